"""GPU parity of the FWI path (vip_forward, vip_grad_logpost) against the FP64
oracle.  Tolerances: receiver data <= 1e-5 relative L2, gradients <= 1e-4
relative L2 per particle, log-posterior <= 1e-5 relative.

The log-posterior bound follows from the data bound: J = |r|^2 / (2 sigma^2)
with r = d - dobs, so |dJ| / J <= 2 |dd| / |r|, and for particles drawn from
the prior |r| is of the order of |d|."""
import numpy as np
import pytest
import torch

from oracle import fwi as ofwi
from paper_2310_13325_amd import binding as vb
from paper_2310_13325_amd import configs
from tests.cases import build_case, small_problem, f32
from tests.gpu_helpers import ctx, dev, grid_geom, rel

pytestmark = pytest.mark.gpu

WAVE_TOL = 1e-5
GRAD_TOL = 1e-4
LOGPOST_TOL = 1e-5


TILES = [-1] + list(range(7))


def test_ricker_matches_oracle():
    c = ctx()
    w = vb.vip_ricker(c, 700, 1e-3, 10.0).cpu().numpy()
    ref = ofwi.ricker(700, 1e-3, 10.0)
    assert np.abs(w - ref).max() <= 1e-7


def test_forward_c1_matches_oracle():
    case = build_case(configs.C1)
    c = ctx()
    grid, geom = grid_geom(c, case)
    models = np.stack([case.v_true, case.particles[0], case.particles[5]])
    data = vb.vip_forward(c, grid, geom, dev(models)).cpu().numpy()
    for p in range(models.shape[0]):
        ref = ofwi.simulate(models[p], case.ogrid, case.ogeom)
        e = rel(data[p], ref)
        print(f"c1 forward model {p}: rel L2 {e:.3e}", flush=True)
        assert e <= WAVE_TOL
        assert np.all(data[p][:, 0, :] == 0.0)


def _scattered_geometry(prob):
    nx, nz = prob.nx, prob.nz
    src = [(0, 0), (nz - 1, nx - 1), (nz // 2, nx // 3)]
    rec = [(0, 0), (0, nx - 1), (nz - 1, 0), (nz - 1, nx - 1), (2, 5), (2, 6), (nz // 2, 0),
           (nz // 2, nx - 1), (7, 33), (30, 64), (nz - 2, nx // 2), (11, 11)]
    return ofwi.Geometry(src_iz=tuple(s[0] for s in src), src_ix=tuple(s[1] for s in src),
                         rec_iz=tuple(r[0] for r in rec), rec_ix=tuple(r[1] for r in rec),
                         f0=prob.f0)


@pytest.mark.parametrize("tile", TILES)
def test_forward_ragged_grid_scattered_receivers(tile):
    prob = small_problem()
    case = build_case(prob)
    og = _scattered_geometry(prob)
    c = ctx()
    c.set_tile(tile)
    grid = vb.Grid(nx=prob.nx, nz=prob.nz, nt=prob.nt, dx=prob.dx, dt=prob.dt, vmax=case.vmax,
                   nb=prob.nb)
    w = vb.vip_ricker(c, prob.nt, prob.dt, prob.f0)
    geom = vb.Geometry(og.src_iz, og.src_ix, og.rec_iz, og.rec_ix, w)
    data = vb.vip_forward(c, grid, geom, dev(case.particles)).cpu().numpy()
    for p in range(case.particles.shape[0]):
        ref = ofwi.simulate(case.particles[p], case.ogrid, og)
        e = rel(data[p], ref)
        print(f"ragged forward tile {tile} particle {p}: rel L2 {e:.3e}", flush=True)
        assert e <= WAVE_TOL
    c.set_tile(-2)


def _oracle_grad(case, parts):
    return ofwi.grad_logpost(parts, case.ogrid, case.ogeom, case.dobs, case.sigma, case.lo, case.hi)


def test_grad_logpost_c1_matches_oracle():
    case = build_case(configs.C1)
    c = ctx()
    grid, geom = grid_geom(c, case)
    lp, g = vb.vip_grad_logpost(c, grid, geom, dev(case.particles), dev(case.dobs), case.sigma,
                                ckpt_every=50, lo=dev(case.lo), hi=dev(case.hi))
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    lp_ref, g_ref = _oracle_grad(case, case.particles)
    for p in range(case.particles.shape[0]):
        eg = rel(g[p], g_ref[p])
        el = abs(lp[p] - lp_ref[p]) / abs(lp_ref[p])
        print(f"c1 particle {p}: grad rel L2 {eg:.3e}, logpost rel {el:.3e}", flush=True)
        assert eg <= GRAD_TOL and el <= LOGPOST_TOL
    assert c.poll(c.workspace("grad", 0)) == 0


@pytest.mark.parametrize("tile", TILES)
def test_grad_ragged_segments_and_chunks(tile):
    prob = small_problem(nt=181)
    case = build_case(prob)
    c = ctx()
    c.set_tile(tile)
    grid, geom = grid_geom(c, case)
    args = (c, grid, geom, dev(case.particles), dev(case.dobs), case.sigma)
    lp_a, g_a = vb.vip_grad_logpost(*args, ckpt_every=13, live_pairs=4,
                                    lo=dev(case.lo), hi=dev(case.hi), ws_tag="g_a")
    lp_ref, g_ref = _oracle_grad(case, case.particles)
    g_a = g_a.cpu().numpy()
    for p in range(case.particles.shape[0]):
        eg = rel(g_a[p], g_ref[p])
        print(f"ragged tile {tile} particle {p}: grad rel L2 {eg:.3e}", flush=True)
        assert eg <= GRAD_TOL
    assert np.allclose(lp_a.cpu().numpy(), lp_ref, rtol=LOGPOST_TOL, atol=0)
    # chunking pairs does not change any arithmetic: bitwise equal
    lp_b, g_b = vb.vip_grad_logpost(*args, ckpt_every=13, live_pairs=0,
                                    lo=dev(case.lo), hi=dev(case.hi), ws_tag="g_b")
    assert torch.equal(lp_b.cpu(), lp_a.cpu()) and np.array_equal(g_b.cpu().numpy(), g_a)
    # other checkpoint intervals only regroup the FP32 segment sums
    for k in (1, 60, 180, 500):
        _, g_k = vb.vip_grad_logpost(*args, ckpt_every=k, lo=dev(case.lo), hi=dev(case.hi),
                                     ws_tag=f"g_k{k}")
        assert rel(g_k.cpu().numpy(), g_a) <= 1e-6, k
    c.set_tile(-2)


@pytest.mark.parametrize("tile", [-1, 0, 2, 6])
def test_grad_stored_tail_segment(tile):
    """The forward sweep keeps a^n of the last S steps (the blocked kernel stores
    them as it goes, the one-step kernel recomputes them from a checkpoint):
    same gradient as S = 0 up to the regrouping of FP32 segment sums, and the
    oracle's; S covers a multiple of the interval, a ragged value and all steps."""
    prob = small_problem(nt=181)
    case = build_case(prob)
    c = ctx()
    c.set_tile(tile)
    grid, geom = grid_geom(c, case)
    args = (c, grid, geom, dev(case.particles), dev(case.dobs), case.sigma)
    kw = dict(ckpt_every=13, lo=dev(case.lo), hi=dev(case.hi))
    lp0, g0 = vb.vip_grad_logpost(*args, **kw, ws_tag="s0")
    g0 = g0.cpu().numpy()
    lp_ref, g_ref = _oracle_grad(case, case.particles)
    for S in (26, 57, 180):
        c.read_timing()
        c.set_timing(True)
        lp_s, g_s = vb.vip_grad_logpost(*args, **kw, stored_steps=S, ws_tag=f"s{S}")
        c.set_timing(False)
        tm = c.read_timing()
        g_s = g_s.cpu().numpy()
        e0, eo = rel(g_s, g0), max(rel(g_s[p], g_ref[p]) for p in range(g_s.shape[0]))
        print(f"tile {tile} stored {S}: vs S=0 {e0:.2e}, vs oracle {eo:.2e}, "
              f"recompute point-steps {tm['recompute']['point_steps']:.3g}", flush=True)
        assert e0 <= 1e-6 and eo <= GRAD_TOL
        assert np.allclose(lp_s.cpu().numpy(), lp0.cpu().numpy(), rtol=1e-6, atol=0)
        pts = float(grid.nx + 2 * grid.nb) * (grid.nz + 2 * grid.nb) * case.particles.shape[0] * prob.ns
        if tile >= 0:   # the blocked forward stores the tail: only the rest is recomputed
            assert tm["recompute"]["point_steps"] == pts * (prob.nt - 1 - S)
            assert tm["forward_store"]["point_steps"] == pts * S
        else:
            assert tm["recompute"]["point_steps"] == pts * (prob.nt - 1)
    assert c.poll(c.workspace("s180", 0)) == 0
    c.set_tile(-2)


@pytest.mark.parametrize("tile", [-1, 0, 2, 6])
def test_minibatch_shot_subsets_match_oracle(tile):
    """Section 2.4 minibatches: a subset of the shots, read in place from the
    full d_obs, scaled by ns / b (through sigma); every shot in another order
    gives the full-data value."""
    prob = small_problem(nt=181, ns=4)
    case = build_case(prob)
    c = ctx()
    c.set_tile(tile)
    grid, geom = grid_geom(c, case)
    x, dobs = dev(case.particles), dev(case.dobs)
    kw = dict(ckpt_every=13, lo=dev(case.lo), hi=dev(case.hi))
    for shots in ([3, 1], [2], [1, 3, 0, 2]):
        lp, g = vb.vip_grad_logpost_minibatch(c, grid, geom, x, dobs, case.sigma, shots, **kw,
                                              ws_tag="mb")
        lp_ref, g_ref = ofwi.minibatch_grad_logpost(case.particles, case.ogrid, case.ogeom,
                                                    case.dobs, case.sigma, shots, case.lo, case.hi)
        g = g.cpu().numpy()
        e = max(rel(g[p], g_ref[p]) for p in range(g.shape[0]))
        print(f"tile {tile} minibatch {shots}: grad rel L2 {e:.2e}", flush=True)
        assert e <= GRAD_TOL
        assert np.allclose(lp.cpu().numpy(), lp_ref, rtol=LOGPOST_TOL, atol=0)
    lp_f, g_f = vb.vip_grad_logpost(c, grid, geom, x, dobs, case.sigma, **kw, ws_tag="mbf")
    assert rel(g, g_f.cpu().numpy()) <= 1e-6
    assert np.allclose(lp.cpu().numpy(), lp_f.cpu().numpy(), rtol=1e-6, atol=0)
    c.set_tile(-2)


def test_rerun_is_bitwise_identical():
    case = build_case(configs.C1)
    c = ctx()
    grid, geom = grid_geom(c, case)
    args = (c, grid, geom, dev(case.particles), dev(case.dobs), case.sigma)
    lp1, g1 = vb.vip_grad_logpost(*args, ckpt_every=50)
    lp1, g1 = lp1.clone(), g1.clone()
    lp2, g2 = vb.vip_grad_logpost(*args, ckpt_every=50)
    assert torch.equal(lp1, lp2) and torch.equal(g1, g2)


def test_velocity_above_declared_bound_is_flagged():
    case = build_case(configs.C1)
    c = ctx()
    p = case.prob
    grid = vb.Grid(nx=p.nx, nz=p.nz, nt=p.nt, dx=p.dx, dt=p.dt, vmax=2500.0, nb=p.nb)
    w = vb.vip_ricker(c, p.nt, p.dt, p.f0)
    og = case.ogeom
    geom = vb.Geometry(og.src_iz, og.src_ix, og.rec_iz, og.rec_ix, w)
    ws = c.workspace("forward", 0)
    c.poll(ws)
    vb.vip_forward(c, grid, geom, dev(np.full((1, p.nz, p.nx), 2400.0)))
    assert c.poll(c.workspace("forward", 0)) == 0
    vb.vip_forward(c, grid, geom, dev(np.full((1, p.nz, p.nx), 2600.0)))
    assert c.poll(c.workspace("forward", 0)) == vb.VIP_FLAG_VMAX


def test_cfl_violation_is_rejected_before_launch():
    case = build_case(configs.C1)
    c = ctx()
    p = case.prob
    grid = vb.Grid(nx=p.nx, nz=p.nz, nt=p.nt, dx=p.dx, dt=p.dt, vmax=6200.0, nb=p.nb)
    w = vb.vip_ricker(c, p.nt, p.dt, p.f0)
    og = case.ogeom
    geom = vb.Geometry(og.src_iz, og.src_ix, og.rec_iz, og.rec_ix, w)
    with pytest.raises(vb.VipError) as e:
        vb.vip_forward(c, grid, geom, dev(np.full((1, p.nz, p.nx), 2000.0)))
    assert e.value.status == -2


@pytest.mark.parametrize("tile", [-1, 0, 3])
def test_grad_with_dz_unequal_dx(tile):
    """dz != dx: the blocked kernels take each Laplacian pair against 2u with its
    own weight (the fused form that sums the x and z pairs needs dx == dz);
    data, gradients and log-posterior against the oracle on a ragged grid."""
    from paper_2310_13325_amd import synth
    prob = small_problem(nt=181, ns=2)
    case = build_case(prob)
    dz = 12.5
    og = ofwi.Grid(nz=prob.nz, nx=prob.nx, nb=prob.nb, nt=prob.nt, dx=prob.dx, dz=dz, dt=prob.dt,
                   alpha=prob.alpha)
    clean = ofwi.simulate(case.v_true, og, case.ogeom)
    sigma = 0.01 * float(np.sqrt(np.mean(clean ** 2)))
    dobs = f32(clean + sigma * synth.noise(prob))
    c = ctx()
    c.set_tile(tile)
    grid = vb.Grid(nx=prob.nx, nz=prob.nz, nt=prob.nt, dx=prob.dx, dz=dz, dt=prob.dt,
                   vmax=case.vmax, nb=prob.nb, sponge_alpha=prob.alpha)
    _, geom = grid_geom(c, case)
    d = vb.vip_forward(c, grid, geom, dev(case.v_true[None])).cpu().numpy()[0]
    ew = rel(d, clean)
    lp, g = vb.vip_grad_logpost(c, grid, geom, dev(case.particles), dev(dobs), sigma, ckpt_every=13,
                                lo=dev(case.lo), hi=dev(case.hi), ws_tag="dz")
    lp_ref, g_ref = ofwi.grad_logpost(case.particles, og, case.ogeom, dobs, sigma, case.lo, case.hi)
    eg = max(rel(g.cpu().numpy()[p], g_ref[p]) for p in range(g.shape[0]))
    print(f"dz != dx, tile {tile}: data rel L2 {ew:.2e}, grad rel L2 {eg:.2e}", flush=True)
    assert ew <= WAVE_TOL and eg <= GRAD_TOL
    assert np.allclose(lp.cpu().numpy(), lp_ref, rtol=LOGPOST_TOL, atol=0)
    c.set_tile(-2)


def _vertical_line_geometry(prob):
    """Receivers on several rows, including two vertical lines (a borehole
    array: rows 2-12 of column 40 and rows 20-29 of column 0), so that strips
    of the step kernel hold more than one receiver per column."""
    nx, nz = prob.nx, prob.nz
    src = [(0, 3), (nz // 2, nx - 2), (nz - 1, nx // 2)]
    rec = ([(r, 40) for r in range(2, 13)] + [(r, 0) for r in range(20, 30)] +
           [(2, 5), (2, 6), (nz - 1, nx - 1), (11, 11)])
    return ofwi.Geometry(src_iz=tuple(s[0] for s in src), src_ix=tuple(s[1] for s in src),
                         rec_iz=tuple(r[0] for r in rec), rec_ix=tuple(r[1] for r in rec),
                         f0=prob.f0)


def _strips_with_two_receivers(tile, prob, og):
    """Number of (tile, strip, column) cells of the blocked kernel holding two or
    more receivers (checked on the host, so the test knows it exercises them)."""
    ex, ez, rz, tmax = (vb.tile_shape(tile)[k] for k in ("ex", "ez", "rz", "tmax"))
    h = 2 * tmax
    iz = ez - 2 * h
    NZ = prob.nz + 2 * prob.nb
    rows_by_col = {}
    for z, x in zip(og.rec_iz, og.rec_ix):
        rows_by_col.setdefault(x + prob.nb, []).append(z + prob.nb)
    count = 0
    for tz in range(-(-NZ // iz)):
        z0 = tz * iz - h
        for strip in range(ez // rz):
            lo = z0 + strip * rz
            for rows in rows_by_col.values():
                if sum(lo <= r < lo + rz for r in rows) >= 2:
                    count += 1
    return count


@pytest.mark.parametrize("tile", TILES)
def test_grad_vertical_receiver_lines(tile):
    """Several receivers in one column within one strip (the kernel's table path
    for further receivers, in the forward traces and in the adjoint's residual
    injection) and residuals injected on many rows: data and gradients against
    the oracle for every tile shape."""
    from paper_2310_13325_amd import synth
    prob = small_problem(nt=181, ns=3)
    case = build_case(prob)
    og = _vertical_line_geometry(prob)
    if tile >= 0:
        assert _strips_with_two_receivers(tile, prob, og) > 0
    clean = ofwi.simulate(case.v_true, case.ogrid, og)
    sigma = 0.01 * float(np.sqrt(np.mean(clean ** 2)))
    r = np.random.default_rng(11)
    dobs = f32(clean + sigma * r.standard_normal(clean.shape))
    c = ctx()
    c.set_tile(tile)
    grid = vb.Grid(nx=prob.nx, nz=prob.nz, nt=prob.nt, dx=prob.dx, dt=prob.dt, vmax=case.vmax,
                   nb=prob.nb, sponge_alpha=prob.alpha)
    w = vb.vip_ricker(c, prob.nt, prob.dt, prob.f0)
    geom = vb.Geometry(og.src_iz, og.src_ix, og.rec_iz, og.rec_ix, w)
    data = vb.vip_forward(c, grid, geom, dev(case.particles)).cpu().numpy()
    lp, g = vb.vip_grad_logpost(c, grid, geom, dev(case.particles), dev(dobs), sigma,
                                ckpt_every=13, lo=dev(case.lo), hi=dev(case.hi), ws_tag="vline")
    lp_ref, g_ref = ofwi.grad_logpost(case.particles, case.ogrid, og, dobs, sigma, case.lo, case.hi)
    g = g.cpu().numpy()
    for p in range(case.particles.shape[0]):
        ew = rel(data[p], ofwi.simulate(case.particles[p], case.ogrid, og))
        eg = rel(g[p], g_ref[p])
        print(f"vertical lines, tile {tile}, particle {p}: data {ew:.2e}, grad {eg:.2e}", flush=True)
        assert ew <= WAVE_TOL and eg <= GRAD_TOL
    assert np.allclose(lp.cpu().numpy(), lp_ref, rtol=LOGPOST_TOL, atol=0)
    c.set_tile(-2)


def test_logpost_is_minus_infinity_outside_the_uniform_prior():
    """A particle outside its uniform bounds (but below the declared velocity
    bound) has log-posterior -inf, the others keep theirs."""
    case = build_case(configs.C1)
    c = ctx()
    grid, geom = grid_geom(c, case)
    parts = case.particles.copy()
    row = int(np.argmin(case.hi[:, 0]))
    assert case.hi[row, 0] + 1.0 <= case.vmax
    parts[1, row, 7] = case.hi[row, 7] + 1.0
    lp, g = vb.vip_grad_logpost(c, grid, geom, dev(parts), dev(case.dobs), case.sigma,
                                ckpt_every=50, lo=dev(case.lo), hi=dev(case.hi), ws_tag="inf")
    lp = lp.cpu().numpy()
    lp_ref, _ = _oracle_grad(case, parts)
    assert lp_ref[1] == -np.inf and lp[1] == -np.inf
    others = [p for p in range(parts.shape[0]) if p != 1]
    assert np.all(np.isfinite(lp[others]))
    assert np.allclose(lp[others], lp_ref[others], rtol=LOGPOST_TOL, atol=0)
    assert c.poll(c.workspace("inf", 0)) == 0
