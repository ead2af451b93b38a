"""The persistent, pipelined step kernel (tile shape 6) against the kernel that
runs one block per tile (shape 0, the same 112 x 112 extended tile and 8 steps
per launch).  Both do the same operations in the same order on every tile, so
receiver data, log-posteriors and gradients must be bitwise equal:

* on a ragged grid with fewer tiles than compute units (most persistent blocks
  find no tile), forward only and full gradients with checkpoints, chunked
  pairs and stored tails (every sweep mode: forward, forward with a^n store,
  recompute, adjoint);
* on the 240 x 160 padded grid of the benchmark workload with 128 particles and
  10 shots (3,840 tiles per launch, 15 per block), in the benchmark's memory
  schedule and in the recompute schedule.

The first case is also held against the FP64 oracle at the usual tolerances."""
import numpy as np
import pytest
import torch

from oracle import fwi as ofwi
from paper_2310_13325_amd import binding as vb
from paper_2310_13325_amd import configs
from tests.cases import build_case, small_problem
from tests.gpu_helpers import ctx, dev, grid_geom, rel

pytestmark = pytest.mark.gpu

PIPE, BLOCK = 6, 0


def _same_shape():
    a, b = vb.tile_shape(PIPE), vb.tile_shape(BLOCK)
    assert all(a[k] == b[k] for k in ("ex", "ez", "rz", "tmax"))


def _grad(c, tile, args, **kw):
    c.set_tile(tile)
    lp, g = vb.vip_grad_logpost(*args, **kw)
    torch.cuda.synchronize()
    c.set_tile(-2)
    return lp.cpu(), g.cpu()


def test_pipe_forward_and_gradients_bitwise_on_a_ragged_grid():
    _same_shape()
    prob = small_problem(nt=181)
    case = build_case(prob)
    c = ctx()
    grid, geom = grid_geom(c, case)
    x = dev(case.particles)
    outs = {}
    for tile in (BLOCK, PIPE):
        c.set_tile(tile)
        outs[tile] = vb.vip_forward(c, grid, geom, x).cpu()
    c.set_tile(-2)
    assert torch.equal(outs[PIPE], outs[BLOCK])
    ref = ofwi.simulate(case.particles[0], case.ogrid, case.ogeom)
    e = rel(outs[PIPE][0].numpy(), ref)
    print(f"pipe forward vs oracle: {e:.2e}", flush=True)
    assert e <= 1e-5

    args = (c, grid, geom, x, dev(case.dobs), case.sigma)
    lo, hi = dev(case.lo), dev(case.hi)
    for kw in (dict(ckpt_every=13, live_pairs=4), dict(ckpt_every=13, stored_steps=57),
               dict(ckpt_every=50, stored_steps=180, live_pairs=5), dict(ckpt_every=1)):
        a = _grad(c, BLOCK, args, lo=lo, hi=hi, ws_tag="pipe_a", **kw)
        b = _grad(c, PIPE, args, lo=lo, hi=hi, ws_tag="pipe_b", **kw)
        print(f"pipe gradients {kw}: bitwise {torch.equal(a[1], b[1])}", flush=True)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), kw
    lp_ref, g_ref = ofwi.grad_logpost(case.particles, case.ogrid, case.ogeom, case.dobs,
                                      case.sigma, case.lo, case.hi)
    g = b[1].numpy()
    for p in range(g.shape[0]):
        e = rel(g[p], g_ref[p])
        print(f"pipe particle {p}: grad vs oracle {e:.2e}", flush=True)
        assert e <= 1e-4
    for tag in ("pipe_a", "pipe_b"):
        assert c.poll(c.workspace(tag, 0)) == 0
        c._ws.pop(tag, None)


def test_pipe_bitwise_with_many_tiles_per_block():
    """The benchmark grid and ensemble with a shorter record (0.6 s, long
    enough for the direct wave to reach the receivers at 360 m): every
    persistent block steps 15 tiles per launch, and its loads for the next
    tile overlap the current one's steps."""
    base = configs.C2
    prob = configs.Problem("c2short", nx=base.nx, nz=base.nz, dx=base.dx, nt=301, dt=base.dt,
                           ns=base.ns, np=base.np, f0=base.f0, src_iz=base.src_iz,
                           rec_iz=base.rec_iz, model=base.model, prior=base.prior,
                           noise=base.noise, seed=base.seed, water_rows=base.water_rows)
    case = build_case(prob)
    assert case.particles.shape[0] == 128
    c = ctx()
    grid, geom = grid_geom(c, case)
    # the noise rule of the full record (2 % of the median trace maximum) gives
    # almost nothing here, where most traces are still quiet: 2 % of the
    # largest sample instead
    sigma = 0.02 * float(np.abs(case.dobs).max())
    args = (c, grid, geom, dev(case.particles), dev(case.dobs), sigma)
    lo, hi = dev(case.lo), dev(case.hi)
    for kw in (dict(ckpt_every=50, stored_steps=prob.nt - 1, live_pairs=640),
               dict(ckpt_every=50)):
        a = _grad(c, BLOCK, args, lo=lo, hi=hi, ws_tag="pipe_c", **kw)
        b = _grad(c, PIPE, args, lo=lo, hi=hi, ws_tag="pipe_d", **kw)
        assert torch.isfinite(a[0]).all() and torch.isfinite(a[1]).all()
        same = torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        if not same:
            d = (a[1] - b[1]).abs().reshape(a[1].shape[0], -1).amax(dim=1)
            print(f"pipe c2short {kw}: particles differing {int((d > 0).sum())}", flush=True)
        print(f"pipe c2short {kw}: bitwise {same}", flush=True)
        assert same, kw
        for tag in ("pipe_c", "pipe_d"):
            assert c.poll(c.workspace(tag, 0)) == 0
            c._ws.pop(tag, None)
    torch.cuda.empty_cache()


def test_pipe_batch_of_uneven_problems_bitwise_equals_single_runs():
    """Three problems of different grids, record lengths and shot counts in
    one batched call with shape 6: launches whose problems share the sweep mode
    run the persistent kernel over all their tiles (a block's run crosses from
    one problem to the next), the others the one-block-per-tile batch kernel;
    either way each problem's result is bitwise its single-problem result."""
    c = ctx()
    cases = [build_case(small_problem("u1", nx=70, nz=37, nt=181, ns=3, seed=11)),
             build_case(small_problem("u2", nx=90, nz=50, nt=150, ns=2, seed=12)),
             build_case(small_problem("u3", nx=120, nz=64, nt=201, ns=4, seed=13))]
    probs = []
    for case in cases:
        grid, geom = grid_geom(c, case)
        probs.append(vb.Problem(grid, geom, dev(case.particles), dev(case.dobs), case.sigma,
                                lo=dev(case.lo), hi=dev(case.hi)))
    c.set_tile(PIPE)
    for k in (13, 50):
        vb.vip_grad_logpost_multi(c, probs, ckpt_every=k)
        torch.cuda.synchronize()
        for j, p in enumerate(probs):
            lp, g = vb.vip_grad_logpost(c, p.grid, p.geom, p.vel, p.dobs, p.sigma, ckpt_every=k,
                                        lo=p.lo, hi=p.hi, ws_tag=f"pipe_single{j}")
            same = torch.equal(lp, p.logpost) and torch.equal(g, p.grad)
            print(f"pipe batch k={k} problem {j}: bitwise {same}", flush=True)
            assert same, (k, j)
    c.set_tile(-2)
    for j in range(3):
        c._ws.pop(f"pipe_single{j}", None)


def _layout_case(kind):
    """Receiver and sponge layouts that take each path of the persistent
    kernel's tile set-up: receivers on three rows sharing columns (the LDS
    receiver tables, with several receivers of one column in one strip), a
    borehole line of 11 rows plus other rows (more receiver rows than the LDS
    tables hold: ids from global memory), and a 64-cell sponge (wider than the
    LDS profile: sponge factors from global memory)."""
    if kind == "wide_sponge":
        prob = configs.Problem("wide_sponge", nx=40, nz=30, dx=10.0, nt=121, dt=1e-3, ns=2, np=3,
                               f0=18.0, src_iz=1, rec_iz=2, model="layers_anomalies",
                               prior="rowmean_pm500", noise="rms_1pct", seed=21, nb=64)
        case = build_case(prob)
        return prob, case, case.ogeom
    prob = small_problem(nt=151, ns=3)
    case = build_case(prob)
    nx, nz = prob.nx, prob.nz
    src = [(0, 3), (nz // 2, nx - 2), (nz - 1, nx // 2)]
    if kind == "rows3":
        rec = [(z, x) for z in (2, 5, 9) for x in range(4, nx - 4, 3)] + [(nz - 1, 7)]
    else:
        rec = ([(r, 40) for r in range(2, 13)] + [(r, 0) for r in range(20, 30)] +
               [(2, 5), (2, 6), (nz - 1, nx - 1)])
    og = ofwi.Geometry(src_iz=tuple(s[0] for s in src), src_ix=tuple(s[1] for s in src),
                       rec_iz=tuple(r[0] for r in rec), rec_ix=tuple(r[1] for r in rec), f0=prob.f0)
    return prob, case, og


@pytest.mark.parametrize("kind", ["rows3", "many_rows", "wide_sponge"])
def test_pipe_bitwise_across_receiver_and_sponge_layouts(kind):
    _same_shape()
    prob, case, og = _layout_case(kind)
    nrows = len(set(og.rec_iz))
    two_in_strip = kind != "wide_sponge"
    print(f"layout {kind}: {nrows} receiver rows, sponge {prob.nb}", flush=True)
    clean = ofwi.simulate(case.v_true, case.ogrid, og)
    sigma = 0.01 * float(np.sqrt(np.mean(clean ** 2)))
    dobs = (clean + sigma * np.random.default_rng(5).standard_normal(clean.shape)).astype(np.float32)
    c = ctx()
    grid = vb.Grid(nx=prob.nx, nz=prob.nz, nt=prob.nt, dx=prob.dx, dt=prob.dt, vmax=case.vmax,
                   nb=prob.nb, sponge_alpha=prob.alpha)
    w = vb.vip_ricker(c, prob.nt, prob.dt, prob.f0)
    geom = vb.Geometry(og.src_iz, og.src_ix, og.rec_iz, og.rec_ix, w)
    x = dev(case.particles)
    outs = {}
    for tile in (BLOCK, PIPE):
        c.set_tile(tile)
        outs[tile] = vb.vip_forward(c, grid, geom, x).cpu()
    c.set_tile(-2)
    assert torch.equal(outs[PIPE], outs[BLOCK]), kind
    args = (c, grid, geom, x, dev(dobs), sigma)
    lo, hi = dev(case.lo), dev(case.hi)
    for kw in (dict(ckpt_every=13), dict(ckpt_every=50, stored_steps=prob.nt - 1)):
        a = _grad(c, BLOCK, args, lo=lo, hi=hi, ws_tag="pipe_l0", **kw)
        b = _grad(c, PIPE, args, lo=lo, hi=hi, ws_tag="pipe_l6", **kw)
        same = torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        print(f"layout {kind} {kw}: bitwise {same}", flush=True)
        assert same, (kind, kw)
    lp_ref, g_ref = ofwi.grad_logpost(case.particles, case.ogrid, og, dobs, sigma, case.lo, case.hi)
    for p in range(g_ref.shape[0]):
        ew = rel(outs[PIPE][p].numpy(), ofwi.simulate(case.particles[p], case.ogrid, og))
        eg = rel(b[1][p].numpy(), g_ref[p])
        print(f"layout {kind} particle {p}: data {ew:.2e}, grad {eg:.2e}", flush=True)
        assert ew <= 1e-5 and eg <= 1e-4
    if two_in_strip:
        # (the host-side count of strips holding two receivers of one column)
        from tests.test_gpu_fwi import _strips_with_two_receivers
        assert _strips_with_two_receivers(PIPE, prob, og) > 0
    for tag in ("pipe_l0", "pipe_l6"):
        c._ws.pop(tag, None)
