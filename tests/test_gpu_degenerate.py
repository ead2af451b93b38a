"""Degenerate FWI shapes against the FP64 oracle, for the one-step kernel, the
blocked kernel at two tile shapes and the persistent kernel:

* a grid far smaller than one tile (6 x 5 cells, a 2-cell sponge) with one
  particle, one shot, and nt = 3 (two time steps: the shortest record the
  interface takes that lets a receiver next to the source see it);
* a 3 x 3 grid with no sponge at all (nb = 0), two particles;
* sources and receivers in the grid's corners and on its edges, two shots,
  with the receivers on three rows (the first and last of them the grid's).

Receiver data to 1e-5 and gradients to 1e-4 relative L2 (the stated
tolerances), log-posteriors to 1e-5."""
import numpy as np
import pytest

from oracle import fwi as ofwi
from paper_2310_13325_amd import binding as vb
from paper_2310_13325_amd import configs
from tests.cases import build_case
from tests.gpu_helpers import ctx, dev, rel

pytestmark = pytest.mark.gpu

TILES = [-1, 0, 3, 6]


def _case(kind):
    if kind == "tiny_nt3":
        prob = configs.Problem("tiny_nt3", nx=6, nz=5, dx=10.0, nt=3, dt=1e-3, ns=1, np=1, f0=18.0,
                               src_iz=1, rec_iz=2, model="layers_anomalies", prior="rowmean_pm500",
                               noise="rms_1pct", seed=3, nb=2)
        case = build_case(prob)
        return prob, case, case.ogeom
    if kind == "no_sponge":
        prob = configs.Problem("no_sponge", nx=3, nz=3, dx=10.0, nt=40, dt=1e-3, ns=1, np=2, f0=18.0,
                               src_iz=0, rec_iz=0, model="layers_anomalies", prior="rowmean_pm500",
                               noise="rms_1pct", seed=4, nb=0)
        case = build_case(prob)
        return prob, case, case.ogeom
    prob = configs.Problem("corners", nx=9, nz=7, dx=10.0, nt=60, dt=1e-3, ns=2, np=2, f0=18.0,
                           src_iz=1, rec_iz=2, model="layers_anomalies", prior="rowmean_pm500",
                           noise="rms_1pct", seed=5, nb=3)
    case = build_case(prob)
    nx, nz = prob.nx, prob.nz
    src = [(0, 0), (nz - 1, nx - 1)]
    rec = [(0, nx - 1), (nz - 1, 0), (0, 0), (nz - 1, nx - 1), (nz // 2, 0), (nz // 2, nx - 1),
           (0, nx // 2)]
    og = ofwi.Geometry(src_iz=tuple(s[0] for s in src), src_ix=tuple(s[1] for s in src),
                       rec_iz=tuple(r[0] for r in rec), rec_ix=tuple(r[1] for r in rec), f0=prob.f0)
    return prob, case, og


@pytest.mark.parametrize("kind", ["tiny_nt3", "no_sponge", "corners"])
@pytest.mark.parametrize("tile", TILES)
def test_degenerate_shapes_match_oracle(kind, tile):
    prob, case, og = _case(kind)
    clean = ofwi.simulate(case.v_true, case.ogrid, og)
    # noise at 1 % of the clean data's RMS (or of its largest sample when the
    # record is too short for the wave to arrive in most traces)
    scale = float(np.sqrt(np.mean(clean ** 2))) or float(np.abs(clean).max())
    sigma = 0.01 * scale
    dobs = (clean + sigma * np.random.default_rng(9).standard_normal(clean.shape)).astype(np.float32)
    c = ctx()
    c.set_tile(tile)
    grid = vb.Grid(nx=prob.nx, nz=prob.nz, nt=prob.nt, dx=prob.dx, dt=prob.dt, vmax=case.vmax,
                   nb=prob.nb, sponge_alpha=prob.alpha)
    w = vb.vip_ricker(c, prob.nt, prob.dt, prob.f0)
    geom = vb.Geometry(og.src_iz, og.src_ix, og.rec_iz, og.rec_ix, w)
    x = dev(case.particles)
    data = vb.vip_forward(c, grid, geom, x).cpu().numpy()
    lp, g = vb.vip_grad_logpost(c, grid, geom, x, dev(dobs), sigma, ckpt_every=2,
                                lo=dev(case.lo), hi=dev(case.hi), ws_tag="degenerate")
    c.set_tile(-2)
    lp_ref, g_ref = ofwi.grad_logpost(case.particles, case.ogrid, og, dobs, sigma, case.lo, case.hi)
    g = g.cpu().numpy()
    for p in range(case.particles.shape[0]):
        ew = rel(data[p], ofwi.simulate(case.particles[p], case.ogrid, og))
        eg = rel(g[p], g_ref[p])
        print(f"{kind}, tile {tile}, particle {p}: data {ew:.2e}, grad {eg:.2e}", flush=True)
        assert np.isfinite(g[p]).all()
        assert ew <= 1e-5 and eg <= 1e-4, (kind, tile, p, ew, eg)
    assert np.allclose(lp.cpu().numpy(), lp_ref, rtol=1e-5, atol=0)
    c._ws.pop("degenerate", None)
