"""Uneven batching (c4 workload): three independent inversions on 96x96,
150x100 and 256x128 grids (nt 800 / 1200 / 1600, 4 / 6 / 8 shots, 32 particles
each) share every launch of the time-stepping kernel; tile shape from the
autotuner; sSVGD of the three 32-particle ensembles with FP64 Cholesky.

Checks: the batch equals each problem run alone with the same tile shape, bit
for bit; sampled particles match the FP64 oracle (<= 1e-4); graph replays of
the batch equal eager; the autotuner's choice is persisted and reused; the
sSVGD batch matches the oracle per ensemble with the same normals."""
import os

import numpy as np
import pytest
import torch

from oracle import cref
from oracle import svgd as osvgd
from paper_2310_13325_amd import autotune
from paper_2310_13325_amd import binding as vb
from paper_2310_13325_amd import configs, synth
from tests.cases import build_case_c, workers
from tests.gpu_helpers import ctx, dev, grid_geom, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c4():
    cases = [build_case_c(p) for p in configs.C4]
    c = ctx()
    probs = []
    for case in cases:
        grid, geom = grid_geom(c, case)
        probs.append(vb.Problem(grid, geom, dev(case.particles), dev(case.dobs), case.sigma,
                                lo=dev(case.lo), hi=dev(case.hi)))
    return cases, probs


def _fresh(probs):
    return [vb.Problem(p.grid, p.geom, p.vel, p.dobs, p.sigma, p.lo, p.hi) for p in probs]


def test_batch_autotuned_equals_separate_runs_and_oracle(c4, tmp_path):
    cases, probs = c4
    c = ctx()
    table = autotune.TileTable(str(tmp_path / "tiles.json"))
    key = autotune.key_for_batch(probs)
    best = autotune.tune(c, lambda: vb.vip_grad_logpost_multi(c, _fresh(probs), ckpt_every=50),
                         key, table, tiles=range(vb.lib().vip_tile_count()))
    print(f"c4 autotuned tile {best}: {table.entries[key]['ms']}", flush=True)
    assert os.path.exists(table.path)
    assert autotune.TileTable(table.path).get(key) == best
    batch = _fresh(probs)
    vb.vip_grad_logpost_multi(c, batch, ckpt_every=50)
    for k, (case, p) in enumerate(zip(cases, batch)):
        lp, g = vb.vip_grad_logpost(c, p.grid, p.geom, p.vel, p.dobs, p.sigma, ckpt_every=50,
                                    lo=p.lo, hi=p.hi, ws_tag=f"single{k}")
        assert torch.equal(lp, p.logpost) and torch.equal(g, p.grad), k
        # FP64 oracle on two sampled particles
        sel = [0, case.particles.shape[0] - 1]
        lp_ref, g_ref = cref.grad_logpost(case.particles[sel], case.ogrid, case.ogeom, case.dobs,
                                          case.sigma, workers=workers())
        gg = p.grad.cpu().numpy()[sel]
        for j in range(2):
            e = rel(gg[j], g_ref[j])
            print(f"c4 problem {k} particle {sel[j]}: grad rel L2 {e:.2e}", flush=True)
            assert e <= 1e-4
        assert np.allclose(p.logpost.cpu().numpy()[sel], lp_ref, rtol=1e-5, atol=0)
    c.set_tile(-2)


def test_batch_graph_replay_equals_eager(c4):
    _, probs = c4
    eager, graph = ctx(False), ctx(True)
    a = _fresh(probs)
    vb.vip_grad_logpost_multi(eager, a, ckpt_every=50, ws_tag="multi_e")
    b = _fresh(probs)
    for rep in range(3):
        vb.vip_grad_logpost_multi(graph, b, ckpt_every=50, ws_tag="multi_g")
        torch.cuda.synchronize()
        for pa, pb in zip(a, b):
            assert torch.equal(pa.logpost, pb.logpost) and torch.equal(pa.grad, pb.grad), rep


def test_ssvgd_batch_with_cholesky_matches_oracle(c4):
    cases, probs = c4
    c = ctx()
    batch = _fresh(probs)
    # seeded gradient-like inputs on both sides (a pull towards the true model
    # plus noise); the batched gradients are checked in the test above
    xs, gs, gs_np, xis, eps, los, his = [], [], [], [], [], [], []
    for k, (case, p) in enumerate(zip(cases, batch)):
        n, d = case.particles.shape[0], case.prob.d
        xs.append(p.vel.view(n, d).clone())
        r = np.random.default_rng(case.prob.seed + 101)
        G = np.float32(-(case.particles.reshape(n, d) - case.v_true.reshape(1, d)) / 100.0 ** 2
                       + 1e-4 * r.standard_normal((n, d))).astype(np.float64)
        gs_np.append(G)
        gs.append(dev(G))
        xi = synth.normals(case.prob.seed, n, d).astype(np.float32)
        xis.append(dev(xi))
        eps.append(5.0 / float(np.abs(G).max()))
        los.append(p.lo.view(-1))
        his.append(p.hi.view(-1))
    ws = vb.vip_ssvgd_step_multi(c, xs, gs, eps, xis=xis, lo=los, hi=his,
                                 gram_prec=vb.VIP_GRAM_FP32)
    assert c.poll(ws) == 0
    for k, case in enumerate(cases):
        n, d = case.particles.shape[0], case.prob.d
        xi = synth.normals(case.prob.seed, n, d).astype(np.float32).astype(np.float64)
        Xr, info = osvgd.ssvgd_step(case.particles.reshape(n, d), gs_np[k], eps[k], xi,
                                    case.lo.reshape(-1), case.hi.reshape(-1))
        e = rel(xs[k].cpu().numpy(), Xr)
        print(f"c4 sSVGD ensemble {k} (n={n}, d={d}): x' rel L2 {e:.2e}, cholesky retries "
              f"{info['retries']}", flush=True)
        assert e <= 1e-6
