"""Differentiation pattern (c3 workload: 400x200 at 12.5 m, nt = 4000, 20 shots,
400 receivers, checkpoints every 50 steps): the torch.autograd op built on the
checkpointed adjoint agrees with vip_grad_logpost, with the FP64 oracle
gradient (<= 1e-4 relative L2) and with central differences of the library's
own forward on 32 cells (edges and corners included)."""
import numpy as np
import pytest
import torch

from oracle import cref
from paper_2310_13325_amd import binding as vb
from paper_2310_13325_amd import configs, synth
from paper_2310_13325_amd.autograd import FwiOperator, fwi_forward
from tests.cases import build_case_c, workers
from tests.gpu_helpers import ctx, dev, grid_geom, rel

pytestmark = pytest.mark.gpu


def _misfit(data, dobs, sigma):
    r = data.double() - dobs.double()
    return 0.5 * (r * r).sum() / sigma ** 2


def test_c3_autograd_against_adjoint_oracle_and_differences():
    prob = configs.C3
    case = build_case_c(prob, 1)
    c = ctx()
    grid, geom = grid_geom(c, case)
    dobs = dev(case.dobs)
    op = FwiOperator(c, grid, geom, ckpt_every=50)
    vel = dev(case.particles).requires_grad_(True)
    data = fwi_forward(vel, op)
    loss = _misfit(data[0], dobs, case.sigma)
    loss.backward()
    g_auto = vel.grad.detach().cpu().numpy().astype(np.float64)[0]
    print(f"c3 autograd: loss {loss.item():.6e}", flush=True)

    # same gradient through vip_grad_logpost (residual and misfit on the device)
    lp, g = vb.vip_grad_logpost(c, grid, geom, vel.detach(), dobs, case.sigma, ckpt_every=50,
                                ws_tag="c3")
    assert rel(-g.cpu().numpy()[0], g_auto) <= 1e-6
    assert abs(-lp.item() - loss.item()) <= 1e-6 * loss.item()

    # FP64 oracle (C, threads over shots)
    lp_ref, g_ref = cref.grad_logpost(case.particles, case.ogrid, case.ogeom, case.dobs,
                                      case.sigma, workers=workers())
    e = rel(g_auto, -g_ref[0])
    print(f"c3 autograd vs oracle: rel L2 {e:.3e}; misfit rel {abs(loss.item() + lp_ref[0]) / abs(lp_ref[0]):.2e}",
          flush=True)
    assert e <= 1e-4
    assert abs(loss.item() + lp_ref[0]) <= 1e-5 * abs(lp_ref[0])

    # central differences of the library's forward, all 64 perturbed models in one call
    cells = synth.fd_cells(prob, 32)
    delta = 1.0
    models = np.repeat(case.particles, 64, axis=0)
    for k, (i, j) in enumerate(cells):
        models[2 * k, i, j] += delta
        models[2 * k + 1, i, j] -= delta
    with torch.no_grad():
        d = vb.vip_forward(c, grid, geom, dev(models))
        r = d.double() - dobs.double()[None]
        J = 0.5 * (r * r).sum(dim=(1, 2, 3)).cpu().numpy() / case.sigma ** 2
    gmax = np.abs(g_auto).max()
    worst = 0.0
    for k, (i, j) in enumerate(cells):
        fd = (J[2 * k] - J[2 * k + 1]) / (2 * delta)
        worst = max(worst, abs(fd - g_auto[i, j]) / gmax)
    print(f"c3 central differences: worst |fd - g| / max|g| = {worst:.2e}", flush=True)
    assert worst <= 1e-3


def test_autograd_forwards_before_backwards_keep_their_own_tapes():
    """Two forwards (the second with more particles) before one backward: each
    backward runs on its own forward's checkpoints, bit for bit the gradient
    of that forward taken alone."""
    from tests.cases import build_case, small_problem
    case = build_case(small_problem("tapes", nx=50, nz=33, nt=140, ns=2, np_=4))
    c = ctx()
    grid, geom = grid_geom(c, case)
    dobs = dev(case.dobs)
    op = FwiOperator(c, grid, geom, ckpt_every=13)
    v1 = dev(case.particles[:2]).requires_grad_(True)
    v2 = dev(case.particles[1:4]).requires_grad_(True)
    loss = (_misfit(fwi_forward(v1, op), dobs[None], case.sigma)
            + 2.0 * _misfit(fwi_forward(v2, op), dobs[None], case.sigma))
    loss.backward()
    refs = []
    for v, w in ((case.particles[:2], 1.0), (case.particles[1:4], 2.0)):
        vr = dev(v).requires_grad_(True)
        (w * _misfit(fwi_forward(vr, op), dobs[None], case.sigma)).backward()
        refs.append(vr.grad)
    assert torch.equal(v1.grad, refs[0]) and torch.equal(v2.grad, refs[1])


def test_c3_autograd_all_64_particles():
    """The differentiation workload at its stated size: 64 particles x 20 shots,
    checkpoints every 50 steps (an 85 GB tape).  Sampled particles against the
    FP64 oracle (gradient <= 1e-4, misfit <= 1e-5); all 64 against
    vip_grad_logpost (the same adjoint through the library's own residual)."""
    prob = configs.C3
    case = build_case_c(prob)
    assert case.particles.shape[0] == 64
    c = ctx()
    grid, geom = grid_geom(c, case)
    dobs = dev(case.dobs)
    op = FwiOperator(c, grid, geom, ckpt_every=50)
    vel = dev(case.particles).requires_grad_(True)
    print("c3 autograd: 64 particles forward", flush=True)
    data = fwi_forward(vel, op)
    J = 0.5 * ((data - dobs[None]) ** 2).sum(dim=(1, 2, 3)) / case.sigma ** 2
    J.sum().backward()
    J = J.detach().cpu().numpy().astype(np.float64)
    g_auto = vel.grad.detach().cpu().numpy().astype(np.float64)
    del data, vel
    op._ws = None
    torch.cuda.empty_cache()
    print("c3 autograd: backward done", flush=True)

    sampled = [0, 31, 63]
    lp_ref, g_ref = cref.grad_logpost(case.particles[sampled], case.ogrid, case.ogeom, case.dobs,
                                      case.sigma, workers=workers())
    for k, p in enumerate(sampled):
        e = rel(g_auto[p], -g_ref[k])
        ej = abs(J[p] + lp_ref[k]) / abs(lp_ref[k])
        print(f"c3 autograd particle {p}: grad rel L2 {e:.2e}, misfit rel {ej:.2e}", flush=True)
        assert e <= 1e-4 and ej <= 1e-5

    lp, g = vb.vip_grad_logpost(c, grid, geom, dev(case.particles), dobs, case.sigma,
                                ckpt_every=50, live_pairs=640, ws_tag="c3all")
    g = g.cpu().numpy()
    c._ws.pop("c3all", None)
    torch.cuda.empty_cache()
    worst = max(rel(-g[p], g_auto[p]) for p in range(64))
    print(f"c3 autograd vs vip_grad_logpost, 64 particles: worst {worst:.2e}", flush=True)
    assert worst <= 1e-5
