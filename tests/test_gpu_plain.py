"""The plain per-pair GPU path computes the same gradient as the batched path
(same scheme in FP32; the plain path sums the Laplacian in the difference form
and the imaging term in FP64 directly, the batched path takes each symmetric
pair against 2u and sums the imaging term per checkpoint segment) and both
match the FP64 oracle."""
import numpy as np
import pytest

from oracle import fwi as ofwi
from paper_2310_13325_amd import binding as vb
from tests.cases import build_case, small_problem
from tests.gpu_helpers import ctx, dev, grid_geom, rel

pytestmark = pytest.mark.gpu


def test_plain_path_matches_oracle_and_batched_path():
    prob = small_problem("plain", nx=52, nz=41, nt=160, ns=2, np_=2)
    case = build_case(prob)
    c = ctx()
    grid, geom = grid_geom(c, case)
    args = (c, grid, geom, dev(case.particles), dev(case.dobs), case.sigma)
    lp_p, g_p = vb.vip_grad_logpost_plain(*args, lo=dev(case.lo), hi=dev(case.hi))
    lp_b, g_b = vb.vip_grad_logpost(*args, ckpt_every=20, lo=dev(case.lo), hi=dev(case.hi))
    lp_ref, g_ref = ofwi.grad_logpost(case.particles, case.ogrid, case.ogeom, case.dobs,
                                      case.sigma, case.lo, case.hi)
    g_p, g_b = g_p.cpu().numpy(), g_b.cpu().numpy()
    for p in range(case.particles.shape[0]):
        assert rel(g_p[p], g_ref[p]) <= 1e-4
        assert rel(g_p[p], g_b[p]) <= 1e-5
    assert np.allclose(lp_p.cpu().numpy(), lp_ref, rtol=1e-5, atol=0)
    assert np.allclose(lp_b.cpu().numpy(), lp_ref, rtol=1e-5, atol=0)
    # Two FP32 roundings of the same misfit: each is within the data error of
    # the oracle (|dJ|/J <= 2 |dd|/|r|, about 1e-6 here), so they agree to 1e-6.
    assert np.allclose(lp_p.cpu().numpy(), lp_b.cpu().numpy(), rtol=1e-6, atol=0)
