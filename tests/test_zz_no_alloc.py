"""The allocation-free SVGD step (vip_svgd_step_noalloc, the library's fixed
per-device array in place of a caller workspace) against vip_svgd_step with a
workspace: the same kernels on the same inputs give the same particles and
bandwidth bit for bit.  Two calls in a row, the second on a smaller ensemble,
so the second runs on an array still holding the first call's contents; both
Gram precisions, with and without the clip prior; a step whose workspace
would exceed the array is rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_2310_13325_amd import binding as vb
from tests.gpu_helpers import ctx, dev

pytestmark = pytest.mark.gpu


def _ensemble(n, d, seed):
    r = np.random.default_rng(seed)
    X = np.float32(3000.0 + 100.0 * r.standard_normal((n, d)))
    G = np.float32(-(X - 3000.0) / 1e4 + 1e-4 * r.standard_normal((n, d)))
    return X, G


@pytest.mark.parametrize("prec", [vb.VIP_GRAM_BF16, vb.VIP_GRAM_FP32])
@pytest.mark.parametrize("clip", [False, True])
def test_noalloc_step_equals_workspace_step(prec, clip):
    c = ctx()
    for n, d, seed in ((128, 24000, 1), (37, 4101, 2)):   # the second call smaller
        print(f"noalloc step: n={n} d={d} gram_prec={prec} clip={clip}", flush=True)
        X, G = _ensemble(n, d, seed)
        lo = dev(np.full(d, 2850.0)) if clip else None
        hi = dev(np.full(d, 3150.0)) if clip else None
        g = dev(G)
        x_ref, x_na = dev(X), dev(X)
        h2_ref = torch.zeros(1, dtype=torch.float64, device="cuda")
        h2_na = torch.zeros(1, dtype=torch.float64, device="cuda")
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        ws = vb.vip_svgd_step(c, x_ref, g, 2000.0, gram_prec=prec, lo=lo, hi=hi, h2_out=h2_ref,
                              ws_tag="noalloc_ref")
        vb.vip_svgd_step_noalloc(c, x_na, g, 2000.0, gram_prec=prec, lo=lo, hi=hi, h2_out=h2_na,
                                 status=status)
        torch.cuda.synchronize()
        assert c.poll(ws) == 0 and int(status.item()) == 0
        assert torch.equal(h2_ref, h2_na)
        assert torch.equal(x_ref, x_na)
        assert not torch.equal(x_na, dev(X))          # the step moved the particles
    c._ws.pop("noalloc_ref", None)


def test_noalloc_step_rejects_ensembles_beyond_the_array():
    c = ctx()
    n, d = 256, 24000
    assert vb.svgd_workspace_bytes(n, d) > vb.VIP_NOALLOC_SCRATCH_BYTES
    x = torch.ones(n, d, device="cuda")
    g = torch.zeros(n, d, device="cuda")
    with pytest.raises(vb.VipError) as e:
        vb.vip_svgd_step_noalloc(c, x, g, 1.0)
    assert e.value.status == -8
    torch.cuda.synchronize()
    assert bool((x == 1.0).all())
