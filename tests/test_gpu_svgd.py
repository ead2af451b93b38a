"""GPU parity of the SVGD / sSVGD update (vip_svgd_step, vip_ssvgd_step) against
the FP64 oracle, and of the Philox generator against the oracle's.

Tolerances (relative L2 unless stated):
  FP32 Gram: D <= 1e-5, K <= 1e-5, phi <= 1e-4, x' <= 1e-6 (x' ~ 3e3, update ~ 1e1);
  BF16 Gram (d >= 4096): D <= 2e-4, K <= 2e-3, phi <= 2e-3, x' <= 1e-5.
BF16 keeps 8 significant bits: the centred coordinates carry a relative
rounding error of about 1e-3 each, which averages to about 2e-3/sqrt(d) in a
squared distance, and K amplifies a relative error of D by D / (2 h^2)
(about ln(n+1) at the median).
The median bandwidth is checked exactly: h^2 must equal the median rule applied
to the library's own distance matrix, so the radix select is pinned bit for bit.
"""
import math

import numpy as np
import pytest
import torch

from oracle import philox as ophilox
from oracle import svgd as osvgd
from paper_2310_13325_amd import binding as vb
from tests.gpu_helpers import ctx, dev, rel

pytestmark = pytest.mark.gpu


def _ensemble(n, d, seed, spread=100.0, base=3000.0):
    r = np.random.default_rng(seed)
    X = base + spread * r.standard_normal((n, d))
    G = -(X - base) / spread ** 2 + 0.01 * r.standard_normal((n, d))
    f = lambda a: a.astype(np.float32).astype(np.float64)
    return f(X), f(G)


def _inspect(ws, n, d):
    lay = vb.svgd_layout(n, d)
    D = vb.workspace_view(ws, lay.D, n * n, torch.float32).cpu().numpy().reshape(n, n)
    K = vb.workspace_view(ws, lay.K, n * n, torch.float32).cpu().numpy().reshape(n, n)
    h2 = float(vb.workspace_view(ws, lay.h2, 1, torch.float64).cpu().numpy()[0])
    phi = vb.workspace_view(ws, lay.phi, n * d, torch.float32).cpu().numpy().reshape(n, d)
    L = vb.workspace_view(ws, lay.L, n * n, torch.float64).cpu().numpy().reshape(n, n)
    return D, K, h2, phi, L


def _run(n, d, seed, gram, eps=50.0, mode=vb.VIP_BW_MEDIAN_ALL, prior=False):
    X, G = _ensemble(n, d, seed)
    lo = hi = None
    if prior:
        lo = np.full(d, 2990.0, dtype=np.float32).astype(np.float64)
        hi = np.full(d, 3010.0, dtype=np.float32).astype(np.float64)
    c = ctx()
    x = dev(X)
    h2o = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = vb.vip_svgd_step(c, x, dev(G), eps, bw_mode=mode, gram_prec=gram,
                          lo=None if lo is None else dev(lo), hi=None if hi is None else dev(hi),
                          h2_out=h2o, ws_tag=f"svgd{n}_{d}")
    D, K, h2, phi, _ = _inspect(ws, n, d)
    Xn = x.cpu().numpy().astype(np.float64)
    assert h2o.item() == h2
    Xr, info = osvgd.svgd_step(X, G, eps, lo, hi, mode=mode)
    return dict(D=D, K=K, h2=h2, phi=phi, X=Xn), dict(D=info["D"], K=info["K"], h2=info["h2"],
                                                      phi=info["phi"], X=Xr), c, ws


def _median_rule(D, n, mode):
    vals = D[np.triu_indices(n, 1)] if mode == vb.VIP_BW_MEDIAN_OFFDIAG else D.ravel()
    med = float(np.median(vals.astype(np.float64))) if vals.size else 0.0
    return 1.0 if med == 0.0 else med / (2.0 * math.log(n + 1.0))


@pytest.mark.parametrize("n,d", [(7, 37), (64, 1000), (130, 515), (300, 777)])
def test_svgd_fp32_gram_matches_oracle(n, d):
    g, r, c, ws = _run(n, d, seed=n + d, gram=vb.VIP_GRAM_FP32)
    print(f"fp32 n={n} d={d}: D {rel(g['D'], r['D']):.2e} K {rel(g['K'], r['K']):.2e} "
          f"phi {rel(g['phi'], r['phi']):.2e} X {rel(g['X'], r['X']):.2e}", flush=True)
    assert rel(g["D"], r["D"]) <= 1e-5
    assert rel(g["K"], r["K"]) <= 1e-5
    assert rel(g["phi"], r["phi"]) <= 1e-4
    assert rel(g["X"], r["X"]) <= 1e-6
    assert g["h2"] == pytest.approx(_median_rule(g["D"], n, vb.VIP_BW_MEDIAN_ALL), rel=1e-15)
    assert abs(g["h2"] - r["h2"]) <= 1e-5 * r["h2"]
    assert np.all(np.diag(g["D"]) == 0) and np.array_equal(g["D"], g["D"].T)
    assert c.poll(ws) == 0


@pytest.mark.parametrize("n,d", [(8, 4096), (128, 4096), (300, 4100)])
def test_svgd_bf16_gram_matches_oracle(n, d):
    g, r, c, ws = _run(n, d, seed=3 * n + d, gram=vb.VIP_GRAM_BF16)
    eD, eK, ep, eX = (rel(g[k], r[k]) for k in ("D", "K", "phi", "X"))
    print(f"bf16 n={n} d={d}: D {eD:.2e} K {eK:.2e} phi {ep:.2e} X {eX:.2e}", flush=True)
    assert eD <= 2e-4 and eK <= 2e-3 and ep <= 2e-3 and eX <= 1e-5
    assert g["h2"] == pytest.approx(_median_rule(g["D"], n, vb.VIP_BW_MEDIAN_ALL), rel=1e-15)


@pytest.mark.parametrize("n,d", [(1, 5), (2, 37), (33, 257), (257, 33)])
def test_bf16_path_small_and_ragged_shapes(n, d):
    """The BF16 path (BF16 Gram, split-BF16 update: K rows padded to 32, B
    pairs padded in both directions) on shapes that are not multiples of its
    tiles.  With few coordinates the BF16 Gram is coarse (2^-9 per product,
    little averaging over d), so the bound is phi within 5e-3; indexing and
    padding mistakes show as O(1) errors or non-finite values."""
    g, r, c, ws = _run(n, d, seed=7 * n + d, gram=vb.VIP_GRAM_BF16)
    e_phi = rel(g["phi"], r["phi"])
    print(f"bf16 path n={n} d={d}: phi rel L2 {e_phi:.2e}", flush=True)
    assert np.isfinite(g["phi"]).all() and np.isfinite(g["X"]).all()
    assert e_phi <= 5e-3
    assert c.poll(ws) == 0


@pytest.mark.parametrize("n,d", [(5, 300_001), (2100, 40)])
def test_centring_beyond_the_register_cache(n, d):
    """The centring kernel keeps up to 2048 rows per column in registers and
    addresses X with 32-bit offsets below 2^31 bytes: (5, 300001) exceeds that
    and takes the instance without the cache; (2100, 40) reads its last 52
    rows past the cache.  Both with the RBF kernel and with the diagonal
    matrix-valued kernel (whose variance pass reads the same values)."""
    g, r, c, ws = _run(n, d, seed=n + d, gram=vb.VIP_GRAM_FP32)
    errs = dict(D=rel(g["D"], r["D"]), K=rel(g["K"], r["K"]), phi=rel(g["phi"], r["phi"]),
                X=rel(g["X"], r["X"]))
    print(f"centring n={n} d={d}: {errs}", flush=True)
    assert errs["D"] <= 1e-5 and errs["K"] <= 1e-5 and errs["phi"] <= 1e-4 and errs["X"] <= 1e-6
    assert c.poll(ws) == 0
    X, G = _ensemble(n, d, seed=n + d + 1)
    x = dev(X)
    ws = vb.vip_svgd_step_ex(c, x, dev(G), 50.0, kernel=vb.VIP_KERNEL_DIAG_VAR,
                             gram_prec=vb.VIP_GRAM_FP32)
    D, _, _, phi, _ = _inspect(ws, n, d)
    Xr, info = osvgd.svgd_step_diag(X, G, 50.0)
    e = dict(D=rel(D, info["D"]), phi=rel(phi, info["phi"]), X=rel(x.cpu().numpy() - X, Xr - X))
    print(f"centring, diagonal kernel n={n} d={d}: {e}", flush=True)
    assert e["D"] <= 1e-5 and e["phi"] <= 1e-4 and e["X"] <= 1e-4


@pytest.mark.parametrize("n", [300, 1025, 2048])
@pytest.mark.parametrize("dup", [False, True])
def test_median_exact_at_larger_n(n, dup):
    """The radix select over many blocks (n^2 keys, an odd n leaving a ragged
    tail of keys), both median modes, with and without duplicated particles
    (many equal keys and zeros): h^2 is the median rule applied to the
    library's own D, bit for bit."""
    d = 24
    X, G = _ensemble(n, d, seed=n + 3 * dup)
    if dup:
        X[n // 3:] = X[np.arange(n - n // 3) % 7]   # the last two thirds copy the first 7 rows
    c = ctx()
    for mode in (vb.VIP_BW_MEDIAN_ALL, vb.VIP_BW_MEDIAN_OFFDIAG):
        x = dev(X)
        ws = vb.vip_svgd_step(c, x, dev(G), 1.0, bw_mode=mode, gram_prec=vb.VIP_GRAM_FP32,
                              ws_tag=f"med{n}")
        D, _, h2, _, _ = _inspect(ws, n, d)
        assert np.array_equal(D, D.T) and np.all(np.diag(D) == 0.0)
        assert h2 == _median_rule(D, n, mode), (mode, h2)
        assert c.poll(ws) == 0


def test_bf16_path_with_clip_prior():
    """The split-BF16 update's epilogue with the clip of the uniform prior
    (bounds read once per column): x' within [lo, hi], some coordinates on the
    bounds, and x' against the oracle within the BF16 bound."""
    n, d = 300, 4100
    g, r, c, ws = _run(n, d, seed=17, gram=vb.VIP_GRAM_BF16, eps=50.0, prior=True)
    assert np.all(g["X"] >= np.float32(2990.0)) and np.all(g["X"] <= np.float32(3010.0))
    assert np.any(g["X"] == np.float32(2990.0)) or np.any(g["X"] == np.float32(3010.0))
    e = rel(g["X"], r["X"])
    print(f"bf16 path with clip: x' rel L2 {e:.2e}", flush=True)
    assert e <= 1e-5
    assert c.poll(ws) == 0


@pytest.mark.parametrize("n", [1, 2, 5, 6])
def test_median_modes_small_n(n):
    k12 = {vb.VIP_BW_MEDIAN_ALL: 1.0 / 9.0, vb.VIP_BW_MEDIAN_OFFDIAG: 1.0 / 3.0}
    for mode in (vb.VIP_BW_MEDIAN_ALL, vb.VIP_BW_MEDIAN_OFFDIAG):
        g, r, _, _ = _run(n, 33, seed=11 * n, gram=vb.VIP_GRAM_FP32, mode=mode)
        assert g["h2"] == pytest.approx(_median_rule(g["D"], n, mode), rel=1e-15)
        assert rel(g["X"], r["X"]) <= 1e-6
        if n == 1:
            assert g["h2"] == 1.0 and g["K"][0, 0] == 1.0
        if n == 2:
            assert abs(g["K"][0, 1] - k12[mode]) <= 1e-6


def test_fixed_bandwidth_and_clip():
    n, d = 9, 50
    X, G = _ensemble(n, d, 5, spread=5.0)
    c = ctx()
    lo = np.full(d, 2995.0)
    hi = np.full(d, 3005.0)
    x = dev(X)
    vb.vip_svgd_step(c, x, dev(G), 2000.0, bw_mode=vb.VIP_BW_FIXED, h_fixed=7.0,
                     gram_prec=vb.VIP_GRAM_FP32, lo=dev(lo), hi=dev(hi), ws_tag="svgd_fixed")
    Xr, info = osvgd.svgd_step(X, G, 2000.0, lo, hi, mode=osvgd.BW_FIXED, h_fixed=7.0)
    xg = x.cpu().numpy()
    assert np.all(xg >= 2995.0) and np.all(xg <= 3005.0)
    assert np.any(xg == 2995.0) or np.any(xg == 3005.0)
    assert rel(xg, Xr) <= 1e-6


def test_ssvgd_with_given_normals_matches_oracle():
    n, d, eps = 24, 3001, 20.0
    X, G = _ensemble(n, d, 21)
    xi = np.random.default_rng(22).standard_normal((n, d)).astype(np.float32).astype(np.float64)
    c = ctx()
    x = dev(X)
    ws = vb.vip_ssvgd_step(c, x, dev(G), eps, xi=dev(xi), gram_prec=vb.VIP_GRAM_FP32,
                           ws_tag="ssvgd")
    D, K, h2, phi, L = _inspect(ws, n, d)
    Xr, info = osvgd.ssvgd_step(X, G, eps, xi)
    eL = rel(L, info["L"])
    eX = rel(x.cpu().numpy(), Xr)
    print(f"ssvgd: L {eL:.2e} X {eX:.2e}", flush=True)
    assert eL <= 1e-5 and eX <= 1e-6
    assert np.allclose(L, np.tril(L)) and np.all(np.diag(L) > 0)
    assert c.poll(ws) == 0


def test_ssvgd_coincident_particles_need_jitter():
    n, d = 6, 40
    X = np.full((n, d), 2500.0)
    G = np.zeros((n, d))
    c = ctx()
    x = dev(X)
    xi = np.random.default_rng(3).standard_normal((n, d)).astype(np.float32).astype(np.float64)
    ws = vb.vip_ssvgd_step(c, x, dev(G), 1.0, xi=dev(xi), gram_prec=vb.VIP_GRAM_FP32,
                           ws_tag="ssvgd_j")
    flags = c.poll(ws)
    _, _, h2, _, L = _inspect(ws, n, d)
    Xr, info = osvgd.ssvgd_step(X, G, 1.0, xi)
    assert info["retries"] >= 1 and flags == vb.VIP_FLAG_JITTER and h2 == 1.0
    assert np.abs(L @ L.T - np.ones((n, n)) / n).max() <= 1e-6
    assert rel(x.cpu().numpy(), Xr) <= 1e-5


def test_ssvgd_philox_noise_is_reproducible_and_normal():
    n, d = 16, 2000
    X, G = _ensemble(n, d, 31)
    c = ctx()
    x1, x2, x3 = dev(X), dev(X), dev(X)
    for x, seed in ((x1, 5), (x2, 5), (x3, 6)):
        vb.vip_ssvgd_step(c, x, dev(G), 10.0, xi=None, seed=seed, stream=9,
                          gram_prec=vb.VIP_GRAM_FP32, ws_tag="ssvgd_p")
    assert torch.equal(x1, x2) and not torch.equal(x1, x3)
    xi = ophilox.normals(n * d, 5, 9).reshape(n, d)
    Xr, _ = osvgd.ssvgd_step(X, G, 10.0, xi)
    assert rel(x1.cpu().numpy(), Xr) <= 1e-6


def test_philox_words_bitwise_and_normals():
    c = ctx()
    seed, stream = 0x0123456789ABCDEF, 0xFEDCBA9876543210
    words = vb.vip_philox_uint32(c, 1000, seed, stream).cpu().numpy().view(np.uint32)
    ref = np.array([ophilox.uint_block(q, seed, stream) for q in range(1000)], dtype=np.uint32)
    assert np.array_equal(words.reshape(1000, 4), ref)
    z = vb.vip_philox_normals(c, 4003, seed, stream).cpu().numpy()
    zr = ophilox.normals(4003, seed, stream)
    assert np.abs(z - zr).max() <= 2e-5


@pytest.mark.parametrize("kind", [vb.VIP_OPT_SGD, vb.VIP_OPT_ADAGRAD, vb.VIP_OPT_ADADELTA,
                                  vb.VIP_OPT_ADAM])
@pytest.mark.parametrize("gram", [vb.VIP_GRAM_FP32, vb.VIP_GRAM_BF16])
def test_svgd_step_rules_match_oracle_over_three_steps(kind, gram):
    """SGD / AdaGrad / AdaDelta / Adam on the SVGD direction: three steps with
    the state carried, against the FP64 oracle fed the same directions; on the
    FP32 path (bound 1e-4) and on the BF16 path with its split update (bound
    5e-3: few coordinates leave the BF16 Gram coarse, as in the ragged test)."""
    from oracle import optim
    n, d = 40, 777
    # centred particles and step scales giving displacements of ~10, far above
    # the FP32 spacing of x, so the displacement read back from x is exact enough
    X, G = _ensemble(n, d, 91, base=0.0)
    c = ctx()
    x, g = dev(X), dev(G)
    b1 = 0.95 if kind == vb.VIP_OPT_ADADELTA else 0.9
    eps = {vb.VIP_OPT_SGD: 2000.0, vb.VIP_OPT_ADAGRAD: 10.0, vb.VIP_OPT_ADADELTA: 5000.0,
           vb.VIP_OPT_ADAM: 10.0}[kind]
    opt = vb.Optimizer(kind, x, beta1=b1, beta2=0.999, delta=1e-6)
    tol = 1e-4 if gram == vb.VIP_GRAM_FP32 else 5e-3
    Xr, st = X.copy(), {}
    for it in range(3):
        vb.vip_svgd_step_opt(c, x, g, eps, opt, gram_prec=gram)
        phi = osvgd.svgd_direction(Xr, G)["phi"]
        Xr = Xr + optim.step(kind, phi, st, eps, b1, 0.999, 1e-6)
        e = rel(x.cpu().numpy() - X, Xr - X)
        print(f"step rule {kind} gram {gram} step {it}: displacement rel L2 {e:.2e}", flush=True)
        assert e <= tol
    if kind != vb.VIP_OPT_SGD:
        assert rel(opt.s1.cpu().numpy(), st["s1"]) <= tol


@pytest.mark.parametrize("gram,n,d", [(vb.VIP_GRAM_FP32, 64, 1000), (vb.VIP_GRAM_FP32, 130, 515),
                                      (vb.VIP_GRAM_BF16, 300, 4100)])
def test_diag_matrix_kernel_svgd_matches_oracle(gram, n, d):
    """Diagonal matrix-valued kernel (Q = 1 / per-coordinate variance): the
    Q-weighted distances, the median bandwidth on them, Q^-1 on the gradients."""
    r = np.random.default_rng(n + d)
    scales = np.float32(np.exp(r.uniform(-2.0, 3.0, d))).astype(np.float64)
    X = np.float32(100.0 * r.standard_normal((n, d)) * scales).astype(np.float64)
    G = np.float32(-X / (100.0 * scales) ** 2 + 0.01 * r.standard_normal((n, d)) / scales
                   ).astype(np.float64)
    c = ctx()
    x = dev(X)
    eps = 50.0
    ws = vb.vip_svgd_step_ex(c, x, dev(G), eps, kernel=vb.VIP_KERNEL_DIAG_VAR, gram_prec=gram)
    D, K, h2, phi, _ = _inspect(ws, n, d)
    Xr, info = osvgd.svgd_step_diag(X, G, eps)
    tol = dict(D=1e-5, phi=1e-4) if gram == vb.VIP_GRAM_FP32 else dict(D=2e-4, phi=2e-3)
    errs = dict(D=rel(D, info["D"]), K=rel(K, info["K"]), phi=rel(phi, info["phi"]),
                X=rel(x.cpu().numpy() - X, Xr - X))
    print(f"diag kernel gram={gram} n={n} d={d}: {errs}", flush=True)
    assert errs["D"] <= tol["D"] and errs["phi"] <= tol["phi"] and errs["X"] <= tol["phi"]


def test_diag_matrix_kernel_ssvgd_matches_oracle():
    n, d, eps = 24, 3001, 20.0
    r = np.random.default_rng(41)
    scales = np.float32(np.exp(r.uniform(-1.0, 2.0, d))).astype(np.float64)
    X = np.float32(3000.0 + 100.0 * r.standard_normal((n, d)) * scales).astype(np.float64)
    G = np.float32(-(X - 3000.0) / (100.0 * scales) ** 2).astype(np.float64)
    xi = np.float32(r.standard_normal((n, d))).astype(np.float64)
    c = ctx()
    x = dev(X)
    vb.vip_svgd_step_ex(c, x, dev(G), eps, kernel=vb.VIP_KERNEL_DIAG_VAR, noise=True, xi=dev(xi),
                        gram_prec=vb.VIP_GRAM_FP32)
    Xr, info = osvgd.ssvgd_step_diag(X, G, eps, xi)
    e = rel(x.cpu().numpy() - X, Xr - X)
    print(f"diag kernel sSVGD: displacement rel L2 {e:.2e}", flush=True)
    assert e <= 1e-4


@pytest.mark.parametrize("n", [129, 600, 1000, 2048])
def test_ssvgd_blocked_cholesky_matches_oracle(n):
    """sSVGD beyond one workgroup's LDS (n > 128): the blocked FP64 Cholesky of
    K/n (32-column panels) and the noise L Xi with the same normals on both
    sides, d = 4096, FP32 Gram: L <= 1e-5, x' <= 1e-6, displacement <= 1e-3,
    and L L^T within 1e-13 (relative to its largest entry) of K/n formed in
    FP64 from the library's own D and h^2.
    The displacement (about 0.5 per coordinate here) is bounded by the FP32
    storage of x' itself: half an ulp at x ~ 3000 is 1.2e-4, so its relative
    error cannot go much below 1e-4 whatever the arithmetic."""
    from oracle import cref
    from tests.cases import workers
    d, eps = 4096, 20.0
    X, G = _ensemble(n, d, 40 + n)
    xi = np.random.default_rng(41 + n).standard_normal((n, d)).astype(np.float32).astype(np.float64)
    c = ctx()
    x = dev(X)
    print(f"blocked cholesky n={n}", flush=True)
    ws = vb.vip_ssvgd_step(c, x, dev(G), eps, xi=dev(xi), gram_prec=vb.VIP_GRAM_FP32,
                           ws_tag=f"chol{n}")
    flags = c.poll(ws)
    D, K, h2, phi, L = _inspect(ws, n, d)
    info = osvgd.svgd_direction(X, G, D=cref.sqdist(X, workers=workers()))
    eta, L_ref, retries = osvgd.ssvgd_noise(info["K"], eps, xi)
    Xr = X + eps * info["phi"] + eta
    xn = x.cpu().numpy().astype(np.float64)
    eL, eX, edX = rel(L, L_ref), rel(xn, Xr), rel(xn - X, Xr - X)
    # backward error of the factorisation itself, against K/n formed in FP64
    # from the library's own D and h^2
    A = np.exp(-D.astype(np.float64) / (2.0 * h2)) / n
    eB = np.abs(L @ L.T - A).max() / A.max()
    print(f"  L {eL:.2e}, x' {eX:.2e}, displacement {edX:.2e}, oracle retries {retries}, "
          f"|LL^T - K/n| / max {eB:.2e}", flush=True)
    assert flags == 0 and retries == 0
    assert eL <= 1e-5 and eX <= 1e-6 and edX <= 1e-3
    assert eB <= 1e-13   # Cholesky's backward error is of order n unit roundoffs at most
    assert np.array_equal(L, np.tril(L)) and np.all(np.diag(L) > 0)
    c._ws.pop(f"chol{n}", None)


@pytest.mark.parametrize("n, ndup", [(200, 200), (300, 10)])
def test_ssvgd_blocked_cholesky_coincident_particles(n, ndup):
    """Coincident particles make K/n singular: the blocked factorisation fails,
    the jitter retries succeed (flag VIP_FLAG_JITTER), L L^T reproduces the
    jittered K/n, and the update matches the oracle's (which also retries)."""
    d, eps = 512, 5.0
    X, G = _ensemble(n, d, 60 + n)
    X[1:ndup] = X[0]
    G[1:ndup] = G[0]
    xi = np.random.default_rng(61 + n).standard_normal((n, d)).astype(np.float32).astype(np.float64)
    c = ctx()
    x = dev(X)
    ws = vb.vip_ssvgd_step(c, x, dev(G), eps, xi=dev(xi), gram_prec=vb.VIP_GRAM_FP32,
                           ws_tag="chol_dup")
    flags = c.poll(ws)
    D, K, h2, phi, L = _inspect(ws, n, d)
    Xr, info = osvgd.ssvgd_step(X, G, eps, xi)
    A = np.exp(-D.astype(np.float64) / (2.0 * h2)) / n
    e = rel(x.cpu().numpy(), Xr)
    print(f"coincident n={n} dup={ndup}: flags {flags}, oracle retries {info['retries']}, "
          f"|LL^T - K/n| {np.abs(L @ L.T - A).max():.2e}, x' {e:.2e}", flush=True)
    assert info["retries"] >= 1 and flags == vb.VIP_FLAG_JITTER
    assert np.abs(L @ L.T - A).max() <= 1e-6 * A.max()
    assert e <= 1e-5
    c._ws.pop("chol_dup", None)


@pytest.mark.parametrize("n, d", [(200, 1024), (201, 1001), (600, 4096)])
def test_ssvgd_bf16_noise_product_matches_fp64(n, d):
    """The BF16 path's noise product beyond one workgroup's Cholesky (L and Xi
    each split into a BF16 pair, three products on the BF16 matrix cores).
    With the particles near 0, x' keeps the noise to FP32 precision, and
    x' - x - eps phi (the library's own phi) matches sqrt(2 eps) L Xi, formed in
    FP64 from the library's own L and the same normals, to 1e-4 relative L2.
    Odd n and d take the element-wise staging."""
    eps = 0.5
    rng = np.random.default_rng(90 + n)
    X = (0.1 * rng.standard_normal((n, d))).astype(np.float32).astype(np.float64)
    G = rng.standard_normal((n, d)).astype(np.float32).astype(np.float64)
    xi = rng.standard_normal((n, d)).astype(np.float32).astype(np.float64)
    c = ctx()
    x = dev(X)
    print(f"BF16 noise product n={n} d={d}", flush=True)
    ws = vb.vip_ssvgd_step(c, x, dev(G), eps, xi=dev(xi), gram_prec=vb.VIP_GRAM_BF16,
                           ws_tag=f"noise16_{n}")
    flags = c.poll(ws)
    D, K, h2, phi, L = _inspect(ws, n, d)
    eta = x.cpu().numpy().astype(np.float64) - X - eps * phi.astype(np.float64)
    eta_ref = np.sqrt(2.0 * eps) * (L @ xi)
    e = rel(eta, eta_ref)
    print(f"  noise vs FP64 L Xi: {e:.2e}", flush=True)
    assert flags & ~vb.VIP_FLAG_JITTER == 0
    assert e <= 1e-4
    c._ws.pop(f"noise16_{n}", None)


@pytest.mark.parametrize("n", [600, 2048])
def test_ssvgd_bf16_path_matches_oracle(n):
    """sSVGD on the BF16 path (BF16 Gram in 256 x 256 blocks, K in BF16 times
    the split B on the BF16 matrix cores, blocked FP64 Cholesky, noise L Xi as
    three BF16 products of split pairs) with the same normals on both sides, d = 4096: phi
    and L to 1e-3 relative L2 (the BF16 path's tolerance), the displacement
    x' - x to 1e-3."""
    from oracle import cref
    from tests.cases import workers
    d, eps = 4096, 20.0
    X, G = _ensemble(n, d, 80 + n)
    xi = np.random.default_rng(81 + n).standard_normal((n, d)).astype(np.float32).astype(np.float64)
    c = ctx()
    x = dev(X)
    ws = vb.vip_ssvgd_step(c, x, dev(G), eps, xi=dev(xi), gram_prec=vb.VIP_GRAM_BF16,
                           ws_tag=f"ssvgd16_{n}")
    flags = c.poll(ws)
    D, K, h2, phi, L = _inspect(ws, n, d)
    info = osvgd.svgd_direction(X, G, D=cref.sqdist(X, workers=workers()))
    eta, L_ref, retries = osvgd.ssvgd_noise(info["K"], eps, xi)
    Xr = X + eps * info["phi"] + eta
    xn = x.cpu().numpy().astype(np.float64)
    ephi, eL, edX = rel(phi, info["phi"]), rel(L, L_ref), rel(xn - X, Xr - X)
    print(f"sSVGD BF16 path n={n}: phi {ephi:.2e}, L {eL:.2e}, displacement {edX:.2e}", flush=True)
    assert flags & ~vb.VIP_FLAG_JITTER == 0 and retries == 0
    assert ephi <= 1e-3 and eL <= 1e-3 and edX <= 1e-3
    c._ws.pop(f"ssvgd16_{n}", None)
