"""GPU parity of ADVI (section 2.2, eq:gradient_mu, eq:gradient_L; the
mean-field family of section 5) through the C ABI against the FP64 oracle.

Bars: samples and gradients elementwise within 1e-5 of the scale of the
terms they sum (FP32 sums of up to d products); updated parameters within
1e-6 relative L2 after three steps of every step rule; the ELBO estimate
within 1e-12 relative plus 1e-6 per diagonal entry (FP64 sums; the device's L
carries FP32 rounding of earlier steps); entries of L above the diagonal and
the padding past column d never written (a NaN sentinel stays bitwise
intact and never reaches a result); the FWI loop (transform prior) within
1e-3 of the oracle's displacement of mu and L after three iterations."""
import math

import numpy as np
import pytest
import torch

from oracle import advi as oadvi
from oracle import optim as ooptim
from oracle import prior as oprior
from paper_2310_13325_amd import binding as vb
from tests.cases import build_case, small_problem
from tests.gpu_helpers import ctx, dev, grid_geom, rel

pytestmark = pytest.mark.gpu

RULES = [vb.VIP_OPT_SGD, vb.VIP_OPT_ADAGRAD, vb.VIP_OPT_ADADELTA, vb.VIP_OPT_ADAM]


def _f32(a):
    return np.float32(a).astype(np.float64)


def _full_case(r, d, ldl, S):
    mu = _f32(r.normal(0.0, 1.0, d))
    L = _f32(np.tril(r.normal(0.0, 0.3, (d, d)), -1) + np.diag(r.uniform(0.5, 2.0, d)))
    eta = _f32(r.standard_normal((S, d)))
    arr = np.full((d, ldl), np.nan, dtype=np.float32)
    arr[np.tril_indices(d)] = L[np.tril_indices(d)]
    return mu, L, eta, arr


def _q_from(arr, mu, family, kind, ldl):
    d = mu.shape[0]
    q = vb.Advi.__new__(vb.Advi)
    q.d, q.family, q.ldl = d, family, ldl if family == vb.VIP_ADVI_FULL_RANK else 0
    q.mu = dev(mu)
    q.L = dev(arr)
    q.opt_mu = vb.Optimizer(kind, q.mu, 0.9, 0.999, 1e-8)
    q.opt_L = vb.Optimizer(kind, q.L, 0.9, 0.999, 1e-8)
    return q


@pytest.mark.parametrize("d,ldl,S", [(1, 1, 1), (7, 7, 3), (1001, 1004, 8), (2050, 2057, 11),
                                     (600, 600, 32)])
def test_full_rank_sample_matches_oracle(d, ldl, S):
    r = np.random.default_rng(100 + d + S)
    mu, L, eta, arr = _full_case(r, d, ldl, S)
    c = ctx()
    q = _q_from(arr, mu, vb.VIP_ADVI_FULL_RANK, vb.VIP_OPT_SGD, ldl)
    th = vb.vip_advi_sample(c, q, dev(eta)).cpu().numpy().astype(np.float64)
    ref = oadvi.sample(mu, L, eta)
    scale = np.abs(mu)[None, :] + np.abs(eta) @ np.abs(L).T
    err = np.abs(th - ref) / scale
    print(f"full-rank sample d={d} ldl={ldl} S={S}: max err / scale {err.max():.2e}", flush=True)
    assert np.isfinite(th).all() and err.max() <= 1e-5
    assert np.array_equal(np.isnan(q.L.cpu().numpy()), np.isnan(arr))


@pytest.mark.parametrize("d,S", [(1, 1), (4099, 5)])
def test_mean_field_sample_matches_oracle(d, S):
    r = np.random.default_rng(200 + d)
    mu, l, eta = _f32(r.normal(0, 1, d)), _f32(r.uniform(0.5, 2, d)), _f32(r.standard_normal((S, d)))
    c = ctx()
    q = _q_from(l, mu, vb.VIP_ADVI_MEAN_FIELD, vb.VIP_OPT_SGD, 0)
    th = vb.vip_advi_sample(c, q, dev(eta)).cpu().numpy()
    ref = oadvi.sample(mu, l, eta, oadvi.MEAN_FIELD)
    assert np.abs(th - ref).max() <= 1e-6 * (np.abs(mu).max() + np.abs(l).max() * np.abs(eta).max())


def _oracle_rule(kind):
    return {"beta1": 0.9, "beta2": 0.999, "delta": 1e-8} if kind != vb.VIP_OPT_SGD else {}


@pytest.mark.parametrize("kind", RULES)
@pytest.mark.parametrize("d,ldl,S", [(777, 782, 5), (300, 300, 1)])
def test_full_rank_step_matches_oracle(kind, d, ldl, S):
    r = np.random.default_rng(300 + kind + d)
    mu, L, _, arr = _full_case(r, d, ldl, S)
    c = ctx()
    q = _q_from(arr, mu, vb.VIP_ADVI_FULL_RANK, kind, ldl)
    eps = 1e-3
    st_mu, st_L = {}, {}
    mu_r, L_r = mu.copy(), L.copy()
    for step in range(3):
        eta = _f32(r.standard_normal((S, d)))
        g = _f32(r.normal(0.0, 5.0, (S, d)))
        lp = r.normal(-1e4, 10.0, S)
        ref_elbo = oadvi.elbo(lp, L_r)   # the oracle's own L before the step
        elbo, gm, gL = vb.vip_advi_step(c, q, dev(eta), dev(g), eps,
                                        logpost=dev(lp, torch.float64), grads=True)
        mu_r, L_r, gm_r, gL_r = oadvi.step(mu_r, L_r, eta, g, eps, kind, st_mu, st_L,
                                           oadvi.FULL_RANK, **_oracle_rule(kind))
        gm = gm.cpu().numpy()
        gLd = gL.cpu().numpy()[:, :d]
        scale_L = np.abs(g).T @ np.abs(eta) / S + np.diag(np.abs(1.0 / np.diag(L_r)))
        low = np.tril_indices(d)
        e_gm = np.abs(gm - gm_r).max() / (np.abs(g).mean(axis=0).max())
        e_gL = (np.abs(gLd - gL_r)[low] / scale_L[low]).max()
        Lg = q.L.cpu().numpy()
        e_mu = rel(q.mu.cpu().numpy(), mu_r)
        e_L = rel(Lg[:, :d][low], L_r[low])
        # FP64 sums on both sides; the device's L_ii carry FP32 rounding of the
        # earlier steps, at most ~1e-6 relative each, so |d log L_ii| <= 1e-6
        e_elbo = abs(elbo.item() - ref_elbo) / (1e-12 * abs(ref_elbo) + 1e-6 * d)
        print(f"rule {kind} d={d} S={S} step {step}: grad_mu {e_gm:.1e} grad_L {e_gL:.1e} "
              f"mu {e_mu:.1e} L {e_L:.1e} elbo {e_elbo:.1e}", flush=True)
        assert e_gm <= 1e-5 and e_gL <= 1e-5
        assert e_mu <= 1e-6 and e_L <= 1e-6
        assert e_elbo <= 1.0
        # untouched: NaN sentinel above the diagonal and in the padding columns,
        # state arrays there still zero
        up = np.triu_indices(d, 1)
        assert np.isnan(Lg[:, :d][up]).all() and np.isnan(Lg[:, d:]).all()
        if q.opt_L.s1 is not None:
            s1 = q.opt_L.s1.cpu().numpy()
            assert (s1[:, :d][up] == 0).all() and (s1[:, d:] == 0).all()


@pytest.mark.parametrize("kind", RULES)
def test_mean_field_step_matches_oracle(kind):
    r = np.random.default_rng(400 + kind)
    d, S = 5000, 3
    mu, l = _f32(r.normal(0, 1, d)), _f32(r.uniform(0.5, 2, d))
    c = ctx()
    q = _q_from(l, mu, vb.VIP_ADVI_MEAN_FIELD, kind, 0)
    st_mu, st_l = {}, {}
    mu_r, l_r = mu.copy(), l.copy()
    for step in range(3):
        eta = _f32(r.standard_normal((S, d)))
        g = _f32(r.normal(0.0, 5.0, (S, d)))
        lp = r.normal(-1e4, 10.0, S)
        ref_elbo = oadvi.elbo(lp, l_r, oadvi.MEAN_FIELD)
        elbo, gm, gl = vb.vip_advi_step(c, q, dev(eta), dev(g), 1e-3,
                                        logpost=dev(lp, torch.float64), grads=True)
        mu_r, l_r, gm_r, gl_r = oadvi.step(mu_r, l_r, eta, g, 1e-3, kind, st_mu, st_l,
                                           oadvi.MEAN_FIELD, **_oracle_rule(kind))
        scale = np.abs(g * eta).mean(axis=0) + 1.0 / np.abs(l_r)
        assert (np.abs(gl.cpu().numpy() - gl_r) / scale).max() <= 1e-5
        assert np.abs(gm.cpu().numpy() - gm_r).max() <= 1e-5 * np.abs(g).mean(axis=0).max()
        assert rel(q.mu.cpu().numpy(), mu_r) <= 1e-6 and rel(q.L.cpu().numpy(), l_r) <= 1e-6
        assert abs(elbo.item() - ref_elbo) <= 1e-12 * abs(ref_elbo) + 1e-6 * d


def test_step_rejects_bad_arguments():
    c = ctx()
    d = 8
    q = vb.Advi(d, vb.VIP_ADVI_FULL_RANK, kind=vb.VIP_OPT_SGD)
    eta = torch.zeros(1, d, device="cuda")
    L = vb.lib()
    args = (c.handle, 0, d, 1, q.mu.data_ptr(), q.L.data_ptr(), q.ldl, eta.data_ptr(),
            eta.data_ptr(), 0.1, None, None, None, None, None, None)
    assert L.vip_advi_step(*args) == vb.VIP_OK
    bad = list(args)
    bad[1] = 7                                  # family
    assert L.vip_advi_step(*bad) == -1
    bad = list(args)
    bad[3] = vb.VIP_ADVI_MAX_SAMPLES + 1        # S
    assert L.vip_advi_step(*bad) == -1
    bad = list(args)
    bad[6] = d - 1                              # ldl < d
    assert L.vip_advi_step(*bad) == -1
    bad = list(args)
    bad[15] = q.mu.data_ptr()                   # elbo without logpost
    assert L.vip_advi_step(*bad) == -1
    assert L.vip_advi_sample(c.handle, 0, d, 0, q.mu.data_ptr(), q.L.data_ptr(), q.ldl,
                             eta.data_ptr(), eta.data_ptr()) == -1
    torch.cuda.synchronize()


def test_full_rank_advi_on_gaussian_target_reaches_it():
    """The GPU loop (sample, torch target gradient, step) reaches the ELBO
    optimum N(m, A^-1) of a Gaussian target, as the oracle does."""
    r = np.random.default_rng(17)
    d = 5
    B = r.standard_normal((d, d))
    A = B @ B.T / d + 0.5 * np.eye(d)
    m = r.standard_normal(d)
    At, mt = dev(A), dev(m)
    c = ctx()
    gen = torch.Generator(device="cuda").manual_seed(5)
    for family in (vb.VIP_ADVI_FULL_RANK, vb.VIP_ADVI_MEAN_FIELD):
        q = vb.Advi(d, family, kind=vb.VIP_OPT_ADAM)
        for it in range(5000):
            S = 4 if it < 3000 else 16
            eps = 0.01 if it < 3000 else 0.002
            if it == 3000:
                q.opt_mu = vb.Optimizer(vb.VIP_OPT_ADAM, q.mu)
                q.opt_L = vb.Optimizer(vb.VIP_OPT_ADAM, q.L)
            eta = torch.randn(S, d, device="cuda", generator=gen)
            th = vb.vip_advi_sample(c, q, eta)
            g = -(th - mt) @ At.T
            vb.vip_advi_step(c, q, eta, g.contiguous(), eps)
        mu = q.mu.cpu().numpy()
        cov = q.covariance().cpu().numpy()
        if family == vb.VIP_ADVI_FULL_RANK:
            target = np.linalg.inv(A)
            assert np.abs(cov - target).max() <= 0.1 * np.abs(target).max()
        else:
            assert np.allclose(np.diag(cov), 1.0 / np.diag(A), rtol=0.1)
        assert np.abs(mu - m).max() <= 0.05 * np.sqrt(np.diag(np.linalg.inv(A))).max()


def test_fwi_advi_iterations_match_oracle():
    """Three ADVI iterations on a small FWI posterior (transform prior, two
    samples per iteration, SGD) from the same normals on both sides."""
    case = build_case(small_problem(nt=181, ns=2))
    d = case.lo.size
    lo, hi = case.lo.reshape(-1), case.hi.reshape(-1)
    c = ctx()
    grid, geom = grid_geom(c, case)
    pr = vb.Prior.transform(dev(case.lo), dev(case.hi))
    mid = _f32(oprior.to_theta(np.clip(case.particles.reshape(case.particles.shape[0], -1).mean(0),
                                       lo + 5.0, hi - 5.0), lo, hi))
    S, eps = 2, 1e-6
    r = np.random.default_rng(23)
    etas = [_f32(r.standard_normal((S, d))) for _ in range(3)]
    for family in (vb.VIP_ADVI_MEAN_FIELD, vb.VIP_ADVI_FULL_RANK):
        q = vb.Advi(d, family, kind=vb.VIP_OPT_SGD, mu0=dev(mid), scale=0.05)
        L0 = q.L.clone()
        for eta in etas:
            e = dev(eta)
            th = vb.vip_advi_sample(c, q, e)
            lp, g = vb.vip_grad_logpost(c, grid, geom, th.view(S, grid.nz, grid.nx),
                                        dev(case.dobs), case.sigma, ckpt_every=13, prior=pr,
                                        ws_tag="advi_fwi")
            vb.vip_advi_step(c, q, e, g.view(S, d), eps)
        fam = oadvi.FULL_RANK if family == vb.VIP_ADVI_FULL_RANK else oadvi.MEAN_FIELD
        L0r = 0.05 * (np.eye(d) if fam == oadvi.FULL_RANK else np.ones(d))

        def f(th):
            lp, g = oprior.transformed_grad_logpost(th.reshape(S, grid.nz, grid.nx), case.ogrid,
                                                    case.ogeom, case.dobs, case.sigma,
                                                    case.lo, case.hi)
            return lp, g.reshape(S, d)
        mu_r, L_r, _ = oadvi.run(f, mid, L0r, etas, eps, ooptim.SGD, fam)
        dmu = q.mu.cpu().numpy() - mid
        e_mu = rel(dmu, mu_r - mid)
        if fam == oadvi.FULL_RANK:
            dL = (q.L - L0).cpu().numpy()[:, :d]
            e_L = rel(np.tril(dL), np.tril(L_r - L0r))
        else:
            e_L = rel((q.L - L0).cpu().numpy(), L_r - L0r)
        print(f"FWI ADVI family {family}: displacement error mu {e_mu:.2e} L {e_L:.2e} "
              f"(|dmu| {np.linalg.norm(mu_r - mid):.3e})", flush=True)
        assert e_mu <= 1e-3 and e_L <= 1e-3


def test_iteration_helper_equals_the_call_sequence():
    case = build_case(small_problem(nt=181, ns=2))
    d = case.lo.size
    c = ctx()
    grid, geom = grid_geom(c, case)
    pr = vb.Prior.transform(dev(case.lo), dev(case.hi))
    qa = vb.Advi(d, vb.VIP_ADVI_MEAN_FIELD, scale=0.1)
    qb = vb.Advi(d, vb.VIP_ADVI_MEAN_FIELD, scale=0.1)
    elbo = vb.vip_advi_iteration(c, qa, grid, geom, dev(case.dobs), case.sigma, pr, 3, 1e-3,
                                 seed=9, it=4, ckpt_every=13)
    eta = vb.vip_philox_normals(c, 3 * d, 9, 4).view(3, d)
    th = vb.vip_advi_sample(c, qb, eta)
    lp, g = vb.vip_grad_logpost(c, grid, geom, th.view(3, grid.nz, grid.nx), dev(case.dobs),
                                case.sigma, ckpt_every=13, prior=pr, ws_tag="advi_b")
    elbo_b, _, _ = vb.vip_advi_step(c, qb, eta, g.view(3, d), 1e-3, logpost=lp)
    assert torch.equal(qa.mu, qb.mu) and torch.equal(qa.L, qb.L) and torch.equal(elbo, elbo_b)
    assert math.isfinite(elbo.item())


def test_full_rank_at_the_benchmark_size_on_sampled_rows():
    """d = 24,000 (the c2 model), S = 8 and the Adam rule, as the benchmark
    times the full-rank kernels: sampled rows of theta, of grad_L and of the
    updated L against the oracle computed one row at a time."""
    d, S = 24000, 8
    r = np.random.default_rng(2024)
    L = r.standard_normal((d, d), dtype=np.float32)
    L *= np.float32(0.01)
    L = np.tril(L)
    L[np.diag_indices(d)] = r.uniform(0.5, 2.0, d).astype(np.float32)
    mu = _f32(r.normal(0.0, 1.0, d))
    eta = _f32(r.standard_normal((S, d)))
    g = _f32(r.normal(0.0, 5.0, (S, d)))
    rows = [0, 1, 255, 256, 4097, 12345, 23998, 23999]
    L_rows = [L[i].astype(np.float64) for i in rows]
    c = ctx()
    q = _q_from(L, mu, vb.VIP_ADVI_FULL_RANK, vb.VIP_OPT_ADAM, d)
    del L
    th = vb.vip_advi_sample(c, q, dev(eta)).cpu().numpy().astype(np.float64)
    ref = oadvi.sample_rows(mu, L_rows, eta, rows)
    scale = np.stack([np.abs(mu[i]) + np.abs(eta[:, : i + 1]) @ np.abs(L_rows[k][: i + 1])
                      for k, i in enumerate(rows)], axis=1)
    e_th = (np.abs(th[:, rows] - ref) / scale).max()
    _, _, gL = vb.vip_advi_step(c, q, dev(eta), dev(g), 1e-3, grads=True)
    g_ref = oadvi.gradient_rows(L_rows, eta, g, rows)
    idx = torch.tensor(rows, device="cuda")
    gL_rows = gL.index_select(0, idx).cpu().numpy().astype(np.float64)
    L_new = q.L.index_select(0, idx).cpu().numpy().astype(np.float64)
    e_g = e_L = 0.0
    for k, i in enumerate(rows):
        gs = np.abs(g[:, i]) @ np.abs(eta[:, : i + 1]) / S
        gs[i] += 1.0 / abs(L_rows[k][i])
        e_g = max(e_g, (np.abs(gL_rows[k][: i + 1] - g_ref[k]) / gs).max())
        inc = ooptim.step(ooptim.ADAM, g_ref[k], {}, 1e-3, beta1=0.9, beta2=0.999, delta=1e-8)
        # Adam's first step is eps g / (|g| + delta): where |g| is within FP32
        # rounding of 0 its sign is not determined, so those entries are left out
        keep = np.abs(g_ref[k]) > 1e-5 * gs
        e_L = max(e_L, np.abs(L_new[k][: i + 1] - (L_rows[k][: i + 1] + inc))[keep].max())
        assert (L_new[k][i + 1:] == 0).all()
    print(f"d={d} S={S} sampled rows: theta {e_th:.2e}, grad_L {e_g:.2e}, L' max abs {e_L:.2e}",
          flush=True)
    assert e_th <= 1e-5 and e_g <= 1e-5 and e_L <= 1e-6
    del q, gL
    torch.cuda.empty_cache()
