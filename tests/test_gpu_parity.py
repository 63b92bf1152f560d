"""GPU parity of the HIP path (called through the C ABI) against the FP64
oracle on the same seeded inputs.

Tolerances
  FP64 path      e_p <= 1e-10   (both sides double; only summation order differs)
  FP32 path      e_p <= 1e-5    (tighter than the 1e-4 target; float unit roundoff
                                 6e-8 times the growth of k=100 dependent steps)
  BF16 split     e_p <= 1e-3    (hi+lo planes carry ~16 significant bits)
  e_p = |var_gpu - var_oracle| / prior(x*)  (prior = interpolated k(x*, x*))
"""
import numpy as np
import pytest
import torch

from oracle import love_fp64 as O
from paper_1803_06058_amd import binding as B
from paper_1803_06058_amd import workloads as WL

from gpu_helpers import build, cfg_of, dev, errors, oracle_cache, spec_of, tdev, torch_dtype

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


# ---------------------------------------------------------------------------
# Operator pieces: K_UU and Khat products
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("toeplitz", ["direct", "fft", "auto"])
@pytest.mark.parametrize("case", ["1d_long_f32", "1d_long_f64", "1d_short_f32", "2d_f32", "4d_f64"])
def test_apply_kuu_parity(case, toeplitz):
    if case == "1d_long_f32":
        P = WL.config(2, scale=0.2)          # m = 2000 (long-line split-K kernel)
    elif case == "1d_long_f64":
        P = WL.config(2, scale=0.2, dtype="f64", precision="fp64")
    elif case == "1d_short_f32":
        P = WL.config(1, dtype="f32", precision="fp32")   # m = 100 (line kernel)
    elif case == "2d_f32":
        P = WL.config(3, scale=0.01)
    else:
        P = WL.config(4, scale=0.002, dtype="f64", precision="fp64")
    print(case, toeplitz, P.m, flush=True)
    cache = build(P, k=8, flags=B.FLAG_NO_MEAN, toeplitz=toeplitz)
    info = cache.info()
    if toeplitz == "fft":
        assert all(info.toeplitz_mode[e] == 2 for e in range(P.d))
    spec = spec_of(P)
    g = np.random.default_rng(0).standard_normal(spec.mtot)
    dt = torch_dtype(P)
    out = host(cache.apply_kuu(tdev(g, dt)))
    ref = O.K_apply(spec, g.astype(np.float32 if dt == torch.float32 else np.float64).astype(np.float64))
    tol = 1e-12 if dt == torch.float64 else 2e-6
    assert np.max(np.abs(out - ref)) <= tol * np.max(np.abs(ref)) * np.sqrt(spec.mtot)
    cache.free()


@pytest.mark.parametrize("cfgi,scale", [(1, 1.0), (2, 0.05), (3, 0.004), (4, 0.002)])
def test_apply_khat_parity(cfgi, scale):
    P = WL.config(cfgi, scale=scale)
    print(P.name, P.n, P.m, flush=True)
    cache = build(P, k=8, flags=B.FLAG_NO_MEAN)
    spec = spec_of(P)
    v = np.random.default_rng(1).standard_normal(P.n)
    dt = torch_dtype(P)
    vv = v.astype(np.float32 if dt == torch.float32 else np.float64)
    out = host(cache.apply_khat(tdev(vv, dt)))
    ref = O.KissOperator(P.x.astype(np.float64), spec).khat(vv.astype(np.float64))
    rel = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    assert rel <= (1e-12 if dt == torch.float64 else 1e-5), rel
    cache.free()


@pytest.mark.parametrize("case", ["1d_f32", "1d_f64", "2d_f32"])
def test_apply_khat_heavy_cells_parity(case):
    """Cells holding >= 64 rows on average take the two-stage W^T v (one wave
    per cell, then per-node sums): 1-D with ~330 rows per cell and 2-D with
    ~620, against the dense product."""
    if case == "2d_f32":
        P = WL.make_problem("heavy2d", d=2, n=50_000, m=(12, 12), kernel="rbf",
                            lengthscale=(0.2, 0.3), noise=0.01, k=8, t=10,
                            target="sincos4", ynoise=0.05)
    else:
        f64 = case == "1d_f64"
        P = WL.make_problem("heavy1d", d=1, n=20_000, m=(64,), kernel="rbf",
                            lengthscale=(0.1,), noise=0.01, k=8, t=10, target="sin6",
                            ynoise=0.1, dtype="f64" if f64 else "f32",
                            precision="fp64" if f64 else "fp32")
    print(P.name, P.n, P.m, flush=True)
    cache = build(P, flags=B.FLAG_NO_MEAN)
    spec = spec_of(P)
    v = np.random.default_rng(1).standard_normal(P.n)
    dt = torch_dtype(P)
    vv = v.astype(np.float32 if dt == torch.float32 else np.float64)
    out = host(cache.apply_khat(tdev(vv, dt)))
    ref = O.KissOperator(P.x.astype(np.float64), spec).khat(vv.astype(np.float64))
    rel = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    assert rel <= (1e-12 if dt == torch.float64 else 1e-5), rel
    cache.free()


def test_heavy_cells_build_parity():
    """A whole build (float Lanczos, double mean CG) through the two-stage
    W^T v: 1-D, 2e4 points on 64 nodes (~330 rows per cell), against the
    oracle."""
    P = WL.make_problem("heavy1d", d=1, n=20_000, m=(64,), kernel="rbf", lengthscale=(0.1,),
                        noise=0.01, k=40, t=2000, target="sin6", ynoise=0.1)
    print(P.name, P.n, P.m, flush=True)
    cache = build(P)
    mu, var = cache.predict_mean_var(tdev(P.xs, torch.float32))
    oc = oracle_cache(P)
    m_ref, v_ref = O.love_predict(oc, P.xs)
    e = errors(host(var), v_ref, O.prior_var(P.xs, spec_of(P)), host(mu), m_ref, P.y)
    print(cache.info().k_eff, e, flush=True)
    assert e["e_p_max"] <= 1e-5
    assert e["mean_err_rel_rms_y"] <= 1e-4
    cache.free()


# ---------------------------------------------------------------------------
# Full build + query
# ---------------------------------------------------------------------------
def test_config1_fp64_parity():
    P = WL.config(1)
    cache = build(P)
    info = cache.info()
    mu, var = cache.predict_mean_var(tdev(P.xs, torch.float64))
    oc = oracle_cache(P, cg_tol=1e-12)
    m_ref, v_ref = O.love_predict(oc, P.xs)
    mA, vA = O.exact_route_A(P.x, P.y, P.xs, spec_of(P))
    p = O.prior_var(P.xs, spec_of(P))
    e = errors(host(var), v_ref, p, host(mu), m_ref, P.y)
    print(info.k_eff, oc.lanczos.k_eff, info.cg_iters, e, flush=True)
    assert abs(info.k_eff - oc.lanczos.k_eff) <= 2
    assert e["e_p_max"] <= 1e-10
    assert e["mean_err_rel_rms_y"] <= 1e-9
    assert np.max(np.abs(host(var) - vA) / p) <= 1e-10     # saturated: exact KISS-GP
    cache.free()


@pytest.mark.parametrize("scale,toeplitz", [(0.02, "auto"), (0.1, "auto"), (0.1, "fft")])
def test_config2_fp32_parity_small(scale, toeplitz):
    P = WL.config(2, scale=scale, k_sample=0)
    print(P.name, P.n, P.m, P.t, toeplitz, flush=True)
    cache = build(P, toeplitz=toeplitz)
    info = cache.info()
    xs = P.xs[:20000]
    mu, var = cache.predict_mean_var(tdev(xs, torch.float32))
    oc = oracle_cache(P)
    m_ref, v_ref = O.love_predict(oc, xs)
    p = O.prior_var(xs, spec_of(P))
    e = errors(host(var), v_ref, p, host(mu), m_ref, P.y)
    print(info.k_eff, info.cg_iters, info.status_flags, e, flush=True)
    assert e["e_p_max"] <= 1e-5
    assert e["mean_err_rel_rms_y"] <= 1e-4
    assert (host(var) <= p * (1 + 1e-6)).all()
    cache.free()


def test_config2_full_size_sampled():
    """Bench configuration (n=1e5, m=1e4, k=100, t=1e6): all 1e6 outputs on the
    GPU, 4000 of them checked against the oracle one by one."""
    P = WL.config(2, k_sample=0)
    cache = build(P)
    xs_all = tdev(P.xs, torch.float32)
    mu, var = cache.predict_mean_var(xs_all)
    torch.cuda.synchronize()
    idx = np.random.default_rng(11).choice(P.t, 4000, replace=False)
    oc = oracle_cache(P)
    xs = P.xs[idx]
    m_ref, v_ref = O.love_predict(oc, xs)
    p = O.prior_var(xs, spec_of(P))
    e = errors(host(var)[idx], v_ref, p, host(mu)[idx], m_ref, P.y)
    print(cache.info().k_eff, cache.info().cg_iters, e, flush=True)
    assert e["e_p_max"] <= 1e-5
    assert e["mean_err_rel_rms_y"] <= 1e-4
    assert np.isfinite(host(var)).all()
    cache.free()


def test_covar_pairs_parity():
    P = WL.config(2, scale=0.02, k_sample=0)
    cache = build(P)
    rng = np.random.default_rng(4)
    xa = rng.uniform(0, 1, (3000, 1)).astype(np.float32)
    xb = np.clip(xa + rng.normal(0, 0.01, xa.shape), 0, 1).astype(np.float32)
    cov = host(cache.predict_covar_pairs(tdev(xa, torch.float32), tdev(xb, torch.float32)))
    oc = oracle_cache(P)
    ref = O.love_covariance(oc, xa.astype(np.float64), xb.astype(np.float64))
    p = np.sqrt(O.prior_var(xa, spec_of(P)) * O.prior_var(xb, spec_of(P)))
    assert np.max(np.abs(cov - ref) / p) <= 1e-5
    cache.free()


def test_covar_block_parity():
    """Every pair of two ragged point sets (300 x 200: partial 32 x 32 tiles)
    against the oracle's paired covariance on the expanded pairs; the block of
    a set with itself is symmetric and its diagonal is the variance."""
    P = WL.config(2, scale=0.02, k_sample=0)
    cache = build(P)
    rng = np.random.default_rng(7)
    xa = rng.uniform(0, 1, (300, 1)).astype(np.float32)
    xb = rng.uniform(0, 1, (200, 1)).astype(np.float32)
    cov = host(cache.predict_covar_block(tdev(xa, torch.float32), tdev(xb, torch.float32)))
    assert cov.shape == (300, 200)
    oc = oracle_cache(P)
    xi = np.repeat(xa, 200, axis=0).astype(np.float64)
    xj = np.tile(xb, (300, 1)).astype(np.float64)
    ref = O.love_covariance(oc, xi, xj).reshape(300, 200)
    spec = spec_of(P)
    p = np.sqrt(np.outer(O.prior_var(xa, spec), O.prior_var(xb, spec)))
    assert np.max(np.abs(cov - ref) / p) <= 1e-5
    same = host(cache.predict_covar_block(tdev(xa, torch.float32), tdev(xa, torch.float32)))
    pa = O.prior_var(xa, spec)
    assert np.max(np.abs(same - same.T) / np.sqrt(np.outer(pa, pa))) <= 1e-6
    _, var = cache.predict_mean_var(tdev(xa, torch.float32))
    assert np.max(np.abs(np.diag(same) - host(var)) / pa) <= 1e-6
    # an out-of-domain point gives a NaN row; empty sets are a no-op
    xo = np.array([[0.5], [1.5], [0.25]], np.float32)
    blk = host(cache.predict_covar_block(tdev(xo, torch.float32), tdev(xb[:5], torch.float32)))
    assert np.isnan(blk[1]).all() and np.isfinite(blk[[0, 2]]).all()
    assert cache.predict_covar_block(tdev(xa[:0], torch.float32), tdev(xb, torch.float32)).numel() == 0
    cache.free()


# ---------------------------------------------------------------------------
# Sampling
# ---------------------------------------------------------------------------
def _sampler_case(scale, s=2000):
    P = WL.config(2, scale=scale, s=s)
    cache = build(P)
    ex = cache.export()
    S, a = host(ex["s"]), host(ex["a"])
    xs = P.xs_sample
    spec = spec_of(P)
    out = host(cache.sample_posterior(tdev(xs, torch.float32), tdev(P.z, torch.float32)))
    Ws = O.interp_matrix(xs.astype(np.float64), spec)
    return P, cache, ex, S, a, xs, spec, out, Ws


def test_sampler_draw_and_saturated_parity():
    """m = 100 <= k' = 100: the second Lanczos spans the grid space, so the
    implied covariance W* S S^T W*^T equals W*(K - R^T R')W*^T on both sides."""
    P, cache, ex, S, a, xs, spec, out, Ws = _sampler_case(0.01)
    # the draw kernel: out = mu + W* S z (float rounding only)
    ref_draw = (Ws @ a)[:, None] + Ws @ (S @ P.z[: S.shape[1]].astype(np.float64))
    assert np.max(np.abs(out - ref_draw)) <= 1e-5 * (1 + np.max(np.abs(ref_draw)))
    oc = oracle_cache(P)
    osm = O.love_sampler(oc, P.k_sample)
    sub = slice(0, 300)
    F = Ws[sub] @ S
    Sig_gpu = F @ F.T
    Sig_or = O.sample_covariance_implied(oc, osm, xs[sub].astype(np.float64))
    p = O.prior_var(xs[sub], spec)
    scale = np.sqrt(np.outer(p, p))
    err = np.max(np.abs(Sig_gpu - Sig_or) / scale)
    print(cache.info().k_eff_sample, osm.k_chol, err, flush=True)
    assert err <= 1e-5
    _, var = cache.predict_mean_var(tdev(xs[sub], torch.float32))
    assert np.max(np.abs(np.diag(Sig_gpu) - host(var)) / p) <= 1e-5
    cache.free()


def test_sampler_truncated_vs_oracle():
    """k' = 100 < m = 200: both sides truncate the second Lanczos at the same
    k', half the grid, where the Krylov space has not converged and its
    unconverged part follows the rounding of each side's operator (the float
    cache against the double one).  Element by element, the GPU's implied
    covariance W* S S^T W*^T is then within 1.5x the oracle's own truncation
    error (|oracle - W*(K - R^T R')W*^T|, relative to the prior) of the
    oracle's, and as close to W*(K - R^T R')W*^T as the oracle is.  The
    full-size 1-D workload (m = 1e4, k' = 100), where the spectrum has decayed
    by k', is compared to 1e-5 of the prior in test_gpu_fullsize.py."""
    P, cache, ex, S, a, xs, spec, out, Ws = _sampler_case(0.02)
    oc = oracle_cache(P)
    osm = O.love_sampler(oc, P.k_sample)
    sub = slice(0, 300)
    Wd = Ws[sub].toarray()
    target = Wd @ (O.K_dense(spec) - oc.Rt @ oc.Rt.T) @ Wd.T
    F = Ws[sub] @ S
    sig_or = O.sample_covariance_implied(oc, osm, xs[sub].astype(np.float64))
    p = O.prior_var(xs[sub], spec)
    scale = np.sqrt(np.outer(p, p))
    e_go = np.max(np.abs(F @ F.T - sig_or) / scale)
    e_gt = np.max(np.abs(F @ F.T - target) / scale)
    e_ot = np.max(np.abs(sig_or - target) / scale)
    print(cache.info().k_eff_sample, osm.k_chol, e_go, e_gt, e_ot, flush=True)
    assert e_go <= 1.5 * e_ot
    assert e_gt <= 1.5 * e_ot
    cache.free()


@pytest.mark.parametrize("scale", [0.02, 1.0])
def test_sampler_eigensolver_paths_agree(scale):
    """The sampler's T' eigen-decomposition has a parallel fast path
    (multisection + twisted factorisation) and an implicit-QL path; the
    implied covariance W* S S^T W*^T must agree between them."""
    P = WL.config(2, scale=scale, s=16)
    xs = P.xs_sample[:300]
    spec = spec_of(P)
    Ws = O.interp_matrix(xs.astype(np.float64), spec)
    p = O.prior_var(xs, spec)
    covs, kk = [], []
    for flags in (0, B.FLAG_EIG_QL):
        cache = build(P, flags=flags)
        inf = cache.info()
        kk.append((inf.k_eff_sample, inf.status_flags & ~32))
        F = Ws @ host(cache.export()["s"])
        covs.append(F @ F.T)
        cache.free()
    print(kk, flush=True)
    assert kk[0] == kk[1]
    err = np.max(np.abs(covs[0] - covs[1]) / np.sqrt(np.outer(p, p)))
    print(err, flush=True)
    assert err <= 1e-6


@pytest.mark.parametrize("scale", [0.05, 1.0])
def test_partial_sum_routes_agree(scale, monkeypatch):
    """The Lanczos runs add their per-block partial rows either in column-sum
    launches or inside the consuming kernels (chosen by row-block count;
    LOVE_PSUM_MAX_NB moves the limit).  Both routes give the same variances
    and sampler covariance up to summation order, and both meet the oracle."""
    P = WL.config(2, scale=scale, s=16)
    xs = P.xs_sample[:300]
    spec = spec_of(P)
    Ws = O.interp_matrix(xs.astype(np.float64), spec)
    p = O.prior_var(xs, spec)
    oc = oracle_cache(P)
    _, v_ref = O.love_predict(oc, xs)
    res = []
    for lim in ("0", "1000000"):
        monkeypatch.setenv("LOVE_PSUM_MAX_NB", lim)
        cache = build(P)
        inf = cache.info()
        _, var = cache.predict_mean_var(tdev(xs, torch.float32))
        F = Ws @ host(cache.export()["s"])
        res.append((inf.k_eff, inf.k_eff_sample, host(var), F @ F.T))
        cache.free()
    monkeypatch.delenv("LOVE_PSUM_MAX_NB")
    (k0, ks0, v0, c0), (k1, ks1, v1, c1) = res
    assert (k0, ks0) == (k1, ks1)
    print(k0, ks0, np.max(np.abs(v0 - v1) / p), flush=True)
    assert np.max(np.abs(v0 - v1) / p) <= 1e-6
    assert np.max(np.abs(c0 - c1) / np.sqrt(np.outer(p, p))) <= 1e-6
    for v in (v0, v1):
        assert np.max(np.abs(v - v_ref) / p) <= 1e-5


def test_sampler_monte_carlo():
    """Sample mean and covariance of 20000 GPU draws at 12 points against the
    implied covariance (statistical tolerance, 6 standard errors)."""
    P = WL.config(2, scale=0.01, s=20000, t_sample=12)
    cache = build(P)
    ex = cache.export()
    S = host(ex["s"])
    xs = P.xs_sample
    out = host(cache.sample_posterior(tdev(xs, torch.float32), tdev(P.z, torch.float32)))
    mu, _ = cache.predict_mean_var(tdev(xs, torch.float32))
    Ws = O.interp_matrix(xs.astype(np.float64), spec_of(P))
    F = Ws @ S
    ref = F @ F.T
    s = out.shape[1]
    level = np.sqrt((np.outer(np.diag(ref), np.diag(ref)) + ref ** 2) / s)
    assert np.all(np.abs(np.cov(out) - ref) < 6 * level + 1e-12)
    assert np.all(np.abs(out.mean(1) - host(mu)) < 6 * np.sqrt(np.diag(ref) / s) + 1e-7)
    cache.free()


# ---------------------------------------------------------------------------
# Precision form (2-D, bf16 split) and 4-D Matern
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("toeplitz", ["direct", "fft"])
def test_config3_bf16split_small(toeplitz):
    P = WL.config(3, scale=0.01)
    print(P.name, P.n, P.m, flush=True)
    cache = build(P, toeplitz=toeplitz)
    xs = P.xs[:5000]
    mu, var = cache.predict_mean_var(tdev(xs, torch.float32))
    oc = oracle_cache(P)
    m_ref, v_ref = O.love_predict(oc, xs)
    p = O.prior_var(xs, spec_of(P))
    e = errors(host(var), v_ref, p, host(mu), m_ref, P.y)
    print(cache.info().k_eff, e, flush=True)
    assert e["e_p_max"] <= 1e-3
    assert e["mean_err_rel_rms_y"] <= 1e-4
    cache.free()


def test_config4_matern_small():
    P = WL.config(4, scale=0.01)
    print(P.name, P.n, P.m, flush=True)
    cache = build(P)
    xs = P.xs[:3000]
    mu, var = cache.predict_mean_var(tdev(xs, torch.float32))
    oc = oracle_cache(P)
    m_ref, v_ref = O.love_predict(oc, xs)
    p = O.prior_var(xs, spec_of(P))
    e = errors(host(var), v_ref, p, host(mu), m_ref, P.y)
    print(cache.info().k_eff, e, flush=True)
    assert e["e_p_max"] <= 1e-5
    assert e["mean_err_rel_rms_y"] <= 1e-4
    cache.free()


# ---------------------------------------------------------------------------
# Mean cache on 2-D .. 4-D grids: grid-space solve (B = kron(V_e) diag(sqrt lam))
# ---------------------------------------------------------------------------
SF_CG_NOCONV = 16


def test_grid_space_mean_2d_mid():
    """64 x 64 grid, 5e4 points, the 2-D precision-form kernel: the grid-space
    solve converges in tens of iterations (the oracle's plain CG needs ~4800)
    and matches the oracle's mean (its CG run to 1e-10, checked converged)."""
    P = WL.make_problem("c3_mid", d=2, n=50_000, m=(64, 64), kernel="rbf",
                        lengthscale=(0.05, 0.08), noise=0.0025, k=50, t=4000,
                        target="sincos4", ynoise=0.05)
    print(P.name, P.n, P.m, flush=True)
    cache = build(P)
    info = cache.info()
    print("cg_iters", info.cg_iters, "status", info.status_flags, flush=True)
    assert not (info.status_flags & SF_CG_NOCONV)
    assert 0 < info.cg_iters < 100
    mu, var = cache.predict_mean_var(tdev(P.xs, torch.float32))
    # the oracle's plain CG needs ~4800 iterations here
    oc = O.love_build(P.x.astype(np.float64), P.y.astype(np.float64), spec_of(P), P.k,
                      cg_tol=1e-10, cg_maxit=20000)
    assert oc.cg_iters < 20000
    m_ref, v_ref = O.love_predict(oc, P.xs)
    e = errors(host(var), v_ref, O.prior_var(P.xs, spec_of(P)), host(mu), m_ref, P.y)
    print(e, "oracle cg", oc.cg_iters, flush=True)
    assert e["mean_err_rel_rms_y"] <= 1e-4
    assert e["e_p_max"] <= 1e-5
    cache.free()


def test_grid_space_mean_3d():
    """Odd d (the axis passes end in the other buffer): 12^3 grid, 2e4 points,
    mean and variance against the oracle."""
    P = WL.make_problem("d3", d=3, n=20_000, m=(12, 12, 12), kernel="rbf",
                        lengthscale=(0.15, 0.2, 0.25), noise=0.01, k=40, t=3000,
                        target="sumsin", ynoise=0.1)
    print(P.name, P.n, P.m, flush=True)
    cache = build(P)
    info = cache.info()
    print("cg_iters", info.cg_iters, "status", info.status_flags, flush=True)
    assert not (info.status_flags & SF_CG_NOCONV)
    assert 0 < info.cg_iters < 100
    mu, var = cache.predict_mean_var(tdev(P.xs, torch.float32))
    oc = oracle_cache(P)
    assert oc.cg_iters < 5000
    m_ref, v_ref = O.love_predict(oc, P.xs)
    e = errors(host(var), v_ref, O.prior_var(P.xs, spec_of(P)), host(mu), m_ref, P.y)
    print(e, flush=True)
    assert e["mean_err_rel_rms_y"] <= 1e-4
    assert e["e_p_max"] <= 1e-5
    cache.free()


def test_large_grid_first_pass_3d():
    """A 28^3 grid (21,952 nodes: 86 tiles of 256 rows, the last one ragged)
    under 70,001 points: the grid-space first pass takes one block per tile and
    a column-sum launch adds their rows, and with 256-row blocks (n >= 65,536)
    the second pass gathers each row's 64-node stencil with two threads.
    Mean and variance against the oracle at 3000 points."""
    P = WL.make_problem("d3_big", d=3, n=70_001, m=(28, 28, 28), kernel="rbf",
                        lengthscale=(0.1, 0.12, 0.15), noise=0.2, k=30, t=3000,
                        target="sumsin", ynoise=0.1)
    print(P.name, P.n, P.m, flush=True)
    assert -(-int(np.prod(P.m)) // 256) > 64 and P.n >= 65_536
    cache = build(P)
    info = cache.info()
    mu, var = cache.predict_mean_var(tdev(P.xs, torch.float32))
    oc = oracle_cache(P)
    m_ref, v_ref = O.love_predict(oc, P.xs)
    e = errors(host(var), v_ref, O.prior_var(P.xs, spec_of(P)), host(mu), m_ref, P.y)
    print("k_eff", info.k_eff, oc.lanczos.k_eff, e, flush=True)
    assert info.k_eff == oc.lanczos.k_eff
    assert e["mean_err_rel_rms_y"] <= 1e-4
    assert e["e_p_max"] <= 1e-5
    cache.free()


def test_grid_space_mean_fp64_parity():
    """Double 2-D build (grid-space mean in double, tolerance 1e-12 of
    sigma ||y||): mean and variance against the oracle at double tolerance."""
    P = WL.make_problem("d2_f64", d=2, n=4000, m=(16, 16), kernel="rbf", lengthscale=(0.15, 0.2),
                        noise=0.01, k=60, t=1000, target="sincos4", ynoise=0.05, dtype="f64",
                        precision="fp64")
    cache = build(P)
    info = cache.info()
    print("cg_iters", info.cg_iters, flush=True)
    assert not (info.status_flags & SF_CG_NOCONV)
    mu, var = cache.predict_mean_var(tdev(P.xs, torch.float64))
    oc = O.love_build(P.x, P.y, spec_of(P), P.k, cg_tol=1e-13, cg_maxit=20000)
    m_ref, v_ref = O.love_predict(oc, P.xs)
    e = errors(host(var), v_ref, O.prior_var(P.xs, spec_of(P)), host(mu), m_ref, P.y)
    print(e, flush=True)
    assert e["e_p_max"] <= 1e-10
    assert e["mean_err_rel_rms_y"] <= 1e-9
    cache.free()


def test_batched_2d_grid_space_equals_single():
    """Two 2-D GPs of different size in one batch: the grid-space mean and the
    Kronecker operator run batched and give each GP its own build bit for bit."""
    Ps = [WL.make_problem("b2d_%d" % i, d=2, n=n, m=m, kernel="rbf", lengthscale=(0.1, 0.15),
                          noise=0.005, k=k, t=1000, target="sincos4", ynoise=0.05, seed=i)
          for i, (n, m, k) in enumerate([(20_000, (24, 24), 40), (8_000, (16, 20), 30)])]
    cfgs = [cfg_of(P) for P in Ps]
    xs = [tdev(P.x, torch.float32) for P in Ps]
    ys = [tdev(P.y, torch.float32) for P in Ps]
    caches = B.build_cache_batched(cfgs, xs, ys)
    qs = [tdev(P.xs, torch.float32) for P in Ps]
    for g, P in enumerate(Ps):
        single = build(P)
        m0, v0 = caches[g].predict_mean_var(qs[g])
        m1, v1 = single.predict_mean_var(qs[g])
        assert caches[g].info().cg_iters == single.info().cg_iters
        assert torch.equal(v0, v1) and torch.equal(m0, m1)
        single.free()
    for c in caches:
        c.free()


@pytest.mark.parametrize("f64", [False, True])
def test_apply_khat_3d_parity(f64):
    """3-D product (two-stage W^T v, lane per cell) against the dense product."""
    P = WL.make_problem("d3op", d=3, n=6000, m=(8, 9, 10), kernel="matern52",
                        lengthscale=(0.3, 0.25, 0.2), noise=0.01, k=8, t=10, target="sumsin",
                        ynoise=0.1, dtype="f64" if f64 else "f32", precision="fp64" if f64 else "fp32")
    cache = build(P, flags=B.FLAG_NO_MEAN)
    spec = spec_of(P)
    v = np.random.default_rng(2).standard_normal(P.n)
    dt = torch_dtype(P)
    vv = v.astype(np.float64 if f64 else np.float32)
    out = host(cache.apply_khat(tdev(vv, dt)))
    ref = O.KissOperator(P.x.astype(np.float64), spec).khat(vv.astype(np.float64))
    rel = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    assert rel <= (1e-12 if f64 else 1e-5), rel
    cache.free()


def test_batched_3d_equals_single():
    """Two 3-D GPs in one batch (two-stage W^T v in the Lanczos and the mean
    solve): each equals its own build bit for bit."""
    Ps = [WL.make_problem("b3d_%d" % i, d=3, n=n, m=m, kernel="rbf", lengthscale=(0.2, 0.25, 0.3),
                          noise=0.01, k=30, t=500, target="sumsin", ynoise=0.1, seed=i)
          for i, (n, m) in enumerate([(6000, (10, 10, 10)), (3000, (8, 9, 8))])]
    caches = B.build_cache_batched([cfg_of(P) for P in Ps], [tdev(P.x, torch.float32) for P in Ps],
                                   [tdev(P.y, torch.float32) for P in Ps])
    for g, P in enumerate(Ps):
        q = tdev(P.xs, torch.float32)
        single = build(P)
        m0, v0 = caches[g].predict_mean_var(q)
        m1, v1 = single.predict_mean_var(q)
        assert torch.equal(v0, v1) and torch.equal(m0, m1)
        single.free()
    for c in caches:
        c.free()


def test_batched_large_grid_equals_single():
    """A GP whose grid-space first pass needs the column-sum launch (28^3
    nodes under 70,001 points) batched with one that sums its rows in the
    second pass (12^3 under 20,000): each equals its own build bit for bit."""
    Ps = [WL.make_problem("blg_%d" % i, d=3, n=n, m=m, kernel="rbf", lengthscale=(0.1, 0.12, 0.15),
                          noise=0.2, k=30, t=500, target="sumsin", ynoise=0.1, seed=i)
          for i, (n, m) in enumerate([(70_001, (28, 28, 28)), (20_000, (12, 12, 12))])]
    caches = B.build_cache_batched([cfg_of(P) for P in Ps], [tdev(P.x, torch.float32) for P in Ps],
                                   [tdev(P.y, torch.float32) for P in Ps])
    for g, P in enumerate(Ps):
        q = tdev(P.xs, torch.float32)
        single = build(P)
        m0, v0 = caches[g].predict_mean_var(q)
        m1, v1 = single.predict_mean_var(q)
        assert torch.equal(v0, v1) and torch.equal(m0, m1)
        single.free()
    for c in caches:
        c.free()


@pytest.mark.parametrize("case", ["2d", "4d", "4d_sparse"])
def test_grid_space_mean_equals_data_space_cg(case):
    """The two mean solvers (grid space by default for d >= 2, data-space CG on
    request) give the same predictive mean on reduced 2-D and 4-D workloads;
    4d_sparse has about 1.5 points per grid node.  The grid-space solve takes
    fewer iterations in each case."""
    if case == "2d":
        P = WL.make_problem("c3_red", d=2, n=20_000, m=(24, 24), kernel="rbf",
                            lengthscale=(0.05, 0.08), noise=0.0025, k=50, t=2000,
                            target="sincos4", ynoise=0.05)
    elif case == "4d":
        P = WL.make_problem("c4_red", d=4, n=60_000, m=(9,) * 4, kernel="matern52",
                            lengthscale=(0.2,) * 4, noise=0.01, k=64, t=2000,
                            target="sumsin", ynoise=0.1)
    else:
        P = WL.config(4, scale=0.05)
    print(P.name, P.n, P.m, flush=True)
    assert P.n >= int(np.prod(P.m)) > P.k
    xs = tdev(P.xs[:2000], torch.float32)
    c1 = build(P)
    c2 = build(P, flags=B.FLAG_MEAN_KRYLOV, cg_maxit=20000)   # needs > 1000 steps in 2-D
    i1, i2 = c1.info(), c2.info()
    print("iters grid", i1.cg_iters, "data", i2.cg_iters, flush=True)
    assert not (i1.status_flags & SF_CG_NOCONV) and not (i2.status_flags & SF_CG_NOCONV)
    m1, v1 = c1.predict_mean_var(xs)
    m2, v2 = c2.predict_mean_var(xs)
    assert i1.cg_iters < min(100, i2.cg_iters)
    rms = float(np.sqrt(np.mean(P.y.astype(np.float64) ** 2)))
    assert float(np.max(np.abs(host(m1) - host(m2)))) / rms <= 1e-4
    assert torch.equal(v1, v2)      # the variance cache does not depend on the mean solver
    c1.free()
    c2.free()


# ---------------------------------------------------------------------------
# Accuracy against the number of Lanczos steps (Sec. 6, accuracy vs. Lanczos
# iterations): exponential decrease, then a floor set by float rounding
# ---------------------------------------------------------------------------
def test_error_vs_lanczos_steps():
    """1-D, n = 2e4, m = 1000 (lengthscale 20 grid spacings): SMAE of the FP32
    GPU variances against the exact KISS-GP variances (route B) for k = 10 ..
    120.  The error never grows with k, falls by more than 1e4 between k = 20
    and k = 80, reaches the FP32 floor by k = 100, and follows the FP64 oracle's
    LOVE at the same k while the truncation error dominates."""
    P = WL.make_problem("err_vs_k", d=1, n=20_000, m=(1000,), kernel="rbf", lengthscale=(0.02,),
                        noise=0.01, k=100, t=2000, target="sin6_40", ynoise=0.1)
    X, y, xs = (a.astype(np.float64) for a in (P.x, P.y, P.xs))
    _, v_ex = O.exact_route_B(X, y, xs, spec_of(P))
    prior = O.prior_var(xs, spec_of(P))
    xs_d = tdev(P.xs, torch.float32)
    rows = []
    for k in (10, 20, 40, 60, 80, 100, 120):
        c = build(P, k=k)
        _, v = c.predict_mean_var(xs_d)
        vg = host(v)
        c.free()
        oc = O.love_build(X, y, spec_of(P), k, cg_tol=1e-8, cg_maxit=3000)
        _, vo = O.love_predict(oc, xs)
        rows.append((k, O.smae(vg, v_ex, y), O.smae(vo, v_ex, y),
                     float(np.max(np.abs(vg - v_ex) / prior))))
        print("k %3d  smae gpu %.3e  oracle %.3e  e_p max %.3e" % rows[-1], flush=True)
    sm = [r[1] for r in rows]
    for a, b in zip(sm, sm[1:]):
        assert b <= a * 1.05 + 1e-7
    assert sm[1] >= 1e4 * sm[4]
    assert rows[5][3] <= 1e-5 and rows[6][3] <= 1e-5
    for k, sg, so, _ in rows:
        if so > 1e-4:
            assert abs(sg - so) <= 1e-2 * so


# ---------------------------------------------------------------------------
# Backward
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cfgi,scale", [(1, 1.0), (4, 0.01)])
def test_backward_parity(cfgi, scale):
    P = WL.config(cfgi, scale=scale)
    cache = build(P)
    dt = torch_dtype(P)
    xs = P.xs[:2000]
    xs = np.clip(xs, 1e-3, 1 - 1e-3).astype(P.np_dtype)
    rng = np.random.default_rng(3)
    gm = rng.standard_normal(xs.shape[0]).astype(P.np_dtype)
    gv = rng.standard_normal(xs.shape[0]).astype(P.np_dtype)
    gx, _ = cache.predict_backward(tdev(xs, dt), tdev(gm, dt), tdev(gv, dt))
    oc = oracle_cache(P)
    ref = O.love_predict_grad(oc, xs.astype(np.float64), gm.astype(np.float64), gv.astype(np.float64))
    rel = np.max(np.abs(host(gx) - ref)) / np.max(np.abs(ref))
    print(rel, flush=True)
    assert rel <= (1e-9 if dt == torch.float64 else 1e-4)
    # autograd wrapper
    xt = tdev(xs, dt).requires_grad_(True)
    mu, var = B.LovePredict.apply(xt, cache)
    (mu * tdev(gm, dt) + var * tdev(gv, dt)).sum().backward()
    assert torch.allclose(xt.grad, gx.view_as(xt))
    cache.free()


@pytest.mark.parametrize("cfgi,scale,tol", [(1, 1.0, 1e-6), (2, 0.02, 1e-4), (3, 0.01, 3e-3),
                                            (4, 0.01, 1e-4)])
def test_grad_rt_parity(cfgi, scale, tol):
    """d(sum g_var var)/d Rt = -2 W*^T diag(g) W* Rt (love_grad_rt) on product
    grids.  Rt is only defined up to the Krylov basis (the float and double
    Lanczos vectors differ), so the comparison is on G Rt^T, which is
    -2 W*^T diag(g) W* Rt Rt^T on both sides and, Rt having full column rank,
    zero only if G is.  The gradient is float and summed per grid node in a
    fixed order: two calls agree bit for bit."""
    P = WL.config(cfgi, scale=scale)
    cache = build(P)
    dt = torch_dtype(P)
    xs = P.xs[:3000]
    gv = np.random.default_rng(8).standard_normal(xs.shape[0]).astype(P.np_dtype)
    xt, gt = tdev(xs, dt), tdev(gv, dt)
    _, g1 = cache.predict_backward(xt, None, gt, want_grt=True)
    _, g2 = cache.predict_backward(xt, None, gt, want_grt=True)
    assert torch.equal(g1, g2)
    ex = cache.export()
    rt = host(ex["rt64"] if dt == torch.float64 else ex["rt"])
    oc = oracle_cache(P)
    ref = O.love_grad_rt(oc, xs.astype(np.float64), gv.astype(np.float64)) @ oc.Rt.T
    got = host(g1) @ rt.T
    rel = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(P.name, P.m, cache.info().k_eff, oc.k, rel, flush=True)
    assert rel <= tol
    cache.free()


# ---------------------------------------------------------------------------
# Determinism, batching, edge cases
# ---------------------------------------------------------------------------
def test_build_is_bitwise_deterministic():
    P = WL.config(2, scale=0.05)
    c1, c2 = build(P), build(P)
    e1, e2 = c1.export(), c2.export()
    for key in e1:
        assert torch.equal(e1[key], e2[key]), key
    c1.free()
    c2.free()


def test_batched_equals_single():
    Ps = WL.batched_config(G=5, scale=0.02, t_per_gp=2000)
    cfgs = [cfg_of(P) for P in Ps]
    xs = [tdev(P.x, torch.float32) for P in Ps]
    ys = [tdev(P.y, torch.float32) for P in Ps]
    caches = B.build_cache_batched(cfgs, xs, ys)
    qs = [tdev(P.xs, torch.float32) for P in Ps]
    means, vars_ = B.predict_mean_var_batched(caches, qs)
    for g, P in enumerate(Ps):
        single = build(P)
        m1, v1 = single.predict_mean_var(qs[g])
        assert torch.equal(v1, vars_[g]) and torch.equal(m1, means[g])
        single.free()
    for c in caches:
        c.free()


def test_batched_mixed_sizes_equal_single():
    """A batch whose GPs span n = 3.7e3 .. 1.2e5 (the large ones run the row
    kernels with 4 rows per lane, the small ones with 1): every GP's cache
    equals its single build bit for bit, and matches the FP64 oracle."""
    Ps = WL.batched_config(G=6, seed=1, scale=1.0, t_per_gp=2000, n_lo=2000, n_hi=150000)
    print([(P.n, P.m[0], P.k) for P in Ps], flush=True)
    cfgs = [cfg_of(P) for P in Ps]
    xs = [tdev(P.x, torch.float32) for P in Ps]
    ys = [tdev(P.y, torch.float32) for P in Ps]
    caches = B.build_cache_batched(cfgs, xs, ys)
    qs = [tdev(P.xs, torch.float32) for P in Ps]
    means, vars_ = B.predict_mean_var_batched(caches, qs)
    for g, P in enumerate(Ps):
        single = build(P)
        m1, v1 = single.predict_mean_var(qs[g])
        assert torch.equal(v1, vars_[g]) and torch.equal(m1, means[g])
        assert single.info().k_eff == caches[g].info().k_eff
        single.free()
    # the smallest GP against the oracle (same k)
    g = int(np.argmin([P.n for P in Ps]))
    P = Ps[g]
    oc = oracle_cache(P)
    m_ref, v_ref = O.love_predict(oc, P.xs)
    e = errors(host(vars_[g]), v_ref, O.prior_var(P.xs, spec_of(P)), host(means[g]), m_ref, P.y)
    print(e, flush=True)
    assert e["e_p_max"] <= 1e-4 and e["mean_err_rel_rms_y"] <= 1e-4
    for c in caches:
        c.free()


def test_batched_grid_and_row_first_pass_equal_single():
    """A batch mixing GPs whose first Gram-Schmidt pass runs in grid space
    (m <= n) with GPs whose pass runs over the data rows (m > n): each GP's
    cache equals its single build bit for bit, and the m > n GP matches the
    FP64 oracle."""
    Pa = WL.config(2, scale=0.02, k_sample=0)                 # n = 2000, m = 200
    Pb = WL.config(2, scale=0.02, k_sample=0, m=(3000,))      # n = 2000, m = 3000
    Pc = WL.config(2, scale=0.05, k_sample=0)                 # n = 5000, m = 500
    Ps = [Pa, Pb, Pc]
    print([(P.n, P.m[0], P.k) for P in Ps], flush=True)
    cfgs = [cfg_of(P) for P in Ps]
    xs = [tdev(P.x, torch.float32) for P in Ps]
    ys = [tdev(P.y, torch.float32) for P in Ps]
    caches = B.build_cache_batched(cfgs, xs, ys)
    qs = [tdev(P.xs, torch.float32) for P in Ps]
    means, vars_ = B.predict_mean_var_batched(caches, qs)
    for g, P in enumerate(Ps):
        single = build(P)
        m1, v1 = single.predict_mean_var(qs[g])
        assert torch.equal(v1, vars_[g]) and torch.equal(m1, means[g])
        assert single.info().k_eff == caches[g].info().k_eff
        single.free()
    oc = oracle_cache(Pb)
    m_ref, v_ref = O.love_predict(oc, Pb.xs)
    e = errors(host(vars_[1]), v_ref, O.prior_var(Pb.xs, spec_of(Pb)), host(means[1]), m_ref, Pb.y)
    print(e, flush=True)
    assert e["e_p_max"] <= 1e-4 and e["mean_err_rel_rms_y"] <= 1e-4
    for c in caches:
        c.free()


def test_keff_without_sync_matches_info():
    """love_cache_keff returns the counts a synchronous build recorded, and
    reads them from the device after an asynchronous build."""
    P = WL.config(2, scale=0.02, k_sample=40, s=8)
    c1 = build(P)
    i1 = c1.info()
    assert c1.keff() == (i1.k_eff, i1.k_eff_sample) and i1.k_eff_sample > 0
    c2 = build(P, flags=B.FLAG_ASYNC)
    assert c2.keff() == (i1.k_eff, i1.k_eff_sample)
    c1.free()
    c2.free()


@pytest.mark.parametrize("case", ["fp32_sampler", "fp64", "bf16split"])
def test_cache_import_roundtrip(case):
    """export -> import: the imported cache (no training data) answers every
    query bit for bit like the built one."""
    if case == "fp32_sampler":
        P = WL.config(2, scale=0.02, k_sample=40, s=64)
    elif case == "fp64":
        P = WL.config(1)
    else:
        P = WL.config(3, scale=0.01)
    dt = torch.float64 if P.precision == "fp64" else torch.float32
    cache = build(P)
    parts = cache.export()
    imp = B.import_cache(cfg_of(P), parts)
    i0, i1 = cache.info(), imp.info()
    assert (i1.k_eff, i1.k_eff_sample, i1.n) == (i0.k_eff, i0.k_eff_sample, 0)
    assert cache.keff() == imp.keff() == (i0.k_eff, i0.k_eff_sample)
    xs = tdev(P.xs[:5000], dt)
    m0, v0 = cache.predict_mean_var(xs)
    m1, v1 = imp.predict_mean_var(xs)
    assert torch.equal(m0, m1) and torch.equal(v0, v1)
    assert torch.equal(cache.predict_covar_block(xs[:100], xs[100:300]),
                       imp.predict_covar_block(xs[:100], xs[100:300]))
    g = torch.ones(xs.shape[0], device=xs.device, dtype=dt)
    assert torch.equal(cache.predict_backward(xs, g, g)[0], imp.predict_backward(xs, g, g)[0])
    if i0.k_eff_sample > 0:
        xss, z = tdev(P.xs_sample, dt), tdev(P.z, torch.float32)
        assert torch.equal(cache.sample_posterior(xss, z), imp.sample_posterior(xss, z))
    with pytest.raises(B.LoveError):
        imp.apply_khat(torch.zeros(P.n, device=xs.device, dtype=dt))
    imp.free()
    cache.free()


def test_edge_cases():
    P = WL.config(2, scale=0.01, k_sample=0)
    cache = build(P)
    # empty query
    mu, var = cache.predict_mean_var(torch.empty(0, 1, device=dev()))
    assert var.numel() == 0
    # query outside the domain -> NaN and a status flag, others unaffected
    xs = torch.tensor([[0.5], [1.5], [0.0], [1.0]], device=dev())
    mu, var = cache.predict_mean_var(xs)
    v = host(var)
    assert np.isnan(v[1]) and np.isfinite(v[[0, 2, 3]]).all()
    assert cache.info().status_flags & 1
    cache.free()
    # k larger than n is clamped
    P2 = WL.config(2, scale=0.0005, k_sample=0)   # n = 50
    c = build(P2, k=100)
    assert c.info().k_eff <= P2.n
    c.free()
    # all training points identical: invariant subspace after few steps (breakdown, not an error)
    P3 = WL.config(2, scale=0.01, k_sample=0, dtype="f64", precision="fp64")
    P3.x[:] = 0.37
    c = build(P3)
    inf = c.info()
    assert inf.k_eff < 10 and inf.status_flags & 8
    _, var = c.predict_mean_var(tdev(P3.xs[:100], torch.float64))
    assert np.isfinite(host(var)).all()
    c.free()
    # training point outside the domain -> EDOMAIN ; non-finite target -> ENONFINITE
    P4 = WL.config(2, scale=0.01, k_sample=0)
    P4.x[5] = 1.25
    with pytest.raises(B.LoveError) as ei:
        build(P4)
    assert ei.value.code == -2
    P5 = WL.config(2, scale=0.01, k_sample=0)
    P5.y[7] = np.nan
    with pytest.raises(B.LoveError) as ei:
        build(P5)
    assert ei.value.code == -6
    # ragged n (not a multiple of any tile) and tiny grid
    P6 = WL.config(2, scale=0.0123, k_sample=0, m=(4,))
    c = build(P6, k=4)
    _, var = c.predict_mean_var(tdev(P6.xs[:50], torch.float32))
    oc = oracle_cache(P6, k=4)
    _, v_ref = O.love_predict(oc, P6.xs[:50])
    p = O.prior_var(P6.xs[:50], spec_of(P6))
    assert np.max(np.abs(host(var) - v_ref) / p) <= 1e-5
    c.free()
