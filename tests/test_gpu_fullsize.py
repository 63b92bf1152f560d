"""Parity at the full sizes of the benchmark workloads, through the C ABI.

  1-D sampler   n = 1e5, m = 1e4, k = k' = 100: the implied covariance
                W* S S^T W*^T of the GPU's sampling matrix against the oracle's
                (Sec. 3.3, eqs. lancapprox, pred_covar_ski_interp_form),
                element by element at 300 of the 1e4 sample points
  4-D FD        n = 2e5, m = 20^4, k = 64 in FP64 on the GPU: the backward
                (d mean / d x*, d var / d x*) against central finite
                differences of the forward (h = 1e-3, smaller next to grid
                lines), per point and axis
  2-D / 4-D     the FP64 oracle's answers at 2000 sampled test points of the
                full workloads (tests/golden/make_fullsize.py writes them: its
                mean CG takes thousands of iterations at these sizes)
"""
import os

import numpy as np
import pytest
import torch

from oracle import love_fp64 as O
from paper_1803_06058_amd import workloads as WL

from gpu_helpers import build, errors, oracle_cache, spec_of, tdev, torch_dtype

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def test_config2_sampler_full_size_elementwise():
    """k' = 100 < m = 1e4: both sides truncate the second Lanczos at the same
    k', on operators that differ by the rounding of the float cache.  The
    implied covariances must agree element by element to 1e-5 of the prior,
    and each must lie within that of W*(K - Rt Rt^T)W*^T (the oracle's Rt)."""
    P = WL.config(2, s=16)
    print(P.name, P.n, P.m, P.k, P.k_sample, flush=True)
    cache = build(P)
    info = cache.info()
    S = host(cache.export()["s"])
    cache.free()
    xs = P.xs_sample[:300].astype(np.float64)
    spec = spec_of(P)
    Ws = O.interp_matrix(xs, spec)
    F = Ws @ S
    sig_gpu = F @ F.T
    oc = oracle_cache(P)
    osm = O.love_sampler(oc, P.k_sample)
    sig_or = O.sample_covariance_implied(oc, osm, xs)
    Wd = Ws.toarray()
    U = Wd @ oc.Rt
    target = Wd @ O.K_apply(spec, Wd.T) - U @ U.T
    p = O.prior_var(xs, spec)
    scale = np.sqrt(np.outer(p, p))
    e_go = np.max(np.abs(sig_gpu - sig_or) / scale)
    e_gt = np.max(np.abs(sig_gpu - target) / scale)
    e_ot = np.max(np.abs(sig_or - target) / scale)
    print(f"k_eff_sample gpu {info.k_eff_sample} oracle {osm.k_chol}: |gpu-oracle| {e_go:.3e} "
          f"|gpu-target| {e_gt:.3e} |oracle-target| {e_ot:.3e}", flush=True)
    assert e_go <= 1e-5
    assert e_gt <= 1e-5 and e_ot <= 1e-5


def test_config4_fp64_finite_differences():
    """The GPU's FP64 backward (d mean / d x*, d var / d x*) against central
    differences D(h) = (f(x + h e) - f(x - h e)) / 2h of its own forward, at
    2000 points x 4 axes of the full 4-D workload.

    Inside one grid cell the Keys interpolant is a polynomial in x_e (degree 3
    for the mean, 6 for the variance), so D(h) = f' + c2 h^2 + c4 h^4 + c6 h^6
    with c6 = f^(7) / 5040 = 0: the two-level Richardson value
    (64 D(h) - 20 D(2h) + D(4h)) / 45 is f' exactly, up to rounding.  Where
    [x - 4h, x + 4h] would cross a grid line the second derivative jumps and
    the expansion does not hold; there the step is shrunk to 0.2 of the
    distance to the line, so every window stays in the cell.  h = 1e-3 for
    every other point.  Each Richardson value must match the backward to 1e-8
    of the axis's largest derivative; the errors of the plain D(1e-3) and of
    one Richardson level are reported."""
    P = WL.config(4, dtype="f64", precision="fp64", k_sample=0)
    print(P.name, P.n, P.m, P.k, flush=True)
    cache = build(P)
    rng = np.random.default_rng(5)
    idx = rng.choice(P.t, 2000, replace=False)
    h = 1e-3
    xs = np.clip(P.xs[idx], 4 * h, 1 - 4 * h)
    xt = tdev(xs, torch.float64)
    ones = torch.ones(xs.shape[0], device=xt.device, dtype=torch.float64)
    zeros = torch.zeros_like(ones)
    ad = {"mean": host(cache.predict_backward(xt, ones, zeros)[0]),
          "var": host(cache.predict_backward(xt, zeros, ones)[0])}

    def central(e, step):
        xp, xm = xs.copy(), xs.copy()
        xp[:, e] += step
        xm[:, e] -= step
        mp, vp = cache.predict_mean_var(tdev(xp, torch.float64))
        mm, vm = cache.predict_mean_var(tdev(xm, torch.float64))
        return {"mean": (host(mp) - host(mm)) / (2 * step),
                "var": (host(vp) - host(vm)) / (2 * step)}

    hg = (P.hi[0] - P.lo[0]) / (P.m[0] - 3)
    n_shrunk = 0
    plain = {"mean": 0.0, "var": 0.0}
    worst = {"mean": 0.0, "var": 0.0}
    one = {"mean": 0.0, "var": 0.0}
    for e in range(P.d):
        u = (xs[:, e] - P.lo[e]) / hg
        dist = np.minimum(u - np.floor(u), np.ceil(u) - u) * hg
        step = np.minimum(h, 0.2 * dist)
        n_shrunk += int(np.sum(step < h))
        d1, d2, d4 = central(e, step), central(e, 2 * step), central(e, 4 * step)
        d_plain = central(e, np.full(xs.shape[0], h))
        for name in ("mean", "var"):
            a = ad[name][:, e]
            scale = np.max(np.abs(a))
            rich2 = (64 * d1[name] - 20 * d2[name] + d4[name]) / 45
            rich1 = (4 * d1[name] - d2[name]) / 3
            err = float(np.max(np.abs(a - rich2)) / scale)
            worst[name] = max(worst[name], err)
            one[name] = max(one[name], float(np.max(np.abs(a - rich1)) / scale))
            plain[name] = max(plain[name], float(np.max(np.abs(a - d_plain[name])) / scale))
            assert err <= 1e-8, (name, e, err)
    print(f"points with a shrunk step {n_shrunk} of {xs.shape[0] * P.d}; "
          f"two-level Richardson vs backward: mean {worst['mean']:.2e} var {worst['var']:.2e}; "
          f"one level: mean {one['mean']:.2e} var {one['var']:.2e}; "
          f"plain D(1e-3) vs backward: mean {plain['mean']:.2e} var {plain['var']:.2e}",
          flush=True)
    cache.free()


def _golden(name):
    path = os.path.join(GOLDEN, name)
    return dict(np.load(path, allow_pickle=False))


def test_config3_full_size_bf16split_and_fp32():
    """n = 5e5, m = 128 x 128, k = 100: the BF16-split cache within e_p 1e-3 of
    the oracle (route C, same k) and the plain FP32 cache within 1e-5, at 2000
    sampled points; both means within 1e-4 RMS(y)."""
    G = _golden("c3_full.npz")
    P = WL.config(3)
    xs = tdev(P.xs[G["idx"]], torch.float32)
    assert np.array_equal(P.xs[G["idx"]].astype(np.float64), G["xs"])
    for precision, tol in (("bf16split", 1e-3), ("fp32", 1e-5)):
        cache = build(P, precision=precision)
        mu, var = cache.predict_mean_var(xs)
        info = cache.info()
        e = errors(host(var), G["var"], G["prior"], host(mu), G["mean"], P.y)
        print(precision, "k_eff", info.k_eff, "oracle", int(G["k_eff"]), "cg", info.cg_iters, e,
              flush=True)
        assert e["e_p_max"] <= tol
        assert e["mean_err_rel_rms_y"] <= 1e-4
        cache.free()


def test_config4_full_size_forward_backward():
    """n = 2e5, m = 20^4, k = 64 (FP32): mean, variance and the backward
    (d mean_i / d x*_i, d var_i / d x*_i) at 2000 sampled points against the
    oracle (love_predict, love_predict_grad): e_p <= 1e-5, mean and d mean
    within 1e-4 of their scale, d var within 1e-5 of its terms' size."""
    G = _golden("c4_full.npz")
    P = WL.config(4)
    assert np.array_equal(P.xs[G["idx"]].astype(np.float64), G["xs"])
    cache = build(P)
    xt = tdev(P.xs[G["idx"]], torch.float32)
    mu, var = cache.predict_mean_var(xt)
    e = errors(host(var), G["var"], G["prior"], host(mu), G["mean"], P.y)
    ones = torch.ones(xt.shape[0], device=xt.device)
    zeros = torch.zeros_like(ones)
    dm = host(cache.predict_backward(xt, ones, zeros)[0])
    dv = host(cache.predict_backward(xt, zeros, ones)[0])
    r_m = np.max(np.abs(dm - G["dmean"])) / np.max(np.abs(G["dmean"]))
    # the variance gradient dp/dx - 2 u . du cancels like the variance itself:
    # its error, per point and axis, relative to the size of the two terms
    # (|dp/dx| + 2 ||u|| ||du||, from the oracle), as e_p is relative to the prior
    r_v = np.max(np.abs(dv - G["dvar"]) / G["dvar_scale"])
    print("k_eff", cache.info().k_eff, "oracle", int(G["k_eff"]), e, "dmean", r_m, "dvar", r_v,
          flush=True)
    assert e["e_p_max"] <= 1e-5
    assert e["mean_err_rel_rms_y"] <= 1e-4
    assert r_m <= 1e-4
    assert r_v <= 1e-5
    cache.free()
