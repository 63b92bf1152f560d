"""Restart with a new probe (Sec. 5, "Ensuring Lanczos solves are accurate")
through the C ABI against the oracle's love_build with the same restart
settings: the solve Q H^{-1} Q^T is checked on 8 averaged columns of W K, a
failing check appends restart_k Lanczos steps from the worst residual, and the
cache takes the dense Cholesky factor of H = Q^T Khat Q over both blocks.
Cases are built to need a restart (k far below what the solve needs): 1-D in
FP64 and FP32 (grid-space first pass, m <= n) and 4-D with m > n (W^T Q then
comes from a scatter after the run); a loose tolerance takes no restart and
leaves the cache bit for bit as a build without the check."""
import numpy as np
import pytest
import torch

from oracle import love_fp64 as O
from paper_1803_06058_amd import binding as B
from paper_1803_06058_amd import workloads as WL

from gpu_helpers import build, cfg_of, errors, spec_of, tdev, torch_dtype

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def oracle_restart(P, k, tol, rk, rmax=1):
    return O.love_build(P.x.astype(np.float64), P.y.astype(np.float64), spec_of(P), k,
                        cg_tol=1e-10, cg_maxit=5000, restart_tol=tol, restart_k=rk,
                        max_restarts=rmax, check_groups_n=8)


CASES = {
    # name: (problem, k, restart_k, restart_max, e_p tolerance)
    "1d_f64": (lambda: WL.config(2, scale=0.02, k_sample=0, dtype="f64", precision="fp64"),
               8, 20, 2, 1e-10),
    "1d_f32": (lambda: WL.config(2, scale=0.02, k_sample=0), 10, 30, 1, 1e-5),
    "4d_f32_m_gt_n": (lambda: WL.config(4, scale=0.01, k_sample=0), 10, 30, 1, 1e-5),
}


@pytest.mark.parametrize("case", list(CASES))
def test_restart_parity(case):
    mk, k, rk, rmax, tol = CASES[case]
    P = mk()
    rtol = 1e-4
    cache = build(P, k=k, restart_tol=rtol, restart_k=rk, restart_max=rmax)
    info = cache.info()
    oc = oracle_restart(P, k, rtol, rk, rmax)
    xs = P.xs[:3000]
    mu, var = cache.predict_mean_var(tdev(xs, torch_dtype(P)))
    m_ref, v_ref = O.love_predict(oc, xs.astype(np.float64))
    p = O.prior_var(xs, spec_of(P))
    e = errors(host(var), v_ref, p, host(mu), m_ref, P.y)
    print(case, "gpu restarts", info.restarts, "k_eff", info.k_eff, "residual", info.solve_residual,
          "| oracle restarts", oc.restarts, "k", oc.k, "residuals", oc.residuals, e, flush=True)
    assert oc.restarts >= 1, "the case must need a restart"
    assert info.restarts == oc.restarts
    assert info.k_eff == oc.k
    assert e["e_p_max"] <= tol
    assert e["mean_err_rel_rms_y"] <= (1e-9 if tol < 1e-8 else 1e-4)
    # the last check's worst residual, as the oracle's
    assert abs(info.solve_residual - oc.residuals[-1]) <= 1e-3 * oc.residuals[-1] + 1e-5
    cache.free()


def test_restart_not_needed_changes_nothing():
    """A tolerance the first run meets: no restart, and Rt, the mean cache and
    the variances equal those of a build without the check, bit for bit."""
    P = WL.config(2, scale=0.02, k_sample=0)
    xs = tdev(P.xs[:3000], torch.float32)
    a = build(P)
    b = build(P, restart_tol=0.5, restart_k=10)
    info = b.info()
    oc = oracle_restart(P, P.k, 0.5, 10)
    assert info.restarts == 0 and oc.restarts == 0
    # float Lanczos vectors: the check's residual carries their rounding
    assert abs(info.solve_residual - oc.residuals[0]) <= 1e-3 * oc.residuals[0] + 1e-5
    ea, eb = a.export(), b.export()
    for key in ("rt", "a", "alpha", "beta"):
        assert torch.equal(ea[key], eb[key]), key
    assert torch.equal(a.predict_mean_var(xs)[1], b.predict_mean_var(xs)[1])
    a.free()
    b.free()


def test_restart_arguments():
    P = WL.config(2, scale=0.02, k_sample=0)
    dt = torch_dtype(P)
    x, y = tdev(P.x, dt), tdev(P.y, dt)
    with pytest.raises(B.LoveError) as ei:      # restart_k missing
        B.build_cache(cfg_of(P, restart_tol=1e-3, restart_k=0), x, y)
    assert ei.value.code == -1
    with pytest.raises(B.LoveError) as ei:      # k + restart_max restart_k > LOVE_MAX_K
        B.build_cache(cfg_of(P, k=100, restart_tol=1e-3, restart_k=20, restart_max=2), x, y)
    assert ei.value.code == -1
    with pytest.raises(B.LoveError) as ei:      # batched builds do not restart
        B.build_cache_batched([cfg_of(P, restart_tol=1e-3, restart_k=10)] * 2, [x, x], [y, y])
    assert ei.value.code == -7
    with pytest.raises(B.LoveError) as ei:      # nor with the hyper-parameter factor
        B.build_cache(cfg_of(P, restart_tol=1e-3, restart_k=10, flags=B.FLAG_HYPER), x, y)
    assert ei.value.code == -7
