"""FP64 CPU oracle for LOVE (LanczOs Variance Estimates) on KISS-GP.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
GPU path is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and this
module imports nothing from the library.

Everything is float64 numpy / scipy, written from the paper (Pleiss, Gardner,
Weinberger, Wilson, "Constant-Time Predictive Distributions for Gaussian
Processes", ICML 2018):

  * GP posterior mean / covariance .............. Sec. 2, eqs. pred_mean, pred_covar
  * Lanczos tridiagonalisation ................... Sec. 2.2
  * SKI / KISS-GP interpolation ................. Sec. 2.3, eq. ski
  * constant-time mean a = K W^T Khat^-1 y ...... Sec. 2.3, eq. pred_mean_ski
  * exact KISS-GP covariance (naive cache C) .... Sec. 3.1, eqs. pred_covar_approx,
                                                    pred_covar_ski_cache
  * LOVE cache R, R' and the O(k) query ......... Sec. 3.2, eq. pred_covar_ski_fast,
                                                    Algorithm 1
  * LOVE sampling matrix S ...................... Sec. 3.3, eqs. pred_covar_ski_interp_form12,
                                                    lancapprox, pred_covar_ski_interp_form
  * full reorthogonalisation .................... Sec. 5, "Numerical stability of Lanczos"
  * additive kernel compositions ................ Sec. 3.4, eq. multi_dimensional_kernel_block

Readings of points the paper leaves open (each is listed in the design notes):
  grid      padded regular grid, h = (hi-lo)/(m-3), u_j = lo + (j-1) h
  Keys      cubic convolution kernel with a = -1/2
  stencil   base j = clamp(floor((x-lo)/h), 0, m-4), s = (x-lo)/h - j
  d-D       tensor-product weights, row-major flattening (last dim fastest),
            K = outputscale * (T_1 kron ... kron T_d)
  prior     the interpolated prior p(x*) = w*^T K w* is the k_{x*x*} term
  Lanczos   alpha_j = q_j^T A q_j, three-term recurrence, two classical
            Gram-Schmidt passes against all previous vectors every step,
            stop when beta_j <= tol * max|alpha|
  sampler   second Lanczos probe b' = (1/m) (K - R^T R') 1, k' = k, Cholesky
            of T'; when T' is not positive definite (K - R^T R' is only
            positive semi-definite, and rounding can push Ritz values below
            zero) S = Q' V diag(max(lam, 0))^{1/2} from T' = V diag(lam) V^T,
            which gives the same S S^T whenever the Cholesky exists
  noise     `noise` is sigma^2 (a variance)
  additive  k(x, x') = outputscale * sum_d k_d(x_d, x'_d): one 1-D component per
            dimension on that dimension's grid; the stacked grid holds the
            axes one after another (axis 0 first), K is block diagonal
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# Problem description
# ---------------------------------------------------------------------------
@dataclass
class Spec:
    """A KISS-GP problem: regular grid, product stationary kernel, noise.

    m[d], lo[d], hi[d]: grid points and data domain per dimension (Sec. 2.3).
    kernel: "rbf" or "matern52" (product over dimensions, or a sum of 1-D
    components when additive: Sec. 3.4).
    lengthscale[d], outputscale, noise (= sigma^2, eq. pred_covar).
    """
    m: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    kernel: str = "rbf"
    lengthscale: Tuple[float, ...] = (0.1,)
    outputscale: float = 1.0
    noise: float = 0.01
    additive: bool = False

    @property
    def d(self) -> int:
        return len(self.m)

    @property
    def mtot(self) -> int:
        return int(np.sum(self.m)) if self.additive else int(np.prod(self.m))

    def offset(self, dim: int) -> int:
        """First index of axis `dim`'s block in the stacked additive grid."""
        return int(np.sum(self.m[:dim]))

    def h(self, dim: int) -> float:
        return (self.hi[dim] - self.lo[dim]) / (self.m[dim] - 3)


# ---------------------------------------------------------------------------
# Sec. 2.3: cubic interpolation (Keys 1981, a = -1/2)
# ---------------------------------------------------------------------------
def keys_psi(r):
    """Keys cubic convolution kernel psi(r), a = -1/2."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    near = r <= 1.0
    far = (r > 1.0) & (r < 2.0)
    rn, rf = r[near], r[far]
    out[near] = 1.5 * rn**3 - 2.5 * rn**2 + 1.0
    out[far] = -0.5 * rf**3 + 2.5 * rf**2 - 4.0 * rf + 2.0
    return out


def keys_dpsi(r):
    """d psi / d r for r >= 0 (psi is C^1, so the value at the knots is unique)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    near = (r >= 0.0) & (r <= 1.0)
    far = (r > 1.0) & (r < 2.0)
    rn, rf = r[near], r[far]
    out[near] = 4.5 * rn**2 - 5.0 * rn
    out[far] = -1.5 * rf**2 + 5.0 * rf - 4.0
    return out


def grid_nodes(spec: Spec, dim: int) -> np.ndarray:
    """Regular grid along one axis, padded by one cell on each side."""
    h = spec.h(dim)
    return spec.lo[dim] + (np.arange(spec.m[dim], dtype=np.float64) - 1.0) * h


def stencil_axis(x, spec: Spec, dim: int):
    """Per-axis cubic stencil: base node j, weights w[4], d w / d x [4].

    Nodes j..j+3 sit at offsets 1+s, s, 1-s, 2-s (in cells) from x.
    """
    x = np.asarray(x, dtype=np.float64)
    h = spec.h(dim)
    tau = (x - spec.lo[dim]) / h
    j = np.clip(np.floor(tau), 0, spec.m[dim] - 4).astype(np.int64)
    s = tau - j
    w = np.stack([keys_psi(1.0 + s), keys_psi(s), keys_psi(1.0 - s), keys_psi(2.0 - s)], axis=-1)
    # d/ds psi(|1+s|) = psi'(1+s); d/ds psi(|s|) = psi'(s); d/ds psi(1-s) = -psi'(1-s) ...
    dw = np.stack([keys_dpsi(1.0 + s), keys_dpsi(s), -keys_dpsi(1.0 - s), -keys_dpsi(2.0 - s)], axis=-1) / h
    return j, w, dw


def interp_matrix(X, spec: Spec) -> sp.csr_matrix:
    """W (n x m): row i is w(x_i)^T with 4^d non-zeros (eq. ski, transposed).

    Additive (Sec. 3.4): row i stacks the d per-axis vectors w^(e)(x_ie),
    4 d non-zeros (eq. multi_dimensional_kernel_block)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    if X.shape[1] != spec.d:
        X = X.reshape(-1, spec.d)
    n, d = X.shape
    if spec.additive:
        return _stacked(X, spec, [stencil_axis(X[:, e], spec, e)[1] for e in range(d)])
    cols = np.zeros((n, 1), dtype=np.int64)
    vals = np.ones((n, 1), dtype=np.float64)
    for dim in range(d):
        j, w, _ = stencil_axis(X[:, dim], spec, dim)
        idx = j[:, None] + np.arange(4)[None, :]
        cols = (cols[:, :, None] * spec.m[dim] + idx[:, None, :]).reshape(n, -1)
        vals = (vals[:, :, None] * w[:, None, :]).reshape(n, -1)
    rows = np.repeat(np.arange(n), cols.shape[1])
    W = sp.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(n, spec.mtot))
    return W


def _stacked(X, spec: Spec, wts) -> sp.csr_matrix:
    """Additive block form: axis e's 4 weights wts[e] at columns offset(e) + j_e + 0..3."""
    n, d = X.shape
    cols, vals = [], []
    for e in range(d):
        j, _, _ = stencil_axis(X[:, e], spec, e)
        cols.append(spec.offset(e) + j[:, None] + np.arange(4)[None, :])
        vals.append(wts[e])
    cols = np.concatenate(cols, axis=1)
    vals = np.concatenate(vals, axis=1)
    rows = np.repeat(np.arange(n), cols.shape[1])
    return sp.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(n, spec.mtot))


def interp_grad_matrices(X, spec: Spec) -> List[sp.csr_matrix]:
    """d W / d x_dim for each dim: same sparsity, derivative weights in dim `dim`.

    Additive: only axis dim's block depends on x_dim (the others are zero)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64)).reshape(-1, spec.d)
    n, d = X.shape
    per = [stencil_axis(X[:, e], spec, e) for e in range(d)]
    if spec.additive:
        return [_stacked(X, spec, [per[e][2] if e == dim else np.zeros_like(per[e][1])
                                   for e in range(d)]) for dim in range(d)]
    out = []
    for dim in range(d):
        cols = np.zeros((n, 1), dtype=np.int64)
        vals = np.ones((n, 1), dtype=np.float64)
        for e in range(d):
            j, w, dw = per[e]
            ww = dw if e == dim else w
            idx = j[:, None] + np.arange(4)[None, :]
            cols = (cols[:, :, None] * spec.m[e] + idx[:, None, :]).reshape(n, -1)
            vals = (vals[:, :, None] * ww[:, None, :]).reshape(n, -1)
        rows = np.repeat(np.arange(n), cols.shape[1])
        out.append(sp.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(n, spec.mtot)))
    return out


# ---------------------------------------------------------------------------
# Sec. 2.3: K_UU on a regular grid is Toeplitz / Kronecker of Toeplitz
# ---------------------------------------------------------------------------
def kernel_1d(r, kind: str, ell: float):
    r = np.abs(np.asarray(r, dtype=np.float64))
    if kind == "rbf":
        return np.exp(-0.5 * (r / ell) ** 2)
    if kind == "matern52":
        z = math.sqrt(5.0) * r / ell
        return (1.0 + z + z * z / 3.0) * np.exp(-z)
    raise ValueError(kind)


def toeplitz_column(spec: Spec, dim: int) -> np.ndarray:
    """First column of T_dim: k_dim(|i| h_dim), i = 0..m_dim-1 (outputscale not included)."""
    return kernel_1d(np.arange(spec.m[dim]) * spec.h(dim), spec.kernel, spec.lengthscale[dim])


def K_dense(spec: Spec) -> np.ndarray:
    """Dense K_UU = outputscale * kron(T_1, ..., T_d) (small grids only);
    additive: outputscale * blockdiag(T_1, ..., T_d)."""
    if spec.additive:
        return spec.outputscale * sla.block_diag(
            *[sla.toeplitz(toeplitz_column(spec, e)) for e in range(spec.d)])
    K = np.ones((1, 1))
    for dim in range(spec.d):
        K = np.kron(K, sla.toeplitz(toeplitz_column(spec, dim)))
    return spec.outputscale * K


def K_apply(spec: Spec, G: np.ndarray) -> np.ndarray:
    """K_UU @ G for G of shape (m,) or (m, B), through the Kronecker axes.

    Each axis is a symmetric Toeplitz product (scipy's matmul_toeplitz, i.e. a
    library Toeplitz product)."""
    G = np.asarray(G, dtype=np.float64)
    vec = G.ndim == 1
    B = 1 if vec else G.shape[1]
    if spec.additive:
        # block diagonal: each axis's own block of the stacked grid (Sec. 3.4)
        G2 = G.reshape(spec.mtot, B)
        Y = np.empty_like(G2)
        for e in range(spec.d):
            blk = slice(spec.offset(e), spec.offset(e) + spec.m[e])
            c = toeplitz_column(spec, e)
            if spec.m[e] <= 512:
                Y[blk] = sla.toeplitz(c) @ G2[blk]
            else:
                Y[blk] = sla.matmul_toeplitz((c, c), G2[blk], check_finite=False)
        Y = spec.outputscale * Y
        return Y[:, 0] if vec else Y
    Y = G.reshape(*spec.m, B)
    for dim in range(spec.d):
        c = toeplitz_column(spec, dim)
        Y = np.moveaxis(Y, dim, 0)
        sh = Y.shape
        Y2 = Y.reshape(sh[0], -1)
        if sh[0] <= 512:
            Y2 = sla.toeplitz(c) @ Y2
        else:
            Y2 = sla.matmul_toeplitz((c, c), Y2, check_finite=False)
        Y = np.moveaxis(Y2.reshape(sh), 0, dim)
    Y = spec.outputscale * Y.reshape(spec.mtot, B)
    return Y[:, 0] if vec else Y


def prior_var(Xs, spec: Spec) -> np.ndarray:
    """p(x*) = w*^T K_UU w*  (interpolated prior variance, the k_{x*x*} term).

    For tensor-product w and Kronecker K this is outputscale * prod_d w_d^T T_d w_d,
    where only the 4x4 block of T_d on the stencil nodes enters; additive:
    outputscale * sum_d w_d^T T_d w_d."""
    Xs = np.atleast_2d(np.asarray(Xs, dtype=np.float64)).reshape(-1, spec.d)
    if spec.additive:
        p = np.zeros(Xs.shape[0])
        for dim in range(spec.d):
            _, w, _ = stencil_axis(Xs[:, dim], spec, dim)
            T4 = sla.toeplitz(toeplitz_column(spec, dim)[:4])
            p += np.einsum("ia,ab,ib->i", w, T4, w)
        return spec.outputscale * p
    p = np.full(Xs.shape[0], spec.outputscale)
    for dim in range(spec.d):
        _, w, _ = stencil_axis(Xs[:, dim], spec, dim)
        c = toeplitz_column(spec, dim)[:4]
        T4 = sla.toeplitz(c)
        p *= np.einsum("ia,ab,ib->i", w, T4, w)
    return p


def prior_var_grad(Xs, spec: Spec) -> np.ndarray:
    """d p / d x*_dim (t x d)."""
    Xs = np.atleast_2d(np.asarray(Xs, dtype=np.float64)).reshape(-1, spec.d)
    if spec.additive:
        g = np.empty_like(Xs)
        for dim in range(spec.d):
            _, w, dw = stencil_axis(Xs[:, dim], spec, dim)
            T4 = sla.toeplitz(toeplitz_column(spec, dim)[:4])
            g[:, dim] = 2.0 * spec.outputscale * np.einsum("ia,ab,ib->i", dw, T4, w)
        return g
    per = []
    for dim in range(spec.d):
        _, w, dw = stencil_axis(Xs[:, dim], spec, dim)
        T4 = sla.toeplitz(toeplitz_column(spec, dim)[:4])
        per.append((np.einsum("ia,ab,ib->i", w, T4, w), 2.0 * np.einsum("ia,ab,ib->i", dw, T4, w)))
    g = np.empty_like(Xs)
    for dim in range(spec.d):
        prod = np.full(Xs.shape[0], spec.outputscale)
        for e in range(spec.d):
            prod = prod * (per[e][1] if e == dim else per[e][0])
        g[:, dim] = prod
    return g


# ---------------------------------------------------------------------------
# The training operator  Khat = W K W^T + sigma^2 I  (Alg. 1 input mvm_K_XX)
# ---------------------------------------------------------------------------
class Operator:
    def __init__(self, X, spec: Spec):
        self.spec = spec
        self.W = interp_matrix(X, spec)
        self.WT = self.W.T.tocsr()
        self.n = self.W.shape[0]

    def mvm_K_UX(self, V):
        """K_UU W^T V  (Alg. 1 input mvm_K_UX)."""
        return K_apply(self.spec, self.WT @ V)

    def mvm_K_XX(self, V):
        """(W K W^T + sigma^2 I) V."""
        return self.W @ self.mvm_K_UX(V) + self.spec.noise * V

    def dense(self) -> np.ndarray:
        Wd = self.W.toarray()
        return Wd @ K_dense(self.spec) @ Wd.T + self.spec.noise * np.eye(self.n)


# ---------------------------------------------------------------------------
# Exact KISS-GP predictions (the targets LOVE approximates)
# ---------------------------------------------------------------------------
def exact_route_A(X, y, Xs, spec: Spec):
    """Dense n-space: mean and variance from eqs. pred_mean_ski / pred_covar_approx.

    Returns (mean, var) with var = p(x*) - k~_{X x*}^T Khat^{-1} k~_{X x*}."""
    op = Operator(X, spec)
    A = op.dense()
    L = np.linalg.cholesky(A)
    Wd = op.W.toarray()
    K = K_dense(spec)
    KWt = K @ Wd.T                                  # m x n
    Ws = interp_matrix(Xs, spec).toarray()          # t x m
    kxs = (Ws @ KWt).T                              # n x t : k~_{X x*}
    alpha = sla.cho_solve((L, True), np.asarray(y, dtype=np.float64))
    mean = kxs.T @ alpha
    V = sla.solve_triangular(L, kxs, lower=True)
    var = prior_var(Xs, spec) - np.sum(V * V, axis=0)
    return mean, var


def exact_route_B(X, y, Xs, spec: Spec):
    """m-space identity: Sigma_U = K - K W^T Khat^{-1} W K = B (I + BW^TWB/sigma^2)^{-1} B,
    B = K^{1/2}.  var = ||L_B^{-1} B w*||^2; mean through Woodbury.  No cancellation."""
    op = Operator(X, spec)
    s2 = spec.noise
    K = K_dense(spec)
    lam, U = np.linalg.eigh(K)
    lam = np.clip(lam, 0.0, None)
    B = (U * np.sqrt(lam)) @ U.T
    WtW = (op.WT @ op.W).toarray()
    M = np.eye(spec.mtot) + (B @ WtW @ B) / s2
    LB = np.linalg.cholesky(M)
    Ws = interp_matrix(Xs, spec).toarray()
    Z = sla.solve_triangular(LB, B @ Ws.T, lower=True)
    var = np.sum(Z * Z, axis=0)
    # Khat^{-1} y = (y - G (s2 I + G^T G)^{-1} G^T y) / s2,  G = W B
    yv = np.asarray(y, dtype=np.float64)
    G = op.W @ B
    Gty = G.T @ yv
    inner = np.linalg.solve(s2 * np.eye(spec.mtot) + G.T @ G, Gty)
    sol = (yv - G @ inner) / s2
    a = K @ (op.WT @ sol)
    mean = Ws @ a
    return mean, var


def exact_covariance_grid(X, spec: Spec) -> np.ndarray:
    """Sigma_U = K - K W^T Khat^{-1} W K (m x m), the grid-space posterior covariance."""
    op = Operator(X, spec)
    K = K_dense(spec)
    A = op.dense()
    KWt = K @ op.W.toarray().T
    L = np.linalg.cholesky(A)
    V = sla.solve_triangular(L, KWt.T, lower=True)
    return K - V.T @ V


# ---------------------------------------------------------------------------
# Sec. 2.1: linear conjugate gradients (mean cache, eq. pred_mean_ski)
# ---------------------------------------------------------------------------
def cg(matvec, b, tol=1e-12, maxit=2000):
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    bn = math.sqrt(b @ b)
    it = 0
    while it < maxit and math.sqrt(rr) > tol * bn:
        Ap = matvec(p)
        step = rr / (p @ Ap)
        x += step * p
        r -= step * Ap
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def mean_cache(op: Operator, y, tol=1e-12, maxit=2000):
    """a = K_UU W^T (W K W^T + sigma^2 I)^{-1} y (eq. pred_mean_ski), solve by CG."""
    sol, it = cg(op.mvm_K_XX, y, tol=tol, maxit=maxit)
    return op.mvm_K_UX(sol), it


# ---------------------------------------------------------------------------
# Sec. 2.2 + Sec. 5: Lanczos with full reorthogonalisation
# ---------------------------------------------------------------------------
@dataclass
class LanczosResult:
    Q: np.ndarray          # n x k_eff, orthonormal columns
    alpha: np.ndarray      # k_eff
    beta: np.ndarray       # k_eff - 1 off-diagonal of T, plus beta[k_eff-1] = residual norm
    k_eff: int

    def T(self) -> np.ndarray:
        k = self.k_eff
        return np.diag(self.alpha[:k]) + np.diag(self.beta[: k - 1], 1) + np.diag(self.beta[: k - 1], -1)


def lanczos(matvec, b, k: int, tol: float = 1e-12) -> LanczosResult:
    """k steps of Lanczos on the symmetric operator `matvec` with probe `b`.

    q_1 = b/||b||; alpha_j = q_j^T A q_j; r = A q_j - alpha_j q_j - beta_{j-1} q_{j-1};
    r is then orthogonalised against every previous q twice (classical
    Gram-Schmidt, two passes); beta_j = ||r||; q_{j+1} = r / beta_j.
    Stops early (k_eff < k) when beta_j <= tol * max_i |alpha_i|."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    k = min(k, n)
    Q = np.zeros((n, k))
    alpha = np.zeros(k)
    beta = np.zeros(k)
    Q[:, 0] = b / np.linalg.norm(b)
    k_eff = k
    for j in range(k):
        q = Q[:, j]
        w = matvec(q)
        alpha[j] = q @ w
        r = w - alpha[j] * q
        if j > 0:
            r -= beta[j - 1] * Q[:, j - 1]
        Qj = Q[:, : j + 1]
        for _ in range(2):
            r -= Qj @ (Qj.T @ r)
        beta[j] = np.linalg.norm(r)
        if j + 1 == k:
            break
        if beta[j] <= tol * np.max(np.abs(alpha[: j + 1])):
            k_eff = j + 1
            break
        Q[:, j + 1] = r / beta[j]
    return LanczosResult(Q[:, :k_eff].copy(), alpha[:k_eff].copy(), beta[:k_eff].copy(), k_eff)


def tridiag_cholesky(alpha: np.ndarray, beta: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """T = L L^T for symmetric tridiagonal T (diag alpha, off-diag beta[:k-1]).

    Returns (ldiag, lsub): L has ldiag on the diagonal and lsub below it.
    Raises numpy.linalg.LinAlgError if T is not positive definite."""
    k = alpha.shape[0]
    ldiag = np.zeros(k)
    lsub = np.zeros(max(k - 1, 0))
    for i in range(k):
        piv = alpha[i] - (lsub[i - 1] ** 2 if i > 0 else 0.0)
        if not piv > 0.0:
            raise np.linalg.LinAlgError("T not positive definite at %d" % i)
        ldiag[i] = math.sqrt(piv)
        if i + 1 < k:
            lsub[i] = beta[i] / ldiag[i]
    return ldiag, lsub


# ---------------------------------------------------------------------------
# Sec. 3.2 + Algorithm 1: the LOVE cache
# ---------------------------------------------------------------------------
@dataclass
class LoveCache:
    spec: Spec
    R: np.ndarray           # k x m,  R  = Q_k^T W^T K   (Alg. 1)
    Rp: np.ndarray          # k x m,  R' = T_k^{-1} R    (Alg. 1, Cholesky solve)
    a: np.ndarray           # m,      mean cache (eq. pred_mean_ski)
    lanczos: LanczosResult
    cg_iters: int


def probe_vector(op: Operator) -> np.ndarray:
    """b = (1/m) W K 1, the average column of W_X^T K_UU (Sec. 3.2 / Alg. 1 input)."""
    m = op.spec.mtot
    return op.W @ K_apply(op.spec, np.ones(m)) / m


def love_build(X, y, spec: Spec, k: int, tol: float = 1e-12, cg_tol: float = 1e-12,
               cg_maxit: int = 2000) -> LoveCache:
    """Precomputation of Algorithm 1: Lanczos on Khat with probe b, Cholesky of T,
    R = (mvm_K_UX(Q_k))^T, R' = cholesky_solve(R, L); plus the mean cache a."""
    op = Operator(X, spec)
    b = probe_vector(op)
    lz = lanczos(op.mvm_K_XX, b, k, tol)
    ldiag, lsub = tridiag_cholesky(lz.alpha, lz.beta)
    L = np.diag(ldiag) + np.diag(lsub, -1)
    R = op.mvm_K_UX(lz.Q).T                           # k x m
    Rp = sla.cho_solve((L, True), R)                  # T^{-1} R
    a, it = mean_cache(op, y, tol=cg_tol, maxit=cg_maxit)
    return LoveCache(spec, R, Rp, a, lz, it)


def love_predict(cache: LoveCache, Xs):
    """Constant-time mean w*^T a and variance p(x*) - (R w*)^T (R' w*) (Alg. 1, i = j)."""
    Ws = interp_matrix(Xs, cache.spec)
    u = (Ws @ cache.R.T)                              # t x k : rows are (R w*)^T
    v = (Ws @ cache.Rp.T)                             # t x k : rows are (R' w*)^T
    var = prior_var(Xs, cache.spec) - np.sum(u * v, axis=1)
    mean = Ws @ cache.a
    return mean, var


def love_covariance(cache: LoveCache, Xi, Xj):
    """Cross-covariance k(x*_i, x*_j) = w_i^T K w_j - (R w_i)^T (R' w_j) for paired points."""
    Wi = interp_matrix(Xi, cache.spec)
    Wj = interp_matrix(Xj, cache.spec)
    kij = np.asarray((Wi.multiply(K_apply(cache.spec, Wj.T.toarray()).T)).sum(axis=1)).ravel()
    u = Wi @ cache.R.T
    v = Wj @ cache.Rp.T
    return kij - np.sum(u * v, axis=1)


def love_predict_grad(cache: LoveCache, Xs, g_mean=None, g_var=None):
    """Gradient of sum(g_mean * mean + g_var * var) with respect to x* (t x d).

    d mean/dx = (dw/dx)^T a;  d var/dx = dp/dx - (R dw)^T(R' w) - (R w)^T(R' dw)."""
    Xs = np.atleast_2d(np.asarray(Xs, dtype=np.float64)).reshape(-1, cache.spec.d)
    t, d = Xs.shape
    g_mean = np.zeros(t) if g_mean is None else np.asarray(g_mean, dtype=np.float64)
    g_var = np.zeros(t) if g_var is None else np.asarray(g_var, dtype=np.float64)
    Ws = interp_matrix(Xs, cache.spec)
    dWs = interp_grad_matrices(Xs, cache.spec)
    u = Ws @ cache.R.T
    v = Ws @ cache.Rp.T
    dp = prior_var_grad(Xs, cache.spec)
    out = np.empty((t, d))
    for dim in range(d):
        du = dWs[dim] @ cache.R.T
        dv = dWs[dim] @ cache.Rp.T
        dmean = dWs[dim] @ cache.a
        dvar = dp[:, dim] - np.sum(du * v, axis=1) - np.sum(u * dv, axis=1)
        out[:, dim] = g_mean * dmean + g_var * dvar
    return out


# ---------------------------------------------------------------------------
# Sec. 3.3: the sampling matrix S
# ---------------------------------------------------------------------------
@dataclass
class SamplerCache:
    S: np.ndarray          # m x k'_eff
    lanczos: LanczosResult
    k_chol: int            # columns of S
    used_cholesky: bool


def love_sampler(cache: LoveCache, k_sample: int, tol: float = 1e-12) -> SamplerCache:
    """Lanczos on K - R^T R' (eq. lancapprox) with probe (1/m)(K - R^T R') 1,
    then S = Q' L_{T'} (eq. pred_covar_ski_interp_form).  If T' is not
    numerically positive definite, S = Q' V sqrt(max(lam, 0)) instead (columns
    with lam <= 0 dropped), which has the same S S^T as the Cholesky route
    whenever that exists."""
    spec = cache.spec
    m = spec.mtot

    def mvm(v):
        return K_apply(spec, v) - cache.R.T @ (cache.Rp @ v)

    b = mvm(np.ones(m)) / m
    lz = lanczos(mvm, b, k_sample, tol)
    T = lz.T()
    amax = np.max(np.abs(lz.alpha))
    try:
        ldiag, lsub = tridiag_cholesky(lz.alpha, lz.beta)
        if np.min(ldiag ** 2) <= tol * amax:
            raise np.linalg.LinAlgError("numerically singular")
        L = np.diag(ldiag) + np.diag(lsub, -1)
        S = lz.Q @ L
        return SamplerCache(S, lz, S.shape[1], True)
    except np.linalg.LinAlgError:
        lam, V = np.linalg.eigh(T)
        keep = lam > 0
        S = lz.Q @ (V[:, keep] * np.sqrt(lam[keep]))
        return SamplerCache(S, lz, S.shape[1], False)


def love_sample(cache: LoveCache, sampler: SamplerCache, Xs, Z):
    """Samples mu(X*) + W_{X*}^T S v for each column v of Z (eq. sample): t x s."""
    Ws = interp_matrix(Xs, cache.spec)
    mean = Ws @ cache.a
    Z = np.asarray(Z, dtype=np.float64)[: sampler.S.shape[1]]
    return mean[:, None] + Ws @ (sampler.S @ Z)


def sample_covariance_implied(cache: LoveCache, sampler: SamplerCache, Xs) -> np.ndarray:
    """W* S S^T W*^T, the covariance the samples are drawn from (t x t)."""
    Ws = interp_matrix(Xs, cache.spec)
    F = Ws @ sampler.S
    return F @ F.T


# ---------------------------------------------------------------------------
# Metrics
# ---------------------------------------------------------------------------
def smae(pred, ref, y):
    """Scaled mean absolute error: mean |pred - ref| / Var(y) (Sec. 4 footnote)."""
    return float(np.mean(np.abs(np.asarray(pred) - np.asarray(ref))) / np.var(np.asarray(y, dtype=np.float64)))
