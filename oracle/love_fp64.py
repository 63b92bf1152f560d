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
  * LOVE cache and the O(k) query .............. Sec. 3.2, eqs. pred_covar_ski_cache,
                                                    pred_covar_ski_fast, lanczos_solve
  * Lanczos restart with a new probe ............ Sec. 5, "Ensuring Lanczos solves are accurate"
  * gradients w.r.t. x*, Rt and hyper-parameters  derived from eqs. pred_mean_ski,
                                                    pred_covar_approx, pred_covar_ski_fast
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
  cache     one m x k factor Rt = K W^T Q L^{-T} with R^T R' = Rt Rt^T (T = L L^T)
  restart   the solve is checked on run-averaged columns of W K; the new probe is
            the residual of the worst one; the two Krylov blocks are combined by
            the projected matrix H = Q^T Khat Q and its dense Cholesky factor
  hyper     hyper-parameters: lengthscale per dimension, outputscale, sigma^2;
            gradients of the LOVE variance take every solve Khat^{-1} as the
            cached Lanczos solve Q H^{-1} Q^T
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
# Derivatives of the grid kernel with respect to its hyper-parameters
# ---------------------------------------------------------------------------
def kernel_1d_dell(r, kind: str, ell: float):
    """d k(r) / d ell for the 1-D kernels of kernel_1d.

    RBF: k = exp(-r^2 / (2 ell^2)), so dk/dell = k r^2 / ell^3.
    Matern-5/2: k = (1 + z + z^2/3) e^{-z} with z = sqrt(5) r / ell; dk/dz =
    -z (1 + z) e^{-z} / 3 and dz/dell = -z / ell, so dk/dell = z^2 (1 + z) e^{-z} / (3 ell)."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    if kind == "rbf":
        return np.exp(-0.5 * (r / ell) ** 2) * r * r / ell ** 3
    if kind == "matern52":
        z = math.sqrt(5.0) * r / ell
        return z * z * (1.0 + z) * np.exp(-z) / (3.0 * ell)
    raise ValueError(kind)


def hyper_names(spec: Spec) -> List[str]:
    """Hyper-parameters in the order the gradients are returned: one lengthscale
    per dimension, then the outputscale, then the noise variance sigma^2."""
    return [f"lengthscale{e}" for e in range(spec.d)] + ["outputscale", "noise"]


def _toeplitz_apply(c: np.ndarray, G2: np.ndarray) -> np.ndarray:
    """Symmetric Toeplitz matrix with first column c times G2 (dense for short
    axes, scipy's FFT Toeplitz product for long ones)."""
    if c.shape[0] <= 512:
        return sla.toeplitz(c) @ G2
    return sla.matmul_toeplitz((c, c), G2, check_finite=False)


def K_apply_dtheta(spec: Spec, which: int, G: np.ndarray) -> np.ndarray:
    """(d K_UU / d theta_which) @ G for G of shape (m,) or (m, B), theta in
    hyper_names order: the product form differentiates one Kronecker factor,
    the additive form one diagonal block; d K / d outputscale = K / outputscale;
    the noise does not enter K_UU (zero)."""
    G = np.asarray(G, dtype=np.float64)
    if which == spec.d + 1:
        return np.zeros_like(G)
    if which == spec.d:
        return K_apply(spec, G) / spec.outputscale
    vec = G.ndim == 1
    B = 1 if vec else G.shape[1]
    e = which
    dcol = kernel_1d_dell(np.arange(spec.m[e]) * spec.h(e), spec.kernel, spec.lengthscale[e])
    if spec.additive:
        G2 = G.reshape(spec.mtot, B)
        Y = np.zeros_like(G2)
        blk = slice(spec.offset(e), spec.offset(e) + spec.m[e])
        Y[blk] = _toeplitz_apply(dcol, G2[blk])
    else:
        Y = G.reshape(*spec.m, B)
        for dim in range(spec.d):
            c = dcol if dim == e else toeplitz_column(spec, dim)
            Y = np.moveaxis(Y, dim, 0)
            sh = Y.shape
            Y = np.moveaxis(_toeplitz_apply(c, Y.reshape(sh[0], -1)).reshape(sh), 0, dim)
        Y = Y.reshape(spec.mtot, B)
    Y = spec.outputscale * Y
    return Y[:, 0] if vec else Y


def prior_var_dtheta(Xs, spec: Spec) -> np.ndarray:
    """d p(x*) / d theta (t x (d + 2), hyper_names order), p = w*^T K w*: only the
    4 x 4 blocks of the axis matrices on each point's stencil enter."""
    Xs = np.atleast_2d(np.asarray(Xs, dtype=np.float64)).reshape(-1, spec.d)
    t, d = Xs.shape
    quad, dquad = [], []
    for e in range(d):
        _, w, _ = stencil_axis(Xs[:, e], spec, e)
        r = np.arange(4) * spec.h(e)
        T4 = sla.toeplitz(toeplitz_column(spec, e)[:4])
        D4 = sla.toeplitz(kernel_1d_dell(r, spec.kernel, spec.lengthscale[e]))
        quad.append(np.einsum("ia,ab,ib->i", w, T4, w))
        dquad.append(np.einsum("ia,ab,ib->i", w, D4, w))
    out = np.zeros((t, d + 2))
    s = spec.outputscale
    for e in range(d):
        if spec.additive:
            out[:, e] = s * dquad[e]
        else:
            prod = np.full(t, s)
            for f in range(d):
                prod = prod * (dquad[f] if f == e else quad[f])
            out[:, e] = prod
    out[:, d] = prior_var(Xs, spec) / s
    return out


# ---------------------------------------------------------------------------
# The KISS-GP training operator (Sec. 2.3, eq. ski)
# ---------------------------------------------------------------------------
class KissOperator:
    """Khat = W K W^T + sigma^2 I with W the n x m interpolation matrix
    (the transpose of the paper's m x n W_X), and the grid-side product
    K W^T V (the paper's K_UU W_X V, an approximation of K_UX V)."""

    def __init__(self, X, spec: Spec):
        self.spec = spec
        self.W = interp_matrix(X, spec)
        self.WT = self.W.T.tocsr()
        self.n = self.W.shape[0]

    def to_grid(self, V):
        """K W^T V: n-space vectors mapped onto the grid (m x ...)."""
        return K_apply(self.spec, self.WT @ V)

    def khat(self, V):
        """(W K W^T + sigma^2 I) V."""
        return self.W @ self.to_grid(V) + self.spec.noise * V

    def dense(self) -> np.ndarray:
        Wd = self.W.toarray()
        return Wd @ K_dense(self.spec) @ Wd.T + self.spec.noise * np.eye(self.n)


# ---------------------------------------------------------------------------
# Exact KISS-GP predictions (the targets LOVE approximates)
# ---------------------------------------------------------------------------
def exact_route_A(X, y, Xs, spec: Spec):
    """Dense n-space: mean and variance from eqs. pred_mean_ski / pred_covar_approx.

    Returns (mean, var) with var = p(x*) - k~_{X x*}^T Khat^{-1} k~_{X x*}."""
    op = KissOperator(X, spec)
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
    op = KissOperator(X, spec)
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
    op = KissOperator(X, spec)
    K = K_dense(spec)
    A = op.dense()
    KWt = K @ op.W.toarray().T
    L = np.linalg.cholesky(A)
    V = sla.solve_triangular(L, KWt.T, lower=True)
    return K - V.T @ V


def _var_hyper_grad(spec: Spec, W, Xs, Z, g, with_scale: bool = False):
    """sum_i g_i d var_i / d theta (hyper_names order) for
    var_i = w_i^T K w_i - w_i^T K W^T z_i, z_i = Khat^{-1} W K w_i (column i of
    Z, n x t), by the product rule:
      d var_i = w_i^T dK w_i - 2 w_i^T dK W^T z_i + z_i^T (W dK W^T + d sigma^2 I) z_i
    (the last term has a plus sign because d(A^{-1}) = -A^{-1} dA A^{-1}).
    W is the training interpolation matrix (n x m, sparse).  with_scale also
    returns sum_i |g_i| (|w_i^T dK w_i| + 2 |w_i^T dK W^T z_i| + |third term|)
    per theta: the three terms nearly cancel (the variance is a small
    remainder of the prior), and this is the size rounding errors scale with."""
    Ws = interp_matrix(Xs, spec)
    g = np.asarray(g, dtype=np.float64)
    Y = np.asarray(W.T @ Z)                         # m x t : W^T z_i
    dp = prior_var_dtheta(Xs, spec)                 # t x (d + 2) : w_i^T dK w_i
    out = np.zeros(spec.d + 2)
    scale = np.zeros(spec.d + 2)
    for th in range(spec.d + 2):
        DY = K_apply_dtheta(spec, th, Y)
        cross = np.asarray(Ws.multiply(DY.T).sum(axis=1)).ravel()      # w_i^T dK W^T z_i
        quad = np.sum(Y * DY, axis=0)                                   # z_i^T W dK W^T z_i
        if th == spec.d + 1:
            quad = quad + np.sum(Z * Z, axis=0)
        out[th] = np.sum(g * (dp[:, th] - 2.0 * cross + quad))
        scale[th] = np.sum(np.abs(g) * (np.abs(dp[:, th]) + 2.0 * np.abs(cross) + np.abs(quad)))
    return (out, scale) if with_scale else out


def exact_var_hyper_grad(X, Xs, spec: Spec, g_var) -> np.ndarray:
    """Gradient of sum_i g_i var(x*_i) with respect to the hyper-parameters
    (hyper_names order) for the exact KISS-GP variance
    var = w^T K w - w^T K W^T Khat^{-1} W K w (eqs. pred_covar_approx,
    pred_covar_ski_cache), with z_i = Khat^{-1} W K w_i from a dense solve."""
    op = KissOperator(X, spec)
    Ws = interp_matrix(Xs, spec)
    Z = np.linalg.solve(op.dense(), op.W @ K_apply(spec, Ws.T.toarray()))
    return _var_hyper_grad(spec, op.W, Xs, Z, g_var)


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


def mean_cache(op: KissOperator, y, tol=1e-12, maxit=2000):
    """a = K_UU W^T (W K W^T + sigma^2 I)^{-1} y (eq. pred_mean_ski), solve by CG."""
    sol, it = cg(op.khat, y, tol=tol, maxit=maxit)
    return op.to_grid(sol), it


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


def lanczos(matvec, b, k: int, tol: float = 1e-12, basis=None) -> LanczosResult:
    """k steps of Lanczos on the symmetric operator `matvec` with probe `b`.

    q_1 = b/||b||; alpha_j = q_j^T A q_j; r = A q_j - alpha_j q_j - beta_{j-1} q_{j-1};
    r is then orthogonalised against every previous q twice (classical
    Gram-Schmidt, two passes); beta_j = ||r||; q_{j+1} = r / beta_j.
    Stops early (k_eff < k) when beta_j <= tol * max_i |alpha_i|.

    basis (n x p, orthonormal columns, optional): vectors of an earlier run
    that every new vector, b included, is also orthogonalised against (the
    second block of a restart, Sec. 5 "Ensuring Lanczos solves are accurate")."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    P = np.zeros((n, 0)) if basis is None else basis
    k = min(k, n - P.shape[1])
    Q = np.zeros((n, k))
    alpha = np.zeros(k)
    beta = np.zeros(k)
    for _ in range(2):
        b = b - P @ (P.T @ b)
    Q[:, 0] = b / np.linalg.norm(b)
    k_eff = k
    for j in range(k):
        q = Q[:, j]
        w = matvec(q)
        alpha[j] = q @ w
        r = w - alpha[j] * q
        if j > 0:
            r -= beta[j - 1] * Q[:, j - 1]
        Qj = np.concatenate([P, Q[:, : j + 1]], axis=1)
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
# Sec. 3.2: the LOVE cache
#
# C = K W^T Khat^{-1} W K (eq. pred_covar_ski_cache).  The Lanczos solve of
# eq. lanczos_solve replaces Khat^{-1} by Q T^{-1} Q^T; with T = L L^T this is
# C ~ (K W^T Q L^{-T}) (K W^T Q L^{-T})^T.  The cache is the one m x k factor
# Rt = K W^T Q L^{-T}: the paper's R^T R' equals Rt Rt^T, and a (co)variance
# is w_i^T K w_j - (Rt^T w_i) . (Rt^T w_j) (eq. pred_covar_ski_fast).
# ---------------------------------------------------------------------------
@dataclass
class LoveCache:
    spec: Spec
    Rt: np.ndarray          # m x k, C ~ Rt Rt^T
    a: np.ndarray           # m, mean cache (eq. pred_mean_ski)
    lanczos: LanczosResult  # Q of every block; alpha, beta of the first
    L: np.ndarray           # k x k lower factor of the projected matrix H = Q^T Khat Q
    cg_iters: int
    restarts: int = 0
    residuals: np.ndarray = field(default_factory=lambda: np.zeros(0))  # check residuals per round

    @property
    def k(self) -> int:
        return self.Rt.shape[1]


def probe_vector(op: KissOperator) -> np.ndarray:
    """b = (1/m) W K 1, the average column of W K (Sec. 3.2)."""
    m = op.spec.mtot
    return op.W @ K_apply(op.spec, np.ones(m)) / m


def check_groups(spec: Spec, groups: int) -> List[np.ndarray]:
    """Grid nodes split into `groups` runs of consecutive (flattened) indices."""
    bounds = np.linspace(0, spec.mtot, groups + 1).round().astype(np.int64)
    return [np.arange(bounds[g], bounds[g + 1]) for g in range(groups) if bounds[g + 1] > bounds[g]]


def solve_residuals(op: KissOperator, Q: np.ndarray, H: np.ndarray, groups: int):
    """Accuracy of the Lanczos solve Khat^{-1} c ~ Q H^{-1} Q^T c (eq.
    lanczos_solve) on the columns of W K the cache stands for: for each run g of
    grid nodes, c_g = W K 1_g / |g| (the average column of W K over the run), its
    relative residual ||c_g - Khat Q H^{-1} Q^T c_g|| / ||c_g||, and the
    residual vector.  Returns (relative residuals, residual vectors n x G)."""
    spec = op.spec
    C = np.empty((op.n, 0))
    cols = []
    for idx in check_groups(spec, groups):
        e = np.zeros(spec.mtot)
        e[idx] = 1.0 / idx.size
        cols.append(op.W @ K_apply(spec, e))
    C = np.stack(cols, axis=1)
    Xs = Q @ np.linalg.solve(H, Q.T @ C)
    Rr = C - op.khat(Xs)
    rel = np.linalg.norm(Rr, axis=0) / np.linalg.norm(C, axis=0)
    return rel, Rr


def love_build(X, y, spec: Spec, k: int, tol: float = 1e-12, cg_tol: float = 1e-12,
               cg_maxit: int = 2000, restart_tol: float = 0.0, restart_k: int = 0,
               max_restarts: int = 1, check_groups_n: int = 8) -> LoveCache:
    """The LOVE pre-computation (Sec. 3.2): k Lanczos steps on Khat from the
    probe b = (1/m) W K 1, the Cholesky factor of the projected matrix, the
    factor Rt = K W^T Q L^{-T}, and the mean cache a.

    Restart (Sec. 5, "Ensuring Lanczos solves are accurate"): with
    restart_tol > 0 the solve is checked on the run-averaged columns of W K
    (solve_residuals); while the worst relative residual exceeds restart_tol
    (and at most max_restarts times) restart_k further Lanczos steps are taken
    from a new probe, that run's residual vector, orthogonalised against all
    earlier vectors.  Q then holds both blocks, H = Q^T Khat Q is no longer
    tridiagonal (the blocks couple), and L is its dense Cholesky factor."""
    op = KissOperator(X, spec)
    lz = lanczos(op.khat, probe_vector(op), k, tol)
    ldiag, lsub = tridiag_cholesky(lz.alpha, lz.beta)
    Q = lz.Q
    L = np.diag(ldiag) + np.diag(lsub, -1)
    restarts = 0
    res_hist = []
    if restart_tol > 0.0:
        for _ in range(max_restarts + 1):
            H = L @ L.T
            rel, Rr = solve_residuals(op, Q, H, check_groups_n)
            res_hist.append(float(np.max(rel)))
            if np.max(rel) <= restart_tol or restarts == max_restarts or Q.shape[1] >= op.n:
                break
            worst = int(np.argmax(rel))
            lz2 = lanczos(op.khat, Rr[:, worst], restart_k, tol, basis=Q)
            Q = np.concatenate([Q, lz2.Q], axis=1)
            H = Q.T @ op.khat(Q)
            H = 0.5 * (H + H.T)
            L = np.linalg.cholesky(H)
            restarts += 1
        lz = LanczosResult(Q, lz.alpha, lz.beta, lz.k_eff)
    Rt = sla.solve_triangular(L, op.to_grid(Q).T, lower=True).T
    a, it = mean_cache(op, y, tol=cg_tol, maxit=cg_maxit)
    return LoveCache(spec, Rt, a, lz, L, it, restarts, np.array(res_hist))


def love_predict(cache: LoveCache, Xs):
    """Constant-time mean w*^T a (eq. pred_mean_ski) and variance
    p(x*) - ||Rt^T w*||^2 (eq. pred_covar_ski_fast with i = j)."""
    Ws = interp_matrix(Xs, cache.spec)
    u = Ws @ cache.Rt                                 # t x k
    var = prior_var(Xs, cache.spec) - np.sum(u * u, axis=1)
    mean = Ws @ cache.a
    return mean, var


def love_covariance(cache: LoveCache, Xi, Xj):
    """Cross-covariance w_i^T K w_j - (Rt^T w_i) . (Rt^T w_j) for paired points."""
    Wi = interp_matrix(Xi, cache.spec)
    Wj = interp_matrix(Xj, cache.spec)
    kij = np.asarray((Wi.multiply(K_apply(cache.spec, Wj.T.toarray()).T)).sum(axis=1)).ravel()
    return kij - np.sum((Wi @ cache.Rt) * (Wj @ cache.Rt), axis=1)


def love_predict_grad(cache: LoveCache, Xs, g_mean=None, g_var=None):
    """Gradient of sum(g_mean * mean + g_var * var) with respect to x* (t x d).

    d mean/dx = (dw/dx)^T a;  d var/dx = dp/dx - 2 (Rt^T w) . (Rt^T dw/dx)."""
    Xs = np.atleast_2d(np.asarray(Xs, dtype=np.float64)).reshape(-1, cache.spec.d)
    t, d = Xs.shape
    g_mean = np.zeros(t) if g_mean is None else np.asarray(g_mean, dtype=np.float64)
    g_var = np.zeros(t) if g_var is None else np.asarray(g_var, dtype=np.float64)
    Ws = interp_matrix(Xs, cache.spec)
    dWs = interp_grad_matrices(Xs, cache.spec)
    u = Ws @ cache.Rt
    dp = prior_var_grad(Xs, cache.spec)
    out = np.empty((t, d))
    for dim in range(d):
        du = dWs[dim] @ cache.Rt
        dmean = dWs[dim] @ cache.a
        dvar = dp[:, dim] - 2.0 * np.sum(u * du, axis=1)
        out[:, dim] = g_mean * dmean + g_var * dvar
    return out


def love_grad_rt(cache: LoveCache, Xs, g_var) -> np.ndarray:
    """d(sum_i g_i var(x*_i)) / d Rt (m x k): var_i depends on Rt only through
    -||Rt^T w_i||^2, whose derivative is -2 w_i (Rt^T w_i)^T."""
    Ws = interp_matrix(Xs, cache.spec)
    u = Ws @ cache.Rt
    g = np.asarray(g_var, dtype=np.float64)
    return -2.0 * (Ws.T @ (g[:, None] * u))


def love_var_hyper_grad(cache: LoveCache, X, Xs, g_var, with_scale: bool = False):
    """Gradient of sum_i g_i var(x*_i) with respect to the hyper-parameters
    (hyper_names order) through the LOVE cache: the product rule of
    exact_var_hyper_grad with every solve Khat^{-1} taken as the cached Lanczos
    solve Q H^{-1} Q^T (eq. lanczos_solve, H = L L^T), so
    z_i = Q L^{-T} L^{-1} Q^T W K w_i = Q L^{-T} u_i with u_i = Rt^T w_i.  Equal to
    the exact gradient once the Krylov space holds every column of W K."""
    spec = cache.spec
    op = KissOperator(X, spec)
    U = interp_matrix(Xs, spec) @ cache.Rt                                     # t x k
    Z = cache.lanczos.Q @ sla.solve_triangular(cache.L.T, U.T, lower=False)   # n x t
    return _var_hyper_grad(spec, op.W, Xs, Z, g_var, with_scale)


# ---------------------------------------------------------------------------
# Sec. 3.3: the sampling matrix S
# ---------------------------------------------------------------------------
@dataclass
class SamplerCache:
    S: np.ndarray          # m x k'_eff
    lanczos: LanczosResult
    k_chol: int            # columns of S
    used_cholesky: bool
    probe: np.ndarray      # b', the second Lanczos probe


def sampler_operator(cache: LoveCache):
    """v -> (K - R^T R') v = (K - Rt Rt^T) v, the test-independent part of the
    predictive covariance (eq. pred_covar_ski_interp_form12)."""
    spec = cache.spec
    return lambda v: K_apply(spec, v) - cache.Rt @ (cache.Rt.T @ v)


def sampler_probe(cache: LoveCache) -> np.ndarray:
    """b' = (1/m) (K - R^T R') 1: the average column of the sampler's operator,
    chosen as the first probe (1/m) W K 1 is for Khat (Sec. 3.3 names no probe)."""
    m = cache.spec.mtot
    return sampler_operator(cache)(np.ones(m)) / m


def love_sampler(cache: LoveCache, k_sample: int, tol: float = 1e-12,
                 factor: str = "auto") -> SamplerCache:
    """Lanczos on K - R^T R' (eq. lancapprox) from sampler_probe, then
    S = Q' L_{T'} (eq. pred_covar_ski_interp_form).  factor = "auto" takes the
    Cholesky factor when T' is numerically positive definite, else
    S = Q' V diag(max(lam, 0))^{1/2} from T' = V diag(lam) V^T (columns with
    lam <= 0 dropped), which has the same S S^T whenever the Cholesky exists;
    "cholesky" / "eigh" force one branch ("cholesky" raises LinAlgError when T'
    is not positive definite)."""
    mvm = sampler_operator(cache)
    b = sampler_probe(cache)
    lz = lanczos(mvm, b, k_sample, tol)
    T = lz.T()
    amax = np.max(np.abs(lz.alpha))
    if factor in ("auto", "cholesky"):
        try:
            ldiag, lsub = tridiag_cholesky(lz.alpha, lz.beta)
            if np.min(ldiag ** 2) <= tol * amax:
                raise np.linalg.LinAlgError("numerically singular")
            L = np.diag(ldiag) + np.diag(lsub, -1)
            S = lz.Q @ L
            return SamplerCache(S, lz, S.shape[1], True, b)
        except np.linalg.LinAlgError:
            if factor == "cholesky":
                raise
    lam, V = np.linalg.eigh(T)
    keep = lam > 0
    S = lz.Q @ (V[:, keep] * np.sqrt(lam[keep]))
    return SamplerCache(S, lz, S.shape[1], False, b)


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


def sample_covariance_mae(samples, ref_cov) -> float:
    """Element-wise mean absolute error between the sample covariance of the
    columns of `samples` (t x s) and a reference t x t covariance (the
    sample-accuracy metric of the sampling experiments, Sec. 4)."""
    S = np.asarray(samples, dtype=np.float64)
    emp = np.cov(S)
    return float(np.mean(np.abs(emp - np.asarray(ref_cov, dtype=np.float64))))
