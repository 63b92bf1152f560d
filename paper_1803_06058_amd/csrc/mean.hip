// Mean cache by a grid-space solve, for Kronecker grids (d >= 2) whose axes
// have at most SPEC_MAXM points.
//
// The mean cache is a = K W^T Khat^{-1} y, the SKI predictive mean of Sec. 3
// with W the cubic interpolation and K = kron(T_1, ..., T_d).  For any B with
// K = B B^T the push-through identity gives
//   a = B (sigma^2 I + B^T W^T W B)^{-1} B^T W^T y,
// an m-space system whose matrix is sigma^2 I plus the nonzero spectrum of
// W K W^T.  B is taken as kron(B_e) with B_e B_e^T = T_e, chosen so that the
// system's expectation over evenly spread data is diagonal:
//   E[W^T W] = n kron(S_e), S_e the mean Gram matrix of one axis's four Keys
//   weights over a cell;  T_e = V_e diag(lam) V_e^T;
//   M_e = diag(sqrt lam) V_e^T S_e V_e diag(sqrt lam) = U_e diag(D_e) U_e^T;
//   B_e = V_e diag(sqrt lam) U_e,  so B_e B_e^T = T_e and B_e^T S_e B_e = D_e.
// Both eigen-decompositions are one-block parallel Jacobi runs in double
// (m_e <= 128).  CG then takes the diagonal preconditioner
// 1 / (sigma^2 + n prod_e D_e), the exact inverse of the expected matrix; only
// the sampling fluctuation of W^T W about its mean is left for CG.  CG on the
// data-space system Khat x = y needs about sqrt(cond(Khat)) iterations, which
// reaches thousands for 2-D and 4-D grids at these noise levels.
//
// Stopping rule: ||r|| <= tol sigma ||y||.  Since the matrix is at least
// sigma^2 I, the training-point mean W a then differs from the exact solve
// by at most tol ||y|| in the 2-norm.
//
// One iteration: u = B p (d axis passes), W u (gather), W^T (scatter),
// B^T (d axis passes) + sigma^2 p, the CG update, the scalar step, the new
// direction.  The CG scalars stay on the device (Ctl); the host checks for
// convergence every few iterations.
#include <algorithm>
#include <cmath>

#include "internal.h"
#include "ops.h"

namespace love {

namespace {

constexpr int EIG_THREADS = 512;
constexpr int SPB = 256;   // threads of the m- and n-length kernels

// buffer codes of the axis passes
enum : int { SB_Z = 0, SB_R, SB_P, SB_Q, SB_T0, SB_T1 };
__device__ inline double* spec_buf(const SpecJob& J, int b) {
  switch (b) {
    case SB_Z: return J.z;
    case SB_R: return J.r;
    case SB_P: return J.p;
    case SB_Q: return J.q;
    case SB_T0: return J.t0;
    default: return J.t1;
  }
}

// axis pass modes
enum : int {
  KP_FWD = 1,      // out_i = sum_j B[i][j] in_j   (else B^T)
  KP_ADD_SP = 2,   // output += sigma^2 p
  KP_DOT_P = 4,    // partial sums of p^T out (column 0)
  KP_FORCE = 8     // run after the solve has stopped (final a = B z)
};

// Sum of column c of the first nr partial rows, by one wave in a fixed order.
__device__ inline double spec_colsum(const double* __restrict__ part, int nr, int c) {
  const int lane = threadIdx.x & (WAVE - 1);
  double acc = 0.0;
  for (int b = lane; b < nr; b += WAVE) acc += part[(size_t)b * SPW + c];
  return wave_sum(acc);
}

// G[a][b] = integral over s in [0, 1] of w_a(s) w_b(s), the four Keys weights
// of a point at fraction s of its cell; 4-point Gauss-Legendre is exact for
// these degree-6 products.
__device__ inline void keys_gram(double G[4][4]) {
  const double xg[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563,
                        0.8611363115940526};
  const double wg[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461,
                        0.3478548451374538};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) G[a][b] = 0.0;
  for (int q = 0; q < 4; ++q) {
    double w[4];
    keys_weights<double>(0.5 * (xg[q] + 1.0), w);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) G[a][b] += 0.5 * wg[q] * w[a] * w[b];
  }
}

constexpr int HALF = SPEC_MAXM / 2;   // largest half problem

struct JacobiShared {
  double c[HALF / 2], s[HALF / 2];
  int p[HALF / 2], q[HALF / 2];
  double scr[16];
  int rotated;
};

// Symmetric A (mp x mp, mp even, row-major, LDS) -> diag by cyclic parallel
// Jacobi; V (LDS) <- V J accumulates the rotations.  Each round applies mp/2
// disjoint rotations (circle-method pairing): A <- J^T A J one 2 x 2 block per
// item, and every row of V mixes its column pairs.  Sweeps stop once a whole
// sweep finds every |a_pq| <= 1e-17 ||A||_F (at most 40).  Whole block; ends
// with a barrier.
__device__ void jacobi_block(double* A, double* V, int mp, JacobiShared& sh) {
  const int t = threadIdx.x, np = mp / 2, nt = blockDim.x;
  double fro = 0.0;
  for (int idx = t; idx < mp * mp; idx += nt) fro += A[idx] * A[idx];
  fro = block_sum(fro, sh.scr);
  const double thr = 1e-17 * sqrt(fro);
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (t == 0) sh.rotated = 0;
    __syncthreads();
    for (int rd = 0; rd < mp - 1; ++rd) {
      if (t < np) {
        // position 0 holds index 0, the others rotate one place per round
        const int pa = t, pb = mp - 1 - t;
        int p = pa == 0 ? 0 : ((pa - 1 + rd) % (mp - 1)) + 1;
        int q = ((pb - 1 + rd) % (mp - 1)) + 1;
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        const double apq = A[p * mp + q];
        double cc = 1.0, ss = 0.0;
        if (fabs(apq) > thr) {
          const double app = A[p * mp + p], aqq = A[q * mp + q];
          const double th = (aqq - app) / (2.0 * apq);
          const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          cc = 1.0 / sqrt(tt * tt + 1.0);
          ss = tt * cc;
          sh.rotated = 1;
        }
        sh.p[t] = p;
        sh.q[t] = q;
        sh.c[t] = cc;
        sh.s[t] = ss;
      }
      __syncthreads();
      for (int it = t; it < np * np; it += nt) {
        const int k1 = it / np, k2 = it % np;
        const double c1 = sh.c[k1], s1 = sh.s[k1], c2 = sh.c[k2], s2 = sh.s[k2];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int p1 = sh.p[k1], q1 = sh.q[k1], p2 = sh.p[k2], q2 = sh.q[k2];
        const double x00 = A[p1 * mp + p2], x01 = A[p1 * mp + q2];
        const double x10 = A[q1 * mp + p2], x11 = A[q1 * mp + q2];
        const double y00 = c1 * x00 - s1 * x10, y01 = c1 * x01 - s1 * x11;
        const double y10 = s1 * x00 + c1 * x10, y11 = s1 * x01 + c1 * x11;
        A[p1 * mp + p2] = c2 * y00 - s2 * y01;
        A[q1 * mp + q2] = s2 * y10 + c2 * y11;
        A[p1 * mp + q2] = (k1 == k2) ? 0.0 : s2 * y00 + c2 * y01;
        A[q1 * mp + p2] = (k1 == k2) ? 0.0 : c2 * y10 - s2 * y11;
      }
      for (int it = t; it < mp * np; it += nt) {
        const int i = it / np, k = it % np;
        const double cc = sh.c[k], ss = sh.s[k];
        if (ss == 0.0) continue;
        const int p = sh.p[k], q = sh.q[k];
        const double vp = V[i * mp + p], vq = V[i * mp + q];
        V[i * mp + p] = cc * vp - ss * vq;
        V[i * mp + q] = ss * vp + cc * vq;
      }
      __syncthreads();
    }
    const int done = !sh.rotated;
    __syncthreads();
    if (done) break;
  }
}

// Entry (i, j) of S_e: sum over cells c of G[i - c][j - c], over the cell count.
__device__ inline double s_entry(const double (&G)[4][4], int m, int i, int j) {
  if (abs(i - j) > 3) return 0.0;
  const int c0 = max(max(i, j) - 3, 0), c1 = min(min(i, j), m - 4);
  double v = 0.0;
  for (int c = c0; c <= c1; ++c) v += G[i - c][j - c];
  return v / (double)(m - 3);
}

// Entry (i, j) of X restricted to parity pi (0 even, 1 odd) for a centrosymmetric
// m x m matrix X (X[m-1-i][m-1-j] = X[i][j]): in the basis (e_i +- e_{m-1-i})/sqrt 2,
// i < m/2, plus e_mid (odd m, even part, index m/2) the matrix splits into
// X_pi[i][j] = X[i][j] +- X[i][m-1-j], X_+[i][mid] = sqrt2 X[i][mid], X_+[mid][mid] = X[mid][mid].
template <typename F>
__device__ inline double half_entry(F X, int m, int pi, int i, int j) {
  const int h = m / 2;
  const bool odd = m & 1;
  if (pi == 0 && odd) {
    const int mid = h;
    if (i == h && j == h) return X(mid, mid);
    if (i == h) return sqrt(2.0) * X(j, mid);
    if (j == h) return sqrt(2.0) * X(i, mid);
  }
  return X(i, j) + (pi == 0 ? 1.0 : -1.0) * X(i, m - 1 - j);
}

// ---------------------------------------------------------------------------
// Per-axis transform, one block per (GP, axis, parity).  T_e and S_e are
// centrosymmetric (Toeplitz; a cell sum of the Keys Gram matrix, which is
// invariant under s -> 1 - s), so both split into an even and an odd half of
// size <= 64.  For each half (all in LDS):
//   T_pi = V diag(lam) V^T;  M = diag(sqrt lam+) V^T S_pi V diag(sqrt lam+) = U diag(D) U^T;
//   B_pi = V diag(sqrt lam+) U.
// B_e has the even modes in columns [0, n_even) and the odd ones after them;
// its rows expand each half back to the grid: row r takes B_pi[min(r, m-1-r)] / sqrt 2,
// negated on the mirrored row of the odd half, and row mid of the even half as is.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(EIG_THREADS) void k_spec_axis(Tab tab,
                                                           const SpecJob* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SpecJob& J = jobs[gp];
  const int e = lb >> 1, pi = lb & 1;
  const int m = J.m[e], ld = J.ldv[e], h = m / 2;
  const bool odd = m & 1;
  const int nh = (pi == 0) ? h + (odd ? 1 : 0) : h;   // size of this half
  const int mp = (nh + 1) & ~1;
  const int off = pi == 0 ? 0 : h + (odd ? 1 : 0);     // first mode column
  const double* __restrict__ col = J.c64[e];
  __shared__ double A[HALF * HALF], V[HALF * HALF], W[HALF * HALF];
  __shared__ JacobiShared sh;
  __shared__ double sl[HALF];   // sqrt(max(lam, 0))
  const int t = threadIdx.x;
  const int mm = mp * mp;
  auto tx = [&](int i, int j) { return col[abs(i - j)]; };
  for (int idx = t; idx < mm; idx += blockDim.x) {
    const int i = idx / mp, j = idx % mp;
    A[idx] = (i < nh && j < nh) ? half_entry(tx, m, pi, i, j) : 0.0;
    V[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_block(A, V, mp, sh);
  for (int i = t; i < mp; i += blockDim.x) sl[i] = i < nh ? sqrt(fmax(A[i * mp + i], 0.0)) : 0.0;
  __syncthreads();
  double G[4][4];
  keys_gram(G);
  auto sx = [&](int i, int j) { return s_entry(G, m, i, j); };
  // W = S_pi V
  for (int idx = t; idx < mm; idx += blockDim.x) {
    const int i = idx / mp, j = idx % mp;
    double v = 0.0;
    if (i < nh)
      for (int k = 0; k < nh; ++k) v += half_entry(sx, m, pi, i, k) * V[k * mp + j];
    W[idx] = v;
  }
  __syncthreads();
  // A = M = diag(sl) V^T W diag(sl), symmetrised (the two products round differently)
  for (int idx = t; idx < mm; idx += blockDim.x) {
    const int i = idx / mp, j = idx % mp;
    if (i > j) continue;
    double v = 0.0, w = 0.0;
    if (sl[i] > 0.0 && sl[j] > 0.0)
      for (int k = 0; k < mp; ++k) {
        v += V[k * mp + i] * W[k * mp + j];
        w += V[k * mp + j] * W[k * mp + i];
      }
    const double a = 0.5 * sl[i] * (v + w) * sl[j];
    A[i * mp + j] = a;
    A[j * mp + i] = a;
  }
  __syncthreads();
  for (int idx = t; idx < mm; idx += blockDim.x) W[idx] = (idx / mp == idx % mp) ? 1.0 : 0.0;
  __syncthreads();
  jacobi_block(A, W, mp, sh);
  for (int j = t; j < nh; j += blockDim.x) J.D[e][off + j] = fmax(A[j * mp + j], 0.0);
  // A = B_pi = V diag(sl) U (A's diagonal has been read)
  __syncthreads();
  for (int idx = t; idx < mm; idx += blockDim.x) {
    const int i = idx / mp, j = idx % mp;
    double v = 0.0;
    for (int k = 0; k < mp; ++k) v += V[i * mp + k] * sl[k] * W[k * mp + j];
    A[idx] = v;
  }
  __syncthreads();
  // expand to the grid rows of B_e
  const double rs2 = sqrt(0.5);
  for (int idx = t; idx < m * nh; idx += blockDim.x) {
    const int r = idx / nh, j = idx % nh;
    double v;
    if (odd && r == h) {
      v = pi == 0 ? A[h * mp + j] : 0.0;
    } else {
      const int i = min(r, m - 1 - r);
      v = A[i * mp + j] * rs2;
      if (pi == 1 && r != i) v = -v;
    }
    J.B[e][(size_t)r * ld + off + j] = v;
  }
}

// pinv and z = 0 over the grid
__global__ __launch_bounds__(SPB) void k_spec_prep(Tab tab, const SpecJob* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SpecJob& J = jobs[gp];
  const int64_t idx = (int64_t)lb * SPB + threadIdx.x;
  if (idx >= J.mtot) return;
  double dprod = 1.0;
  int64_t rem = idx;
  for (int e = 0; e < J.d; ++e) {
    const int ie = (int)(rem / J.inner[e]);
    rem -= (int64_t)ie * J.inner[e];
    dprod *= J.D[e][ie];
  }
  J.pinv[idx] = 1.0 / (J.sigma2 + (double)J.n * dprod);
  J.z[idx] = 0.0;
}

// partial sums of y^T y (column 3)
__global__ __launch_bounds__(SPB) void k_spec_ynorm(Tab tab, const SpecJob* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SpecJob& J = jobs[gp];
  __shared__ double scr[16];
  const int64_t r = (int64_t)lb * SPB + threadIdx.x;
  const double v = r < J.n ? J.y[r] : 0.0;
  const double s = block_sum(v * v, scr);
  if (threadIdx.x == 0) J.part[(size_t)lb * SPW + 3] = s;
}

// One axis pass: out[o, i, in] = sum_j M[i][j] in[o, j, in] along `axis`
// (M = B_e or B_e^T), with the mode's post-processing.
__global__ __launch_bounds__(SPB) void k_spec_kron(Tab tab, const SpecJob* __restrict__ jobs,
                                                   int axis, int mode, int src, int dst) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SpecJob& J = jobs[gp];
  if (!(mode & KP_FORCE) && J.ctl->cg_done) return;
  const int me = J.m[axis], ld = J.ldv[axis];
  const int64_t inner = J.inner[axis];
  const int64_t idx = (int64_t)lb * SPB + threadIdx.x;
  const bool live = idx < J.mtot;
  double acc = 0.0;
  if (live) {
    const int64_t in_ = idx % inner;
    const int64_t oi = idx / inner;
    const int i = (int)(oi % me);
    const int64_t base = (oi - i) * inner + in_;
    const double* __restrict__ x = spec_buf(J, src) + base;
    const double* __restrict__ Bm = J.B[axis];
    if (mode & KP_FWD) {
      for (int j = 0; j < me; ++j) acc += Bm[i * ld + j] * x[j * inner];
    } else {
      for (int j = 0; j < me; ++j) acc += Bm[j * ld + i] * x[j * inner];
    }
    if (mode & KP_ADD_SP) acc += J.sigma2 * J.p[idx];
    spec_buf(J, dst)[idx] = acc;
  }
  if (mode & KP_DOT_P) {
    __shared__ double scr[16];
    const double v = live ? J.p[idx] * acc : 0.0;
    const double s = block_sum(v, scr);
    if (threadIdx.x == 0) J.part[(size_t)lb * SPW + 0] = s;
  }
}

// init = 0: gamma = rz / p^T q (column 0 summed in a fixed order by every
// block), z += gamma p, r -= gamma q.  Then partial sums of r^T pinv r
// (column 1) and r^T r (column 2).
__global__ __launch_bounds__(SPB) void k_spec_update(Tab tab, const SpecJob* __restrict__ jobs,
                                                     int init) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SpecJob& J = jobs[gp];
  if (J.ctl->cg_done) return;
  __shared__ double scr[16];
  __shared__ double s_pq;
  if (!init) {
    if (threadIdx.x < WAVE) {
      const double s = spec_colsum(J.part, J.nbm, 0);
      if (threadIdx.x == 0) s_pq = s;
    }
    __syncthreads();
  }
  const int64_t idx = (int64_t)lb * SPB + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (idx < J.mtot) {
    double rv = J.r[idx];
    if (!init) {
      const double gm = J.ctl->rz / s_pq;
      J.z[idx] += gm * J.p[idx];
      rv -= gm * J.q[idx];
      J.r[idx] = rv;
    }
    rz = rv * J.pinv[idx] * rv;
    rr = rv * rv;
  }
  const double srz = block_sum(rz, scr);
  const double srr = block_sum(rr, scr);
  if (threadIdx.x == 0) {
    J.part[(size_t)lb * SPW + 1] = srz;
    J.part[(size_t)lb * SPW + 2] = srr;
  }
}

// Scalar step, one wave per GP: convergence, iteration limit, direction ratio.
__global__ __launch_bounds__(WAVE) void k_spec_ep(Tab tab, const SpecJob* __restrict__ jobs,
                                                  int init) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SpecJob& J = jobs[gp];
  Ctl* ctl = J.ctl;
  if (ctl->cg_done) return;
  const double rz = spec_colsum(J.part, J.nbm, 1);
  const double rr = spec_colsum(J.part, J.nbm, 2);
  const double yy = init ? spec_colsum(J.part, J.nbn, 3) : 0.0;
  if (threadIdx.x != 0) return;
  if (init) {
    ctl->rr0 = yy;
    ctl->cg_iters = 0;
  } else {
    ctl->cg_iters += 1;
  }
  ctl->rr = rr;
  if (!isfinite(rr) || !isfinite(rz)) {
    ctl->cg_done = 1;
    ctl->status |= SF_NONFINITE;
    return;
  }
  if (!(rr > J.tol2 * ctl->rr0)) {
    ctl->cg_done = 1;
    return;
  }
  if (!init && ctl->cg_iters >= J.maxit) {
    ctl->cg_done = 1;
    ctl->status |= SF_CG_NOCONV;
    return;
  }
  ctl->ratio = init ? 0.0 : rz / ctl->rz;
  ctl->rz = rz;
}

// p = pinv r + ratio p (p = pinv r on the first step)
__global__ __launch_bounds__(SPB) void k_spec_dir(Tab tab, const SpecJob* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SpecJob& J = jobs[gp];
  if (J.ctl->cg_done) return;
  const int64_t idx = (int64_t)lb * SPB + threadIdx.x;
  if (idx >= J.mtot) return;
  const double beta = J.ctl->ratio;
  const double zr = J.pinv[idx] * J.r[idx];
  J.p[idx] = beta == 0.0 ? zr : zr + beta * J.p[idx];
}

// a = u in the cache precision
__global__ __launch_bounds__(SPB) void k_spec_store(Tab tab, const SpecJob* __restrict__ jobs,
                                                    int src) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SpecJob& J = jobs[gp];
  const int64_t idx = (int64_t)lb * SPB + threadIdx.x;
  if (idx >= J.mtot) return;
  const double v = spec_buf(J, src)[idx];
  if (J.a_fp64) ((double*)J.a)[idx] = v;
  else ((float*)J.a)[idx] = (float)v;
}

// The solve's counters into the cache's control block (run on the build stream
// once both streams have joined): iterations, done, and its status bits.
__global__ void k_spec_merge(int G, const SpecJob* __restrict__ jobs) {
  for (int g = threadIdx.x; g < G; g += blockDim.x) {
    const Ctl* own = jobs[g].ctl;
    Ctl* out = jobs[g].ctl_out;
    out->cg_iters = own->cg_iters;
    out->cg_done = 1;
    out->status |= own->status & (SF_NONFINITE | SF_CG_NOCONV);
  }
}

__global__ void k_spec_alldone(int G, const SpecJob* __restrict__ jobs, int* flag) {
  __shared__ int all;
  if (threadIdx.x == 0) all = 1;
  __syncthreads();
  for (int g = threadIdx.x; g < G; g += blockDim.x)
    if (!jobs[g].ctl->cg_done) atomicAnd(&all, 0);
  __syncthreads();
  if (threadIdx.x == 0) *flag = all;
}

}  // namespace

bool spectral_mean_applies(const love_cache* c) {
  if (c->d < 2 || c->add) return false;   // needs the Kronecker (product) structure
  if (c->cfg.flags & (LOVE_FLAG_PLAIN_CG | LOVE_FLAG_MEAN_KRYLOV)) return false;
  for (int e = 0; e < c->d; ++e)
    if (c->mdim[e] > SPEC_MAXM) return false;
  return true;
}

love_status SpectralMean::start(const std::vector<love_cache*>& cs,
                                const std::vector<const double*>& x64,
                                const std::vector<const double*>& y64,
                                const std::vector<double*>& un, hipStream_t s) {
  s_ = s;
  G_ = (int)cs.size();
  d_ = cs[0]->d;
  const int G = G_, d = d_;
  jobs_.assign(G, SpecJob{});
  mem_.assign(G, nullptr);
  std::vector<int64_t> b_m(G), b_n(G), b_axis(G, 2 * d), b_one(G, 1), b_nodes(G);
  for (int g = 0; g < G; ++g) {
    love_cache* c = cs[g];
    SpecJob J{};
    J.g = make_grid<double>(c);
    J.x = x64[g];
    J.cell_start = c->cell_start;
    J.y = y64[g];
    J.n = c->n;
    J.mtot = c->m;
    J.d = d;
    int64_t inner = 1;
    for (int e = d - 1; e >= 0; --e) {
      J.m[e] = c->mdim[e];
      J.ldv[e] = (c->mdim[e] + 1) & ~1;
      J.inner[e] = inner;
      inner *= c->mdim[e];
      J.c64[e] = (const double*)c->toep.ax[e].c64;
    }
    J.nbm = (int)cdiv(J.mtot, SPB);
    J.nbn = (int)cdiv(J.n, SPB);
    // own control block and scatter scratch: the solve runs beside the Lanczos
    static_assert(sizeof(Ctl) <= 256, "control block slot");
    size_t nd = 32;   // the control block's 256-byte slot
    for (int e = 0; e < d; ++e) nd += (size_t)J.ldv[e] * J.ldv[e] + (size_t)J.ldv[e];
    nd += 7 * (size_t)J.mtot + (size_t)std::max(J.nbm, J.nbn) * SPW;
    const size_t sb = scatter_scratch_bytes(c, sizeof(double));
    const size_t cb = sb ? (sb + 255) / 256 * 32 : 0;   // doubles, whole 256-byte blocks
    nd += cb;
    mem_[g] = (char*)ws_alloc(nd * sizeof(double), s);
    if (!mem_[g]) return LOVE_ENOMEM;
    double* q = (double*)mem_[g];
    J.ctl = (Ctl*)q;
    q += 32;
    cellp_.push_back(cb ? q : nullptr);
    q += cb;
    for (int e = 0; e < d; ++e) {
      const size_t l2 = (size_t)J.ldv[e] * J.ldv[e];
      J.B[e] = q;
      J.D[e] = q + l2;
      q = J.D[e] + J.ldv[e];
    }
    J.pinv = q;
    J.z = J.pinv + J.mtot;
    J.r = J.z + J.mtot;
    J.p = J.r + J.mtot;
    J.q = J.p + J.mtot;
    J.t0 = J.q + J.mtot;
    J.t1 = J.t0 + J.mtot;
    J.part = J.t1 + J.mtot;
    J.un = un[g];
    J.sigma2 = c->cfg.noise;
    const double tol = c->cfg.cg_tol > 0 ? c->cfg.cg_tol : (c->fp64 ? 1e-12 : 1e-6);
    J.tol2 = tol * tol * c->cfg.noise;
    J.maxit = c->cfg.cg_maxit > 0 ? c->cfg.cg_maxit : 1000;
    J.ctl_out = c->ctl;
    J.a = c->a;
    J.a_fp64 = c->fp64 ? 1 : 0;
    jobs_[g] = J;
    b_m[g] = J.nbm;
    b_n[g] = J.nbn;
    b_nodes[g] = cdiv(J.mtot, 4);
    LOVE_HIP_TRY(hipMemsetAsync(J.ctl, 0, sizeof(Ctl), s));
  }
  // W u and W^T v jobs (double)
  std::vector<GatherJob<double>> ga(G);
  std::vector<ScatterJob<double>> sy(G), su(G);
  for (int g = 0; g < G; ++g) {
    const SpecJob& J = jobs_[g];
    GatherJob<double> Ga{};
    Ga.g = J.g;
    Ga.x = J.x;
    Ga.n = J.n;
    Ga.kg = (d & 1) ? J.t0 : J.t1;   // output of the last forward pass
    Ga.out = J.un;
    Ga.ctl = J.ctl;
    ga[g] = Ga;
    ScatterJob<double> S{};
    S.g = J.g;
    S.x = J.x;
    S.cell_start = J.cell_start;
    S.v = J.y;
    S.out = J.t0;
    S.ctl = J.ctl;
    S.cellp = cellp_[g];
    sy[g] = S;
    S.v = J.un;
    su[g] = S;
  }
  o_j_ = A_.add(jobs_);
  o_ga_ = A_.add(ga);
  const size_t o_sy = A_.add(sy);
  o_su_ = A_.add(su);
  love_status st = A_.upload(s);
  if (st != LOVE_OK) return st;
  uploaded_ = true;
  dj_ = A_.at<SpecJob>(o_j_);
  t_m_ = make_tab(b_m);
  t_n_ = make_tab(b_n);
  t_one_ = make_tab(b_one);
  t_nodes_ = make_tab(b_nodes);
  const Tab t_axis = make_tab(b_axis);
  kinds_ = scatter_kinds(cs);
  for (const auto& J : jobs_) maxit_ = std::max(maxit_, J.maxit);
  dflag_ = (int*)ws_alloc(sizeof(int), s);
  if (!dflag_) return LOVE_ENOMEM;

  ProfScope ps("mean_spectral", s);
  k_spec_axis<<<tab_blocks(t_axis), EIG_THREADS, 0, s>>>(t_axis, dj_);
  k_spec_prep<<<tab_blocks(t_m_), SPB, 0, s>>>(t_m_, dj_);
  k_spec_ynorm<<<tab_blocks(t_n_), SPB, 0, s>>>(t_n_, dj_);
  // r = b = B^T W^T y ; p = pinv r
  launch_scatter<double>(t_nodes_, A_.at<ScatterJob<double>>(o_sy), d, 0, 2, s, kinds_);
  backward_passes(SB_R, 0);
  k_spec_update<<<tab_blocks(t_m_), SPB, 0, s>>>(t_m_, dj_, 1);
  k_spec_ep<<<tab_blocks(t_one_), WAVE, 0, s>>>(t_one_, dj_, 1);
  k_spec_dir<<<tab_blocks(t_m_), SPB, 0, s>>>(t_m_, dj_);
  iterations(FIRST_CHUNK);
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}

// B^T applied to t0 (d passes ending in `dst`), with `last` mode bits
void SpectralMean::backward_passes(int dst, int last) {
  int src = SB_T0;
  for (int e = 0; e < d_; ++e) {
    const bool fin = e == d_ - 1;
    const int out = fin ? dst : (src == SB_T0 ? SB_T1 : SB_T0);
    tlaunch("spec_kron", k_spec_kron, tab_blocks(t_m_), SPB, 0, s_, t_m_, dj_, e, fin ? last : 0,
            src, out);
    src = out;
  }
}

// B applied to `src` (d passes ending in t0 for odd d, t1 for even d)
void SpectralMean::forward_passes(int src, int extra) {
  int in = src;
  for (int e = 0; e < d_; ++e) {
    const int out = (e & 1) ? SB_T1 : SB_T0;
    tlaunch("spec_kron", k_spec_kron, tab_blocks(t_m_), SPB, 0, s_, t_m_, dj_, e, KP_FWD | extra,
            in, out);
    in = out;
  }
}

void SpectralMean::iterations(int count) {
  for (int qn = 0; qn < count && it_ < maxit_; ++qn, ++it_) {
    forward_passes(SB_P, 0);
    launch_gather<double>(t_n_, A_.at<GatherJob<double>>(o_ga_), d_, 2, s_);
    launch_scatter<double>(t_nodes_, A_.at<ScatterJob<double>>(o_su_), d_, 0, 2, s_, kinds_);
    backward_passes(SB_Q, KP_ADD_SP | KP_DOT_P);
    k_spec_update<<<tab_blocks(t_m_), SPB, 0, s_>>>(t_m_, dj_, 0);
    k_spec_ep<<<tab_blocks(t_one_), WAVE, 0, s_>>>(t_one_, dj_, 0);
    k_spec_dir<<<tab_blocks(t_m_), SPB, 0, s_>>>(t_m_, dj_);
  }
}

love_status SpectralMean::finish() {
  int chunk = 4;   // iterations between convergence checks after the first chunk, doubling to 16
  int hflag = 0;
  while (true) {
    k_spec_alldone<<<1, 64, 0, s_>>>(G_, dj_, dflag_);
    LOVE_HIP_TRY(hipMemcpyAsync(&hflag, dflag_, sizeof(int), hipMemcpyDeviceToHost, s_));
    LOVE_HIP_TRY(hipStreamSynchronize(s_));
    if (hflag || it_ >= maxit_) break;
    iterations(chunk);
    chunk = std::min(16, 2 * chunk);
  }
  // a = B z
  forward_passes(SB_Z, KP_FORCE);
  k_spec_store<<<tab_blocks(t_m_), SPB, 0, s_>>>(t_m_, dj_, (d_ & 1) ? SB_T0 : SB_T1);
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}

void SpectralMean::merge(hipStream_t s) {
  if (uploaded_) k_spec_merge<<<1, 64, 0, s>>>(G_, dj_);
}

void SpectralMean::release(hipStream_t s) {
  // The buffers were allocated on the solve's stream and are freed there,
  // after the build stream's last use of them (merge): the solve's stream
  // first waits for `s`.
  hipStream_t fs = s_ ? s_ : s;
  if (fs != s) {
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess || hipStreamWaitEvent(fs, ev, 0) != hipSuccess)
      (void)hipStreamSynchronize(s);
    if (ev) (void)hipEventDestroy(ev);
  }
  ws_free(dflag_, fs);
  dflag_ = nullptr;
  A_.release(fs);
  for (char* p : mem_)
    ws_free(p, fs);
  mem_.clear();
  uploaded_ = false;
}

}  // namespace love
