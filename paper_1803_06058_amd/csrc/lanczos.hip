// Lanczos with full reorthogonalisation on Khat = W K W^T + sigma^2 I, the
// LOVE cache, and the mean cache (Sec. 2.2, Sec. 3.2, Alg. 1, Sec. 5).
//
// One Lanczos step j (0-based), all on device, no host synchronisation:
//   scatter   g = W^T q_j                                  (grid, m)
//   toeplitz  R_j = K g          -- kept as row j of R = Q^T W^T K (Alg. 1)
//   gdots     v = W R_j + sigma^2 q_j ;  c = Q_{0..j}^T v   (first Gram-Schmidt pass;
//             c_j = alpha_j, c_{j-1} = beta_{j-1} up to rounding)
//   udots     r' = v - Q c ;  c2 = Q^T r' ; ||r'||^2        (second pass; Q tile staged in LDS)
//             alpha_j = c_j + c2_j ; beta_j = sqrt(||r'||^2 - ||c2||^2)
//   finalize  q_{j+1} = (r' - Q c2) / beta_j
// Every reduction is a two-level "last block" reduction in a fixed order, so
// results are bitwise reproducible.  The Lanczos vectors stay in float (or
// double for the FP64 precision); all coefficients are double.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "ops.h"

namespace love {

constexpr int BLK = 256;
constexpr int LDP = MAXK + 8;   // row stride of the partial-sum arrays
constexpr int RGS = 16;         // blocks per first-level reduction group

// ----------------------------------------------------------------------------
// Two-level deterministic reduction of per-block partial vectors.
// Each block has written partial[blockIdx.x * LDP + 0..nv).  Blocks form
// groups of RGS; the last block of a group sums the group's rows, the last
// group sums the group rows.  In both levels every lane loads its values
// before any reduction (W lanes per value, fixed shuffle tree), so a level
// costs one memory round trip, and the order of the sums never changes.
// Returns true in exactly one block, whose `red` (shared, >= nv doubles)
// then holds the sums.  Requires gridDim.x <= RGS * 32.
// ----------------------------------------------------------------------------
template <int W>
__device__ inline void sum_rows(const double* __restrict__ src, int P, int nv, double* dst,
                                bool dst_shared) {
  constexpr int VPW = WAVE / W;                       // values per wave per pass
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  const int q = lane % W, sub = lane / W;
  constexpr int MAXIT = (MAXK + 1 + VPW * 4 - 1) / (VPW * 4);
  double vals[MAXIT];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int c = (it * nw + w) * VPW + sub;
    vals[it] = (q < P && c < nv) ? src[(size_t)q * LDP + c] : 0.0;
  }
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    double v = vals[it];
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
    const int c = (it * nw + w) * VPW + sub;
    if (q == 0 && c < nv) dst[c] = v;
  }
  (void)dst_shared;
}

__device__ bool reduce_partials(double* __restrict__ partial, double* __restrict__ gpartial,
                                unsigned* __restrict__ counters, int nv, double* red) {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned grp = b / RGS, ng = (nb + RGS - 1) / RGS;
  const unsigned gsz = min((unsigned)RGS, nb - grp * RGS);
  if (!last_block_arrive(&counters[grp], gsz)) return false;
  sum_rows<RGS>(partial + (size_t)grp * RGS * LDP, (int)gsz, nv, gpartial + (size_t)grp * LDP, false);
  if (!last_block_arrive(&counters[ng], ng)) return false;
  sum_rows<32>(gpartial, (int)ng, nv, red, true);
  __syncthreads();
  return true;
}

// Dots of the block's rows [r0, r0 + nrows) with columns 0..ncols-1 of Q
// (column-major, stride ldq).  vl holds the block's vector values (LDS).
// Wave w handles columns w, w+4, ...; results go to prow[col].
template <typename T, typename V>
__device__ inline void block_dots(const T* __restrict__ Q, int64_t ldq, int ncols, int64_t r0,
                                  int nrows, const V* vl, double* __restrict__ prow) {
  constexpr int CG = 8;   // columns per wave pass; all their loads are in flight together
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  for (int c0 = w * CG; c0 < ncols; c0 += nw * CG) {
    double acc[CG];
#pragma unroll
    for (int g = 0; g < CG; ++g) acc[g] = 0.0;
    for (int rr = lane; rr < nrows; rr += WAVE) {
      const double vv = (double)vl[rr];
      T qv[CG];
#pragma unroll
      for (int g = 0; g < CG; ++g)
        qv[g] = (c0 + g < ncols) ? Q[(int64_t)(c0 + g) * ldq + r0 + rr] : T(0);
#pragma unroll
      for (int g = 0; g < CG; ++g) acc[g] += (double)qv[g] * vv;
    }
#pragma unroll
    for (int g = 0; g < CG; ++g) {
      const double sum = wave_sum(acc[g]);
      if (lane == 0 && c0 + g < ncols) prow[c0 + g] = sum;
    }
  }
}

// ----------------------------------------------------------------------------
// First pass: v = W R_j + sigma^2 q_j (rows), c = Q_{0..j}^T v.
// ----------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(BLK) void k_lz_gdots(GridT<T> g, const T* __restrict__ x, int64_t n,
                                                  const T* __restrict__ kg, const T* __restrict__ Q,
                                                  int64_t ldq, int j, T sigma2, T* __restrict__ vout,
                                                  int rpb, double* partial, double* gpartial,
                                                  unsigned* counters, double* __restrict__ coef,
                                                  Ctl* ctl) {
  if (ctl->stop) return;
  extern __shared__ unsigned char smem_raw[];
  T* vl = (T*)smem_raw;  // rpb
  __shared__ double red[LDP];
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const T* qj = Q + (int64_t)j * ldq;
  for (int rr = threadIdx.x; rr < rpb; rr += BLK) {
    const int64_t row = r0 + rr;
    T val = T(0);
    if (row < n) {
      val = gather_row_dev<T, D>(g, x, row, kg) + sigma2 * qj[row];
      vout[row] = val;
    }
    vl[rr] = val;
  }
  __syncthreads();
  const int nrows = (int)min<int64_t>(rpb, n - r0);
  block_dots(Q, ldq, j + 1, r0, nrows, vl, partial + (size_t)blockIdx.x * LDP);
  if (!reduce_partials(partial, gpartial, counters, j + 1, red)) return;
  for (int c = threadIdx.x; c <= j; c += BLK) coef[c] = red[c];
}

// ----------------------------------------------------------------------------
// Second pass: r' = v - Q c ; c2 = Q^T r' ; ||r'||^2 ; then alpha_j, beta_j.
// The Q tile of STR rows x ncols is staged in LDS so Q is read once.
// ----------------------------------------------------------------------------
template <typename T, int STR>
__global__ __launch_bounds__(BLK) void k_lz_udots(int64_t n, const T* __restrict__ v,
                                                  const T* __restrict__ Q, int64_t ldq, int j,
                                                  const double* __restrict__ coef,
                                                  T* __restrict__ rout, int rpb, double* partial,
                                                  double* gpartial, unsigned* counters,
                                                  double* __restrict__ c2out,
                                                  double* __restrict__ alpha,
                                                  double* __restrict__ beta, double tol, int klast,
                                                  Ctl* ctl) {
  if (ctl->stop) return;
  const int ncols = j + 1;
  extern __shared__ unsigned char smem_raw[];
  T* qt = (T*)smem_raw;           // ncols x STR
  __shared__ double cl[MAXK];
  __shared__ double dacc[MAXK + 1];
  __shared__ T rl[STR];
  __shared__ double red[LDP];
  __shared__ double scr[16];
  for (int c = threadIdx.x; c < ncols; c += BLK) {
    cl[c] = coef[c];
    dacc[c] = 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  double rr_acc = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  for (int st = 0; st < rpb; st += STR) {
    const int64_t rs = r0 + st;
    for (int t = threadIdx.x; t < STR; t += BLK) {
      const int64_t row = rs + t;
      const bool ok = row < n && st + t < rpb;
      double proj = 0.0;
      for (int c0 = 0; c0 < ncols; c0 += 16) {
        T qv[16];
#pragma unroll
        for (int g = 0; g < 16; ++g)
          qv[g] = (ok && c0 + g < ncols) ? Q[(int64_t)(c0 + g) * ldq + row] : T(0);
#pragma unroll
        for (int g = 0; g < 16; ++g) {
          if (c0 + g < ncols) {
            qt[(c0 + g) * STR + t] = qv[g];
            proj += (double)qv[g] * cl[c0 + g];
          }
        }
      }
      T r = T(0);
      if (ok) {
        r = (T)((double)v[row] - proj);
        rout[row] = r;
        rr_acc += (double)r * (double)r;
      }
      rl[t] = r;
    }
    __syncthreads();
    for (int c = w; c < ncols; c += BLK / WAVE) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < STR / WAVE; ++q) a += (double)qt[c * STR + lane + q * WAVE] * (double)rl[lane + q * WAVE];
      a = wave_sum(a);
      if (lane == 0) dacc[c] += a;
    }
    __syncthreads();
  }
  const double rrb = block_sum(rr_acc, scr);
  double* prow = partial + (size_t)blockIdx.x * LDP;
  for (int c = threadIdx.x; c < ncols; c += BLK) prow[c] = dacc[c];
  if (threadIdx.x == 0) prow[ncols] = rrb;
  if (!reduce_partials(partial, gpartial, counters, ncols + 1, red)) return;
  for (int c = threadIdx.x; c < ncols; c += BLK) c2out[c] = red[c];
  if (threadIdx.x == 0) {
    double c2n = 0.0;
    for (int c = 0; c < ncols; ++c) c2n += red[c] * red[c];
    const double a = coef[j] + red[j];
    const double b2 = red[ncols] - c2n;
    const double b = b2 > 0.0 ? sqrt(b2) : 0.0;
    alpha[j] = a;
    beta[j] = b;
    const double amax = fmax(ctl->amax, fabs(a));
    ctl->amax = amax;
    if (!isfinite(a) || !isfinite(b)) {
      ctl->status |= SF_NONFINITE;
      ctl->stop = 1;
      ctl->k_eff = j;
    } else {
      ctl->k_eff = j + 1;
      if (j < klast && !(b > tol * amax)) {
        ctl->stop = 1;
        ctl->status |= SF_BREAKDOWN;
      }
    }
  }
}

// q_{j+1} = (r' - Q c2) / beta_j
template <typename T>
__global__ __launch_bounds__(BLK) void k_lz_finalize(int64_t n, const T* __restrict__ r,
                                                     T* __restrict__ Q, int64_t ldq, int j,
                                                     const double* __restrict__ c2,
                                                     const double* __restrict__ beta, Ctl* ctl) {
  if (ctl->stop) return;
  __shared__ double cl[MAXK];
  for (int c = threadIdx.x; c <= j; c += BLK) cl[c] = c2[c];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (row >= n) return;
  double acc = (double)r[row];
#pragma unroll 16
  for (int c = 0; c <= j; ++c) acc -= (double)Q[(int64_t)c * ldq + row] * cl[c];
  Q[(int64_t)(j + 1) * ldq + row] = (T)(acc / beta[j]);
}

// ----------------------------------------------------------------------------
// Generic dots of a given vector v with columns 0..ncols-1 of Q plus v^T v.
// mode 0: coef[c] = q_c^T v ; scalar[0] = v^T v.
// mode 1 (probe): also ctl->bnorm = ||v||.
// mode 2 (mean jump start): z = T^{-1} (Q^T v) written to coef; ctl->rr0 = v^T v.
// ----------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BLK) void k_dots(int64_t n, const T* __restrict__ v,
                                              const T* __restrict__ Q, int64_t ldq, int ncols_max,
                                              int rpb, double* partial, double* gpartial,
                                              unsigned* counters, double* __restrict__ coef,
                                              double* __restrict__ scalar, int mode,
                                              const double* __restrict__ ldiag,
                                              const double* __restrict__ lsub, Ctl* ctl) {
  extern __shared__ unsigned char smem_raw[];
  T* vl = (T*)smem_raw;
  __shared__ double red[LDP];
  __shared__ double scr[16];
  const int ncols = (mode == 2) ? min(ncols_max, ctl->k_eff) : ncols_max;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  double ss = 0.0;
  for (int rr = threadIdx.x; rr < rpb; rr += BLK) {
    const int64_t row = r0 + rr;
    const T val = row < n ? v[row] : T(0);
    vl[rr] = val;
    ss += (double)val * (double)val;
  }
  const double ssb = block_sum(ss, scr);
  __syncthreads();
  const int nrows = (int)min<int64_t>(rpb, n - r0);
  double* prow = partial + (size_t)blockIdx.x * LDP;
  if (ncols > 0) block_dots(Q, ldq, ncols, r0, nrows, vl, prow);
  if (threadIdx.x == 0) prow[ncols] = ssb;
  if (!reduce_partials(partial, gpartial, counters, ncols + 1, red)) return;
  if (mode == 2) {
    if (threadIdx.x == 0) {
      // T z = Q^T y with T = L L^T (bidiagonal L): forward then backward substitution
      const int k = ncols;
      double zz[MAXK];
      for (int i = 0; i < k; ++i) {
        double t = red[i] - (i > 0 ? lsub[i - 1] * zz[i - 1] : 0.0);
        zz[i] = t / ldiag[i];
      }
      for (int i = k - 1; i >= 0; --i) {
        double t = zz[i] - (i + 1 < k ? lsub[i] * zz[i + 1] : 0.0);
        zz[i] = t / ldiag[i];
      }
      for (int i = 0; i < k; ++i) coef[i] = zz[i];
      for (int i = k; i < ncols_max; ++i) coef[i] = 0.0;
      ctl->rr0 = red[ncols];
    }
    return;
  }
  for (int c = threadIdx.x; c < ncols; c += BLK) coef[c] = red[c];
  if (threadIdx.x == 0) {
    if (scalar) scalar[0] = red[ncols];
    if (mode == 1) ctl->bnorm = sqrt(red[ncols]);
  }
}

// out = v / ctl->bnorm
template <typename T>
__global__ void k_scale_by_bnorm(int64_t n, const T* __restrict__ v, T* __restrict__ out,
                                 Ctl* ctl) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double b = ctl->bnorm;
  out[i] = (T)((double)v[i] / b);
}

// x0 = Q z (first k_eff columns)
template <typename T, typename TO>
__global__ __launch_bounds__(BLK) void k_q_times(int64_t n, const T* __restrict__ Q, int64_t ldq,
                                                 const double* __restrict__ z,
                                                 TO* __restrict__ out, const Ctl* ctl) {
  __shared__ double zl[MAXK];
  const int k = ctl->k_eff;
  for (int c = threadIdx.x; c < k; c += BLK) zl[c] = z[c];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (row >= n) return;
  double acc = 0.0;
#pragma unroll 16
  for (int c = 0; c < k; ++c) acc += (double)Q[(int64_t)c * ldq + row] * zl[c];
  out[row] = (TO)acc;
}

// Cholesky of the tridiagonal T (alpha, beta) of size ctl->k_eff (one thread).
// A non-positive pivot truncates k_eff there (SF_NOTPD, or SF_SAMPLER_TRUNC
// when `sampler`).  rel_tol: a pivot must exceed rel_tol * max|alpha|.
__global__ void k_tri_chol(const double* __restrict__ alpha, const double* __restrict__ beta,
                           double* __restrict__ ldiag, double* __restrict__ lsub, Ctl* ctl,
                           double rel_tol, int sampler) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = ctl->k_eff;
  double amax = 0.0;
  for (int i = 0; i < k; ++i) amax = fmax(amax, fabs(alpha[i]));
  int keep = k;
  double prev = 0.0;
  for (int i = 0; i < k; ++i) {
    const double piv = alpha[i] - prev * prev;
    if (!(piv > rel_tol * amax) || !isfinite(piv)) {
      keep = i;
      ctl->status |= sampler ? SF_SAMPLER_TRUNC : SF_NOTPD;
      break;
    }
    ldiag[i] = sqrt(piv);
    prev = (i + 1 < k) ? beta[i] / ldiag[i] : 0.0;
    lsub[i] = prev;
  }
  if (sampler) ctl->k_chol = keep;
  else ctl->k_eff = keep;
}

// bf16 round-to-nearest-even from the IEEE-754 bit pattern
__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Rt[u, :] = (L^{-1} R[:, u])^T : bidiagonal forward substitution per grid node.
// split = 1 stores bf16 hi = rne(z), lo = rne(z - hi).
template <typename T>
__global__ void k_rtilde(int64_t m, const T* __restrict__ R, const double* __restrict__ ldiag,
                         const double* __restrict__ lsub, void* __restrict__ rt,
                         uint16_t* __restrict__ rt_lo, int kpad, int split, const Ctl* ctl) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= m) return;
  const int k = ctl->k_eff;
  double z = 0.0;
  for (int i = 0; i < kpad; ++i) {
    double val = 0.0;
    if (i < k) {
      const double rv = (double)R[(int64_t)i * m + u];
      z = (rv - (i > 0 ? lsub[i - 1] * z : 0.0)) / ldiag[i];
      val = z;
    }
    if (split) {
      const float f = (float)val;
      const uint16_t hi = f32_to_bf16_rne(f);
      const uint16_t lo = f32_to_bf16_rne(f - bf16_to_f32(hi));
      ((uint16_t*)rt)[u * kpad + i] = hi;
      rt_lo[u * kpad + i] = lo;
    } else {
      ((T*)rt)[u * kpad + i] = (T)val;
    }
  }
}

// ----------------------------------------------------------------------------
// CG for the mean cache: Khat x = y, started from the Lanczos solve
// x0 = Q T^{-1} Q^T y (eq. lanczos_solve).  Per iteration:
//   scatter  g_p = W^T r + ratio * g_p        (= W^T p_new without forming p first)
//   toeplitz kg = K g_p
//   ap       p = r + ratio * p ; Ap = W kg + sigma^2 p ; gamma = rr / p^T Ap
//   update   x += gamma p ; r -= gamma Ap ; ratio = rr_new / rr
// ----------------------------------------------------------------------------
template <typename T, int D>
__global__ __launch_bounds__(BLK) void k_cg_ap(GridT<T> g, const T* __restrict__ x, int64_t n,
                                               const T* __restrict__ kg, const T* __restrict__ r,
                                               T* __restrict__ p, T* __restrict__ ap, T sigma2,
                                               int rpb, double* partial, double* gpartial,
                                               unsigned* counters, Ctl* ctl) {
  if (ctl->cg_done) return;
  __shared__ double red[LDP];
  __shared__ double scr[16];
  const double ratio = ctl->ratio;
  double d = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  for (int rr = threadIdx.x; rr < rpb; rr += BLK) {
    const int64_t row = r0 + rr;
    if (row >= n) break;
    const T pn = (T)((double)r[row] + ratio * (double)p[row]);
    p[row] = pn;
    const T a = gather_row_dev<T, D>(g, x, row, kg) + sigma2 * pn;
    ap[row] = a;
    d += (double)pn * (double)a;
  }
  const double db = block_sum(d, scr);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * LDP] = db;
  if (!reduce_partials(partial, gpartial, counters, 1, red)) return;
  if (threadIdx.x == 0) ctl->gamma = ctl->rr / red[0];
}

template <typename T>
__global__ __launch_bounds__(BLK) void k_cg_update(int64_t n, T* __restrict__ xs,
                                                   T* __restrict__ r, const T* __restrict__ p,
                                                   const T* __restrict__ ap, int rpb,
                                                   double* partial, double* gpartial,
                                                   unsigned* counters, double tol2, int maxit,
                                                   Ctl* ctl) {
  if (ctl->cg_done) return;
  __shared__ double red[LDP];
  __shared__ double scr[16];
  const double gm = ctl->gamma;
  double d = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  for (int rr = threadIdx.x; rr < rpb; rr += BLK) {
    const int64_t row = r0 + rr;
    if (row >= n) break;
    xs[row] = (T)((double)xs[row] + gm * (double)p[row]);
    const T rn = (T)((double)r[row] - gm * (double)ap[row]);
    r[row] = rn;
    d += (double)rn * (double)rn;
  }
  const double db = block_sum(d, scr);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * LDP] = db;
  if (!reduce_partials(partial, gpartial, counters, 1, red)) return;
  if (threadIdx.x == 0) {
    const double rrn = red[0];
    ctl->ratio = rrn / ctl->rr;
    ctl->rr = rrn;
    ctl->cg_iters += 1;
    if (!(rrn > tol2 * ctl->rr0)) ctl->cg_done = 1;
    else if (ctl->cg_iters >= maxit) {
      ctl->cg_done = 1;
      ctl->status |= SF_CG_NOCONV;
    }
    if (!isfinite(rrn)) {
      ctl->cg_done = 1;
      ctl->status |= SF_NONFINITE;
    }
  }
}

// r = y - A x0 ; p = 0 ; rr = r^T r ; ratio = 0
template <typename T, int D>
__global__ __launch_bounds__(BLK) void k_cg_init(GridT<T> g, const T* __restrict__ x, int64_t n,
                                                 const T* __restrict__ kg, const T* __restrict__ y,
                                                 const T* __restrict__ x0, T* __restrict__ r,
                                                 T* __restrict__ p, T sigma2, int rpb,
                                                 double* partial, double* gpartial,
                                                 unsigned* counters, double tol2, Ctl* ctl) {
  __shared__ double red[LDP];
  __shared__ double scr[16];
  double d = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  for (int rr = threadIdx.x; rr < rpb; rr += BLK) {
    const int64_t row = r0 + rr;
    if (row >= n) break;
    const T ax = gather_row_dev<T, D>(g, x, row, kg) + sigma2 * x0[row];
    const T rv = (T)((double)y[row] - (double)ax);
    r[row] = rv;
    p[row] = T(0);
    d += (double)rv * (double)rv;
  }
  const double db = block_sum(d, scr);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.x * LDP] = db;
  if (!reduce_partials(partial, gpartial, counters, 1, red)) return;
  if (threadIdx.x == 0) {
    ctl->rr = red[0];
    ctl->ratio = 0.0;
    ctl->cg_iters = 0;
    ctl->cg_done = (red[0] > tol2 * ctl->rr0) ? 0 : 1;
  }
}

__global__ void k_ctl_init(Ctl* ctl) {
  Ctl z{};
  *ctl = z;
}

// ----------------------------------------------------------------------------
// Host orchestration
// ----------------------------------------------------------------------------
struct Work {
  double* partial = nullptr;
  double* gpartial = nullptr;
  unsigned* counters = nullptr;
  double* coef = nullptr;
  double* c2 = nullptr;
  double* ldiag = nullptr;
  double* lsub = nullptr;
  double* scalar = nullptr;
  int rpb = BLK;
  int nb = 0;
};

static love_status work_alloc(love_cache* c, Work& wk, int64_t rows, std::vector<void*>& tmp,
                              hipStream_t s) {
  int rpt = (int)cdiv(rows, (int64_t)BLK * 512);
  if (rpt < 1) rpt = 1;
  wk.rpb = BLK * rpt;
  wk.nb = (int)cdiv(rows, wk.rpb);
  const int ng = (int)cdiv(wk.nb, RGS);
  size_t bytes = sizeof(double) * ((size_t)wk.nb * LDP + (size_t)ng * LDP + 5 * LDP) +
                 sizeof(unsigned) * (ng + 1);
  char* p = nullptr;
  LOVE_HIP_TRY(hipMallocAsync((void**)&p, bytes, s));
  tmp.push_back(p);
  wk.partial = (double*)p;
  wk.gpartial = wk.partial + (size_t)wk.nb * LDP;
  wk.coef = wk.gpartial + (size_t)ng * LDP;
  wk.c2 = wk.coef + LDP;
  wk.ldiag = wk.c2 + LDP;
  wk.lsub = wk.ldiag + LDP;
  wk.scalar = wk.lsub + LDP;
  wk.counters = (unsigned*)(wk.scalar + LDP);
  LOVE_HIP_TRY(hipMemsetAsync(wk.counters, 0, sizeof(unsigned) * (ng + 1), s));
  return LOVE_OK;
}

template <typename T>
static void set_smem_limits() {
  static bool done = false;
  if (done) return;
  done = true;
  (void)hipFuncSetAttribute((const void*)k_lz_udots<T, (sizeof(T) == 8 ? 128 : 256)>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 8192);
}

// Mean cache a = K W^T Khat^{-1} y (eq. pred_mean_ski).  The solve runs in
// double whatever the cache precision: in float the true residual of CG
// stalls at ~1e-3 relative on the 1e5-point workload (rounding of the
// operator's float sums times its condition number ~1e5), which leaves the
// mean wrong in the third digit; in double, CG started from the Lanczos solve
// x0 = Q T^{-1} Q^T y (eq. lanczos_solve) needs about a dozen iterations.
template <typename T, int D>
static love_status mean_solve(love_cache* c, const T* Q, int64_t ldq, Work& wk,
                              std::vector<void*>& tmp, hipStream_t s) {
  ProfScope ps("mean_cg", s);
  const int64_t n = c->n, m = c->m;
  const int k = c->k;
  const unsigned nbr = (unsigned)cdiv(n, BLK);
  Ctl* ctl = c->ctl;
  double *x64, *y64, *xs, *rr, *pp, *ap, *gv, *gm;
  {
    const bool own = sizeof(T) != 8;
    size_t bytes = sizeof(double) * ((own ? (size_t)n * (c->d + 1) : 0) + 4 * (size_t)ldq + 2 * (size_t)m);
    char* p = nullptr;
    LOVE_HIP_TRY(hipMallocAsync((void**)&p, bytes, s));
    tmp.push_back(p);
    double* q = (double*)p;
    if (own) {
      x64 = q;
      y64 = x64 + (size_t)n * c->d;
      q = y64 + n;
      launch_convert<T, double>((const T*)c->x, x64, n * c->d, s);
      launch_convert<T, double>((const T*)c->y, y64, n, s);
    } else {
      x64 = (double*)c->x;
      y64 = (double*)c->y;
    }
    xs = q;
    rr = xs + ldq;
    pp = rr + ldq;
    ap = pp + ldq;
    gv = ap + ldq;
    gm = gv + m;
  }
  GridT<double> g = make_grid<double>(c);
  const double sigma2 = c->cfg.noise;
  const bool plain = (c->cfg.flags & LOVE_FLAG_PLAIN_CG) != 0;
  // jump start: z = T^{-1} Q^T y, x0 = Q z (float Q, double z and x0)
  const T* yT = (const T*)c->y;
  k_dots<T><<<wk.nb, BLK, sizeof(T) * wk.rpb, s>>>(n, yT, Q, ldq, plain ? 0 : k, wk.rpb,
                                                   wk.partial, wk.gpartial, wk.counters, wk.coef,
                                                   wk.scalar, 2, wk.ldiag, wk.lsub, ctl);
  if (plain) launch_fill<double>(xs, 0.0, n, s);
  else k_q_times<T, double><<<nbr, BLK, 0, s>>>(n, Q, ldq, wk.coef, xs, ctl);
  const double cgtol = c->cfg.cg_tol > 0 ? c->cfg.cg_tol : (c->fp64 ? 1e-12 : 1e-6);
  const int maxit = c->cfg.cg_maxit > 0 ? c->cfg.cg_maxit : 1000;
  launch_scatter<double>(c, xs, gv, nullptr, nullptr, 0, s, x64);
  toeplitz_apply<double>(c, gv, gm, nullptr, 0, s);
  k_cg_init<double, D><<<wk.nb, BLK, 0, s>>>(g, x64, n, gm, y64, xs, rr, pp, sigma2, wk.rpb,
                                             wk.partial, wk.gpartial, wk.counters, cgtol * cgtol,
                                             ctl);
  launch_fill<double>(gv, 0.0, m, s);   // W^T p with p = 0
  Ctl hctl;
  int it = 0;
  const int chunk = 8;
  while (it < maxit) {
    for (int q = 0; q < chunk && it < maxit; ++q, ++it) {
      launch_scatter<double>(c, rr, gv, gv, ctl, 2 | 4, s, x64);
      toeplitz_apply<double>(c, gv, gm, ctl, 2, s);
      k_cg_ap<double, D><<<wk.nb, BLK, 0, s>>>(g, x64, n, gm, rr, pp, ap, sigma2, wk.rpb,
                                               wk.partial, wk.gpartial, wk.counters, ctl);
      k_cg_update<double><<<wk.nb, BLK, 0, s>>>(n, xs, rr, pp, ap, wk.rpb, wk.partial,
                                                wk.gpartial, wk.counters, cgtol * cgtol, maxit,
                                                ctl);
    }
    LOVE_HIP_TRY(hipMemcpyAsync(&hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    LOVE_HIP_TRY(hipStreamSynchronize(s));
    if (hctl.cg_done) break;
  }
  launch_scatter<double>(c, xs, gv, nullptr, nullptr, 0, s, x64);
  toeplitz_apply<double>(c, gv, gm, nullptr, 0, s);
  if (sizeof(T) == 8) launch_convert<double, double>(gm, (double*)c->a, m, s);
  else launch_convert<double, float>(gm, (float*)c->a, m, s);
  return LOVE_OK;
}

template <typename T, int D>
static love_status lanczos_impl(love_cache* c, hipStream_t s) {
  constexpr int STR = (sizeof(T) == 8) ? 128 : 256;
  set_smem_limits<T>();
  const int64_t n = c->n, m = c->m;
  const int k = c->k;
  const int64_t ldq = cdiv(n, 64) * 64;
  GridT<T> g = make_grid<T>(c);
  const T* x = (const T*)c->x;
  const T sigma2 = (T)c->cfg.noise;
  std::vector<void*> tmp;
  Work wk;
  love_status st = work_alloc(c, wk, n, tmp, s);
  if (st != LOVE_OK) return st;
  // transient buffers: Q (n x k), R (k x m), v, r, grid vectors
  T *Q, *R, *v, *r, *gv, *gm;
  {
    size_t bytes = sizeof(T) * ((size_t)ldq * k + (size_t)k * m + 2 * (size_t)ldq + 2 * (size_t)m);
    char* p = nullptr;
    LOVE_HIP_TRY(hipMallocAsync((void**)&p, bytes, s));
    tmp.push_back(p);
    Q = (T*)p;
    R = Q + (size_t)ldq * k;
    v = R + (size_t)k * m;
    r = v + ldq;
    gv = r + ldq;
    gm = gv + m;
  }
  Ctl* ctl = c->ctl;
  k_ctl_init<<<1, 1, 0, s>>>(ctl);
  const unsigned nbr = (unsigned)cdiv(n, BLK);
  // probe b = (1/m) W K 1 ; q_0 = b / ||b||
  {
    ProfScope ps("probe", s);
    launch_fill<T>(gv, T(1.0 / (double)m), m, s);
    toeplitz_apply<T>(c, gv, gm, nullptr, 0, s);
    launch_gather<T>(c, gm, nullptr, T(0), v, nullptr, s);
    k_dots<T><<<wk.nb, BLK, sizeof(T) * wk.rpb, s>>>(n, v, Q, ldq, 0, wk.rpb, wk.partial, wk.gpartial,
                                                     wk.counters, wk.coef, wk.scalar, 1, nullptr,
                                                     nullptr, ctl);
    k_scale_by_bnorm<T><<<nbr, BLK, 0, s>>>(n, v, Q, ctl);
  }
  const double tol = c->tol_lanczos;
  for (int j = 0; j < k; ++j) {
    launch_scatter<T>(c, Q + (size_t)j * ldq, gv, nullptr, ctl, 1, s);
    toeplitz_apply<T>(c, gv, R + (size_t)j * m, ctl, 1, s);
    {
      ProfScope ps("lz_gdots", s);
      k_lz_gdots<T, D><<<wk.nb, BLK, sizeof(T) * wk.rpb, s>>>(
          g, x, n, R + (size_t)j * m, Q, ldq, j, sigma2, v, wk.rpb, wk.partial, wk.gpartial,
          wk.counters, wk.coef, ctl);
    }
    {
      ProfScope ps("lz_udots", s);
      const size_t shm = sizeof(T) * (size_t)(j + 1) * STR;
      k_lz_udots<T, STR><<<wk.nb, BLK, shm, s>>>(n, v, Q, ldq, j, wk.coef, r, wk.rpb, wk.partial,
                                                 wk.gpartial, wk.counters, wk.c2, c->alpha,
                                                 c->beta, tol, k - 1, ctl);
    }
    if (j + 1 < k) {
      ProfScope ps("lz_finalize", s);
      k_lz_finalize<T><<<nbr, BLK, 0, s>>>(n, r, Q, ldq, j, wk.c2, c->beta, ctl);
    }
  }
  // T = L L^T ; Rt = (L^{-1} R)^T
  k_tri_chol<<<1, 64, 0, s>>>(c->alpha, c->beta, wk.ldiag, wk.lsub, ctl, 0.0, 0);
  {
    ProfScope ps("rtilde", s);
    const int split = c->cfg.precision == LOVE_P_FP32_BF16SPLIT;
    k_rtilde<T><<<cdiv(m, 256), 256, 0, s>>>(m, R, wk.ldiag, wk.lsub, c->rt, (uint16_t*)c->rt_lo,
                                             c->kpad, split, ctl);
  }
  // mean cache a = K W^T Khat^{-1} y
  if (!(c->cfg.flags & LOVE_FLAG_NO_MEAN)) {
    love_status ms = mean_solve<T, D>(c, Q, ldq, wk, tmp, s);
    if (ms != LOVE_OK) return ms;
  }
  for (void* p : tmp) (void)hipFreeAsync(p, s);
  LOVE_HIP_TRY(hipGetLastError());
  return LOVE_OK;
}

template <typename T>
love_status build_lanczos_and_mean(love_cache* c, hipStream_t s) {
  switch (c->d) {
    case 1: return lanczos_impl<T, 1>(c, s);
    case 2: return lanczos_impl<T, 2>(c, s);
    case 3: return lanczos_impl<T, 3>(c, s);
    case 4: return lanczos_impl<T, 4>(c, s);
  }
  return LOVE_EINVAL;
}
template love_status build_lanczos_and_mean<float>(love_cache*, hipStream_t);
template love_status build_lanczos_and_mean<double>(love_cache*, hipStream_t);


// ============================================================================
// Sampling cache (Sec. 3.3): Lanczos on B = K - R^T R' = K - Rt Rt^T in grid
// space (eq. lancapprox), probe b' = (1/m) B 1, then S = Q' L_{T'}
// (eq. pred_covar_ski_interp_form).  B is the difference of two nearly equal
// matrices (the posterior covariance is 1e-4..1e-6 of the prior here), so
// this Lanczos runs in double whatever the cache precision; Rt is read in its
// stored precision and widened.
// ============================================================================
template <typename TR, int SPLIT>
__device__ inline double rt_val(const void* rt, const uint16_t* rt_lo, int64_t idx) {
  if constexpr (SPLIT) {
    const uint16_t* hi = (const uint16_t*)rt;
    return (double)(bf16_to_f32(hi[idx]) + bf16_to_f32(rt_lo[idx]));
  } else {
    return (double)((const TR*)rt)[idx];
  }
}

// s = Rt^T v (columns < keff); lanes own columns, waves split the rows.
template <typename TR, int SPLIT>
__global__ __launch_bounds__(BLK) void k_rt_dots(int64_t m, const double* __restrict__ v,
                                                 const void* __restrict__ rt,
                                                 const uint16_t* __restrict__ rt_lo, int kpad,
                                                 const Ctl* ctl_main, int rpb, double* partial,
                                                 double* gpartial, unsigned* counters,
                                                 double* __restrict__ sout, const Ctl* ctl) {
  if (ctl && ctl->stop) return;
  __shared__ double red[LDP];
  __shared__ double wsum[BLK / WAVE][MAXK];
  const int keff = ctl_main->k_eff;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  const int64_t r1 = min<int64_t>(r0 + rpb, m);
  double a0 = 0.0, a1 = 0.0;
  for (int64_t u = r0 + w; u < r1; u += BLK / WAVE) {
    const double vu = v[u];
    if (lane < keff) a0 += vu * rt_val<TR, SPLIT>(rt, rt_lo, u * kpad + lane);
    if (lane + WAVE < keff) a1 += vu * rt_val<TR, SPLIT>(rt, rt_lo, u * kpad + lane + WAVE);
  }
  wsum[w][lane] = a0;
  wsum[w][lane + WAVE] = a1;
  __syncthreads();
  double* prow = partial + (size_t)blockIdx.x * LDP;
  for (int c = threadIdx.x; c < keff; c += BLK) {
    double s = 0.0;
    for (int q = 0; q < BLK / WAVE; ++q) s += wsum[q][c];
    prow[c] = s;
  }
  if (!reduce_partials(partial, gpartial, counters, keff, red)) return;
  for (int c = threadIdx.x; c < keff; c += BLK) sout[c] = red[c];
}

// v = kv - Rt s (grid rows); then c = Q'_{0..j}^T v  (ncols = j + 1; 0 = probe)
template <typename TR, int SPLIT>
__global__ __launch_bounds__(BLK) void k_sp_apply_dots(int64_t m, const double* __restrict__ kv,
                                                       const void* __restrict__ rt,
                                                       const uint16_t* __restrict__ rt_lo,
                                                       int kpad, const Ctl* ctl_main,
                                                       const double* __restrict__ sv,
                                                       const double* __restrict__ Q, int64_t ldq,
                                                       int ncols, double* __restrict__ vout,
                                                       int rpb, double* partial, double* gpartial,
                                                       unsigned* counters,
                                                       double* __restrict__ coef, Ctl* ctl) {
  if (ctl->stop) return;
  extern __shared__ unsigned char smem_raw[];
  double* vl = (double*)smem_raw;
  __shared__ double red[LDP];
  __shared__ double sl[MAXK];
  const int keff = ctl_main->k_eff;
  for (int c = threadIdx.x; c < keff; c += BLK) sl[c] = sv[c];
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * rpb;
  for (int rr = threadIdx.x; rr < rpb; rr += BLK) {
    const int64_t u = r0 + rr;
    double val = 0.0;
    if (u < m) {
      double acc = kv[u];
#pragma unroll 16
      for (int c = 0; c < keff; ++c) acc -= rt_val<TR, SPLIT>(rt, rt_lo, u * kpad + c) * sl[c];
      val = acc;
      vout[u] = val;
    }
    vl[rr] = val;
  }
  __syncthreads();
  if (ncols == 0) return;
  const int nrows = (int)min<int64_t>(rpb, m - r0);
  block_dots(Q, ldq, ncols, r0, nrows, vl, partial + (size_t)blockIdx.x * LDP);
  if (!reduce_partials(partial, gpartial, counters, ncols, red)) return;
  for (int c = threadIdx.x; c < ncols; c += BLK) coef[c] = red[c];
}

// Eigen-decomposition T' = V diag(lam) V^T of the sampler's symmetric
// tridiagonal (k' <= 128) by implicit QL with Wilkinson shifts (Bowdler,
// Martin, Reinsch and Wilkinson, 1968).  One block of MAXK threads: thread 0
// runs the scalar chase of a sweep and records its plane rotations; then each
// thread applies the sweep's rotations, in order, to its own row of V (held in
// LDS).  Eigenpairs are returned sorted by decreasing eigenvalue; k_chol
// counts the strictly positive ones (negative Ritz values of K - Rt Rt^T are
// rounding noise of the float cache and are clipped to zero).
constexpr int EIG_MAXSWEEP = 40;

__global__ __launch_bounds__(MAXK) void k_tri_eig(const double* __restrict__ alpha,
                                                  const double* __restrict__ beta,
                                                  double* __restrict__ vout,
                                                  double* __restrict__ lam, Ctl* ctl) {
  extern __shared__ unsigned char smem_raw[];
  double* V = (double*)smem_raw;   // MAXK x MAXK, column c of V at V[c * MAXK + row]
  __shared__ double d[MAXK], e[MAXK], rc[MAXK], rs[MAXK];
  __shared__ int ri[MAXK];
  __shared__ int nrot, done, lcur, iters;
  __shared__ int perm[MAXK];
  const int t = threadIdx.x;
  const int k = ctl->k_eff;
  for (int cidx = 0; cidx < k; ++cidx) V[cidx * MAXK + t] = (cidx == t) ? 1.0 : 0.0;
  if (t == 0) {
    for (int i = 0; i < k; ++i) {
      d[i] = alpha[i];
      e[i] = (i + 1 < k) ? beta[i] : 0.0;
    }
    lcur = 0;
    iters = 0;
    done = (k <= 0);
  }
  __syncthreads();
  while (true) {
    if (t == 0) {
      nrot = 0;
      // advance l over converged eigenvalues; stop at the first one needing a sweep
      while (lcur < k) {
        int mm = lcur;
        for (; mm < k - 1; ++mm) {
          const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
          if (fabs(e[mm]) <= 2.220446049250313e-16 * dd) break;
        }
        if (mm == lcur) {
          ++lcur;
          iters = 0;
          continue;
        }
        if (++iters > EIG_MAXSWEEP) {   // give up on this eigenvalue (flagged)
          ctl->status |= SF_NONFINITE;
          ++lcur;
          iters = 0;
          continue;
        }
        const int l = lcur;
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = hypot(g, 1.0);
        g = d[mm] - d[l] + e[l] / (g + copysign(r, g));
        double sv = 1.0, cv = 1.0, p = 0.0;
        int i = mm - 1;
        bool underflow = false;
        for (; i >= l; --i) {
          const double f = sv * e[i], b = cv * e[i];
          r = hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) {
            d[i + 1] -= p;
            e[mm] = 0.0;
            underflow = true;
            break;
          }
          sv = f / r;
          cv = g / r;
          g = d[i + 1] - p;
          r = (d[i] - g) * sv + 2.0 * cv * b;
          p = sv * r;
          d[i + 1] = g + p;
          g = cv * r - b;
          ri[nrot] = i;
          rc[nrot] = cv;
          rs[nrot] = sv;
          ++nrot;
        }
        if (!underflow) {
          d[l] -= p;
          e[l] = g;
          e[mm] = 0.0;
        }
        break;   // one sweep recorded
      }
      done = (lcur >= k) ? 1 : 0;
    }
    __syncthreads();
    const int nr = nrot;
    if (t < k) {
      for (int q = 0; q < nr; ++q) {
        const int i = ri[q];
        const double cv = rc[q], sv = rs[q];
        const double f = V[(i + 1) * MAXK + t];
        const double vi = V[i * MAXK + t];
        V[(i + 1) * MAXK + t] = sv * vi + cv * f;
        V[i * MAXK + t] = cv * vi - sv * f;
      }
    }
    __syncthreads();
    if (done) break;
  }
  if (t == 0) {
    for (int i = 0; i < k; ++i) perm[i] = i;
    for (int i = 0; i < k; ++i) {          // selection sort, decreasing
      int best = i;
      for (int j = i + 1; j < k; ++j)
        if (d[perm[j]] > d[perm[best]]) best = j;
      const int tmpi = perm[i];
      perm[i] = perm[best];
      perm[best] = tmpi;
    }
    int pos = 0;
    for (int i = 0; i < k; ++i) {
      lam[i] = d[perm[i]];
      if (d[perm[i]] > 0.0 && isfinite(d[perm[i]])) pos = i + 1;
    }
    ctl->k_chol = pos;
    if (pos < k) ctl->status |= SF_SAMPLER_TRUNC;
  }
  __syncthreads();
  for (int cidx = 0; cidx < k; ++cidx) vout[cidx * MAXK + t] = V[perm[cidx] * MAXK + t];
}

// S[u, c] = sqrt(lam_c) * sum_i Q'[i][u] V[c][i]  for c < k_chol (zero beyond kspad).
__global__ __launch_bounds__(256) void k_s_from_eig(int64_t m, const double* __restrict__ Q,
                                                    int64_t ldq, const double* __restrict__ vout,
                                                    const double* __restrict__ lam,
                                                    float* __restrict__ S, int kspad,
                                                    const Ctl* ctl) {
  extern __shared__ unsigned char smem_raw[];
  double* Vl = (double*)smem_raw;   // kc x k (row c = eigenvector c)
  const int k = ctl->k_eff, kc = ctl->k_chol;
  for (int idx = threadIdx.x; idx < kc * k; idx += blockDim.x) {
    const int c = idx / k, i = idx % k;
    Vl[idx] = vout[c * MAXK + i] * sqrt(lam[c]);
  }
  __syncthreads();
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= m) return;
  constexpr int CT = 16;
  for (int c0 = 0; c0 < kspad; c0 += CT) {
    double acc[CT];
#pragma unroll
    for (int q = 0; q < CT; ++q) acc[q] = 0.0;
    if (c0 < kc) {
      for (int i = 0; i < k; ++i) {
        const double qv = Q[(int64_t)i * ldq + u];
#pragma unroll
        for (int q = 0; q < CT; ++q)
          if (c0 + q < kc) acc[q] += qv * Vl[(c0 + q) * k + i];
      }
    }
#pragma unroll
    for (int q = 0; q < CT; ++q)
      if (c0 + q < kspad) S[u * kspad + c0 + q] = (float)acc[q];
  }
}

template <typename TR, int SPLIT>
static love_status sampler_impl(love_cache* c, hipStream_t s) {
  set_smem_limits<double>();
  const int64_t m = c->m;
  const int ks = c->ks;
  const int64_t ldq = cdiv(m, 64) * 64;
  std::vector<void*> tmp;
  Work wk;
  love_status st = work_alloc(c, wk, m, tmp, s);
  if (st != LOVE_OK) return st;
  double *Q, *v, *r, *kv, *gv, *sv, *alpha, *beta, *vout, *lam;
  {
    size_t bytes = sizeof(double) * ((size_t)ldq * ks + 4 * (size_t)ldq + 4 * LDP + MAXK * MAXK);
    char* p = nullptr;
    LOVE_HIP_TRY(hipMallocAsync((void**)&p, bytes, s));
    tmp.push_back(p);
    Q = (double*)p;
    v = Q + (size_t)ldq * ks;
    r = v + ldq;
    kv = r + ldq;
    gv = kv + ldq;
    sv = gv + ldq;
    alpha = sv + LDP;
    beta = alpha + LDP;
    lam = beta + LDP;
    vout = lam + LDP;
  }
  Ctl* ctl = c->ctl_s;
  const Ctl* cm = c->ctl;
  k_ctl_init<<<1, 1, 0, s>>>(ctl);
  const unsigned nbm = (unsigned)cdiv(m, BLK);
  const size_t shm = sizeof(double) * wk.rpb;
  {
    ProfScope ps("sampler_probe", s);
    launch_fill<double>(gv, 1.0 / (double)m, m, s);
    toeplitz_apply<double>(c, gv, kv, nullptr, 0, s);
    k_rt_dots<TR, SPLIT><<<wk.nb, BLK, 0, s>>>(m, gv, c->rt, (const uint16_t*)c->rt_lo, c->kpad, cm,
                                               wk.rpb, wk.partial, wk.gpartial, wk.counters, sv,
                                               nullptr);
    k_sp_apply_dots<TR, SPLIT><<<wk.nb, BLK, shm, s>>>(m, kv, c->rt, (const uint16_t*)c->rt_lo,
                                                      c->kpad, cm, sv, Q, ldq, 0, v, wk.rpb,
                                                      wk.partial, wk.gpartial, wk.counters,
                                                      wk.coef, ctl);
    k_dots<double><<<wk.nb, BLK, shm, s>>>(m, v, Q, ldq, 0, wk.rpb, wk.partial, wk.gpartial,
                                           wk.counters, wk.coef, wk.scalar, 1, nullptr, nullptr, ctl);
    k_scale_by_bnorm<double><<<nbm, BLK, 0, s>>>(m, v, Q, ctl);
  }
  const double tol = 1e-12;
  for (int j = 0; j < ks; ++j) {
    ProfScope ps("sampler_step", s);
    const double* qj = Q + (size_t)j * ldq;
    toeplitz_apply<double>(c, qj, kv, ctl, 1, s);
    k_rt_dots<TR, SPLIT><<<wk.nb, BLK, 0, s>>>(m, qj, c->rt, (const uint16_t*)c->rt_lo, c->kpad, cm,
                                               wk.rpb, wk.partial, wk.gpartial, wk.counters, sv,
                                               ctl);
    k_sp_apply_dots<TR, SPLIT><<<wk.nb, BLK, shm, s>>>(m, kv, c->rt, (const uint16_t*)c->rt_lo,
                                                      c->kpad, cm, sv, Q, ldq, j + 1, v, wk.rpb,
                                                      wk.partial, wk.gpartial, wk.counters,
                                                      wk.coef, ctl);
    k_lz_udots<double, 128><<<wk.nb, BLK, sizeof(double) * (size_t)(j + 1) * 128, s>>>(
        m, v, Q, ldq, j, wk.coef, r, wk.rpb, wk.partial, wk.gpartial, wk.counters, wk.c2, alpha,
        beta, tol, ks - 1, ctl);
    if (j + 1 < ks) k_lz_finalize<double><<<nbm, BLK, 0, s>>>(m, r, Q, ldq, j, wk.c2, beta, ctl);
  }
  {
    ProfScope pe("sampler_eig", s);
    (void)hipFuncSetAttribute((const void*)k_tri_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                              sizeof(double) * MAXK * MAXK);
    (void)hipFuncSetAttribute((const void*)k_s_from_eig, hipFuncAttributeMaxDynamicSharedMemorySize,
                              sizeof(double) * MAXK * MAXK);
    k_tri_eig<<<1, MAXK, sizeof(double) * MAXK * MAXK, s>>>(alpha, beta, vout, lam, ctl);
    k_s_from_eig<<<cdiv(m, 256), 256, sizeof(double) * MAXK * MAXK, s>>>(m, Q, ldq, vout, lam, c->S,
                                                                        c->kspad, ctl);
  }
  for (void* p : tmp) (void)hipFreeAsync(p, s);
  LOVE_HIP_TRY(hipGetLastError());
  return LOVE_OK;
}

love_status build_sampler(love_cache* c, hipStream_t s) {
  ProfScope ps("sampler_build", s);
  if (c->fp64) return sampler_impl<double, 0>(c, s);
  if (c->cfg.precision == LOVE_P_FP32_BF16SPLIT) return sampler_impl<float, 1>(c, s);
  return sampler_impl<float, 0>(c, s);
}

}  // namespace love
