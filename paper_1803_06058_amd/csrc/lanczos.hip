// Lanczos with full reorthogonalisation on Khat = W K W^T + sigma^2 I, the
// LOVE cache, the mean cache and the sampling cache (Sec. 2.2, Sec. 3.2,
// Alg. 1, Sec. 3.3, Sec. 5), for a batch of independent GPs run in lock step
// (one launch per phase covers every GP; a single GP is the batch of one).
//
// One Lanczos step j (0-based), all on device, no host synchronisation:
//   scatter   g = W^T q_j                                  (grid, m)
//   toeplitz  R_j = K g          -- kept as row j of R = Q^T W^T K (Alg. 1)
//   gdots     v = W R_j + sigma^2 q_j ;  per-block partials of Q_{0..j}^T v
//   colsum    c = Q_{0..j}^T v   (first Gram-Schmidt pass; c_j = alpha_j)
//   udots     r' = v - Q c ; per-block partials of Q^T r' and ||r'||^2
//   (when m <= n the first pass runs in grid space instead: with G = W^T Q,
//   kept column by column from the scatter, Q^T v = G^T R_j + sigma^2 Q^T q_j,
//   and Q^T q_j is taken as e_j -- the second pass removes what that leaves --
//   so one small kernel (cdots, partial rows over grid blocks) replaces
//   gdots + colsum, and udots forms v itself and adds the cdots rows)
//   colsum    c2, ||r'||^2       (second pass)
//   finalize  alpha_j = c_j + c2_j, beta_j = sqrt(||r'||^2 - ||c2||^2),
//             stop test, q_{j+1} = (r' - Q c2) / beta_j
// Row kernels work on blocks of 256 rows: lane l of every wave owns rows
// 4l..4l+3 (one 16-byte load per column), the block's 4 waves split the
// columns of Q, and a wave reduces 8 columns at once with a transposing
// butterfly (10 shuffles instead of 48).  Grid-wide sums never use
// device-scope fences inside a kernel (on this GPU a device-scope release
// writes back the whole L2 of the issuing XCD, once per block); instead a
// producer kernel writes one partial row per block and a second small kernel
// adds the rows in a fixed order, so results are bitwise reproducible and the
// kernel boundary provides visibility.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "internal.h"
#include "ops.h"
#include "toep_dev.h"

namespace love {

constexpr int BLK = 256;          // small kernels
constexpr int CWV = 8;            // column waves of a row-kernel block
constexpr int RBLK = CWV * WAVE;  // threads of a row-kernel block

// ----------------------------------------------------------------------------
// Reductions
// ----------------------------------------------------------------------------
// sum_b partial[b][c], one wave; every lane issues all its loads before adding
__device__ __forceinline__ double colsum_wave(const double* __restrict__ partial, int nb, int c) {
  const int lane = threadIdx.x & (WAVE - 1);
  double acc = 0.0;
  for (int b0 = 0; b0 < nb; b0 += WAVE * 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int b = b0 + lane + WAVE * q;
      v[q] = (b < nb) ? partial[(size_t)b * LDP + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += v[q];
  }
  return wave_sum(acc);
}

// Sum of NV per-lane values over the wave, all at once: each butterfly stage
// exchanges half of the remaining values with the partner lane, so after
// log2(NV) stages a lane holds one partial sum, of value index
// (lane >> (6 - log2 NV)) & (NV - 1); plain xor stages finish the sum.
template <int NV>
__device__ __forceinline__ double bfly_sum(double (&a)[NV]) {
  const int lane = threadIdx.x & (WAVE - 1);
  int mask = WAVE / 2;
#pragma unroll
  for (int h = NV / 2; h >= 1; h /= 2) {
    const bool upper = (lane & mask) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const double send = upper ? a[i] : a[i + h];
      const double keep = upper ? a[i + h] : a[i];
      a[i] = keep + __shfl_xor(send, mask, WAVE);
    }
    mask >>= 1;
  }
  double s = a[0];
  for (int off = mask; off >= 1; off >>= 1) s += __shfl_xor(s, off, WAVE);
  return s;
}
constexpr int BF_NV = 8;
constexpr int BF_SHIFT = 3;   // 6 - log2(BF_NV)

// RPL consecutive rows of one column starting at `row` (aligned: ldq and
// the lane's first row are multiples of RPL)
template <int RPL>
__device__ __forceinline__ void loadr(const float* __restrict__ col, int64_t row,
                                      float (&q)[RPL]) {
  if constexpr (RPL == 4) {
    const float4 v = *reinterpret_cast<const float4*>(col + row);
    q[0] = v.x;
    q[1] = v.y;
    q[2] = v.z;
    q[3] = v.w;
  } else if constexpr (RPL == 2) {
    const float2 v = *reinterpret_cast<const float2*>(col + row);
    q[0] = v.x;
    q[1] = v.y;
  } else {
    q[0] = col[row];
  }
}
template <int RPL>
__device__ __forceinline__ void loadr(const double* __restrict__ col, int64_t row,
                                      double (&q)[RPL]) {
  if constexpr (RPL == 4) {
    const double2 a = *reinterpret_cast<const double2*>(col + row);
    const double2 b = *reinterpret_cast<const double2*>(col + row + 2);
    q[0] = a.x;
    q[1] = a.y;
    q[2] = b.x;
    q[3] = b.y;
  } else if constexpr (RPL == 2) {
    const double2 a = *reinterpret_cast<const double2*>(col + row);
    q[0] = a.x;
    q[1] = a.y;
  } else {
    q[0] = col[row];
  }
}

// prow[c] = sum over the block's 64 RPL rows of Q[c][row] * vv (c < ncols);
// the lane's rows are rowL..rowL+RPL-1 with values vv; wave w takes
// c = w, w+CWV, ...  Rows past the GP's n hold zeros in Q and vv.
template <typename T, int RPL>
__device__ __forceinline__ void coldots(const T* __restrict__ Q, int64_t ldq, int ncols,
                                        int64_t rowL, const double (&vv)[RPL],
                                        double* __restrict__ prow) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  for (int base = w; base < ncols; base += CWV * BF_NV) {
    T q[BF_NV][RPL];
#pragma unroll
    for (int i = 0; i < BF_NV; ++i) {
      const int c = min(base + CWV * i, ncols - 1);
      loadr<RPL>(Q + (int64_t)c * ldq, rowL, q[i]);
    }
    double a[BF_NV];
#pragma unroll
    for (int i = 0; i < BF_NV; ++i) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) s += (double)q[i][r] * vv[r];
      a[i] = (base + CWV * i < ncols) ? s : 0.0;
    }
    const double tot = bfly_sum<BF_NV>(a);
    const int c = base + CWV * ((lane >> BF_SHIFT) & (BF_NV - 1));
    if ((lane & ((1 << BF_SHIFT) - 1)) == 0 && c < ncols) prow[c] = tot;
  }
}

// Per-wave projection rows in LDS: local row t = RPL lane + r is kept at
// r * RPAD + lane, so that the RPL-strided rows of a lane do not fall on the
// same LDS banks when written (lanes contiguous) or read (row order).
constexpr int RPAD = WAVE + 4;
constexpr int REDW = 4 * RPAD;    // doubles per wave (RPL <= 4)
template <int RPL>
__device__ __forceinline__ int red_at(int t) {
  return (t % RPL) * RPAD + t / RPL;
}

// row RPL lane + r of red[w] (at red_at) = sum over the wave's columns c (w, w+CWV, ...) of
// Q[c][rowL + r] * cl[c]; the caller adds the CWV waves' rows in wave order.
template <typename T, int RPL>
__device__ __forceinline__ void colproj(const T* __restrict__ Q, int64_t ldq, int ncols,
                                        int64_t rowL, const double* __restrict__ cl,
                                        double (*red)[REDW]) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  double acc[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) acc[r] = 0.0;
  for (int base = w; base < ncols; base += CWV * BF_NV) {
    T q[BF_NV][RPL];
#pragma unroll
    for (int i = 0; i < BF_NV; ++i) {
      const int c = min(base + CWV * i, ncols - 1);
      loadr<RPL>(Q + (int64_t)c * ldq, rowL, q[i]);
    }
#pragma unroll
    for (int i = 0; i < BF_NV; ++i) {
      const int c = base + CWV * i;
      const double f = c < ncols ? cl[min(c, ncols - 1)] : 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) acc[r] += (double)q[i][r] * f;
    }
  }
#pragma unroll
  for (int r = 0; r < RPL; ++r) red[w][r * RPAD + lane] = acc[r];
}

// A block's 64 RPL rows of the columns of Q that wave w handles (w + CWV i,
// i < 2 BF_NV), loaded once into registers: a pass's projection and its dot
// products share one read of Q, and the loads go out before the
// coefficients they meet are known.  Same column order as colproj / coldots.
static_assert(MAXK <= 2 * CWV * BF_NV, "two column groups per wave cover MAXK");
template <typename T, int RPL>
struct QRegs {
  T q[2][BF_NV][RPL];
};
template <typename T, int RPL>
__device__ __forceinline__ void qregs_load(QRegs<T, RPL>& R, const T* __restrict__ Q, int64_t ldq,
                                           int ncols, int64_t rowL) {
  const int w = threadIdx.x / WAVE;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int base = w + it * CWV * BF_NV;
    if (base < ncols) {
#pragma unroll
      for (int i = 0; i < BF_NV; ++i) {
        const int c = min(base + CWV * i, ncols - 1);
        loadr<RPL>(Q + (int64_t)c * ldq, rowL, R.q[it][i]);
      }
    }
  }
}
// colproj on the register tile (REWIDEN: widen each value at its use, which
// keeps the register count down where the tile has no later use)
template <typename T, int RPL, bool REWIDEN = false>
__device__ __forceinline__ void colproj_regs(const QRegs<T, RPL>& R, int ncols,
                                             const double* __restrict__ cl, double (*red)[REDW]) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  double acc[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) acc[r] = 0.0;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int base = w + it * CWV * BF_NV;
    if (base < ncols) {
#pragma unroll
      for (int i = 0; i < BF_NV; ++i) {
        const int c = base + CWV * i;
        const double f = c < ncols ? cl[min(c, ncols - 1)] : 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          T qv = R.q[it][i][r];
          if constexpr (REWIDEN) asm volatile("" : "+v"(qv));
          acc[r] += (double)qv * f;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPL; ++r) red[w][r * RPAD + lane] = acc[r];
}
// coldots on the register tile
template <typename T, int RPL>
__device__ __forceinline__ void coldots_regs(const QRegs<T, RPL>& R, int ncols,
                                             const double (&vv)[RPL], double* __restrict__ prow) {
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int base = w + it * CWV * BF_NV;
    if (base < ncols) {
      double a[BF_NV];
#pragma unroll
      for (int i = 0; i < BF_NV; ++i) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          // widen again here rather than keep colproj's widened copies alive
          // (twice the registers of the tile)
          T qv = R.q[it][i][r];
          asm volatile("" : "+v"(qv));
          s += (double)qv * vv[r];
        }
        a[i] = (base + CWV * i < ncols) ? s : 0.0;
      }
      const double tot = bfly_sum<BF_NV>(a);
      const int c = base + CWV * ((lane >> BF_SHIFT) & (BF_NV - 1));
      if ((lane & ((1 << BF_SHIFT) - 1)) == 0 && c < ncols) prow[c] = tot;
    }
  }
}

// sum of the column waves' projections of local row t, in wave order
template <int RPL>
__device__ __forceinline__ double red_sum(const double (*red)[REDW], int t) {
  const int at = red_at<RPL>(t);
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < CWV; ++q) s += red[q][at];
  return s;
}

// this lane's RPL values of a per-block row vector staged in LDS
template <int RPL>
__device__ __forceinline__ void lane_rows(const double* vl, double (&vv)[RPL]) {
  const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
  for (int r = 0; r < RPL; ++r) vv[r] = vl[RPL * lane + r];
}

// Column sums of per-block partial rows, batched: out[c] = sum_b partial[b][c]
// for c < nv + nv_add; one wave per column.
struct SumJob {
  const double* partial;
  double* out;
  const Ctl* ctl;
  int nb;
  int nv;
};

__device__ __forceinline__ void colsum_block(const SumJob& J, int lb, int nv_add) {
  const int c = lb * (BLK / WAVE) + threadIdx.x / WAVE;
  if (c >= J.nv + nv_add) return;
  const double s = colsum_wave(J.partial, J.nb, c);
  if ((threadIdx.x & (WAVE - 1)) == 0) J.out[c] = s;
}
__global__ __launch_bounds__(BLK) void k_colsum(Tab tab, const SumJob* __restrict__ jobs,
                                                int nv_add, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SumJob& J = jobs[gp];
  if (ctl_skip(J.ctl, mode)) return;
  colsum_block(J, lb, nv_add);
}

// Rows per lane of the row kernels for a run over `rows` rows: 4 (256-row
// blocks, 16-byte loads) while that still gives >= 256 blocks, else 1
// (64-row blocks) so small problems still spread over the chip.  Chosen per
// GP, so a GP's row blocking (hence its summation order) is the same in a
// batch as in its own build.
// Whether a Lanczos run over nb row blocks sums its partial rows inside the
// consuming kernels (every block adds all nb rows, so the cost grows as nb^2)
// rather than in column-sum launches: measured about even at 160 blocks and
// slower at 391.  The environment variable LOVE_PSUM_MAX_NB=<blocks> moves the
// limit (declared in love.h).
static bool lz_psum(int64_t nb) {
  const char* env = std::getenv("LOVE_PSUM_MAX_NB");
  const int64_t lim = env ? std::atoll(env) : 160;
  return nb <= lim;
}

static int rows_per_lane(int64_t rows) { return cdiv(rows, 256) >= 256 ? 4 : 1; }

// launch over G GPs with nv_g + nv_add columns each (nv_g equal to the jobs' nv)
static void launch_colsum(const SumJob* jobs, const std::vector<int>& nv, int nv_add, int mode,
                          hipStream_t s) {
  std::vector<int64_t> nbk(nv.size());
  for (size_t g = 0; g < nv.size(); ++g) nbk[g] = cdiv(std::max(nv[g] + nv_add, 0), BLK / WAVE);
  const Tab t = make_tab(nbk);
  if (tab_blocks(t)) tlaunch("colsum", k_colsum, tab_blocks(t), BLK, 0, s, t, jobs, nv_add, mode);
}

// ----------------------------------------------------------------------------
// Lanczos steps (batched over GPs; LzJob per GP)
// ----------------------------------------------------------------------------
// Row kernels run on blocks of 64 RPL rows (RPL rows per lane): threads
// t < 64 RPL own row r0 + t in the per-row phases; ldq is a multiple of 256.
// partial[lb][0] = sum of v^2 over the block's rows
template <typename T, int RPL>
__device__ __forceinline__ void lz_norm_body(const LzJob<T>& J, int lb) {
  __shared__ double scr[16];
  constexpr int RBK = WAVE * RPL;
  const int64_t row = (int64_t)lb * RBK + threadIdx.x;
  const double v = (threadIdx.x < RBK && row < J.n) ? (double)J.v[row] : 0.0;
  const double s = block_sum(v * v, scr);
  if (threadIdx.x == 0) J.partial[(size_t)lb * LDP] = s;
}
template <typename T>
__global__ __launch_bounds__(RBLK) void k_lz_norm(Tab tab, const LzJob<T>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const LzJob<T>& J = jobs[gp];
  if (J.rpl == 4) lz_norm_body<T, 4>(J, lb);
  else lz_norm_body<T, 1>(J, lb);
}

// ctl->bnorm = sqrt(sum_b partial[b][0]); one block of one wave per GP
template <typename T>
__global__ void k_lz_bnorm(Tab tab, const LzJob<T>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const LzJob<T>& J = jobs[gp];
  const double s = colsum_wave(J.partial, J.nb, 0);
  if (threadIdx.x == 0) J.ctl->bnorm = sqrt(s);
}

// q_0 = v / ||v|| (zeros on the padding rows n..ldq-1)
template <typename T, int RPL>
__device__ __forceinline__ void lz_start_body(const LzJob<T>& J, int lb) {
  constexpr int RBK = WAVE * RPL;
  if (threadIdx.x >= RBK) return;
  const int64_t row = (int64_t)lb * RBK + threadIdx.x;
  const double b = J.ctl->bnorm;
  J.Q[row] = row < J.n ? (T)((double)J.v[row] / b) : T(0);
}
template <typename T>
__global__ __launch_bounds__(RBLK) void k_lz_start(Tab tab, const LzJob<T>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const LzJob<T>& J = jobs[gp];
  if (J.rpl == 4) lz_start_body<T, 4>(J, lb);
  else lz_start_body<T, 1>(J, lb);
}

// First pass: v = W R_j + sigma^2 q_j (rows), partial rows of Q_{0..j}^T v.
template <typename T, int D, int RPL>
__device__ __forceinline__ void lz_gdots_body(const LzJob<T>& J, int lb, int j) {
  if (J.ctl->stop) return;
  constexpr int RBK = WAVE * RPL;
  __shared__ double vl[RBK];
  const int64_t r0 = (int64_t)lb * RBK;
  const int64_t n = J.n;
  if (threadIdx.x < RBK) {
    const int64_t row = r0 + threadIdx.x;
    double val = 0.0;
    if (row < n) {
      const T* qj = J.Q + (int64_t)j * J.ldq;
      const T vv = gather_row_dev<T, D>(J.g, J.x, row, J.R + (int64_t)j * J.m) + J.sigma2 * qj[row];
      J.v[row] = vv;
      val = (double)vv;
    }
    vl[threadIdx.x] = val;
  }
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  double vv[RPL];
  lane_rows<RPL>(vl, vv);
  coldots<T, RPL>(J.Q, J.ldq, j + 1, r0 + RPL * lane, vv, J.partial + (size_t)lb * LDP);
}
template <typename T, int D>
__global__ __launch_bounds__(RBLK) void k_lz_gdots(Tab tab, const LzJob<T>* __restrict__ jobs,
                                                  int j) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const LzJob<T>& J = jobs[gp];
  if (J.rpl == 4) lz_gdots_body<T, D, 4>(J, lb, j);
  else lz_gdots_body<T, D, 1>(J, lb, j);
}

// Blocks of the grid-space first pass: one per 256-row tile up to
// GPASS_NBC_SUM tiles, whose partial rows the second pass adds itself;
// larger grids take one block per tile (at most GPASS_NBC_MAX) and a
// column-sum launch adds their rows (the second pass would otherwise read
// them all in every block).
constexpr int GPASS_NBC_SUM = 64;
constexpr int GPASS_NBC_MAX = 1024;
static inline int gpass_blocks(int64_t m) {
  const int64_t t = cdiv(m, RB);
  return (int)(t <= GPASS_NBC_SUM ? t : std::min<int64_t>(t, GPASS_NBC_MAX));
}

// Grid-space first pass: partial rows of G_{0..j}^T R_j over the GP's nbc
// blocks; block lb takes the 256-row tiles lb, lb + nbc, ... (lane: 4 rows),
// the waves split the columns as in coldots and keep one running sum per
// column group across tiles.  R_j has no padding rows (masked); G's padding
// rows are zero.
template <typename T>
__global__ __launch_bounds__(RBLK) void k_lz_cdots(Tab tab, const LzJob<T>* __restrict__ jobs,
                                                  int j) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const LzJob<T>& J = jobs[gp];
  if (J.ctl->stop) return;
  static_assert(MAXK <= 2 * CWV * BF_NV, "two column groups per wave");
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int ncols = j + 1;
  const T* Rj = J.R + (int64_t)j * J.m;
  double acc[2] = {0.0, 0.0};
  for (int64_t t0 = (int64_t)lb * RB; t0 < J.m; t0 += (int64_t)J.nbc * RB) {
    const int64_t row = t0 + 4 * lane;
    double vv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) vv[r] = row + r < J.m ? (double)Rj[row + r] : 0.0;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int base = w + it * CWV * BF_NV;
      if (base >= ncols) break;
      T q[BF_NV][4];
#pragma unroll
      for (int i = 0; i < BF_NV; ++i) {
        const int c = min(base + CWV * i, ncols - 1);
        loadr<4>(J.G + (int64_t)c * J.ldg, row, q[i]);
      }
      double a[BF_NV];
#pragma unroll
      for (int i = 0; i < BF_NV; ++i) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) s += (double)q[i][r] * vv[r];
        a[i] = (base + CWV * i < ncols) ? s : 0.0;
      }
      acc[it] += bfly_sum<BF_NV>(a);
    }
  }
  if ((lane & ((1 << BF_SHIFT) - 1)) == 0) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int c = w + it * CWV * BF_NV + CWV * ((lane >> BF_SHIFT) & (BF_NV - 1));
      if (c < ncols) J.gpart[(size_t)lb * LDP + c] = acc[it];
    }
  }
}

// c_i = sum of the nbc cdots rows (+ sigma^2 at i = j), into cl; block 0
// also stores them as the first-pass coefficients.  Rows are added in a
// fixed order (4 interleaved parts, then the parts in order).
template <typename T>
__device__ __forceinline__ void gpass_coef(const LzJob<T>& J, int j, int lb, double* cl) {
  __shared__ double part[RBLK / 128][128];
  const int ncols = j + 1;
  const int c = threadIdx.x & 127, p = threadIdx.x >> 7;
  double s = 0.0;
  if (c < ncols) {
#pragma unroll 4
    for (int b = p; b < J.nbc; b += RBLK / 128) s += J.gpart[(size_t)b * LDP + c];
  }
  part[p][c] = s;
  __syncthreads();
  if (threadIdx.x < ncols) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < RBLK / 128; ++q) t += part[q][threadIdx.x];
    if ((int)threadIdx.x == j) t += (double)J.sigma2;
    cl[threadIdx.x] = t;
    if (lb == 0) J.coef[threadIdx.x] = t;
  }
}

// cl[c] = sum of the rows b < nrows of part (stride LDP) at column c, for
// c < ncols <= LDP.  Columns go in chunks of 128 (64 for a last chunk of
// <= 64); each chunk's rows are added in a fixed order (RBLK / chunk width
// interleaved row sets, then the sets in order), so every block gets the
// same sums.  BATCH > 0: a thread issues its rows BATCH masked loads at a
// time (the same sums in the same order; more registers, fewer round trips
// to rows other blocks just wrote).
template <int BATCH = 0>
__device__ __forceinline__ void rows_sum(const double* part, int nrows, int ncols, double* cl) {
  __shared__ double ps[RBLK];
  for (int c0 = 0; c0 < ncols; c0 += 128) {
    const int sh = ncols - c0 <= 64 ? 6 : 7;
    const int w = 1 << sh, np = RBLK >> sh;
    const int c = threadIdx.x & (w - 1), p = threadIdx.x >> sh;
    double s = 0.0;
    if (c0 + c < ncols) {
      if constexpr (BATCH > 0) {
        for (int b0 = p; b0 < nrows; b0 += BATCH * np) {
          double v[BATCH];
#pragma unroll
          for (int q = 0; q < BATCH; ++q) {
            const int b = b0 + q * np;
            v[q] = b < nrows ? part[(size_t)b * LDP + c0 + c] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < BATCH; ++q) s += v[q];
        }
      } else {
#pragma unroll 8
        for (int b = p; b < nrows; b += np) s += part[(size_t)b * LDP + c0 + c];
      }
    }
    ps[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < w && c0 + (int)threadIdx.x < ncols) {
      double t = 0.0;
      for (int q = 0; q < np; ++q) t += ps[q * w + threadIdx.x];
      cl[c0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// Second pass: r' = v - Q c ; partial rows of [Q^T r', ||r'||^2].  With the
// grid-space first pass, v = W R_j + sigma^2 q_j is formed here and c comes
// from the cdots rows.
// Row-sum load batches of the in-kernel sums: the double runs (the sampler's,
// at most 160 blocks, never register-bound) batch 20 loads; the float main
// runs keep the short loop, whose register count keeps two blocks per CU.
template <typename T>
constexpr int RS_BATCH_OF = sizeof(T) == 8 ? 20 : 0;

template <typename T, int D, int RPL>
__device__ __forceinline__ void lz_udots_body(const LzJob<T>& J, int lb, int j) {
  if (J.ctl->stop) return;
  constexpr int RBK = WAVE * RPL;
  __shared__ double cl[MAXK];
  __shared__ double red[CWV][REDW];
  __shared__ double rl[RBK];
  __shared__ double scr[16];
  // 3-D and 4-D stencils (64 and 256 nodes per row) with 256-row blocks: two
  // threads per row, each gathering half of the stencil
  constexpr bool SPLIT = D >= 3 && RPL == 4;
  static_assert(!SPLIT || RBLK == 2 * WAVE * RPL, "two threads per row");
  __shared__ T gh[2][WAVE * RPL];
  const int ncols = j + 1;
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)lb * RBK;
  const int64_t row = r0 + t;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t rowL = r0 + RPL * lane;
  QRegs<T, RPL> qr;
  qregs_load<T, RPL>(qr, J.Q, J.ldq, ncols, rowL);
  T vrow = T(0);
  if (J.gpath) {
    if constexpr (SPLIT) {
      const int rr = t & (RBK - 1), hf = t / RBK;
      const int64_t gr = r0 + rr;
      T part = T(0);
      if (gr < J.n) {
        T xr[D];
#pragma unroll
        for (int e = 0; e < D; ++e) xr[e] = J.x[gr * D + e];
        part = gather_row_part<T, D>(J.g, xr, J.R + (int64_t)j * J.m, hf);
      }
      gh[hf][rr] = part;
    } else {
      if (t < RBK && row < J.n)
        vrow = gather_row_dev<T, D>(J.g, J.x, row, J.R + (int64_t)j * J.m) +
               J.sigma2 * J.Q[(int64_t)j * J.ldq + row];
    }
    if (J.gcs) {
      // the first pass's rows summed by the column-sum launch (into c2)
      for (int c = threadIdx.x; c < ncols; c += RBLK) {
        const double t = J.c2[c] + (c == j ? (double)J.sigma2 : 0.0);
        cl[c] = t;
        if (lb == 0) J.coef[c] = t;
      }
    } else {
      gpass_coef<T>(J, j, lb, cl);
    }
  } else if (J.psum) {
    if (t < RBK && row < J.n) vrow = J.v[row];
    rows_sum<RS_BATCH_OF<T>>(J.partial, J.nb, ncols, cl);
    if (lb == 0)
      for (int c = threadIdx.x; c < ncols; c += RBLK) J.coef[c] = cl[c];
  } else {
    if (t < RBK && row < J.n) vrow = J.v[row];
    for (int c = threadIdx.x; c < ncols; c += RBLK) cl[c] = J.coef[c];
  }
  __syncthreads();
  if constexpr (SPLIT) {
    if (J.gpath && t < RBK && row < J.n)
      vrow = (gh[0][t] + gh[1][t]) + J.sigma2 * J.Q[(int64_t)j * J.ldq + row];
  }
  colproj_regs<T, RPL>(qr, ncols, cl, red);
  __syncthreads();
  double rv = 0.0;
  if (t < RBK) {
    if (row < J.n) {
      const double proj = red_sum<RPL>(red, t);
      const T r = (T)((double)vrow - proj);
      J.r[row] = r;
      rv = (double)r;
    }
    rl[t] = rv;
  }
  const double rrb = block_sum(rv * rv, scr);
  __syncthreads();
  double vv[RPL];
  lane_rows<RPL>(rl, vv);
  double* prow = (J.psum ? J.partial2 : J.partial) + (size_t)lb * LDP;
  coldots_regs<T, RPL>(qr, ncols, vv, prow);
  if (threadIdx.x == 0) prow[ncols] = rrb;
}
// The 4-D float instance is held to 128 registers (four waves per SIMD, two
// blocks per CU) at the cost of a small spill: measured faster than one
// block per CU at 153 registers.
template <typename T, int D>
__global__ __launch_bounds__(RBLK)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && D == 4 ? 4 : 1)))
void k_lz_udots(Tab tab, const LzJob<T>* __restrict__ jobs, int j) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const LzJob<T>& J = jobs[gp];
  if (J.rpl == 4) lz_udots_body<T, D, 4>(J, lb, j);
  else lz_udots_body<T, D, 1>(J, lb, j);
}

// alpha_j, beta_j, stop test (every block, identically), then
// q_{j+1} = (r' - Q c2) / beta_j on rows 0..ldq-1 (zeros past n).  Block 0
// records the step.  At j = k - 1 the run stops (no new vector).
template <typename T, int RPL>
__device__ __forceinline__ void lz_finalize_body(const LzJob<T>& J, int lb, int j) {
  Ctl* ctl = J.ctl;
  if (ctl->stop) return;
  constexpr int RBK = WAVE * RPL;
  __shared__ double cl[MAXK];
  __shared__ double red[CWV][REDW];
  __shared__ double s_beta;
  __shared__ int s_stop;
  __shared__ double c2l[LDP];
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t r0 = (int64_t)lb * RBK, rowL = r0 + RPL * lane;
  QRegs<T, RPL> qr;
  qregs_load<T, RPL>(qr, J.Q, J.ldq, j + 1, rowL);
  const double* c2rr = J.c2;
  if (J.psum) {
    rows_sum<RS_BATCH_OF<T>>(J.partial2, J.nb, j + 2, c2l);
    c2rr = c2l;
  }
  for (int c = threadIdx.x; c <= j; c += RBLK) cl[c] = c2rr[c];
  if (threadIdx.x < WAVE) {
    double c2n = 0.0;
    for (int c = lane; c <= j; c += WAVE) c2n += c2rr[c] * c2rr[c];
    c2n = wave_sum(c2n);
    if (threadIdx.x == 0) {
      const double a = J.coef[j] + c2rr[j];
      const double b2 = c2rr[j + 1] - c2n;
      const double b = b2 > 0.0 ? sqrt(b2) : 0.0;
      const double amax = fmax(j > 0 ? J.amax[j - 1] : 0.0, fabs(a));
      int stop = 0;
      unsigned st = 0;
      int keff = j + 1;
      if (!isfinite(a) || !isfinite(b)) {
        stop = 1;
        st = SF_NONFINITE;
        keff = j;
      } else if (j < J.klast && !(b > J.tol * amax)) {
        stop = 1;
        st = SF_BREAKDOWN;
      } else if (j >= J.klast) {
        stop = 1;
      }
      s_beta = b;
      s_stop = stop;
      // Block 0 records; other blocks of this launch that read ctl->stop after
      // it is set reach the same decision from the same inputs.
      if (lb == 0) {
        J.alpha[j] = a;
        J.beta[j] = b;
        J.amax[j] = amax;
        ctl->k_eff = keff;
        if (stop) {
          ctl->stop = 1;
          ctl->status |= st;
        }
      }
    }
  }
  __syncthreads();
  if (s_stop) return;
  colproj_regs<T, RPL, true>(qr, j + 1, cl, red);
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= RBK) return;
  const int64_t row = r0 + t;
  double q = 0.0;
  if (row < J.n) {
    const double proj = red_sum<RPL>(red, t);
    q = ((double)J.r[row] - proj) / s_beta;
  }
  J.Q[(int64_t)(j + 1) * J.ldq + row] = (T)q;
}
template <typename T>
__global__ __launch_bounds__(RBLK) void k_lz_finalize(Tab tab, const LzJob<T>* __restrict__ jobs,
                                                     int j) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const LzJob<T>& J = jobs[gp];
  if (J.rpl == 4) lz_finalize_body<T, 4>(J, lb, j);
  else lz_finalize_body<T, 1>(J, lb, j);
}


// Cholesky of the tridiagonal T (alpha, beta) of size ctl->k_eff; one block
// per GP, one thread working.  A non-positive pivot truncates k_eff there
// (SF_NOTPD).  rel_tol: a pivot must exceed rel_tol * max|alpha|.
template <typename T>
__global__ void k_tri_chol(Tab tab, const LzJob<T>* __restrict__ jobs, double rel_tol) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const LzJob<T>& J = jobs[gp];
  Ctl* ctl = J.ctl;
  // alpha, beta staged in LDS by the whole block; the recurrence (one thread)
  // then reads and writes LDS only, and the factors go out in parallel
  __shared__ double a[MAXK], b[MAXK], ld[MAXK], ls[MAXK];
  __shared__ int s_keep;
  const int k = ctl->k_eff;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    a[i] = J.alpha[i];
    b[i] = J.beta[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double amax = 0.0;
    for (int i = 0; i < k; ++i) amax = fmax(amax, fabs(a[i]));
    int keep = k;
    double prev = 0.0;
    for (int i = 0; i < k; ++i) {
      const double piv = a[i] - prev * prev;
      if (!(piv > rel_tol * amax) || !isfinite(piv)) {
        keep = i;
        ctl->status |= SF_NOTPD;
        break;
      }
      const double l = sqrt(piv);
      ld[i] = l;
      prev = (i + 1 < k) ? b[i] / l : 0.0;
      ls[i] = prev;
    }
    s_keep = keep;
    ctl->k_eff = keep;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < s_keep; i += blockDim.x) {
    J.ldiag[i] = ld[i];
    J.lsub[i] = ls[i];
  }
}

// Rt[u, :] = (L^{-1} R[:, u])^T : bidiagonal forward substitution per grid node.
// split = 1 stores bf16 hi = rne(z), lo = rne(z - hi).
// Rt[u, :] = (L^{-1} R[:, u])^T (and, for the hyper-parameter gradient, B
// from G = W^T Q the same way).  One wave per 64 grid rows, lane = row: the
// forward substitution runs down the k columns (loads of R coalesced over the
// rows), the rows are staged in LDS and leave as one contiguous 64 x kpad slab
// (coalesced stores), in the cache precision or as bf16 hi + bf16 lo.
constexpr int RT_ROWS = WAVE;
template <typename T>
__global__ __launch_bounds__(RT_ROWS) void k_rtilde(Tab tab, const RtJob<T>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const RtJob<T>& J = jobs[gp];
  constexpr int TS = MAXK + 1;   // tile row stride (odd: rows fall on different banks)
  __shared__ T tile[RT_ROWS * TS];
  __shared__ double ld[MAXK], ls[MAXK];
  const int k = J.ctl->k_eff, kpad = J.kpad;
  const int64_t m = J.m, rs = J.ld ? J.ld : J.m;
  const int t = threadIdx.x;
  for (int i = t; i < k; i += RT_ROWS) {
    ld[i] = J.ldiag[i];
    ls[i] = J.lsub[i];
  }
  __syncthreads();
  const int64_t u0 = (int64_t)lb * RT_ROWS, u = u0 + t;
  double z = 0.0;
  // unrolled so that the loads of R for several columns are in flight while
  // the substitution (one divide per column) runs
#pragma unroll 8
  for (int i = 0; i < kpad; ++i) {
    double val = 0.0;
    if (i < k && u < m) {
      const double rv = (double)J.R[(int64_t)i * rs + u];
      z = (rv - (i > 0 ? ls[i - 1] * z : 0.0)) / ld[i];
      val = z;
    }
    tile[t * TS + i] = (T)val;
  }
  __syncthreads();
  const int rows = (int)min<int64_t>(RT_ROWS, m - u0);
  for (int q = t; q < rows * kpad; q += RT_ROWS) {
    const int r = q / kpad, i = q - r * kpad;
    const T val = tile[r * TS + i];
    const int64_t idx = (u0 + r) * kpad + i;
    if (J.split) {
      const float f = (float)val;
      const uint16_t hi = f32_to_bf16_rne(f);
      const uint16_t lo = f32_to_bf16_rne(f - bf16_to_f32(hi));
      ((uint16_t*)J.rt)[idx] = hi;
      J.rt_lo[idx] = lo;
    } else {
      ((T*)J.rt)[idx] = val;
    }
  }
}

// ----------------------------------------------------------------------------
// Mean cache: preconditioned CG on Khat x = y (double vectors), batched.
//
// Preconditioner from the Lanczos decomposition Khat Q ~ Q T that the build
// already holds (Sec. 2.2; the Lanczos solve Q T^{-1} Q^T b of eq.
// lanczos_solve is its action on span(Q)):
//   M^{-1} = Q T^{-1} Q^T + (I - Q Q^T)^2 / sigma^2
//          = I / sigma^2 + Q C Q^T,   C = T^{-1} - (2 I - G) / sigma^2,  G = Q^T Q.
// Both terms are positive semidefinite and their null spaces meet only in 0,
// so M^{-1} is positive definite for any Q (also when the float Lanczos
// vectors are orthonormal only to ~1e-7); on span(Q) it inverts T, and on the
// rest Khat is sigma^2 I plus the spectrum the Lanczos run did not reach.
// With c = Q^T r and d = C c, z = M^{-1} r = r / sigma^2 + Q d and
// r^T z = r^T r / sigma^2 + c^T d, so no extra pass is needed for r^T z.
// Per iteration:
//   scatter  g_p = W^T (z + ratio * p)         (new direction, formed on the fly)
//   toeplitz kg = K g_p
//   ap       p = z + ratio * p ; Ap = W kg + sigma^2 p ; partial rows of p^T Ap
//   update   gamma = rz / p^T Ap ; x += gamma p ; r -= gamma Ap ;
//            partial rows of [Q^T r, r^T r]
//   colsum   c, r^T r
//   pcg_ep   convergence test; d = C c ; rz_new ; ratio = rz_new / rz
//   apply    z = r / sigma^2 + Q d
// With the identity preconditioner (plain CG) c and d are empty and z = r.
// ----------------------------------------------------------------------------
constexpr int PAP_COL = LDP - 1;   // partial-row column of p^T Ap (clear of the dot columns)

struct ConvJob {
  const float* in;
  double* out;
  int64_t n;
};
__global__ void k_convert_b(Tab tab, const ConvJob* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ConvJob& J = jobs[gp];
  const int64_t i = (int64_t)lb * blockDim.x + threadIdx.x;
  if (i < J.n) J.out[i] = (double)J.in[i];
}

template <typename TQ, int D, int RPL>
__device__ __forceinline__ void cg_ap_body(const CgJob<TQ>& J, int lb) {
  if (J.ctl->cg_done) return;
  __shared__ double scr[16];
  constexpr int RBK = WAVE * RPL;
  const double ratio = J.ctl->ratio;
  const int64_t row = (int64_t)lb * RBK + threadIdx.x;
  double d = 0.0;
  if (threadIdx.x < RBK && row < J.n) {
    const double pn = J.z[row] + ratio * J.p[row];
    J.p[row] = pn;
    const double a = gather_row_dev<double, D>(J.g, J.x, row, J.gm) + J.sigma2 * pn;
    J.ap[row] = a;
    d = pn * a;
  }
  const double db = block_sum(d, scr);
  if (threadIdx.x == 0) J.partial[(size_t)lb * LDP + PAP_COL] = db;
}
template <typename TQ, int D>
__global__ __launch_bounds__(RBLK) void k_cg_ap(Tab tab, const CgJob<TQ>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const CgJob<TQ>& J = jobs[gp];
  if (J.rpl == 4) cg_ap_body<TQ, D, 4>(J, lb);
  else cg_ap_body<TQ, D, 1>(J, lb);
}

// partial rows of [Q^T r, r^T r] from the block's residual rows (rl in LDS)
template <typename TQ, int RPL>
__device__ __forceinline__ void pcg_dots(const CgJob<TQ>& J, const double* rl, double ssb, int lb) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int kq = J.kq;
  const int ncols = min(kq, J.ctl->k_eff);
  double* prow = J.partial + (size_t)lb * LDP;
  if (ncols > 0) {
    double vv[RPL];
    lane_rows<RPL>(rl, vv);
    coldots<TQ, RPL>(J.Q, J.ldq, ncols, (int64_t)lb * (WAVE * RPL) + RPL * lane, vv, prow);
  }
  for (int c = max(ncols, 0) + threadIdx.x; c < kq; c += RBLK) prow[c] = 0.0;
  if (threadIdx.x == 0) prow[kq] = ssb;
}

// x = 0, r = y, p = 0, partial rows of [Q^T y, y^T y]
template <typename TQ, int RPL>
__device__ __forceinline__ void pcg_init_body(const CgJob<TQ>& J, int lb) {
  constexpr int RBK = WAVE * RPL;
  __shared__ double rl[RBK];
  __shared__ double scr[16];
  const int64_t row = (int64_t)lb * RBK + threadIdx.x;
  double v = 0.0;
  if (threadIdx.x < RBK) {
    if (row < J.n) {
      v = J.y[row];
      J.xs[row] = 0.0;
      J.r[row] = v;
      J.p[row] = 0.0;
    }
    rl[threadIdx.x] = v;
  }
  const double ssb = block_sum(v * v, scr);
  __syncthreads();
  pcg_dots<TQ, RPL>(J, rl, ssb, lb);
}
template <typename TQ>
__global__ __launch_bounds__(RBLK) void k_pcg_init(Tab tab, const CgJob<TQ>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const CgJob<TQ>& J = jobs[gp];
  if (J.rpl == 4) pcg_init_body<TQ, 4>(J, lb);
  else pcg_init_body<TQ, 1>(J, lb);
}

// gamma = rz / p^T Ap (p^T Ap re-summed by every block from the partial rows
// of k_cg_ap, one wave, fixed order); x += gamma p ; r -= gamma Ap ; dots.
template <typename TQ, int RPL>
__device__ __forceinline__ void pcg_update_body(const CgJob<TQ>& J, int lb) {
  if (J.ctl->cg_done) return;
  constexpr int RBK = WAVE * RPL;
  __shared__ double rl[RBK];
  __shared__ double scr[16];
  __shared__ double s_pap;
  if (threadIdx.x < WAVE) {
    const double sum = colsum_wave(J.partial, J.nb, PAP_COL);
    if (threadIdx.x == 0) s_pap = sum;
  }
  __syncthreads();
  const double gm = J.ctl->rz / s_pap;
  const int64_t row = (int64_t)lb * RBK + threadIdx.x;
  double v = 0.0;
  if (threadIdx.x < RBK) {
    if (row < J.n) {
      J.xs[row] += gm * J.p[row];
      v = J.r[row] - gm * J.ap[row];
      J.r[row] = v;
    }
    rl[threadIdx.x] = v;
  }
  const double ssb = block_sum(v * v, scr);
  __syncthreads();
  pcg_dots<TQ, RPL>(J, rl, ssb, lb);
}
template <typename TQ>
__global__ __launch_bounds__(RBLK) void k_pcg_update(Tab tab, const CgJob<TQ>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const CgJob<TQ>& J = jobs[gp];
  if (J.rpl == 4) pcg_update_body<TQ, 4>(J, lb);
  else pcg_update_body<TQ, 1>(J, lb);
}

// One block per GP.  coef = [c_0 .. c_{kq-1}, r^T r] (column sums of the
// update's partial rows).  Convergence test on ||r|| <= tol ||y||, then
// d = C c, rz = r^T r * rscale + c^T d and the direction ratio.  init: first
// call (sets ||y||^2, ratio 0).
template <typename TQ>
__global__ __launch_bounds__(BLK) void k_pcg_ep(Tab tab, const CgJob<TQ>* __restrict__ jobs,
                                                int init) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const CgJob<TQ>& J = jobs[gp];
  Ctl* ctl = J.ctl;
  if (ctl->cg_done) return;
  __shared__ double cl[MAXK];
  __shared__ double scr[16];
  const int kq = J.kq;
  const int k = min(kq, ctl->k_eff);
  const double* sums = J.coef;
  const int t = threadIdx.x;
  if (t < k) cl[t] = sums[t];
  __syncthreads();
  double cd = 0.0;
  if (t < k) {
    double acc = 0.0;
    const double* row = J.cm + (size_t)t * J.kpad;
    for (int jj = 0; jj < k; ++jj) acc += row[jj] * cl[jj];
    J.dvec[t] = acc;
    cd = cl[t] * acc;
  }
  const double cdb = block_sum(cd, scr);
  if (t != 0) return;
  const double rr = sums[kq];
  if (init) {
    ctl->rr0 = rr;
    ctl->cg_iters = 0;
  } else {
    ctl->cg_iters += 1;
  }
  ctl->rr = rr;
  const double rz = rr * J.rscale + cdb;
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
  if (!(rz > 0.0)) {   // cannot happen for a positive definite M^{-1}; stop cleanly
    ctl->cg_done = 1;
    ctl->status |= SF_CG_NOCONV;
    return;
  }
  ctl->ratio = init ? 0.0 : rz / ctl->rz;
  ctl->rz = rz;
}

// z = r * rscale + Q d  (first min(kq, k_eff) columns)
template <typename TQ, int RPL>
__device__ __forceinline__ void pcg_apply_body(const CgJob<TQ>& J, int lb) {
  if (J.ctl->cg_done) return;
  __shared__ double dl[MAXK];
  __shared__ double red[CWV][REDW];
  const int k = min(J.kq, J.ctl->k_eff);
  for (int c = threadIdx.x; c < k; c += RBLK) dl[c] = J.dvec[c];
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  constexpr int RBK = WAVE * RPL;
  const int64_t r0 = (int64_t)lb * RBK;
  if (k > 0) {
    colproj<TQ, RPL>(J.Q, J.ldq, k, r0 + RPL * lane, dl, red);
    __syncthreads();
  }
  const int t = threadIdx.x;
  const int64_t row = r0 + t;
  if (t >= RBK || row >= J.n) return;
  double acc = J.r[row] * J.rscale;
  if (k > 0) acc += red_sum<RPL>(red, t);
  J.z[row] = acc;
}
template <typename TQ>
__global__ __launch_bounds__(RBLK) void k_pcg_apply(Tab tab, const CgJob<TQ>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const CgJob<TQ>& J = jobs[gp];
  if (J.rpl == 4) pcg_apply_body<TQ, 4>(J, lb);
  else pcg_apply_body<TQ, 1>(J, lb);
}

// Gram matrix G = Q^T Q of the first k_eff columns, in double: per-block
// partial kpad x kpad matrices over row slices.  Thread (ti, tj) of a 16 x 16
// layout owns entries (ti + 16a, tj + 16b), a, b < 8; rows are staged through
// LDS in tiles of GR_TR.
constexpr int GR_TR = 32;
template <typename TQ>
__global__ __launch_bounds__(256) void k_gram(Tab tab, const CgJob<TQ>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const CgJob<TQ>& J = jobs[gp];
  constexpr int NA = 8, KP = 16 * NA;
  __shared__ double tile[GR_TR][KP + 1];
  const int t = threadIdx.x, ti = t / 16, tj = t % 16;
  const int k = min(J.kq, J.ctl->k_eff);
  const int kpad = J.kpad;
  double acc[NA][NA];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NA; ++b) acc[a][b] = 0.0;
  const int64_t rb = (int64_t)lb * J.rpbg;
  const int64_t re = min<int64_t>(rb + J.rpbg, J.n);
  for (int64_t r0 = rb; r0 < re; r0 += GR_TR) {
    for (int e = t; e < GR_TR * KP; e += 256) {
      const int rr = e % GR_TR, cc = e / GR_TR;
      const int64_t row = r0 + rr;
      tile[rr][cc] = (row < re && cc < k) ? (double)J.Q[(int64_t)cc * J.ldq + row] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < GR_TR; ++rr) {
      double qi[NA], qj[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) qi[a] = tile[rr][ti + 16 * a];
#pragma unroll
      for (int b = 0; b < NA; ++b) qj[b] = tile[rr][tj + 16 * b];
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NA; ++b) acc[a][b] += qi[a] * qj[b];
    }
    __syncthreads();
  }
  double* out = J.pg + (size_t)lb * kpad * kpad;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NA; ++b) {
      const int i = ti + 16 * a, jj = tj + 16 * b;
      if (i < kpad && jj < kpad) out[(size_t)i * kpad + jj] = acc[a][b];
    }
}

// T^{-1} from T = L L^T (bidiagonal L): thread i solves T x = e_i; one block
// of MAXK threads per GP.
template <typename TQ>
__global__ void k_tinv(Tab tab, const CgJob<TQ>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const CgJob<TQ>& J = jobs[gp];
  const int i = threadIdx.x;
  const int kpad = J.kpad;
  if (i >= kpad) return;
  const int k = min(J.kq, J.ctl->k_eff);
  const double* ldiag = J.ldiag;
  const double* lsub = J.lsub;
  double* col = J.tinv + (size_t)i * kpad;
  for (int jj = 0; jj < kpad; ++jj) col[jj] = 0.0;
  if (i >= k) return;
  // forward: L w = e_i (w_j = 0 for j < i)
  double w = 1.0 / ldiag[i];
  col[i] = w;
  for (int jj = i + 1; jj < k; ++jj) {
    w = -lsub[jj - 1] * w / ldiag[jj];
    col[jj] = w;
  }
  // backward: L^T x = w
  double xn = col[k - 1] / ldiag[k - 1];
  col[k - 1] = xn;
  for (int jj = k - 2; jj >= 0; --jj) {
    xn = (col[jj] - lsub[jj] * xn) / ldiag[jj];
    col[jj] = xn;
  }
}

// C = T^{-1} - (2 I - G) / sigma^2 with G summed from the k_gram partials in
// block order; ortho = max |G - I| (bit patterns of non-negative doubles
// order like unsigned integers).
template <typename TQ>
__global__ void k_pcg_matrix(Tab tab, const CgJob<TQ>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const CgJob<TQ>& J = jobs[gp];
  const int kpad = J.kpad;
  const int e = lb * blockDim.x + threadIdx.x;
  if (e >= kpad * kpad) return;
  const int i = e / kpad, jj = e % kpad;
  const int k = min(J.kq, J.ctl->k_eff);
  double gsum = 0.0;
  for (int b = 0; b < J.nbg; ++b) gsum += J.pg[(size_t)b * kpad * kpad + e];
  const bool in = i < k && jj < k;
  J.cm[e] = in ? J.tinv[e] - ((i == jj ? 2.0 : 0.0) - gsum) / J.sigma2 : 0.0;
  if (in && J.ortho) {
    const double dev = fabs(gsum - (i == jj ? 1.0 : 0.0));
    atomicMax((unsigned long long*)J.ortho, (unsigned long long)__double_as_longlong(dev));
  }
}

// flags[g] = 1 once GP g's CG is done; one block
template <typename TQ>
__global__ void k_cg_flags(int G, const CgJob<TQ>* __restrict__ jobs, int* flags) {
  for (int g = threadIdx.x; g < G; g += blockDim.x) flags[g] = jobs[g].ctl->cg_done ? 1 : 0;
}

// a[u] = gm[u] in the cache precision
template <typename TQ>
__global__ void k_cg_store_a(Tab tab, const CgJob<TQ>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const CgJob<TQ>& J = jobs[gp];
  const int64_t u = (int64_t)lb * blockDim.x + threadIdx.x;
  if (u >= J.m) return;
  if (J.a_fp64) ((double*)J.a)[u] = J.gm[u];
  else ((float*)J.a)[u] = (float)J.gm[u];
}

__global__ void k_ctl_init(Ctl* ctl) {
  Ctl z{};
  *ctl = z;
}

// ============================================================================
// Sampling cache (Sec. 3.3): Lanczos on B = K - R^T R' = K - Rt Rt^T in grid
// space (eq. lancapprox), probe b' = (1/m) B 1, then a factor S with
// S S^T = Q' T' Q'^T (eq. pred_covar_ski_interp_form).  B is the difference
// of two nearly equal matrices (the posterior covariance is 1e-4..1e-6 of the
// prior here), so this Lanczos runs in double whatever the cache precision;
// Rt is read in its stored precision and widened.  One GP at a time.
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


// partial rows of s = Rt^T v (columns < keff) over blocks of 64 RPL grid
// rows; lanes own columns, waves split the rows.
template <typename TR, int SPLIT, int RPL>
__device__ __forceinline__ void rt_dots_block(int b, int64_t m, const double* __restrict__ v,
                                              const void* __restrict__ rt,
                                              const uint16_t* __restrict__ rt_lo, int kpad,
                                              const Ctl* ctl_main,
                                              double* __restrict__ partial) {
  constexpr int RBK = WAVE * RPL;
  __shared__ double wsum[RBLK / WAVE][MAXK];
  const int keff = ctl_main->k_eff;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int64_t r0 = (int64_t)b * RBK;
  const int64_t r1 = min<int64_t>(r0 + RBK, m);
  double a0 = 0.0, a1 = 0.0;
#pragma unroll 8
  for (int64_t u = r0 + w; u < r1; u += RBLK / WAVE) {
    const double vu = v[u];
    if (lane < keff) a0 += vu * rt_val<TR, SPLIT>(rt, rt_lo, u * kpad + lane);
    if (lane + WAVE < keff) a1 += vu * rt_val<TR, SPLIT>(rt, rt_lo, u * kpad + lane + WAVE);
  }
  wsum[w][lane] = a0;
  wsum[w][lane + WAVE] = a1;
  __syncthreads();
  double* prow = partial + (size_t)b * LDP;
  for (int c = threadIdx.x; c < keff; c += RBLK) {
    double s = 0.0;
    for (int q = 0; q < RBLK / WAVE; ++q) s += wsum[q][c];
    prow[c] = s;
  }
}
template <typename TR, int SPLIT, int RPL>
__global__ __launch_bounds__(RBLK) void k_rt_dots(int64_t m, const double* __restrict__ v,
                                                 const void* __restrict__ rt,
                                                 const uint16_t* __restrict__ rt_lo, int kpad,
                                                 const Ctl* ctl_main,
                                                 double* __restrict__ partial, const Ctl* ctl) {
  if (ctl->stop) return;
  rt_dots_block<TR, SPLIT, RPL>(blockIdx.x, m, v, rt, rt_lo, kpad, ctl_main, partial);
}

// Sampler step, first launch: K q_j by the banded product (blocks [0, nbb),
// the axis job tj) and the partial rows of s = Rt^T q_j (the row blocks after
// them) -- independent work on the same vector, one launch.
static_assert(TB_WAVES * WAVE == RBLK, "band blocks and row blocks have one size");
template <typename TR, int SPLIT, int RPL>
__global__ __launch_bounds__(RBLK) void k_sp_band_rt(Tab tband, const ToepJob<double>* __restrict__ tj,
                                                    int j, int nbb, int64_t m,
                                                    const double* __restrict__ v,
                                                    const void* __restrict__ rt,
                                                    const uint16_t* __restrict__ rt_lo, int kpad,
                                                    const Ctl* ctl_main,
                                                    double* __restrict__ partial, const Ctl* ctl) {
  if (ctl->stop) return;
  if ((int)blockIdx.x < nbb) {
    int gp, lb;
    if (!tab_find(tband, blockIdx.x, gp, lb)) return;
    toep_band_block<double>(tj[gp], lb, j);
  } else {
    rt_dots_block<TR, SPLIT, RPL>(blockIdx.x - nbb, m, v, rt, rt_lo, kpad, ctl_main, partial);
  }
}

// Second launch: the segment sums of the banded product (blocks [0, nrb)) and
// the column sums giving s (the blocks after them).
static_assert(TB_RED == BLK, "reduce blocks and colsum blocks have one size");
__global__ __launch_bounds__(BLK) void k_sp_reduce_sum(Tab tred,
                                                      const ToepJob<double>* __restrict__ tj,
                                                      int j, int nrb,
                                                      const SumJob* __restrict__ sj,
                                                      const Ctl* ctl) {
  if (ctl->stop) return;
  if ((int)blockIdx.x < nrb) {
    int gp, lb;
    if (!tab_find(tred, blockIdx.x, gp, lb)) return;
    toep_reduce_block<double>(tj[gp], lb, j);
  } else {
    colsum_block(*sj, blockIdx.x - nrb, 0);
  }
}

// v = kv - Rt s on the block's 64 RPL grid rows, then partial rows of
// Q'_{0..ncols-1}^T v (none for ncols = 0).  Each wave takes NR rows per
// butterfly: lanes own columns lane and lane + 64 of Rt (columns past k_eff
// hold zeros, and s is zero there), and the NR row dots are reduced by one
// butterfly.  The Rt values, kv and the Q' tile are loaded before s is read.
template <typename TR, int SPLIT>
__device__ __forceinline__ auto rt_raw(const void* rt, const uint16_t* rt_lo, int64_t idx) {
  if constexpr (SPLIT) {
    const uint16_t* hi = (const uint16_t*)rt;
    return bf16_to_f32(hi[idx]) + bf16_to_f32(rt_lo[idx]);
  } else {
    return ((const TR*)rt)[idx];
  }
}
template <typename TR, int SPLIT, int RPL>
__global__ __launch_bounds__(RBLK) void k_sp_apply_dots(int64_t m, const double* __restrict__ kv,
                                                       const void* __restrict__ rt,
                                                       const uint16_t* __restrict__ rt_lo,
                                                       int kpad, const Ctl* ctl_main,
                                                       const double* __restrict__ sv,
                                                       const double* __restrict__ Q, int64_t ldq,
                                                       int ncols, double* __restrict__ vout,
                                                       double* __restrict__ partial,
                                                       const Ctl* ctl,
                                                       const double* __restrict__ rtpart,
                                                       int nbr,
                                                       const double* __restrict__ kseg,
                                                       int nseg, int64_t segL) {
  if (ctl->stop) return;
  constexpr int RBK = WAVE * RPL;
  constexpr int NW = RBLK / WAVE;
  constexpr int NR = RPL == 1 ? 8 : 16;        // rows per butterfly
  constexpr int NIT = RBK / (NW * NR);         // butterflies per wave
  constexpr int SH = NR == 8 ? 3 : 2;          // 6 - log2(NR)
  static_assert(NIT * NW * NR == RBK, "rows split evenly over the waves");
  using RV = decltype(rt_raw<TR, SPLIT>(nullptr, nullptr, 0));
  __shared__ double vl[RBK];
  __shared__ double sl[2 * WAVE];
  __shared__ double kl[RBK];
  const int64_t r0 = (int64_t)blockIdx.x * RBK;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  if (kseg) {
    // K q on the block's rows from the banded segments (a fixed number of
    // masked loads, issued first), added in segment order as the segment-sum
    // kernel adds them (scale 1)
    if ((int)threadIdx.x < RBK) {
      const int64_t u = min<int64_t>(r0 + threadIdx.x, m - 1);
      double sv_[TB_NSEG_MAX];
#pragma unroll
      for (int q = 0; q < TB_NSEG_MAX; ++q) sv_[q] = q < nseg ? kseg[(int64_t)q * segL + u] : 0.0;
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < TB_NSEG_MAX; ++q) acc += sv_[q];
      kl[threadIdx.x] = acc;
    }
  }
  QRegs<double, RPL> qr;   // Q' tile for the dots
  qregs_load<double, RPL>(qr, Q, ldq, ncols, r0 + RPL * lane);
  RV a0[NIT][NR], a1[NIT][NR];
  const bool hi_cols = kpad > WAVE;            // kpad is 64 or 128
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int64_t u = min<int64_t>(r0 + (it * NW + w) * NR + i, m - 1);
      a0[it][i] = rt_raw<TR, SPLIT>(rt, rt_lo, u * kpad + lane);
      a1[it][i] = hi_cols ? rt_raw<TR, SPLIT>(rt, rt_lo, u * kpad + lane + WAVE) : RV(0);
    }
  }
  const int keff = ctl_main->k_eff;
  if (rtpart) {
    // s = Rt^T q from the nbr partial rows (the segment-sum launch is skipped)
    rows_sum<20>(rtpart, nbr, 2 * WAVE, sl);
    for (int c = threadIdx.x; c < 2 * WAVE; c += RBLK)
      if (c >= keff) sl[c] = 0.0;
  } else {
    for (int c = threadIdx.x; c < 2 * WAVE; c += RBLK) sl[c] = c < keff ? sv[c] : 0.0;
  }
  __syncthreads();
  const double s0 = sl[lane], s1 = sl[lane + WAVE];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int rb = (it * NW + w) * NR;
    double part[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) part[i] = (double)a0[it][i] * s0 + (double)a1[it][i] * s1;
    const double tot = bfly_sum<NR>(part);
    if ((lane & ((1 << SH) - 1)) == 0) {
      const int i = (lane >> SH) & (NR - 1);
      const int64_t u = r0 + rb + i;
      double val = 0.0;
      if (u < m) {
        val = (kseg ? kl[rb + i] : kv[u]) - tot;
        vout[u] = val;
      }
      vl[rb + i] = val;
    }
  }
  __syncthreads();
  if (ncols == 0) return;
  double vv[RPL];
  lane_rows<RPL>(vl, vv);
  coldots_regs<double, RPL>(qr, ncols, vv, partial + (size_t)blockIdx.x * LDP);
}

// Eigen-decomposition T' = V diag(lam) V^T of the sampler's symmetric
// tridiagonal (k' <= 128), returned sorted by decreasing eigenvalue in
// vout (column c at vout[c * MAXK + row]) and lam.  k_chol counts the strictly
// positive eigenvalues: negative Ritz values of K - Rt Rt^T come from the
// rounding of the float cache and are clipped to zero.
//
// Fast path, parallel over eigenvalues:
//  * eigenvalues by multisection of Sturm counts (the count of negative
//    pivots of the LDL^T factorisation of T' - x I is the number of
//    eigenvalues below x): one wave per eigenvalue index, its 64 lanes count
//    at 64 interior points of the current bracket, so each round narrows the
//    bracket 65-fold; ten rounds take the Gershgorin interval to rounding
//    level;
//  * eigenvectors by a twisted factorisation (one lane per eigenvalue):
//    forward and backward LDL^T of T' - lam I give
//    gamma_r = D+_r + D-_r - (alpha_r - lam); with r = argmin |gamma_r|, z_r = 1
//    and the two one-term recurrences outward from r solve
//    (T' - lam I) z = gamma_r e_r.  The error of z is ~ eps ||T'|| / gap.
// What matters downstream is V Lambda V^T, to which an eigenvalue lam
// contributes lam * z z^T; so when a neighbour of a non-negligible eigenvalue
// (lam > 1e-9 ||T'||) is closer than 1e-6 lam, or a vector is not finite, the
// fast path hands over to the implicit QL solver below, whose eigenvectors
// are orthogonal to rounding whatever the gaps.
constexpr int EIG_ROUNDS = 10;

__device__ inline int sturm_count(const double* a, const double* b2, int k, double x,
                                  double pivmin) {
  int cnt = 0;
  double q = a[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < k; ++i) {
    q = (a[i] - x) - b2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// Gershgorin interval [gl, gu] of T' and the pivot floor, per thread (k steps).
__device__ inline void tri_bounds(const double* a, const double* b, int k, double& gl, double& gu,
                                  double& pivmin) {
  gl = 1e300;
  gu = -1e300;
  double bmax2 = 0.0;
  for (int i = 0; i < k; ++i) {
    const double off = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < k ? fabs(b[i]) : 0.0);
    gl = fmin(gl, a[i] - off);
    gu = fmax(gu, a[i] + off);
    if (i + 1 < k) bmax2 = fmax(bmax2, b[i] * b[i]);
  }
  pivmin = 2.2250738585072014e-308 * fmax(1.0, bmax2);
  const double tn = fmax(fabs(gl), fabs(gu));
  const double fudge = 4.0 * 2.220446049250313e-16 * tn * (double)k + 4.0 * pivmin;
  gl -= fudge;
  gu += fudge;
}

// lam_asc[e] = e-th smallest eigenvalue; block of EIG_WPB waves, wave per index.
constexpr int EIG_WPB = 4;
__global__ __launch_bounds__(WAVE * EIG_WPB) void k_eig_bisect(const double* __restrict__ alpha,
                                                               const double* __restrict__ beta,
                                                               double* __restrict__ lam_asc,
                                                               const Ctl* ctl) {
  __shared__ double a[MAXK], b[MAXK], b2[MAXK];
  const int k = ctl->k_eff;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    a[i] = alpha[i];
    const double bi = (i + 1 < k) ? beta[i] : 0.0;
    b[i] = bi;
    b2[i] = bi * bi;
  }
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  const int e = blockIdx.x * EIG_WPB + threadIdx.x / WAVE;
  if (e >= k) return;
  double lo, hi, pivmin;
  tri_bounds(a, b, k, lo, hi, pivmin);
  const double eps = 2.220446049250313e-16;
  for (int it = 0; it < EIG_ROUNDS; ++it) {
    const double w = hi - lo;
    if (!(w > 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin)) break;   // uniform
    const double step = w / (double)(WAVE + 1);
    const double x = lo + step * (double)(lane + 1);
    const int cnt = sturm_count(a, b2, k, x, pivmin);
    const uint64_t mask = __ballot(cnt > e);   // lanes whose point lies above lam_e
    if (mask == 0ull) {
      lo = lo + step * (double)WAVE;
    } else {
      const int f = __ffsll((unsigned long long)mask) - 1;
      const double nlo = f > 0 ? lo + step * (double)f : lo;
      hi = lo + step * (double)(f + 1);
      lo = nlo;
    }
  }
  if (lane == 0) lam_asc[e] = 0.5 * (lo + hi);
}

// Eigenvectors by twisted factorisation; one block, one thread per eigenvalue
// (blockDim >= k).  dscr: 2 * MAXK * MAXK doubles (forward / backward pivots,
// [i][e] so a wave's accesses coalesce).  force_ql: always hand over to QL.
__global__ __launch_bounds__(MAXK) void k_eig_vectors(const double* __restrict__ alpha,
                                                      const double* __restrict__ beta,
                                                      const double* __restrict__ lam_asc,
                                                      double* __restrict__ vout,
                                                      double* __restrict__ lam,
                                                      double* __restrict__ dscr, int force_ql,
                                                      Ctl* ctl) {
  __shared__ double a[MAXK], b[MAXK];
  __shared__ int s_bad, s_pos;
  const int k = ctl->k_eff;
  const int e = threadIdx.x;
  for (int i = e; i < k; i += blockDim.x) {
    a[i] = alpha[i];
    b[i] = (i + 1 < k) ? beta[i] : 0.0;
  }
  if (e == 0) {
    s_bad = force_ql;
    s_pos = 0;
  }
  __syncthreads();
  if (e < k) {
    double gl, gu, pivmin;
    tri_bounds(a, b, k, gl, gu, pivmin);
    const double tn = fmax(fabs(gl), fabs(gu));
    const double lm = lam_asc[e];
    int bad = 0;
    if (e + 1 < k) {
      const double ln = lam_asc[e + 1];
      const double big = fmax(fabs(lm), fabs(ln));
      if (big > 1e-9 * tn && (ln - lm) < 1e-6 * big) bad = 1;
    }
    // the two pivot tables do not overlap each other or vout: restrict lets
    // the loads of one iteration be issued ahead of the previous stores
    double* __restrict__ dp = dscr;
    double* __restrict__ dm = dscr + MAXK * MAXK;
    // forward pivots D+
    double q = a[0] - lm;
    if (fabs(q) < pivmin) q = -pivmin;
    dp[e] = q;
    for (int i = 1; i < k; ++i) {
      q = (a[i] - lm) - b[i - 1] * b[i - 1] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      dp[i * MAXK + e] = q;
    }
    // backward pivots D- and the twist index
    q = a[k - 1] - lm;
    if (fabs(q) < pivmin) q = -pivmin;
    dm[(k - 1) * MAXK + e] = q;
    int r = k - 1;
    double gbest = fabs(dp[(k - 1) * MAXK + e] + q - (a[k - 1] - lm));
#pragma unroll 8
    for (int i = k - 2; i >= 0; --i) {
      q = (a[i] - lm) - b[i] * b[i] / q;
      if (fabs(q) < pivmin) q = -pivmin;
      dm[i * MAXK + e] = q;
      const double gm = fabs(dp[i * MAXK + e] + q - (a[i] - lm));
      if (gm < gbest) {
        gbest = gm;
        r = i;
      }
    }
    // z_r = 1, recurrences outward; column c = k-1-e of vout (decreasing order)
    const int c = k - 1 - e;
    double* __restrict__ col = vout + (size_t)c * MAXK;
    double z = 1.0, nrm = 1.0;
    col[r] = 1.0;
#pragma unroll 8
    for (int i = r - 1; i >= 0; --i) {
      z = -(b[i] / dp[i * MAXK + e]) * z;
      col[i] = z;
      nrm += z * z;
    }
    z = 1.0;
#pragma unroll 8
    for (int i = r; i + 1 < k; ++i) {
      z = -(b[i] / dm[(i + 1) * MAXK + e]) * z;
      col[i + 1] = z;
      nrm += z * z;
    }
    if (!isfinite(nrm) || !isfinite(lm)) bad = 1;
    const double inv = 1.0 / sqrt(nrm);
    for (int i = 0; i < k; ++i) col[i] *= inv;
    for (int i = k; i < MAXK; ++i) col[i] = 0.0;
    lam[c] = lm;
    if (bad) atomicOr(&s_bad, 1);
    if (lm > 0.0 && isfinite(lm)) atomicAdd(&s_pos, 1);
  }
  __syncthreads();
  if (e == 0) {
    if (s_bad) {
      ctl->eig_fallback = 1;
    } else {
      ctl->k_chol = s_pos;
      if (s_pos < k) ctl->status |= SF_SAMPLER_TRUNC;
    }
  }
}

// Implicit QL with Wilkinson shifts (Bowdler, Martin, Reinsch and Wilkinson,
// 1968), the fallback above; does nothing unless ctl->eig_fallback.  One wave
// does everything: lane i holds d[i], d[i+64], e[i], e[i+64] in registers; the
// scalar chase runs uniformly on all lanes (values fetched with readlane), and
// every plane rotation is applied at once to the lane's two rows of V (held in
// global scratch), the updated column carried in registers.
constexpr int EIG_MAXSWEEP = 40;

__device__ inline double rl64(double v, int lane) {
  const int2 u = *reinterpret_cast<const int2*>(&v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(u.x, lane);
  r.y = __builtin_amdgcn_readlane(u.y, lane);
  return *reinterpret_cast<const double*>(&r);
}
// value of a 128-entry array held as (lo: entries 0..63, hi: entries 64..127)
__device__ inline double get128(double lo, double hi, int i) {
  return i < WAVE ? rl64(lo, i) : rl64(hi, i - WAVE);
}
__device__ inline void set128(double& lo, double& hi, int i, double v, int lane) {
  if (i < WAVE) lo = (lane == i) ? v : lo;
  else hi = (lane == i - WAVE) ? v : hi;
}

__global__ __launch_bounds__(WAVE) void k_tri_eig(const double* __restrict__ alpha,
                                                  const double* __restrict__ beta,
                                                  double* __restrict__ vout,
                                                  double* __restrict__ lam,
                                                  double* __restrict__ V, Ctl* ctl) {
  if (!ctl->eig_fallback) return;
  // V: column c at V[c * MAXK + row] (global scratch: this path is the rare one)
  __shared__ double dsh[MAXK];
  __shared__ int perm[MAXK];
  const int lane = threadIdx.x;
  const int k = ctl->k_eff;
  for (int cidx = 0; cidx < k; ++cidx) {
    V[cidx * MAXK + lane] = (cidx == lane) ? 1.0 : 0.0;
    V[cidx * MAXK + lane + WAVE] = (cidx == lane + WAVE) ? 1.0 : 0.0;
  }
  double dlo = lane < k ? alpha[lane] : 0.0;
  double dhi = lane + WAVE < k ? alpha[lane + WAVE] : 0.0;
  double elo = lane + 1 < k ? beta[lane] : 0.0;
  double ehi = lane + WAVE + 1 < k ? beta[lane + WAVE] : 0.0;
  unsigned bad = 0;
  for (int l = 0; l < k; ++l) {
    int iter = 0;
    while (true) {
      int mm = l;
      for (; mm < k - 1; ++mm) {
        const double dd = fabs(get128(dlo, dhi, mm)) + fabs(get128(dlo, dhi, mm + 1));
        if (fabs(get128(elo, ehi, mm)) <= 2.220446049250313e-16 * dd) break;
      }
      if (mm == l) break;
      if (++iter > EIG_MAXSWEEP) {
        bad = 1;
        break;
      }
      const double dl = get128(dlo, dhi, l), el = get128(elo, ehi, l);
      double g = (get128(dlo, dhi, l + 1) - dl) / (2.0 * el);
      double r = hypot(g, 1.0);
      g = get128(dlo, dhi, mm) - dl + el / (g + copysign(r, g));
      double sv = 1.0, cv = 1.0, p = 0.0;
      // eigenvector rows of this lane: column mm is the running carry
      double car0 = V[mm * MAXK + lane], car1 = V[mm * MAXK + lane + WAVE];
      int last = -1;
      bool underflow = false;
      for (int i = mm - 1; i >= l; --i) {
        const double ei = get128(elo, ehi, i);
        const double f = sv * ei, b = cv * ei;
        const double ss = f * f + g * g;
        double inv = 0.0;
        if (ss > 0.0) {
          inv = rsqrt(ss);
          inv = inv * (1.5 - 0.5 * ss * inv * inv);   // one Newton step
        }
        r = ss * inv;
        set128(elo, ehi, i + 1, r, lane);
        if (r == 0.0) {
          set128(dlo, dhi, i + 1, get128(dlo, dhi, i + 1) - p, lane);
          set128(elo, ehi, mm, 0.0, lane);
          underflow = true;
          break;
        }
        sv = f * inv;
        cv = g * inv;
        g = get128(dlo, dhi, i + 1) - p;
        r = (get128(dlo, dhi, i) - g) * sv + 2.0 * cv * b;
        p = sv * r;
        set128(dlo, dhi, i + 1, g + p, lane);
        g = cv * r - b;
        // V[:, i+1] <- s V[:, i] + c V[:, i+1] ; V[:, i] <- c V[:, i] - s V[:, i+1]
        const double v0 = V[i * MAXK + lane], v1 = V[i * MAXK + lane + WAVE];
        V[(i + 1) * MAXK + lane] = sv * v0 + cv * car0;
        V[(i + 1) * MAXK + lane + WAVE] = sv * v1 + cv * car1;
        car0 = cv * v0 - sv * car0;
        car1 = cv * v1 - sv * car1;
        last = i;
      }
      if (last >= 0) {
        V[last * MAXK + lane] = car0;
        V[last * MAXK + lane + WAVE] = car1;
      }
      if (!underflow) {
        set128(dlo, dhi, l, get128(dlo, dhi, l) - p, lane);
        set128(elo, ehi, l, g, lane);
        set128(elo, ehi, mm, 0.0, lane);
      }
    }
  }
  dsh[lane] = dlo;
  dsh[lane + WAVE] = dhi;
  __syncthreads();
  if (lane == 0) {
    for (int i = 0; i < k; ++i) perm[i] = i;
    for (int i = 0; i < k; ++i) {          // selection sort, decreasing
      int best = i;
      for (int j = i + 1; j < k; ++j)
        if (dsh[perm[j]] > dsh[perm[best]]) best = j;
      const int tmpi = perm[i];
      perm[i] = perm[best];
      perm[best] = tmpi;
    }
    int pos = 0;
    for (int i = 0; i < k; ++i) {
      lam[i] = dsh[perm[i]];
      if (dsh[perm[i]] > 0.0 && isfinite(dsh[perm[i]])) pos = i + 1;
    }
    ctl->k_chol = pos;
    if (pos < k) ctl->status |= SF_SAMPLER_TRUNC;
    if (bad) ctl->status |= SF_NONFINITE;
  }
  __syncthreads();
  for (int cidx = 0; cidx < k; ++cidx) {
    vout[cidx * MAXK + lane] = V[perm[cidx] * MAXK + lane];
    vout[cidx * MAXK + lane + WAVE] = V[perm[cidx] * MAXK + lane + WAVE];
  }
}

// S[u, c] = sqrt(lam_c) * sum_i Q'[i][u] V[c][i]  for c < k_chol (zero beyond kspad).
__global__ __launch_bounds__(256) void k_s_from_eig(int64_t m, const double* __restrict__ Q,
                                                    int64_t ldq, const double* __restrict__ vout,
                                                    const double* __restrict__ lam,
                                                    float* __restrict__ S, int kspad,
                                                    const Ctl* ctl) {
  constexpr int CT = 16;                      // columns of S per block (blockIdx.y)
  __shared__ double Vl[CT][MAXK];             // sqrt(lam_c) * eigenvector c
  const int k = ctl->k_eff, kc = ctl->k_chol;
  const int c0 = blockIdx.y * CT;
  for (int idx = threadIdx.x; idx < CT * k; idx += blockDim.x) {
    const int q = idx / k, i = idx % k;
    Vl[q][i] = (c0 + q < kc) ? vout[(c0 + q) * MAXK + i] * sqrt(lam[c0 + q]) : 0.0;
  }
  __syncthreads();
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= m) return;
  double acc[CT];
#pragma unroll
  for (int q = 0; q < CT; ++q) acc[q] = 0.0;
  if (c0 < kc) {
    for (int i = 0; i < k; ++i) {
      const double qv = Q[(int64_t)i * ldq + u];
#pragma unroll
      for (int q = 0; q < CT; ++q) acc[q] += qv * Vl[q][i];
    }
  }
#pragma unroll
  for (int q = 0; q < CT; ++q)
    if (c0 + q < kspad) S[u * kspad + c0 + q] = (float)acc[q];
}

template <typename TR, int SPLIT, int RPL>
static love_status sampler_impl(love_cache* c, hipStream_t s) {
  const int64_t m = c->m;
  const int ks = c->ks;
  const int64_t ldq = cdiv(m, RB) * RB;
  const int64_t nb = ldq / (WAVE * RPL);
  double *Q, *v, *r, *kv, *gv, *sv, *alpha, *beta, *vout, *lam, *lasc, *dscr, *tsc, *partial,
      *partial2, *coef, *c2, *amax;
  char* buf = nullptr;
  {
    size_t bytes = sizeof(double) * ((size_t)ldq * ks + 4 * (size_t)ldq + 8 * LDP +
                                     3 * MAXK * MAXK + (size_t)toeplitz_scratch_elems(c) +
                                     2 * (size_t)nb * LDP);
    buf = (char*)ws_alloc(bytes, s);
    if (!buf) return LOVE_ENOMEM;
    Q = (double*)buf;
    v = Q + (size_t)ldq * ks;
    r = v + ldq;
    kv = r + ldq;
    gv = kv + ldq;
    sv = gv + ldq;
    alpha = sv + LDP;
    beta = alpha + LDP;
    lam = beta + LDP;
    lasc = lam + LDP;
    coef = lasc + LDP;
    c2 = coef + LDP;
    amax = c2 + LDP;
    vout = amax + LDP;
    dscr = vout + MAXK * MAXK;
    tsc = dscr + 2 * MAXK * MAXK;
    partial = tsc + toeplitz_scratch_elems(c);
    partial2 = partial + (size_t)nb * LDP;
  }
  Ctl* ctl = c->ctl_s;
  const Ctl* cm = c->ctl;
  LzJob<double> J{};
  J.n = m;
  J.ldq = ldq;
  J.Q = Q;
  J.v = v;
  J.r = r;
  J.partial = partial;
  J.coef = coef;
  J.c2 = c2;
  J.amax = amax;
  J.alpha = alpha;
  J.beta = beta;
  J.ctl = ctl;
  J.tol = 1e-12;
  J.klast = ks - 1;
  J.nb = (int)nb;
  J.rpl = RPL;
  J.psum = lz_psum(nb) ? 1 : 0;
  J.partial2 = partial2;
  SumJob js_rt{partial, sv, ctl, (int)nb, c->k};
  SumJob js_coef{partial, coef, ctl, (int)nb, 1};
  SumJob js_c2{partial, c2, ctl, (int)nb, 2};
  JobArena A;
  // the workspace and the job tables go back on every return path
  struct SpRelease {
    char* buf;
    JobArena& a;
    hipStream_t st;
    ~SpRelease() {
      a.release(st);
      ws_free(buf, st);
    }
  } sp_release{buf, A, s};
  const size_t o_lz = A.add(std::vector<LzJob<double>>{J});
  const size_t o_rt = A.add(std::vector<SumJob>{js_rt});
  const size_t o_coef = A.add(std::vector<SumJob>{js_coef});
  const size_t o_c2 = A.add(std::vector<SumJob>{js_c2});
  ToepRun<double> t_probe, t_step;
  std::vector<love_cache*> one{c};
  toep_prepare<double>(A, t_probe, one, {gv}, {0}, {kv}, {0}, {tsc}, {ctl});
  toep_prepare<double>(A, t_step, one, {Q}, {ldq}, {kv}, {0}, {tsc}, {ctl});
  love_status st = A.upload(s);
  if (st != LOVE_OK) return st;
  const LzJob<double>* dJ = A.at<LzJob<double>>(o_lz);
  const Tab t1 = tab1(1), tnb = tab1(nb);
  const std::vector<int> nv1{1}, nv2{2}, nvk{c->k};   // must match the jobs' nv
  k_ctl_init<<<1, 1, 0, s>>>(ctl);
  const uint16_t* rlo = (const uint16_t*)c->rt_lo;
  {
    ProfScope ps("sampler_probe", s);
    launch_fill<double>(gv, 1.0 / (double)m, m, s);
    toep_run<double>(A, t_probe, 0, 1, s);
    k_rt_dots<TR, SPLIT, RPL><<<(unsigned)nb, RBLK, 0, s>>>(m, gv, c->rt, rlo, c->kpad, cm,
                                                            partial, ctl);
    launch_colsum(A.at<SumJob>(o_rt), nvk, 0, 1, s);
    k_sp_apply_dots<TR, SPLIT, RPL><<<(unsigned)nb, RBLK, 0, s>>>(
        m, kv, c->rt, rlo, c->kpad, cm, sv, Q, ldq, 0, v, partial, ctl, nullptr, 0, nullptr, 0, 0);
    k_lz_norm<double><<<(unsigned)nb, RBLK, 0, s>>>(tnb, dJ);
    k_lz_bnorm<double><<<1, WAVE, 0, s>>>(t1, dJ);
    k_lz_start<double><<<(unsigned)nb, RBLK, 0, s>>>(tnb, dJ);
  }
  // one banded axis: K q_j and s = Rt^T q_j share two launches
  const auto& ax0 = t_step.ax[0];
  const bool fuse = t_step.d == 1 && tab_blocks(ax0.band) > 0 && tab_blocks(ax0.lines) == 0 &&
                    tab_blocks(ax0.fft) == 0;
  // one banded job and in-kernel partial sums: the apply kernel also adds the
  // banded segments of its rows and the Rt^T q partial rows (which then go to
  // the second partial buffer), and the segment-sum launch is skipped
  const bool fold = fuse && J.psum && ax0.band.G == 1;
  const double* kseg = (fold && ax0.nseg0 > 1) ? (const double*)ax0.partial0 : nullptr;
  for (int j = 0; j < ks; ++j) {
    ProfScope ps("sampler_step", s);
    const double* qj = Q + (size_t)j * ldq;
    if (fuse) {
      const ToepJob<double>* tj = A.at<ToepJob<double>>(ax0.jobs);
      const unsigned nbb = tab_blocks(ax0.band), nrb = tab_blocks(ax0.reduce);
      tlaunch("sp_band_rt", k_sp_band_rt<TR, SPLIT, RPL>, nbb + (unsigned)nb, RBLK, 0, s,
              ax0.band, tj, j, (int)nbb, m, qj, c->rt, rlo, c->kpad, cm, fold ? partial2 : partial,
              (const Ctl*)ctl);
      if (!fold)
        tlaunch("sp_reduce_sum", k_sp_reduce_sum, nrb + (unsigned)cdiv(c->k, BLK / WAVE), BLK, 0,
                s, ax0.reduce, tj, j, (int)nrb, A.at<SumJob>(o_rt), (const Ctl*)ctl);
    } else {
      toep_run<double>(A, t_step, j, 1, s);
      tlaunch("rt_dots", k_rt_dots<TR, SPLIT, RPL>, (unsigned)nb, RBLK, 0, s, m, qj, c->rt, rlo,
              c->kpad, cm, partial, (const Ctl*)ctl);
      launch_colsum(A.at<SumJob>(o_rt), nvk, 0, 1, s);
    }
    tlaunch("sp_apply", k_sp_apply_dots<TR, SPLIT, RPL>, (unsigned)nb, RBLK, 0, s, m, kv, c->rt,
            rlo, c->kpad, cm, sv, Q, ldq, j + 1, v, partial, (const Ctl*)ctl,
            fold ? (const double*)partial2 : (const double*)nullptr, (int)nb, kseg,
            (int)ax0.nseg0, (int64_t)ax0.L0);
    if (!J.psum) launch_colsum(A.at<SumJob>(o_coef), nv1, j, 1, s);
    tlaunch("sp_udots", k_lz_udots<double, 1>, (unsigned)nb, RBLK, 0, s, tnb, dJ, j);
    if (!J.psum) launch_colsum(A.at<SumJob>(o_c2), nv2, j, 1, s);
    tlaunch("sp_finalize", k_lz_finalize<double>, (unsigned)nb, RBLK, 0, s, tnb, dJ, j);
  }
  {
    ProfScope pe("sampler_eig", s);
    const int force_ql = (c->cfg.flags & LOVE_FLAG_EIG_QL) ? 1 : 0;
    k_eig_bisect<<<(unsigned)cdiv(ks, EIG_WPB), WAVE * EIG_WPB, 0, s>>>(alpha, beta, lasc, ctl);
    k_eig_vectors<<<1, MAXK, 0, s>>>(alpha, beta, lasc, vout, lam, dscr, force_ql, ctl);
    k_tri_eig<<<1, WAVE, 0, s>>>(alpha, beta, vout, lam, dscr, ctl);
    dim3 sgrid((unsigned)cdiv(m, 256), (unsigned)cdiv(c->kspad, 16));
    k_s_from_eig<<<sgrid, 256, 0, s>>>(m, Q, ldq, vout, lam, c->S, c->kspad, ctl);
  }
  LOVE_HIP_TRY(hipGetLastError());
  return LOVE_OK;
}

template <int RPL>
static love_status sampler_rpl(love_cache* c, hipStream_t s) {
  if (c->fp64) return sampler_impl<double, 0, RPL>(c, s);
  if (c->cfg.precision == LOVE_P_FP32_BF16SPLIT) return sampler_impl<float, 1, RPL>(c, s);
  return sampler_impl<float, 0, RPL>(c, s);
}

static love_status sampler_dispatch(love_cache* c, hipStream_t s) {
  ProfScope ps("sampler_build", s);
  return rows_per_lane(c->m) == 4 ? sampler_rpl<4>(c, s) : sampler_rpl<1>(c, s);
}

// ============================================================================
// Restart with a new probe (Sec. 5, "Ensuring Lanczos solves are accurate").
// After the first run the Lanczos solve Q H^{-1} Q^T is checked on the
// averaged columns c_g = W K 1_g / |g| of W K (1_g: the indicator of the g-th
// run of consecutive grid nodes); if the worst relative residual
// ||c_g - Khat Q H^{-1} Q^T c_g|| / ||c_g|| is too large, more Lanczos steps
// start from that residual (orthogonalised twice against every earlier
// vector; the step kernels then orthogonalise against both blocks), and
// H = Q^T Khat Q = G^T R^T + sigma^2 Q^T Q (G = W^T Q, rows of R = K W^T q_j)
// with its dense Cholesky factor replaces the tridiagonal T.  Single GP.
// ============================================================================
// gv = 1_[lo, hi) / (hi - lo) over the m grid nodes
template <typename T>
__global__ void k_rs_group(T* __restrict__ gv, int64_t m, int64_t lo, int64_t hi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) gv[i] = (i >= lo && i < hi) ? (T)(1.0 / (double)(hi - lo)) : T(0);
}

// D[i * ldd + g] = Q[:, i] . Y[:, g] over n rows, i < k, g < ng; one block per (i, g)
template <typename T>
__global__ __launch_bounds__(256) void k_rs_dots(const T* __restrict__ Q, int64_t ldq,
                                                 const T* __restrict__ Y, int64_t ldy, int64_t n,
                                                 int ng, double* __restrict__ D, int ldd) {
  __shared__ double scr[16];
  const int i = blockIdx.x, g = blockIdx.y;
  const T* q = Q + (int64_t)i * ldq;
  const T* y = Y + (int64_t)g * ldy;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) acc += (double)q[r] * (double)y[r];
  acc = block_sum(acc, scr);
  if (threadIdx.x == 0) D[(int64_t)i * ldd + g] = acc;
}

// X[:, g] = Q[:, :k] Yk[:, g] (rows past n zero); Yk is k x ldy (column g at g)
template <typename T>
__global__ void k_rs_combine(const T* __restrict__ Q, int64_t ldq, int k,
                             const double* __restrict__ Yk, int ldy, int ng,
                             T* __restrict__ X, int64_t ldx, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ldx) return;
  for (int g = 0; g < ng; ++g) {
    double a = 0.0;
    if (r < n)
      for (int i = 0; i < k; ++i) a += (double)Q[(int64_t)i * ldq + r] * Yk[(int64_t)i * ldy + g];
    X[(int64_t)g * ldx + r] = (T)a;
  }
}

// solve (L L^T) y = b for ng right-hand sides in place (B: k x ldb, column g
// at g); L dense lower, k x MAXK row-major, k = ctl->k_eff.  One thread per
// right-hand side.
__global__ void k_rs_solve(const double* __restrict__ L, const Ctl* __restrict__ ctl,
                           double* __restrict__ B, int ldb, int ng) {
  const int g = threadIdx.x;
  if (g >= ng) return;
  const int k = ctl->k_eff;
  for (int i = 0; i < k; ++i) {
    double z = B[(int64_t)i * ldb + g];
    for (int l = 0; l < i; ++l) z -= L[i * MAXK + l] * B[(int64_t)l * ldb + g];
    B[(int64_t)i * ldb + g] = z / L[i * MAXK + i];
  }
  for (int i = k - 1; i >= 0; --i) {
    double z = B[(int64_t)i * ldb + g];
    for (int l = i + 1; l < k; ++l) z -= L[l * MAXK + i] * B[(int64_t)l * ldb + g];
    B[(int64_t)i * ldb + g] = z / L[i * MAXK + i];
  }
}

// dense L (k x MAXK) from the bidiagonal Cholesky factor (ldiag, lsub)
__global__ void k_rs_dense_bidiag(const double* __restrict__ ld, const double* __restrict__ ls,
                                  const Ctl* __restrict__ ctl, double* __restrict__ L) {
  const int k = ctl->k_eff;
  for (int e = threadIdx.x; e < MAXK * MAXK; e += blockDim.x) {
    const int i = e / MAXK, l = e % MAXK;
    double v = 0.0;
    if (i < k && l < k) v = (i == l) ? ld[i] : (i == l + 1 ? ls[l] : 0.0);
    L[e] = v;
  }
}

// nrm[2 g] = ||C_g - KX_g||, nrm[2 g + 1] = ||C_g||; Rr_g = C_g - KX_g; one block per g
template <typename T>
__global__ __launch_bounds__(256) void k_rs_resid(const T* __restrict__ C, const T* __restrict__ KX,
                                                  T* __restrict__ Rr, int64_t ld, int64_t n,
                                                  double* __restrict__ nrm) {
  __shared__ double scr[16];
  const int g = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t r = threadIdx.x; r < ld; r += 256) {
    const int64_t i = (int64_t)g * ld + r;
    const double c = r < n ? (double)C[i] : 0.0;
    const double d = r < n ? c - (double)KX[i] : 0.0;
    Rr[i] = (T)d;
    a += d * d;
    b += c * c;
  }
  a = block_sum(a, scr);
  __syncthreads();
  b = block_sum(b, scr);
  if (threadIdx.x == 0) {
    nrm[2 * g] = sqrt(a);
    nrm[2 * g + 1] = sqrt(b);
  }
}

// v -= Q[:, :k] c (one Gram-Schmidt pass; c from k_rs_dots), rows < n
template <typename T>
__global__ void k_rs_sub(T* __restrict__ v, const T* __restrict__ Q, int64_t ldq, int k,
                         const double* __restrict__ c, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double a = (double)v[r];
  for (int i = 0; i < k; ++i) a -= (double)Q[(int64_t)i * ldq + r] * c[i];
  v[r] = (T)a;
}

// q = v / ||v|| into column j of Q (padding rows zero); one block
template <typename T>
__global__ __launch_bounds__(256) void k_rs_start(const T* __restrict__ v, int64_t n, int64_t ldq,
                                                  T* __restrict__ qj) {
  __shared__ double scr[16];
  double a = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) a += (double)v[r] * (double)v[r];
  a = block_sum(a, scr);
  const double inv = a > 0.0 ? 1.0 / sqrt(a) : 0.0;
  for (int64_t r = threadIdx.x; r < ldq; r += 256) qj[r] = r < n ? (T)((double)v[r] * inv) : T(0);
}

// H[i][j] = G_i . R_j + sigma^2 q_i . q_j for i <= j < k (mirrored); one block per pair
template <typename T>
__global__ __launch_bounds__(256) void k_rs_h(const T* __restrict__ G, int64_t ldg,
                                              const T* __restrict__ R, int64_t m,
                                              const T* __restrict__ Q, int64_t ldq, int64_t n,
                                              double sigma2, const Ctl* __restrict__ ctl,
                                              double* __restrict__ H) {
  __shared__ double scr[16];
  const int i = blockIdx.x, j = blockIdx.y;
  const int k = ctl->k_eff;
  if (i > j || j >= k) return;
  double a = 0.0, b = 0.0;
  for (int64_t u = threadIdx.x; u < m; u += 256)
    a += (double)G[(int64_t)i * ldg + u] * (double)R[(int64_t)j * m + u];
  for (int64_t r = threadIdx.x; r < n; r += 256)
    b += (double)Q[(int64_t)i * ldq + r] * (double)Q[(int64_t)j * ldq + r];
  a = block_sum(a, scr);
  __syncthreads();
  b = block_sum(b, scr);
  if (threadIdx.x == 0) {
    const double h = a + sigma2 * b;
    H[i * MAXK + j] = h;
    H[j * MAXK + i] = h;
  }
}

// Dense Cholesky H = L L^T (k = ctl->k_eff <= MAXK) in double in LDS, column
// by column; a pivot <= rel_tol max|H_ii| truncates k_eff there (SF_NOTPD).
// Also Linv = L^{-1}.  L and Linv: k x MAXK row-major (zero above the diagonal).
__global__ __launch_bounds__(MAXK) void k_rs_chol(const double* __restrict__ H, Ctl* ctl,
                                                  double rel_tol, double* __restrict__ L,
                                                  double* __restrict__ Linv) {
  __shared__ double A[MAXK][MAXK + 1];
  __shared__ int s_keep;
  const int k = ctl->k_eff, t = threadIdx.x;
  for (int e = t; e < MAXK * MAXK; e += MAXK) {
    const int i = e / MAXK, l = e % MAXK;
    A[i][l] = (i < k && l < k) ? H[i * MAXK + l] : 0.0;
  }
  if (t == 0) s_keep = k;
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < k; ++i) dmax = fmax(dmax, fabs(A[i][i]));
  for (int c = 0; c < k; ++c) {
    if (c >= s_keep) break;
    if (t == 0) {
      double d = A[c][c];
      for (int l = 0; l < c; ++l) d -= A[c][l] * A[c][l];
      if (!(d > rel_tol * dmax) || !isfinite(d)) {
        s_keep = c;
      } else {
        A[c][c] = sqrt(d);
      }
    }
    __syncthreads();
    if (c >= s_keep) break;
    if (t > c && t < k) {
      double v = A[t][c];
      for (int l = 0; l < c; ++l) v -= A[t][l] * A[c][l];
      A[t][c] = v / A[c][c];
    }
    __syncthreads();
  }
  const int kk = s_keep;
  // write L; Linv column t by forward substitution of L x = e_t
  for (int e = t; e < MAXK * MAXK; e += MAXK) {
    const int i = e / MAXK, l = e % MAXK;
    L[e] = (i < kk && l <= i) ? A[i][l] : 0.0;
  }
  for (int i = 0; i < MAXK; ++i) Linv[i * MAXK + t] = 0.0;
  if (t < kk) {
    for (int i = t; i < kk; ++i) {
      double z = (i == t) ? 1.0 : 0.0;
      for (int l = t; l < i; ++l) z -= A[i][l] * Linv[l * MAXK + t];
      Linv[i * MAXK + t] = z / A[i][i];
    }
  }
  if (t == 0 && kk < k) {
    ctl->k_eff = kk;
    ctl->status |= SF_NOTPD;
  }
}

// Rt[u, i] = sum_{l <= i} Linv[i][l] R[l][u] for i < k_eff (0 beyond), in the
// cache precision or as bf16 hi + bf16 lo; thread per (u, i)
template <typename T>
__global__ void k_rs_rtilde(const T* __restrict__ R, int64_t m, const double* __restrict__ Linv,
                            const Ctl* __restrict__ ctl, int kpad, int split, void* rt,
                            uint16_t* __restrict__ rt_lo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * kpad) return;
  const int64_t u = idx / kpad;
  const int i = (int)(idx - u * kpad);
  const int k = ctl->k_eff;
  double z = 0.0;
  if (i < k)
    for (int l = 0; l <= i; ++l) z += Linv[i * MAXK + l] * (double)R[(int64_t)l * m + u];
  if (split) {
    const float f = (float)z;
    const uint16_t hi = f32_to_bf16_rne(f);
    ((uint16_t*)rt)[idx] = hi;
    rt_lo[idx] = f32_to_bf16_rne(f - bf16_to_f32(hi));
  } else {
    ((T*)rt)[idx] = (T)z;
  }
}

__global__ void k_rs_set(int* __restrict__ p, int v) { *p = v; }
__global__ void k_rs_unstop(Ctl* ctl) { ctl->stop = 0; }

// ============================================================================
// Batched build: Lanczos + Rt + mean cache for G GPs in lock step.
// ============================================================================
namespace {

// Device buffers of one GP's main run (cache precision T) and mean solve.
template <typename T>
struct GpBufs {
  T *Q = nullptr, *R = nullptr, *v = nullptr, *r = nullptr, *gv = nullptr, *gm = nullptr,
    *tsc = nullptr, *G = nullptr, *Gh = nullptr;
  double* gpart = nullptr;
  int64_t ldg = 0;     // 0: no grid-space first pass
  int64_t ldgh = 0;    // column stride of Gh (W^T Q for B without the grid-space pass)
  double *partial = nullptr, *coef = nullptr, *c2 = nullptr, *amax = nullptr, *ldiag = nullptr,
         *lsub = nullptr;
  // mean solve (double)
  double *x64 = nullptr, *y64 = nullptr, *xs = nullptr, *cr = nullptr, *cz = nullptr,
         *cp = nullptr, *cap = nullptr, *cgv = nullptr, *cgm = nullptr, *ctsc = nullptr,
         *pg = nullptr, *tinv = nullptr, *cm = nullptr, *cpart = nullptr, *ccoef = nullptr,
         *cdvec = nullptr;
  int nbg = 0;
  int64_t rpbg = 0;
  void* cellp = nullptr;   // scatter scratch for d >= 3 (sized for double)
  char* mem = nullptr;
};

template <typename T>
love_status alloc_gp(love_cache* c, GpBufs<T>& b, bool mean, bool plain, hipStream_t s) {
  const int64_t n = c->n, m = c->m, ldq = c->ldq, k = c->k, kpad = c->kpad;
  const int64_t nb = ldq / WAVE;   // row blocks at one row per lane (the most)
  const int64_t ts = toeplitz_scratch_elems(c);
  b.nbg = (int)std::min<int64_t>(256, std::max<int64_t>(1, cdiv(n, 128)));
  b.rpbg = cdiv(n, (int64_t)b.nbg);
  // grid-space first pass when the grid is no larger than the data
  b.ldg = m <= n ? cdiv(m, RB) * RB : 0;
  b.ldgh = ((c->B || c->restart_max > 0) && !b.ldg) ? cdiv(m, RB) * RB : 0;
  size_t tb = sizeof(T) * ((size_t)ldq * k + (size_t)k * m + 2 * (size_t)ldq + 2 * (size_t)m +
                           (size_t)ts + (size_t)b.ldg * k + (size_t)b.ldgh * k);
  tb = (tb + 255) & ~size_t(255);
  size_t db = sizeof(double) * ((size_t)nb * LDP + 6 * LDP +
                                (b.ldg ? (size_t)gpass_blocks(m) * LDP : 0));
  if (mean) {
    const bool own = sizeof(T) != 8;
    db += sizeof(double) * ((own ? (size_t)n * (c->d + 1) : 0) + 5 * (size_t)ldq +
                            2 * (size_t)m + (size_t)ts + (size_t)nb * LDP + 2 * LDP);
    if (!plain) db += sizeof(double) * ((size_t)b.nbg + 2) * kpad * kpad;
  }
  const size_t cb = (scatter_scratch_bytes(c, sizeof(double)) + 255) & ~size_t(255);
  b.mem = (char*)ws_alloc(tb + db + cb, s);
  if (!b.mem) return LOVE_ENOMEM;
  if (cb) b.cellp = b.mem + tb + db;
  T* t = (T*)b.mem;
  b.Q = t;   // Q and G first: their columns start on 16-byte boundaries
  if (b.ldg) {
    b.G = b.Q + (size_t)ldq * k;
    LOVE_HIP_TRY(hipMemsetAsync(b.G, 0, sizeof(T) * (size_t)b.ldg * k, s));
  }
  b.R = b.Q + (size_t)ldq * k + (size_t)b.ldg * k;
  b.v = b.R + (size_t)k * m;
  b.r = b.v + ldq;
  b.gv = b.r + ldq;
  b.gm = b.gv + m;
  b.tsc = b.gm + m;
  if (b.ldgh) b.Gh = b.tsc + ts;
  double* q = (double*)(b.mem + tb);
  b.partial = q;
  b.coef = b.partial + (size_t)nb * LDP;
  b.c2 = b.coef + LDP;
  b.amax = b.c2 + LDP;
  b.ldiag = b.amax + LDP;
  b.lsub = b.ldiag + LDP;
  q = b.lsub + LDP + LDP;
  if (b.ldg) {
    b.gpart = q;
    q += (size_t)gpass_blocks(m) * LDP;
  }
  if (mean) {
    if (sizeof(T) != 8) {
      b.x64 = q;
      b.y64 = b.x64 + (size_t)n * c->d;
      q = b.y64 + n;
    } else {
      b.x64 = (double*)c->x;
      b.y64 = (double*)c->y;
    }
    b.xs = q;
    b.cr = b.xs + ldq;
    b.cz = b.cr + ldq;
    b.cp = b.cz + ldq;
    b.cap = b.cp + ldq;
    b.cgv = b.cap + ldq;
    b.cgm = b.cgv + m;
    b.ctsc = b.cgm + m;
    b.cpart = b.ctsc + ts;
    b.ccoef = b.cpart + (size_t)nb * LDP;
    b.cdvec = b.ccoef + LDP;
    q = b.cdvec + LDP;
    if (!plain) {
      b.pg = q;
      b.tinv = b.pg + (size_t)b.nbg * kpad * kpad;
      b.cm = b.tinv + (size_t)kpad * kpad;
    }
  }
  return LOVE_OK;
}

}  // namespace

template <typename T, int D>
static love_status batch_impl(const std::vector<love_cache*>& cs, hipStream_t s,
                              hipStream_t s_side) {
  const int G = (int)cs.size();
  std::vector<GpBufs<T>> bufs(G);
  const bool mean = !(cs[0]->cfg.flags & LOVE_FLAG_NO_MEAN);
  std::vector<bool> plain(G);
  for (int g = 0; g < G; ++g) {
    plain[g] = (cs[g]->cfg.flags & LOVE_FLAG_PLAIN_CG) != 0;
    love_status st = alloc_gp<T>(cs[g], bufs[g], mean, plain[g], s);
    if (st != LOVE_OK) {
      for (auto& b : bufs)
        ws_free(b.mem, s);
      return st;
    }
  }
  // --- jobs --------------------------------------------------------------------
  std::vector<LzJob<T>> lz(G);
  std::vector<ScatterJob<T>> sc(G);
  std::vector<GatherJob<T>> ga(G);
  std::vector<FillJob<T>> fi(G);
  std::vector<RtJob<T>> rj(G), bj(G);
  std::vector<ScatterJob<T>> sch(G);
  std::vector<int64_t> b_hy(G, 0), b_hsc(G, 0);   // hyper: B rows, scatter node blocks
  std::vector<SumJob> s_coef(G), s_c2(G);
  std::vector<const T*> t_in_probe(G), t_in_step(G);
  std::vector<T*> t_out_probe(G), t_out_step(G), t_scr(G);
  std::vector<int64_t> js0(G, 0), js_m(G);
  std::vector<const Ctl*> ctls(G);
  std::vector<int64_t> b_rows(G), b_nodes(G), b_m(G), b_one(G, 1), b_grid(G);
  std::vector<int> nv1(G, 1);
  std::vector<int> nv2(G, 2);   // columns of the coef / c2 sums at j = 0
  std::vector<int> nvg(G, 1);   // the large-grid first-pass sums
  std::vector<SumJob> s_gco(G);
  bool any_gcs = false;
  std::vector<int64_t> b_gd(G), b_cd(G), js_in(G);
  int kmax = 0;
  for (int g = 0; g < G; ++g) {
    love_cache* c = cs[g];
    GpBufs<T>& b = bufs[g];
    // rows per lane chosen per GP (as for its own single build)
    const int rpl = rows_per_lane(c->ldq);
    const int64_t nb = c->ldq / (WAVE * rpl);
    LzJob<T> J{};
    J.rpl = rpl;
    J.g = make_grid<T>(c);
    J.x = (const T*)c->x;
    J.cell_start = c->cell_start;
    J.sigma2 = (T)c->cfg.noise;
    J.m = c->m;
    J.R = b.R;
    J.n = c->n;
    J.ldq = c->ldq;
    J.Q = b.Q;
    J.v = b.v;
    J.r = b.r;
    J.gv = b.gv;
    J.gm = b.gm;
    J.partial = b.partial;
    J.coef = b.coef;
    J.c2 = b.c2;
    J.amax = b.amax;
    J.alpha = c->alpha;
    J.beta = c->beta;
    J.ldiag = b.ldiag;
    J.lsub = b.lsub;
    J.ctl = c->ctl;
    J.tol = c->tol_lanczos;
    J.klast = c->k1 - 1;
    J.nb = (int)nb;
    J.gpath = b.ldg ? 1 : 0;
    J.G = b.G;
    J.ldg = b.ldg;
    J.gpart = b.gpart;
    J.nbc = b.ldg ? gpass_blocks(c->m) : 0;
    J.gcs = J.nbc > GPASS_NBC_SUM ? 1 : 0;
    lz[g] = J;
    ScatterJob<T> S{};
    S.g = J.g;
    S.x = J.x;
    S.cell_start = c->cell_start;
    S.v = b.Q;
    S.v_js = c->ldq;
    S.out = J.gpath ? b.G : b.gv;
    S.out_js = J.gpath ? b.ldg : 0;
    S.ctl = c->ctl;
    S.cellp = (T*)b.cellp;
    sc[g] = S;
    GatherJob<T> Ga{};
    Ga.g = J.g;
    Ga.x = J.x;
    Ga.n = c->n;
    Ga.kg = b.gm;
    Ga.out = b.v;
    ga[g] = Ga;
    fi[g] = FillJob<T>{b.gv, c->m, (T)(1.0 / (double)c->m)};
    RtJob<T> Rj{};
    Rj.R = b.R;
    Rj.ldiag = b.ldiag;
    Rj.lsub = b.lsub;
    Rj.rt = c->rt;
    Rj.rt_lo = (uint16_t*)c->rt_lo;
    Rj.m = c->m;
    Rj.kpad = c->kpad;
    Rj.split = c->cfg.precision == LOVE_P_FP32_BF16SPLIT;
    Rj.ctl = c->ctl;
    rj[g] = Rj;
    if (b.ldgh) {
      // G = W^T Q after the run, column by column, where the grid-space first
      // pass does not keep it (the factor B and the restart's H need it)
      ScatterJob<T> Sh = S;
      Sh.out = b.Gh;
      Sh.out_js = b.ldgh;
      sch[g] = Sh;
    }
    if (c->B) {
      // B = (L^{-1} G^T)^T from G = W^T Q
      RtJob<T> Bj = Rj;
      Bj.R = b.ldg ? b.G : b.Gh;
      Bj.ld = b.ldg ? b.ldg : b.ldgh;
      Bj.rt = c->B;
      Bj.rt_lo = nullptr;
      Bj.split = 0;
      bj[g] = Bj;
      b_hy[g] = cdiv(c->m, RT_ROWS);
      if (!b.ldg) b_hsc[g] = cdiv(c->m, 4);   // as the step's scatter table
    }
    s_coef[g] = SumJob{b.partial, b.coef, c->ctl, (int)nb, 1};
    nv1[g] = J.gpath ? -(1 << 20) : 1;   // no first-pass sums on the grid-space path
    s_gco[g] = SumJob{b.gpart, b.c2, c->ctl, J.nbc, 1};
    nvg[g] = J.gcs ? 1 : -(1 << 20);
    any_gcs = any_gcs || J.gcs;
    if (J.gpath && lz_psum(nb)) {
      lz[g].psum = 1;
      lz[g].partial2 = b.partial;   // udots reads only the cdots rows here
      nv2[g] = -(1 << 20);
    }
    b_gd[g] = J.gpath ? 0 : nb;
    b_cd[g] = J.nbc;
    js_in[g] = J.gpath ? b.ldg : 0;
    s_c2[g] = SumJob{b.partial, b.c2, c->ctl, (int)nb, 2};
    t_in_probe[g] = b.gv;
    t_out_probe[g] = b.gm;
    t_in_step[g] = J.gpath ? b.G : b.gv;
    t_out_step[g] = b.R;
    js_m[g] = c->m;
    t_scr[g] = b.tsc;
    ctls[g] = c->ctl;
    b_rows[g] = nb;
    b_nodes[g] = cdiv(c->m, 4);
    b_m[g] = cdiv(c->m, 256);
    b_grid[g] = cdiv(c->n, 256);
    kmax = std::max(kmax, c->k1);
  }
  JobArena A;
  SpectralMean sm;
  // Every return releases the build's workspace on s: first the side streams
  // are joined into s (the samplers' and the mean solve's kernels read these
  // buffers), then the job arrays and the GP buffers are freed.
  struct Cleanup {
    hipStream_t s;
    JobArena* A;
    std::vector<GpBufs<T>>* bufs;
    SpectralMean* sm;
    hipStream_t side = nullptr;       // sampler stream, while its work is not joined
    hipEvent_t side_join = nullptr;
    hipStream_t ms = nullptr;         // mean-solve stream, while the solve is live
    bool mean_live = false;
    std::vector<hipEvent_t> events;
    ~Cleanup() {
      if (side) {
        if (!side_join || hipEventRecord(side_join, side) != hipSuccess ||
            hipStreamWaitEvent(s, side_join, 0) != hipSuccess)
          (void)hipStreamSynchronize(side);
      }
      if (mean_live) {
        (void)hipStreamSynchronize(ms);
        sm->release(s);
      }
      A->release(s);
      for (auto& b : *bufs) ws_free(b.mem, s);
      for (hipEvent_t e : events)
        if (e) (void)hipEventDestroy(e);
    }
  } clean{s, &A, &bufs, &sm};
  const size_t o_lz = A.add(lz), o_sc = A.add(sc), o_ga = A.add(ga), o_fi = A.add(fi),
               o_rj = A.add(rj), o_coef = A.add(s_coef), o_c2 = A.add(s_c2),
               o_gco = A.add(s_gco),
               o_bj = A.add(bj), o_sch = A.add(sch);
  ToepRun<T> t_probe, t_step;
  toep_prepare<T>(A, t_probe, cs, t_in_probe, js0, t_out_probe, js0, t_scr,
                  std::vector<const Ctl*>(G, nullptr));
  toep_prepare<T>(A, t_step, cs, t_in_step, js_in, t_out_step, js_m, t_scr, ctls);
  // mean solve jobs
  std::vector<CgJob<T>> cg(G);
  std::vector<ScatterJob<double>> csc(G), cfin(G);
  std::vector<ConvJob> cvx(G), cvy(G);
  std::vector<int64_t> b_cvx(G, 0), b_cvy(G, 0), b_gram(G), b_cmat(G);
  std::vector<int> nvq(G);
  ToepRun<double> t_cg;
  if (mean) {
    std::vector<const double*> ci(G);
    std::vector<double*> co(G), cscr(G);
    for (int g = 0; g < G; ++g) {
      love_cache* c = cs[g];
      GpBufs<T>& b = bufs[g];
      CgJob<T> C{};
      C.g = make_grid<double>(c);
      C.x = b.x64;
      C.y = b.y64;
      C.n = c->n;
      C.m = c->m;
      C.ldq = c->ldq;
      C.xs = b.xs;
      C.r = b.cr;
      C.z = b.cz;
      C.p = b.cp;
      C.ap = b.cap;
      C.gv = b.cgv;
      C.gm = b.cgm;
      C.Q = b.Q;
      C.kq = plain[g] ? 0 : c->k1;
      C.kpad = c->kpad;
      C.ldiag = b.ldiag;
      C.lsub = b.lsub;
      C.pg = b.pg;
      C.tinv = b.tinv;
      C.cm = b.cm;
      C.nbg = b.nbg;
      C.rpbg = b.rpbg;
      C.partial = b.cpart;
      C.coef = b.ccoef;
      C.dvec = b.cdvec;
      C.sigma2 = c->cfg.noise;
      C.rscale = plain[g] ? 1.0 : 1.0 / c->cfg.noise;
      const double cgtol = c->cfg.cg_tol > 0 ? c->cfg.cg_tol : (c->fp64 ? 1e-12 : 1e-6);
      C.tol2 = cgtol * cgtol;
      C.maxit = c->cfg.cg_maxit > 0 ? c->cfg.cg_maxit : 1000;
      C.rpl = lz[g].rpl;
      C.nb = lz[g].nb;
      C.ctl = c->ctl;
      C.ortho = plain[g] ? nullptr : c->ortho;
      C.a = c->a;
      C.a_fp64 = c->fp64 ? 1 : 0;
      cg[g] = C;
      ScatterJob<double> S{};
      S.g = C.g;
      S.x = b.x64;
      S.cell_start = c->cell_start;
      S.v = b.cz;
      S.v2 = b.cp;
      S.out = b.cgv;
      S.ctl = c->ctl;
      S.cellp = (double*)b.cellp;
      csc[g] = S;
      S.v = b.xs;
      S.v2 = nullptr;
      S.ctl = nullptr;
      cfin[g] = S;
      if (sizeof(T) != 8) {
        cvx[g] = ConvJob{(const float*)c->x, b.x64, c->n * c->d};
        cvy[g] = ConvJob{(const float*)c->y, b.y64, c->n};
        b_cvx[g] = cdiv(c->n * c->d, 256);
        b_cvy[g] = cdiv(c->n, 256);
      }
      b_gram[g] = plain[g] ? 0 : b.nbg;
      b_cmat[g] = plain[g] ? 0 : cdiv((int64_t)c->kpad * c->kpad, 256);
      nvq[g] = C.kq + 1;
      ci[g] = b.cgv;
      co[g] = b.cgm;
      cscr[g] = b.ctsc;
    }
    toep_prepare<double>(A, t_cg, cs, ci, js0, co, js0, cscr, ctls);
  }
  const size_t o_cg = A.add(cg), o_csc = A.add(csc), o_cfin = A.add(cfin), o_cvx = A.add(cvx),
               o_cvy = A.add(cvy);
  std::vector<SumJob> s_cg(G);
  for (int g = 0; g < G; ++g) s_cg[g] = SumJob{bufs[g].cpart, bufs[g].ccoef, cs[g]->ctl,
                                                lz[g].nb, nvq[g]};
  const size_t o_scg = A.add(s_cg);
  love_status st = A.upload(s);
  if (st != LOVE_OK) return st;
  const LzJob<T>* dlz = A.at<LzJob<T>>(o_lz);
  const Tab t_rows = make_tab(b_rows), t_nodes = make_tab(b_nodes), t_m = make_tab(b_m),
            t_one = make_tab(b_one), t_gd = make_tab(b_gd), t_cd = make_tab(b_cd);
  for (int g = 0; g < G; ++g) k_ctl_init<<<1, 1, 0, s>>>(cs[g]->ctl);
  // Grid-space mean solve (Kronecker grids): it needs only x, y and the grid,
  // so it starts here on its own stream and runs beside the Lanczos.
  bool spec = mean;
  for (auto* c : cs) spec = spec && spectral_mean_applies(c);
  hipStream_t s_mean = s;
  hipEvent_t ev_mfork = nullptr, ev_mjoin = nullptr;
  if (spec) {
    hipStream_t ms = mean_stream();
    if (ms && hipEventCreateWithFlags(&ev_mfork, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&ev_mjoin, hipEventDisableTiming) == hipSuccess &&
        hipEventRecord(ev_mfork, s) == hipSuccess && hipStreamWaitEvent(ms, ev_mfork, 0) == hipSuccess)
      s_mean = ms;
    clean.events.push_back(ev_mfork);
    clean.events.push_back(ev_mjoin);
    clean.ms = s_mean;
    clean.mean_live = true;
    const Tab t_cvx = make_tab(b_cvx), t_cvy = make_tab(b_cvy);
    if (tab_blocks(t_cvx)) {
      k_convert_b<<<tab_blocks(t_cvx), 256, 0, s_mean>>>(t_cvx, A.at<ConvJob>(o_cvx));
      k_convert_b<<<tab_blocks(t_cvy), 256, 0, s_mean>>>(t_cvy, A.at<ConvJob>(o_cvy));
    }
    std::vector<const double*> sx(G), sy(G);
    std::vector<double*> su(G);
    for (int g = 0; g < G; ++g) {
      sx[g] = bufs[g].x64;
      sy[g] = bufs[g].y64;
      su[g] = bufs[g].cz;
    }
    love_status ss = sm.start(cs, sx, sy, su, s_mean);
    if (ss != LOVE_OK) return ss;
  }
  const int two_st = scatter_kinds(cs);
  // --- probe b = (1/m) W K 1 ; q_0 = b / ||b|| -----------------------------------
  {
    ProfScope ps("probe", s);
    launch_fill<T>(t_m, A.at<FillJob<T>>(o_fi), s);
    toep_run<T>(A, t_probe, 0, 0, s);
    launch_gather<T>(make_tab(b_grid), A.at<GatherJob<T>>(o_ga), D, 0, s);
    k_lz_norm<T><<<tab_blocks(t_rows), RBLK, 0, s>>>(t_rows, dlz);
    k_lz_bnorm<T><<<tab_blocks(t_one), WAVE, 0, s>>>(t_one, dlz);
    k_lz_start<T><<<tab_blocks(t_rows), RBLK, 0, s>>>(t_rows, dlz);
  }
  // --- Lanczos steps -------------------------------------------------------------
  // A GP whose k steps are done drops out of the launch tables (its blocks
  // would only return at once); GPs stopped early by breakdown return through
  // their control block.
  Tab a_nodes = t_nodes, a_cd = t_cd, a_gd = t_gd, a_rows = t_rows;
  ToepRun<T> a_step = t_step;
  std::vector<int> a_nv1 = nv1, a_nv2 = nv2, a_nvg = nvg;
  for (int j = 0; j < kmax; ++j) {
    bool drop = false;
    for (int g = 0; g < G; ++g) drop = drop || cs[g]->k1 == j;
    if (drop) {
      auto keep = [&](const Tab& t) {
        std::vector<int64_t> b(G);
        for (int g = 0; g < G; ++g) b[g] = cs[g]->k1 > j ? t.off[g + 1] - t.off[g] : 0;
        return make_tab(b);
      };
      a_nodes = keep(t_nodes);
      a_cd = keep(t_cd);
      a_gd = keep(t_gd);
      a_rows = keep(t_rows);
      // Toeplitz tables hold t_step.jpg entries per GP
      auto keep_t = [&](const Tab& t) {
        std::vector<int64_t> b(t.G);
        for (int i = 0; i < t.G; ++i)
          b[i] = cs[i / t_step.jpg]->k1 > j ? t.off[i + 1] - t.off[i] : 0;
        return make_tab(b);
      };
      for (int e = 0; e < t_step.d; ++e) {
        a_step.ax[e].band = keep_t(t_step.ax[e].band);
        a_step.ax[e].reduce = keep_t(t_step.ax[e].reduce);
        a_step.ax[e].lines = keep_t(t_step.ax[e].lines);
        a_step.ax[e].fft = keep_t(t_step.ax[e].fft);
      }
      for (int g = 0; g < G; ++g)
        if (cs[g]->k1 <= j) a_nv1[g] = a_nv2[g] = a_nvg[g] = -(1 << 20);
    }
    launch_scatter<T>(a_nodes, A.at<ScatterJob<T>>(o_sc), D, j, 1, s, two_st);
    toep_run<T>(A, a_step, j, 1, s);
    if (tab_blocks(a_cd))
      tlaunch("lz_cdots", k_lz_cdots<T>, tab_blocks(a_cd), RBLK, 0, s, a_cd, dlz, j);
    if (any_gcs) launch_colsum(A.at<SumJob>(o_gco), a_nvg, j, 1, s);
    if (tab_blocks(a_gd)) {
      tlaunch("lz_gdots", k_lz_gdots<T, D>, tab_blocks(a_gd), RBLK, 0, s, a_gd, dlz, j);
      launch_colsum(A.at<SumJob>(o_coef), a_nv1, j, 1, s);
    }
    tlaunch("lz_udots", k_lz_udots<T, D>, tab_blocks(a_rows), RBLK, 0, s, a_rows, dlz, j);
    launch_colsum(A.at<SumJob>(o_c2), a_nv2, j, 1, s);
    tlaunch("lz_finalize", k_lz_finalize<T>, tab_blocks(a_rows), RBLK, 0, s, a_rows, dlz, j);
  }
  // --- T = L L^T ; Rt = (L^{-1} R)^T ---------------------------------------------
  k_tri_chol<T><<<tab_blocks(t_one), 64, 0, s>>>(t_one, dlz, 0.0);
  // --- restart with a new probe when the solve check fails (single GP) ----------
  bool dense_rt = false;
  double* rs_linv = nullptr;
  char* rs_mem = nullptr;
  JobArena A_rs, A_rs2;
  struct RsRelease {   // the restart's workspace goes back on every return path
    char*& mem;
    JobArena& a1;
    JobArena& a2;
    hipStream_t st;
    ~RsRelease() {
      ws_free(mem, st);
      a1.release(st);
      a2.release(st);
    }
  } rs_release{rs_mem, A_rs, A_rs2, s};
  if (G == 1 && cs[0]->restart_max > 0) {
    love_cache* c = cs[0];
    GpBufs<T>& b = bufs[0];
    const int Gc = c->restart_groups;
    const int64_t n = c->n, m = c->m, ldq = c->ldq;
    const size_t tcol = sizeof(T) * (size_t)ldq * Gc;
    const size_t dsz = sizeof(double) * (3 * (size_t)MAXK * MAXK + (size_t)MAXK * Gc + 2 * (size_t)Gc +
                                         MAXK);
    rs_mem = (char*)ws_alloc(4 * tcol + dsz, s);
    if (!rs_mem) return LOVE_ENOMEM;
    T* Cm = (T*)rs_mem;
    T* KX = (T*)(rs_mem + tcol);
    T* Rr = (T*)(rs_mem + 2 * tcol);
    T* X = (T*)(rs_mem + 3 * tcol);
    double* Ld = (double*)(rs_mem + 4 * tcol);
    rs_linv = Ld + MAXK * MAXK;
    double* Hd = rs_linv + MAXK * MAXK;
    double* Dm = Hd + MAXK * MAXK;
    double* nrm = Dm + (size_t)MAXK * Gc;
    double* cvec = nrm + 2 * Gc;
    // jobs: the groups' W K 1_g / |g| and Khat x_g columns, the x_g scatters
    std::vector<GatherJob<T>> gj(2 * Gc);
    std::vector<ScatterJob<T>> sj(Gc);
    for (int g = 0; g < Gc; ++g) {
      GatherJob<T> a = ga[0];
      a.kg = b.gm;
      a.vsig = nullptr;
      a.sigma2 = T(0);
      a.out = Cm + (size_t)g * ldq;
      a.ctl = nullptr;
      gj[g] = a;
      a.vsig = X + (size_t)g * ldq;
      a.sigma2 = (T)c->cfg.noise;
      a.out = KX + (size_t)g * ldq;
      gj[Gc + g] = a;
      ScatterJob<T> sx = sc[0];
      sx.v = X + (size_t)g * ldq;
      sx.v_js = 0;
      sx.out = b.gv;
      sx.out_js = 0;
      sx.ctl = nullptr;
      sj[g] = sx;
    }
    const size_t o_gj = A_rs.add(gj), o_sj = A_rs.add(sj);
    love_status st = A_rs.upload(s);
    if (st != LOVE_OK) return st;
    const Tab tab_m = tab1(cdiv(m, 4)), tab_n = tab1(cdiv(n, 256));
    k_rs_dense_bidiag<<<1, 256, 0, s>>>(b.ldiag, b.lsub, c->ctl, Ld);
    // the checked columns c_g = W K 1_g / |g| (runs of the m grid nodes, bounds
    // rounded half to even)
    const double step = (double)m / Gc;
    for (int g = 0; g < Gc; ++g) {
      const int64_t lo = (int64_t)std::nearbyint(g * step);
      const int64_t hi = g + 1 == Gc ? m : (int64_t)std::nearbyint((g + 1) * step);
      k_rs_group<T><<<(unsigned)cdiv(m, 256), 256, 0, s>>>(b.gv, m, lo, hi);
      toep_run<T>(A, t_probe, 0, 0, s);
      launch_gather<T>(tab_n, A_rs.at<GatherJob<T>>(o_gj) + g, D, 0, s);
    }
    const T* Gsrc = b.ldg ? b.G : b.Gh;
    const int64_t ldgs = b.ldg ? b.ldg : b.ldgh;
    const CgJob<T>* dcg0 = A.at<CgJob<T>>(o_cg);
    for (int round = 0;; ++round) {
      Ctl hc;
      LOVE_HIP_TRY(hipMemcpyAsync(&hc, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
      LOVE_HIP_TRY(hipStreamSynchronize(s));
      const int kq = hc.k_eff;
      if (kq < 1) break;
      // x_g = Q H^{-1} Q^T c_g, then the residuals c_g - Khat x_g
      k_rs_dots<T><<<dim3((unsigned)kq, (unsigned)Gc), 256, 0, s>>>(b.Q, ldq, Cm, ldq, n, Gc, Dm, Gc);
      k_rs_solve<<<1, 64 * (int)cdiv(Gc, 64), 0, s>>>(Ld, c->ctl, Dm, Gc, Gc);
      k_rs_combine<T><<<(unsigned)cdiv(ldq, 256), 256, 0, s>>>(b.Q, ldq, kq, Dm, Gc, Gc, X, ldq, n);
      for (int g = 0; g < Gc; ++g) {
        launch_scatter<T>(tab_m, A_rs.at<ScatterJob<T>>(o_sj) + g, D, 0, 0, s, two_st);
        toep_run<T>(A, t_probe, 0, 0, s);
        launch_gather<T>(tab_n, A_rs.at<GatherJob<T>>(o_gj) + Gc + g, D, 0, s);
      }
      k_rs_resid<T><<<(unsigned)Gc, 256, 0, s>>>(Cm, KX, Rr, ldq, n, nrm);
      std::vector<double> hn(2 * Gc);
      LOVE_HIP_TRY(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * 2 * Gc, hipMemcpyDeviceToHost, s));
      LOVE_HIP_TRY(hipStreamSynchronize(s));
      int worst = 0;
      double wrel = -1.0;
      for (int g = 0; g < Gc; ++g) {
        const double rel = hn[2 * g + 1] > 0.0 ? hn[2 * g] / hn[2 * g + 1] : 0.0;
        if (rel > wrel) {
          wrel = rel;
          worst = g;
        }
      }
      c->solve_residual = wrel;
      if (!(wrel > c->cfg.restart_tol) || round == c->restart_max || kq >= n ||
          kq + c->restart_k > c->k)
        break;
      // new probe: the worst residual, orthogonalised twice against Q
      T* vr = Rr + (size_t)worst * ldq;
      for (int pass = 0; pass < 2; ++pass) {
        k_rs_dots<T><<<dim3((unsigned)kq, 1), 256, 0, s>>>(b.Q, ldq, vr, ldq, n, 1, cvec, 1);
        k_rs_sub<T><<<(unsigned)cdiv(n, 256), 256, 0, s>>>(vr, b.Q, ldq, kq, cvec, n);
      }
      k_rs_start<T><<<1, 256, 0, s>>>(vr, n, ldq, b.Q + (size_t)kq * ldq);
      // the preconditioner of the mean solve keeps the first run's vectors
      if (round == 0 && mean && !plain[0])
        k_rs_set<<<1, 1, 0, s>>>(&(const_cast<CgJob<T>*>(dcg0)->kq), kq);
      k_rs_unstop<<<1, 1, 0, s>>>(c->ctl);
      LzJob<T> J2 = lz[0];
      J2.klast = kq + c->restart_k - 1;
      A_rs2.release(s);
      A_rs2 = JobArena();
      const size_t o_l2 = A_rs2.add(std::vector<LzJob<T>>{J2});
      st = A_rs2.upload(s);
      if (st != LOVE_OK) return st;
      const LzJob<T>* dlz2 = A_rs2.at<LzJob<T>>(o_l2);
      for (int j = kq; j < kq + c->restart_k; ++j) {
        launch_scatter<T>(t_nodes, A.at<ScatterJob<T>>(o_sc), D, j, 1, s, two_st);
        toep_run<T>(A, t_step, j, 1, s);
        if (tab_blocks(t_cd))
          tlaunch("lz_cdots", k_lz_cdots<T>, tab_blocks(t_cd), RBLK, 0, s, t_cd, dlz2, j);
        if (any_gcs) launch_colsum(A.at<SumJob>(o_gco), nvg, j, 1, s);
        if (tab_blocks(t_gd)) {
          tlaunch("lz_gdots", k_lz_gdots<T, D>, tab_blocks(t_gd), RBLK, 0, s, t_gd, dlz2, j);
          launch_colsum(A.at<SumJob>(o_coef), nv1, j, 1, s);
        }
        tlaunch("lz_udots", k_lz_udots<T, D>, tab_blocks(t_rows), RBLK, 0, s, t_rows, dlz2, j);
        launch_colsum(A.at<SumJob>(o_c2), nv2, j, 1, s);
        tlaunch("lz_finalize", k_lz_finalize<T>, tab_blocks(t_rows), RBLK, 0, s, t_rows, dlz2, j);
      }
      // H = Q^T Khat Q over every vector so far, its dense Cholesky factor
      if (!b.ldg)
        for (int j = 0; j < kq + c->restart_k; ++j)
          launch_scatter<T>(tab_m, A.at<ScatterJob<T>>(o_sch), D, j, 0, s, two_st);
      k_rs_h<T><<<dim3((unsigned)c->k, (unsigned)c->k), 256, 0, s>>>(
          Gsrc, ldgs, b.R, m, b.Q, ldq, n, c->cfg.noise, c->ctl, Hd);
      k_rs_chol<<<1, MAXK, 0, s>>>(Hd, c->ctl, 0.0, Ld, rs_linv);
      dense_rt = true;
      c->restarts = round + 1;
    }
  }
  if (dense_rt) {
    love_cache* c = cs[0];
    tlaunch("rtilde", k_rs_rtilde<T>, (unsigned)cdiv(c->m * c->kpad, 256), 256, 0, s,
            (const T*)bufs[0].R, c->m, (const double*)rs_linv, (const Ctl*)c->ctl, c->kpad,
            c->cfg.precision == LOVE_P_FP32_BF16SPLIT ? 1 : 0, c->rt, (uint16_t*)c->rt_lo);
  } else {
    std::vector<int64_t> b_rt(G);
    for (int g = 0; g < G; ++g) b_rt[g] = cdiv(cs[g]->m, RT_ROWS);
    const Tab t_rt = make_tab(b_rt);
    tlaunch("rtilde", k_rtilde<T>, tab_blocks(t_rt), RT_ROWS, 0, s, t_rt, A.at<RtJob<T>>(o_rj));
  }
  // --- B = W^T Q L^{-T} for the hyper-parameter gradient (LOVE_FLAG_HYPER) ------
  {
    int kh = 0;
    for (int g = 0; g < G; ++g)
      if (b_hsc[g]) kh = std::max(kh, cs[g]->k);
    for (int j = 0; j < kh; ++j) {
      std::vector<int64_t> b(G);
      for (int g = 0; g < G; ++g) b[g] = j < cs[g]->k ? b_hsc[g] : 0;
      launch_scatter<T>(make_tab(b), A.at<ScatterJob<T>>(o_sch), D, j, 0, s, two_st);
    }
    const Tab t_hy = make_tab(b_hy);
    if (tab_blocks(t_hy))
      tlaunch("rtilde", k_rtilde<T>, tab_blocks(t_hy), RT_ROWS, 0, s, t_hy,
              A.at<RtJob<T>>(o_bj));
  }
  // The samplers (grid space, need Rt) and the mean solve (needs Q) are
  // independent chains of small kernels: the samplers run on a side stream
  // concurrently with the mean CG, and the caller's stream waits for them.
  bool any_s = false;
  for (auto* c : cs) any_s = any_s || c->ks > 0;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  const bool side = any_s && s_side != nullptr;
  if (any_s) {
    if (side) {
      LOVE_HIP_TRY(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
      clean.events.push_back(ev_fork);
      LOVE_HIP_TRY(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
      clean.events.push_back(ev_join);
      LOVE_HIP_TRY(hipEventRecord(ev_fork, s));
      LOVE_HIP_TRY(hipStreamWaitEvent(s_side, ev_fork, 0));
      clean.side = s_side;
      clean.side_join = ev_join;
    }
    for (auto* c : cs) {
      if (c->ks <= 0) continue;
      love_status ss = sampler_dispatch(c, side ? s_side : s);
      if (ss != LOVE_OK) return ss;
    }
    if (side) LOVE_HIP_TRY(hipEventRecord(ev_join, s_side));
  }
  // --- mean cache a = K W^T Khat^{-1} y --------------------------------------------
  if (mean) {
    ProfScope ps("mean_cg", s);
    const CgJob<T>* dcg = A.at<CgJob<T>>(o_cg);
    const Tab t_cvx = make_tab(b_cvx), t_cvy = make_tab(b_cvy), t_gram = make_tab(b_gram),
              t_cmat = make_tab(b_cmat);
    if (tab_blocks(t_cvx) && !spec) {
      k_convert_b<<<tab_blocks(t_cvx), 256, 0, s>>>(t_cvx, A.at<ConvJob>(o_cvx));
      k_convert_b<<<tab_blocks(t_cvy), 256, 0, s>>>(t_cvy, A.at<ConvJob>(o_cvy));
    }
    if (tab_blocks(t_gram)) {
      for (int g = 0; g < G; ++g)
        if (!plain[g]) LOVE_HIP_TRY(hipMemsetAsync(cs[g]->ortho, 0, sizeof(double), s));
      k_gram<T><<<tab_blocks(t_gram), 256, 0, s>>>(t_gram, dcg);
      k_tinv<T><<<tab_blocks(t_one), MAXK, 0, s>>>(t_one, dcg);
      k_pcg_matrix<T><<<tab_blocks(t_cmat), 256, 0, s>>>(t_cmat, dcg);
    }
    if (spec) {
      love_status ss = sm.finish();
      if (ss != LOVE_OK) return ss;
      if (s_mean != s) {
        LOVE_HIP_TRY(hipEventRecord(ev_mjoin, s_mean));
        LOVE_HIP_TRY(hipStreamWaitEvent(s, ev_mjoin, 0));
      }
      sm.merge(s);
      clean.mean_live = false;
      sm.release(s);
    }
    if (!spec) {
    const SumJob* dscg = A.at<SumJob>(o_scg);
    const std::vector<int> nv0(G, 0);
    k_pcg_init<T><<<tab_blocks(t_rows), RBLK, 0, s>>>(t_rows, dcg);
    launch_colsum(dscg, nvq, 0, 0, s);
    k_pcg_ep<T><<<tab_blocks(t_one), BLK, 0, s>>>(t_one, dcg, 1);
    k_pcg_apply<T><<<tab_blocks(t_rows), RBLK, 0, s>>>(t_rows, dcg);
    int* dflag = nullptr;
    dflag = (int*)ws_alloc(sizeof(int) * G, s);
    if (!dflag) return LOVE_ENOMEM;
    std::vector<int> hflag(G, 0);
    int maxit = 0;
    bool any_plain = false;
    for (int g = 0; g < G; ++g) {
      maxit = std::max(maxit, cg[g].maxit);
      any_plain = any_plain || plain[g];
    }
    // iterations between convergence checks: 4 (8 for plain CG) at first,
    // doubling after each check up to 16 (a long tail then costs few syncs)
    int chunk = any_plain ? 8 : 4;
    // launch tables of the GPs still iterating: at every check the converged
    // GPs drop out (their blocks would only return at once)
    Tab a_nodes = t_nodes, a_rows = t_rows, a_one = t_one;
    ToepRun<double> a_cg = t_cg;
    std::vector<int> a_nvq = nvq;
    int it = 0;
    while (it < maxit) {
      for (int q = 0; q < chunk && it < maxit; ++q, ++it) {
        launch_scatter<double>(a_nodes, A.at<ScatterJob<double>>(o_csc), D, 0, 2 | 4, s, two_st);
        toep_run<double>(A, a_cg, 0, 2, s);
        k_cg_ap<T, D><<<tab_blocks(a_rows), RBLK, 0, s>>>(a_rows, dcg);
        k_pcg_update<T><<<tab_blocks(a_rows), RBLK, 0, s>>>(a_rows, dcg);
        launch_colsum(dscg, a_nvq, 0, 2, s);
        k_pcg_ep<T><<<tab_blocks(a_one), BLK, 0, s>>>(a_one, dcg, 0);
        k_pcg_apply<T><<<tab_blocks(a_rows), RBLK, 0, s>>>(a_rows, dcg);
      }
      k_cg_flags<T><<<1, 64, 0, s>>>(G, dcg, dflag);
      LOVE_HIP_TRY(hipMemcpyAsync(hflag.data(), dflag, sizeof(int) * G, hipMemcpyDeviceToHost, s));
      LOVE_HIP_TRY(hipStreamSynchronize(s));
      int live = 0;
      for (int g = 0; g < G; ++g) live += hflag[g] ? 0 : 1;
      if (!live) break;
      chunk = std::min(16, 2 * chunk);
      auto keep = [&](const Tab& t) {
        std::vector<int64_t> b(G);
        for (int g = 0; g < G; ++g) b[g] = hflag[g] ? 0 : t.off[g + 1] - t.off[g];
        return make_tab(b);
      };
      a_nodes = keep(t_nodes);
      a_rows = keep(t_rows);
      a_one = keep(t_one);
      // Toeplitz tables hold t_cg.jpg entries per GP
      auto keep_t = [&](const Tab& t) {
        std::vector<int64_t> b(t.G);
        for (int i = 0; i < t.G; ++i) b[i] = hflag[i / t_cg.jpg] ? 0 : t.off[i + 1] - t.off[i];
        return make_tab(b);
      };
      for (int e = 0; e < t_cg.d; ++e) {
        a_cg.ax[e].band = keep_t(t_cg.ax[e].band);
        a_cg.ax[e].reduce = keep_t(t_cg.ax[e].reduce);
        a_cg.ax[e].lines = keep_t(t_cg.ax[e].lines);
        a_cg.ax[e].fft = keep_t(t_cg.ax[e].fft);
      }
      for (int g = 0; g < G; ++g) a_nvq[g] = hflag[g] ? 0 : nvq[g];
    }
    ws_free(dflag, s);
    launch_scatter<double>(t_nodes, A.at<ScatterJob<double>>(o_cfin), D, 0, 0, s, two_st);
    toep_run<double>(A, t_cg, 0, 0, s);
    k_cg_store_a<T><<<tab_blocks(t_m), 256, 0, s>>>(t_m, dcg);
    }
  }
  if (side) {
    LOVE_HIP_TRY(hipStreamWaitEvent(s, ev_join, 0));
    clean.side = nullptr;
  }
  LOVE_HIP_TRY(hipGetLastError());
  return LOVE_OK;   // the workspace is released by `clean`
}

template <typename T>
love_status build_batch_lanczos(const std::vector<love_cache*>& cs, hipStream_t s,
                                hipStream_t s_side) {
  switch (cs[0]->d) {
    case 1: return batch_impl<T, 1>(cs, s, s_side);
    case 2: return batch_impl<T, 2>(cs, s, s_side);
    case 3: return batch_impl<T, 3>(cs, s, s_side);
    case 4: return batch_impl<T, 4>(cs, s, s_side);
  }
  return LOVE_EINVAL;
}
template love_status build_batch_lanczos<float>(const std::vector<love_cache*>&, hipStream_t, hipStream_t);
template love_status build_batch_lanczos<double>(const std::vector<love_cache*>&, hipStream_t, hipStream_t);

}  // namespace love
