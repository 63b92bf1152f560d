// Banded direct Toeplitz product (one axis of K_UU) as block-level device
// code, shared by the operator's own kernels and the fused sampler launches.
#pragma once
#include "common.h"
#include "jobs.h"

namespace love {

// ----------------------------------------------------------------------------
// Direct Toeplitz product along a contiguous axis of length L (long lines):
//   out[o, i] = scale * sum_j c[|i - j|] in[o, j],   |i - j| <= bw.
// A GP's blocks are (output tile of TB_OUT = 64 * TB_R outputs, input
// segment, line).  A block stages its input segment and the matching strip of
// signed coefficients cd[delta] = c[|delta|] in LDS; its waves take equal
// slices of the segment.  Each lane owns TB_R consecutive outputs whose
// coefficients slide along a register window (one LDS load per input; the
// input itself is an LDS broadcast).  Wave sums are added in LDS in wave
// order; with several segments, k_toep_reduce adds the segment sums in
// segment order (deterministic throughout).  Coefficients beyond the band bw
// are below the working precision's rounding of the largest term (set at
// plan time).
// ----------------------------------------------------------------------------
constexpr int TB_WAVES = 8;
constexpr int TB_R = 3;                   // odd: lane stride TB_R keeps LDS reads near conflict-free
constexpr int TB_OUT = WAVE * TB_R;       // 192
constexpr int TB_SEG = 2048;              // max inputs per block (one LDS window)
constexpr int TB_NSEG_MAX = 16;

// one block (TB_WAVES waves) of the banded product: block lb of the GP's job J
template <typename T>
__device__ __forceinline__ void toep_band_block(const ToepJob<T>& J, int lb, int j) {
  __shared__ T gl[TB_SEG];
  __shared__ T cd[TB_SEG + TB_OUT];
  __shared__ T red[TB_WAVES][TB_OUT];
  const int L = J.L, bw = J.bw, seglen = J.seglen, nseg = J.nseg;
  const int tile = lb % J.ntiles;
  const int rest = lb / J.ntiles;
  const int seg = rest % nseg;
  const int64_t line = rest / nseg;
  const T* __restrict__ c = J.c;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int i0 = tile * TB_OUT;
  const T* g = J.in + (int64_t)j * J.in_js + line * L;
  const int jlo = max(0, i0 - bw);
  const int jhi = min(L - 1, i0 + TB_OUT - 1 + bw);
  const int jw = jlo + seg * seglen;
  const int nwin = max(0, min(seglen, jhi + 1 - jw));
  const int il = i0 + lane * TB_R;          // first output of this lane
  T acc[TB_R];
#pragma unroll
  for (int r = 0; r < TB_R; ++r) acc[r] = T(0);
  if (nwin > 0) {
    // cd[q] = c[|delta|] for delta = dmin + q, dmin = i0 - (jw + nwin - 1)
    const int dmin = i0 - (jw + nwin - 1);
    const int ncd = nwin + TB_OUT - 1;
#pragma unroll 4
    for (int q = threadIdx.x; q < nwin; q += TB_WAVES * WAVE) gl[q] = g[jw + q];
#pragma unroll 5
    for (int q = threadIdx.x; q < ncd; q += TB_WAVES * WAVE) {
      const int dl = dmin + q;
      const int ad = dl < 0 ? -dl : dl;
      cd[q] = (ad <= bw && ad < L) ? c[ad] : T(0);
    }
    __syncthreads();
    const int per = (nwin + TB_WAVES - 1) / TB_WAVES;
    const int qb = w * per, qe = min(nwin, qb + per);
    if (qb < qe) {
      // coefficient of output il + r and input jw + q: cd[il + r - jw - q - dmin]
      const int base = il - jw - dmin;
      T P[TB_R];
#pragma unroll
      for (int r = 0; r < TB_R; ++r) P[r] = cd[base + r - qb];
      int q = qb;
      for (; q + TB_R <= qe; q += TB_R) {
#pragma unroll
        for (int u = 0; u < TB_R; ++u) {
          const T gv = gl[q + u];
#pragma unroll
          for (int r = 0; r < TB_R; ++r) acc[r] += P[(r - u + TB_R) % TB_R] * gv;
          const int ni = base - (q + u) - 1;
          P[(TB_R - 1 - u) % TB_R] = ni >= 0 ? cd[ni] : T(0);
        }
      }
      for (; q < qe; ++q) {   // tail (fewer than TB_R inputs): direct indexing
        const T gv = gl[q];
#pragma unroll
        for (int r = 0; r < TB_R; ++r) acc[r] += cd[base + r - q] * gv;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < TB_R; ++r) red[w][lane * TB_R + r] = acc[r];
  __syncthreads();
  for (int o = threadIdx.x; o < TB_OUT; o += TB_WAVES * WAVE) {
    T s = T(0);
#pragma unroll
    for (int q = 0; q < TB_WAVES; ++q) s += red[q][o];
    const int i = i0 + o;
    if (i < L) {
      if (nseg == 1) J.out[(int64_t)j * J.out_js + line * L + i] = J.scale * s;
      else J.partial[(line * nseg + seg) * L + i] = s;
    }
  }
}

// out[line, i] = scale * sum_seg partial[line, seg, i] (segment order); one
// block of TB_RED threads
constexpr int TB_RED = 256;
template <typename T>
__device__ __forceinline__ void toep_reduce_block(const ToepJob<T>& J, int lb, int j) {
  const int L = J.L, nseg = J.nseg;
  const int64_t idx = (int64_t)lb * TB_RED + threadIdx.x;
  if (idx >= J.outer * L) return;
  const int64_t line = idx / L, i = idx % L;
  const T* lp = J.partial + line * nseg * (int64_t)L + i;
  T v[TB_NSEG_MAX];
#pragma unroll
  for (int q = 0; q < TB_NSEG_MAX; ++q) v[q] = q < nseg ? lp[(int64_t)q * L] : T(0);
  T acc = T(0);
#pragma unroll
  for (int q = 0; q < TB_NSEG_MAX; ++q) acc += v[q];
  J.out[(int64_t)j * J.out_js + idx] = J.scale * acc;
}

}  // namespace love
