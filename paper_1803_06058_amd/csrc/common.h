// Shared device/host definitions of the LOVE library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace love {

constexpr int WAVE = 64;
constexpr int MAXD = 4;
constexpr int MAXK = 128;

// Grid geometry passed to kernels by value.  The grid has m_i nodes per axis,
// padded by one cell on each side of the data box: h_i = (hi_i - lo_i) / (m_i - 3),
// node j at lo_i + (j - 1) h_i.  A point's stencil base along axis i is
// clamp(floor((x - lo_i) / h_i), 0, m_i - 4), so "cells" run over
// 0..m_i - 4 (cells_i = m_i - 3 of them).  Nodes and cells are flattened
// row-major (last axis fastest).
template <typename T>
struct GridT {
  int d;
  int m[MAXD];
  int cells[MAXD];
  int64_t nstride[MAXD];   // node strides
  int64_t cstride[MAXD];   // cell strides
  int64_t mtot, ctot;
  T lo[MAXD], hi[MAXD], invh[MAXD];
  // The training rows were sorted by stencil cell computed in float when
  // cell_f != 0.  Every kernel then takes the stencil base from that same
  // float computation (so W^T and W agree row by row) and only the fraction
  // s in precision T; s may then leave [0, 1] by a float rounding of
  // (x - lo) / h, where the cubic pieces extend smoothly (weights still sum
  // to 1).
  int cell_f;
  float lo_f[MAXD], invh_f[MAXD];
  // additive composition: add = 1, the grid is the axes' 1-D grids one after
  // another (axis e's nodes from aoff[e], its cells from acoff[e]); the rows
  // are in caller order and aperm lists each axis's rows by cell
  int add;
  int64_t aoff[MAXD], acoff[MAXD];
  const int32_t* aperm;
};

// Keys cubic convolution weights (a = -1/2) for a point at fraction s in [0,1]
// of its cell: nodes at distances 1+s, s, 1-s, 2-s.  Expanded polynomials:
//   psi(1+s) = -s (1-s)^2 / 2        psi(s)   = (3/2 s - 5/2) s^2 + 1
//   psi(1-s) = (3/2 u - 5/2) u^2 + 1  psi(2-s) = -s^2 u / 2,   u = 1 - s.
template <typename T>
__host__ __device__ inline void keys_weights(T s, T w[4]) {
  const T u = T(1) - s;
  w[0] = T(-0.5) * s * u * u;
  w[1] = (T(1.5) * s - T(2.5)) * s * s + T(1);
  w[2] = (T(1.5) * u - T(2.5)) * u * u + T(1);
  w[3] = T(-0.5) * s * s * u;
}

// d w / d s of the four weights above.
template <typename T>
__host__ __device__ inline void keys_dweights(T s, T dw[4]) {
  const T u = T(1) - s;
  dw[0] = T(-0.5) * u * (T(1) - T(3) * s);
  dw[1] = (T(4.5) * s - T(5)) * s;
  dw[2] = -(T(4.5) * u - T(5)) * u;
  dw[3] = T(-0.5) * s * (T(2) - T(3) * s);
}

// Stencil base and fraction along one axis.  Points outside [lo, hi] are
// clamped here; callers that must reject them test in_domain() first.
template <typename T>
__device__ inline int stencil_base(T x, T lo, T invh, int m, T& s) {
  T tau = (x - lo) * invh;
  T f = floor(tau);
  f = f < T(0) ? T(0) : f;
  f = f > T(m - 4) ? T(m - 4) : f;
  s = tau - f;
  return (int)f;
}

// Stencil base and fraction along axis e, consistent with the cell sort.
template <typename T>
__device__ inline int stencil_at(const GridT<T>& g, int e, T x, T& s) {
  if (g.cell_f) {
    float sf;
    const int j = stencil_base<float>((float)x, g.lo_f[e], g.invh_f[e], g.m[e], sf);
    s = (x - g.lo[e]) * g.invh[e] - (T)j;
    return j;
  }
  return stencil_base<T>(x, g.lo[e], g.invh[e], g.m[e], s);
}

template <typename T>
__device__ inline bool in_domain(T x, T lo, T hi) {
  return x >= lo && x <= hi;   // false for NaN
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

// ----------------------------------------------------------------------------
// Wave / block reductions
// ----------------------------------------------------------------------------
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

template <typename T>
__device__ inline T group_sum(T v, int width) {
  for (int off = width / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
  return v;
}

// Sum over the block (blockDim.x multiple of 64, <= 1024); result valid in all threads.
template <typename T>
__device__ inline T block_sum(T v, T* scratch /* >= 16 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  T s = T(0);
  for (int i = 0; i < nw; ++i) s += scratch[i];
  return s;
}

// Status bits shared with the host (mirrors LOVE_SF_* in love.h).
enum : unsigned {
  SF_DOMAIN = 1u, SF_NONFINITE = 2u, SF_NOTPD = 4u, SF_BREAKDOWN = 8u, SF_CG_NOCONV = 16u,
  SF_SAMPLER_TRUNC = 32u
};

// Device-resident control block of one Lanczos / CG run.  Kernels read the
// flags and return early once a run has stopped, so the host can enqueue a
// fixed number of steps without synchronising.
struct Ctl {
  int stop;          // Lanczos: set when beta_j <= tol * max|alpha|
  int k_eff;         // Lanczos steps kept
  int cg_done;       // CG converged (or failed)
  int cg_iters;
  unsigned status;   // SF_* bits
  int k_chol;        // sampler: number of positive eigenvalues of T'
  int eig_fallback;  // sampler: eigenvectors must come from the QL solver
  double amax;       // running max |alpha|
  double rr;         // CG: current r^T r
  double rr0;        // CG: ||y||^2
  double rz;         // CG: current r^T M^{-1} r (preconditioned)
  double ratio;      // CG: rz_new / rz_old (direction update)
  double bnorm;      // probe norm
};

}  // namespace love
