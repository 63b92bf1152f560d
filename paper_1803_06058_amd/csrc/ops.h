// Device helpers shared by the operator, Lanczos and query kernels.
#pragma once
#include "common.h"

namespace love {

// weight of stencil offset o (0..3) at fraction s; 0 for any other offset
template <typename T>
__device__ inline T keys_weight_at(int o, T s) {
  const T u = T(1) - s;
  T w = T(0);
  w = (o == 0) ? T(-0.5) * s * u * u : w;
  w = (o == 1) ? (T(1.5) * s - T(2.5)) * s * s + T(1) : w;
  w = (o == 2) ? (T(1.5) * u - T(2.5)) * u * u + T(1) : w;
  w = (o == 3) ? T(-0.5) * s * s * u : w;
  return w;
}

// Kernels that run inside the Lanczos / CG loops return at once when the
// run has stopped (bit 1: Lanczos stop, bit 2: CG converged).
__device__ inline bool ctl_skip(const Ctl* ctl, int mode) {
  if (!ctl) return false;
  if ((mode & 1) && ctl->stop) return true;
  if ((mode & 2) && ctl->cg_done) return true;
  return false;
}

// (W u)[r] for one row: tensor-product cubic stencil, 4^D grid values (4 D
// for an additive composition, Sec. 3.4).
template <typename T, int D>
__device__ inline T gather_row_vals(const GridT<T>& g, const T (&xr)[D], const T* __restrict__ kg) {
  if (g.add) {
    // additive composition: the four nodes of every axis's own block
    T acc = T(0);
#pragma unroll
    for (int e = 0; e < D; ++e) {
      T s, w[4];
      const int j = stencil_at(g, e, xr[e], s);
      keys_weights(s, w);
      const T* p = kg + g.aoff[e] + j;
      acc += w[0] * p[0] + w[1] * p[1] + w[2] * p[2] + w[3] * p[3];
    }
    return acc;
  }
  T w[D][4];
  int64_t base = 0;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    T s;
    const int j = stencil_at(g, e, xr[e], s);
    keys_weights(s, w[e]);
    base += (int64_t)j * g.nstride[e];
  }
  constexpr int OUTER = 1 << (2 * (D - 1));
  T acc = T(0);
#pragma unroll
  for (int hi = 0; hi < OUTER; ++hi) {
    T wp = T(1);
    int64_t off = base;
#pragma unroll
    for (int e = 0; e < D - 1; ++e) {
      const int o = (hi >> (2 * (D - 2 - e))) & 3;
      wp *= w[e][o];
      off += (int64_t)o * g.nstride[e];
    }
    const T* p = kg + off;
    acc += wp * (w[D - 1][0] * p[0] + w[D - 1][1] * p[1] + w[D - 1][2] * p[2] + w[D - 1][3] * p[3]);
  }
  return acc;
}
// Half `half` (0 or 1) of (W u)[r] for D >= 2: the first axis's stencil
// offsets 2 half and 2 half + 1, in the order gather_row_vals takes them;
// the row's value is half 0 + half 1.  An additive composition's row is all
// in half 0.
template <typename T, int D>
__device__ inline T gather_row_part(const GridT<T>& g, const T (&xr)[D], const T* __restrict__ kg,
                                    int half) {
  static_assert(D >= 2, "the split is over the first axis of a product stencil");
  if (g.add) return half ? T(0) : gather_row_vals<T, D>(g, xr, kg);
  T w[D][4];
  int64_t base = 0;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    T s;
    const int j = stencil_at(g, e, xr[e], s);
    keys_weights(s, w[e]);
    base += (int64_t)j * g.nstride[e];
  }
  const T wa[2] = {half ? w[0][2] : w[0][0], half ? w[0][3] : w[0][1]};
  base += (int64_t)(2 * half) * g.nstride[0];
  constexpr int INNER = 1 << (2 * (D - 2));   // offsets of the axes between the first and the last
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int hi = 0; hi < INNER; ++hi) {
      T wp = wa[a];
      int64_t off = base + (int64_t)a * g.nstride[0];
#pragma unroll
      for (int e = 1; e < D - 1; ++e) {
        const int o = (hi >> (2 * (D - 2 - e))) & 3;
        wp *= w[e][o];
        off += (int64_t)o * g.nstride[e];
      }
      const T* p = kg + off;
      acc += wp * (w[D - 1][0] * p[0] + w[D - 1][1] * p[1] + w[D - 1][2] * p[2] + w[D - 1][3] * p[3]);
    }
  }
  return acc;
}

template <typename T, int D>
__device__ inline T gather_row_dev(const GridT<T>& g, const T* __restrict__ x, int64_t r,
                                   const T* __restrict__ kg) {
  T xr[D];
#pragma unroll
  for (int e = 0; e < D; ++e) xr[e] = x[r * D + e];
  return gather_row_vals<T, D>(g, xr, kg);
}

}  // namespace love
