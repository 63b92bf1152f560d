// Constant-time test-time kernels (Sec. 3.2 test phase, Alg. 1 queries;
// Sec. 3.3 sampling) and the backward of the mean / variance with respect to
// the test inputs.
//
// A query point touches only the 4^d grid nodes of its cubic stencil, so every
// kernel here is a gather of 4^d rows of Rt (m x kpad) plus the mean cache a.
// One wave serves one point: lane l owns columns l and l + 64 of Rt, so every
// row load is a coalesced 256-byte access; ||u||^2 and the prior are summed
// in double and the variance subtraction (which cancels 4-6 digits) is done
// in double.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.h"
#include "ops.h"

namespace love {

__device__ inline float bf16f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <typename T, int SPLIT>
__device__ inline double rt_load(const void* rt, const uint16_t* rt_lo, int64_t idx) {
  if constexpr (SPLIT) {
    return (double)(bf16f(((const uint16_t*)rt)[idx]) + bf16f(rt_lo[idx]));
  } else {
    return (double)((const T*)rt)[idx];
  }
}

struct Stencil4 {
  int base[MAXD];
};

// per-axis weights, derivative weights and the stencil base of one point
template <typename T, int D>
__device__ inline bool point_stencil(const GridT<T>& g, const T* __restrict__ xp, double w[D][4],
                                     double dw[D][4], int64_t& base, bool want_dw) {
  bool ok = true;
  base = 0;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    T xe = xp[e];
    ok = ok && in_domain(xe, g.lo[e], g.hi[e]);
    if (!(xe == xe)) xe = g.lo[e];
    T s;
    const int j = stencil_at(g, e, xe, s);
    T wt[4];
    keys_weights(s, wt);
#pragma unroll
    for (int o = 0; o < 4; ++o) w[e][o] = (double)wt[o];
    if (want_dw) {
      T dt[4];
      keys_dweights(s, dt);
#pragma unroll
      for (int o = 0; o < 4; ++o) dw[e][o] = (double)dt[o] * (double)g.invh[e];
    }
    base += (int64_t)j * g.nstride[e];
  }
  return ok;
}

// point_stencil that also returns each axis's stencil base jb[e]
template <typename T, int D>
__device__ inline bool point_stencil_j(const GridT<T>& g, const T* __restrict__ xp, double w[D][4],
                                       double dw[D][4], int (&jb)[D], int64_t& base, bool want_dw) {
  bool ok = true;
  base = 0;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    T xe = xp[e];
    ok = ok && in_domain(xe, g.lo[e], g.hi[e]);
    if (!(xe == xe)) xe = g.lo[e];
    T s;
    const int j = stencil_at(g, e, xe, s);
    T wt[4];
    keys_weights(s, wt);
#pragma unroll
    for (int o = 0; o < 4; ++o) w[e][o] = (double)wt[o];
    if (want_dw) {
      T dt[4];
      keys_dweights(s, dt);
#pragma unroll
      for (int o = 0; o < 4; ++o) dw[e][o] = (double)dt[o] * (double)g.invh[e];
    }
    jb[e] = j;
    base += (int64_t)j * g.nstride[e];
  }
  return ok;
}

// Stencil entries of one point: 4^D grid nodes of the tensor-product grid,
// or (ADD, Sec. 3.4) the four nodes of each axis's own block, 4 D in all.
template <int D, bool ADD>
struct Entries {
  static constexpr int N = ADD ? 4 * D : 1 << (2 * D);
};
template <typename T, int D, bool ADD>
__device__ inline void stn_entry(const GridT<T>& g, const double (&w)[D][4], int64_t base,
                                 const int (&jb)[D], int a, double& wa, int64_t& node) {
  if constexpr (ADD) {
    wa = w[a >> 2][a & 3];
    node = g.aoff[a >> 2] + jb[a >> 2] + (a & 3);
  } else {
    wa = 1.0;
    node = base;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int o = (a >> (2 * (D - 1 - e))) & 3;
      wa *= w[e][o];
      node += (int64_t)o * g.nstride[e];
    }
  }
}

// w_e^T T_e(4x4) v_e with T_e(4x4)[a][b] = c4[e][|a-b|]
__device__ inline double quad4(const double* c4e, const double* a, const double* b) {
  double s = 0.0;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) s += a[p] * b[q] * c4e[p > q ? p - q : q - p];
  return s;
}

template <typename T>
struct PredJob {
  GridT<T> g;
  const T* xs;
  int64_t t;
  const void* rt;
  const uint16_t* rt_lo;
  int kpad;
  const T* a;          // mean cache (nullable)
  const double* c4;
  T* mean;             // nullable
  T* var;
  unsigned* status;
};

// Each query point is served by PLQ = 16 lanes, four points per wave and
// sixteen per block: lane sub of a point holds the CPL = kpad / 16 consecutive
// columns sub CPL .. sub CPL + CPL - 1 of every stencil row of Rt (one or two
// 16-byte loads per row), so a wave keeps four points' gathers in flight
// instead of one.  u = Rt^T w accumulates per column over the stencil rows in
// row order; ||u||^2 and the mean are then summed over the 16 lanes.
constexpr int PLQ = 16;
constexpr int PPB = 256 / PLQ;   // points per block

template <typename T, int SPLIT, int CPL>
__device__ __forceinline__ void rt_row(const void* rt, const uint16_t* rt_lo, int64_t idx,
                                       double (&v)[CPL]) {
  if constexpr (!SPLIT && sizeof(T) == 4) {
#pragma unroll
    for (int q = 0; q < CPL; q += 4) {
      const float4 f = *reinterpret_cast<const float4*>((const float*)rt + idx + q);
      v[q] = f.x;
      v[q + 1] = f.y;
      v[q + 2] = f.z;
      v[q + 3] = f.w;
    }
  } else if constexpr (!SPLIT) {
#pragma unroll
    for (int q = 0; q < CPL; q += 2) {
      const double2 f = *reinterpret_cast<const double2*>((const double*)rt + idx + q);
      v[q] = f.x;
      v[q + 1] = f.y;
    }
  } else {
#pragma unroll
    for (int q = 0; q < CPL; ++q) v[q] = rt_load<T, SPLIT>(rt, rt_lo, idx + q);
  }
}

template <typename T, int D, int SPLIT, int CPL>
__device__ inline void predict_body(const PredJob<T>& J, int64_t lb) {
  const int lane = threadIdx.x & (WAVE - 1), sub = lane & (PLQ - 1);
  const int64_t p = lb * PPB + threadIdx.x / PLQ;
  const bool live = p < J.t;
  const int64_t pc = live ? p : J.t - 1;   // spare lanes redo the last point, write nothing
  const GridT<T>& g = J.g;
  const int kpad = J.kpad;
  const T* acache = J.a;
  double w[D][4], dw[D][4];
  int64_t base;
  const bool ok = point_stencil<T, D>(g, J.xs + pc * D, w, dw, base, false);
  constexpr int NA = 1 << (2 * D);
  double u[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) u[q] = 0.0;
  double mu = 0.0;
#pragma unroll 4
  for (int a = 0; a < NA; ++a) {
    double wa = 1.0;
    int64_t node = base;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int o = (a >> (2 * (D - 1 - e))) & 3;
      wa *= w[e][o];
      node += (int64_t)o * g.nstride[e];
    }
    double r[CPL];
    rt_row<T, SPLIT, CPL>(J.rt, J.rt_lo, node * kpad + sub * CPL, r);
#pragma unroll
    for (int q = 0; q < CPL; ++q) u[q] += wa * r[q];
    if ((a & (PLQ - 1)) == sub && acache) mu += wa * (double)acache[node];
  }
  double uu = 0.0;
#pragma unroll
  for (int q = 0; q < CPL; ++q) uu += u[q] * u[q];
  uu = group_sum(uu, PLQ);
  mu = group_sum(mu, PLQ);
  if (sub == 0 && live) {
    double pr = 1.0;
#pragma unroll
    for (int e = 0; e < D; ++e) pr *= quad4(J.c4 + 4 * e, w[e], w[e]);
    if (ok) {
      J.var[p] = (T)(pr - uu);
      if (J.mean) J.mean[p] = (T)mu;
    } else {
      J.var[p] = (T)NAN;
      if (J.mean) J.mean[p] = (T)NAN;
      atomicOr(J.status, SF_DOMAIN);
    }
  }
}

// Additive composition (Sec. 3.4): the stacked interpolation vector has the
// four nodes of each axis's own block, 4 D rows of Rt in all, and the prior
// is the sum of the axes' w_e^T T_e w_e (outputscale in every c4 row).
template <typename T, int D, int SPLIT, int CPL>
__device__ inline void predict_body_add(const PredJob<T>& J, int64_t lb) {
  const int lane = threadIdx.x & (WAVE - 1), sub = lane & (PLQ - 1);
  const int64_t p = lb * PPB + threadIdx.x / PLQ;
  const bool live = p < J.t;
  const int64_t pc = live ? p : J.t - 1;
  const GridT<T>& g = J.g;
  const int kpad = J.kpad;
  const T* acache = J.a;
  double w[D][4];
  int64_t base[D];
  bool ok = true;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    T xe = J.xs[pc * D + e];
    ok = ok && in_domain(xe, g.lo[e], g.hi[e]);
    if (!(xe == xe)) xe = g.lo[e];
    T sv, wt[4];
    const int j = stencil_at(g, e, xe, sv);
    keys_weights(sv, wt);
#pragma unroll
    for (int o = 0; o < 4; ++o) w[e][o] = (double)wt[o];
    base[e] = g.aoff[e] + j;
  }
  static_assert(4 * D <= PLQ, "one mean term per lane");
  double u[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) u[q] = 0.0;
  double mu = 0.0;
#pragma unroll
  for (int a = 0; a < 4 * D; ++a) {
    const double wa = w[a >> 2][a & 3];
    const int64_t node = base[a >> 2] + (a & 3);
    double r[CPL];
    rt_row<T, SPLIT, CPL>(J.rt, J.rt_lo, node * kpad + sub * CPL, r);
#pragma unroll
    for (int q = 0; q < CPL; ++q) u[q] += wa * r[q];
    if (a == sub && acache) mu += wa * (double)acache[node];
  }
  double uu = 0.0;
#pragma unroll
  for (int q = 0; q < CPL; ++q) uu += u[q] * u[q];
  uu = group_sum(uu, PLQ);
  mu = group_sum(mu, PLQ);
  if (sub == 0 && live) {
    double pr = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) pr += quad4(J.c4 + 4 * e, w[e], w[e]);
    if (ok) {
      J.var[p] = (T)(pr - uu);
      if (J.mean) J.mean[p] = (T)mu;
    } else {
      J.var[p] = (T)NAN;
      if (J.mean) J.mean[p] = (T)NAN;
      atomicOr(J.status, SF_DOMAIN);
    }
  }
}

template <typename T, int D, int SPLIT>
__device__ __forceinline__ void predict_any(const PredJob<T>& J, int64_t lb) {
  if (J.g.add) {
    if (J.kpad > 64) predict_body_add<T, D, SPLIT, 8>(J, lb);
    else predict_body_add<T, D, SPLIT, 4>(J, lb);
  } else {
    if (J.kpad > 64) predict_body<T, D, SPLIT, 8>(J, lb);
    else predict_body<T, D, SPLIT, 4>(J, lb);
  }
}

template <typename T, int D, int SPLIT>
__global__ __launch_bounds__(256) void k_predict(PredJob<T> J) {
  predict_any<T, D, SPLIT>(J, blockIdx.x);
}

template <typename T, int D, int SPLIT>
__global__ __launch_bounds__(256) void k_predict_b(Tab tab, const PredJob<T>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  predict_any<T, D, SPLIT>(jobs[gp], lb);
}

template <typename T>
static PredJob<T> pred_job(const love_cache* c, const T* xs, int64_t t, T* mean, T* var) {
  PredJob<T> J{};
  J.g = make_grid<T>(c);
  J.xs = xs;
  J.t = t;
  J.rt = c->rt;
  J.rt_lo = (const uint16_t*)c->rt_lo;
  J.kpad = c->kpad;
  J.a = (c->cfg.flags & LOVE_FLAG_NO_MEAN) ? nullptr : (const T*)c->a;
  J.c4 = c->c4_dev;
  J.mean = mean;
  J.var = var;
  J.status = c->status;
  return J;
}

// G == 1: arguments by value (no upload); otherwise one launch for all GPs.
template <typename T>
love_status predict_batch(const std::vector<const love_cache*>& cs,
                          const std::vector<const T*>& xs, const std::vector<int64_t>& ts,
                          const std::vector<T*>& means, const std::vector<T*>& vars,
                          hipStream_t s) {
  const int G = (int)cs.size();
  const int d = cs[0]->d;
  const bool split = cs[0]->cfg.precision == LOVE_P_FP32_BF16SPLIT;
  if (G == 1) {
    if (ts[0] == 0) return LOVE_OK;
    const PredJob<T> J = pred_job<T>(cs[0], xs[0], ts[0], means[0], vars[0]);
    const unsigned nb = (unsigned)cdiv(ts[0], PPB);
#define LAUNCH_P(D)                                                   \
  if (split) tlaunch("predict", k_predict<T, D, 1>, nb, 256, 0, s, J); \
  else tlaunch("predict", k_predict<T, D, 0>, nb, 256, 0, s, J);
    switch (d) {
      case 1: LAUNCH_P(1); break;
      case 2: LAUNCH_P(2); break;
      case 3: LAUNCH_P(3); break;
      case 4: LAUNCH_P(4); break;
    }
#undef LAUNCH_P
    return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
  }
  for (int g0 = 0; g0 < G; g0 += MAXG) {
    const int g1 = std::min(G, g0 + MAXG);
    std::vector<PredJob<T>> jobs;
    std::vector<int64_t> blocks;
    for (int g = g0; g < g1; ++g) {
      jobs.push_back(pred_job<T>(cs[g], xs[g], ts[g], means[g], vars[g]));
      blocks.push_back(cdiv(ts[g], PPB));
    }
    const Tab tab = make_tab(blocks);
    if (!tab_blocks(tab)) continue;
    JobArena A;
    const size_t o = A.add(jobs);
    love_status st = A.upload(s);
    if (st != LOVE_OK) return st;
    const PredJob<T>* dj = A.at<PredJob<T>>(o);
    const unsigned nb = tab_blocks(tab);
#define LAUNCH_PB(D)                                                  \
  if (split) tlaunch("predict", k_predict_b<T, D, 1>, nb, 256, 0, s, tab, dj); \
  else tlaunch("predict", k_predict_b<T, D, 0>, nb, 256, 0, s, tab, dj);
    switch (d) {
      case 1: LAUNCH_PB(1); break;
      case 2: LAUNCH_PB(2); break;
      case 3: LAUNCH_PB(3); break;
      case 4: LAUNCH_PB(4); break;
    }
#undef LAUNCH_PB
    A.release(s);
  }
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}
template love_status predict_batch<float>(const std::vector<const love_cache*>&, const std::vector<const float*>&, const std::vector<int64_t>&, const std::vector<float*>&, const std::vector<float*>&, hipStream_t);
template love_status predict_batch<double>(const std::vector<const love_cache*>&, const std::vector<const double*>&, const std::vector<int64_t>&, const std::vector<double*>&, const std::vector<double*>&, hipStream_t);

// ----------------------------------------------------------------------------
// Cross-covariance of paired points (Alg. 1 with w_i != w_j):
//   cov = w_i^T K w_j - (Rt^T w_i)^T (Rt^T w_j)
// The prior term uses the full first column of each axis factor, since the
// two stencils may be far apart.
// ----------------------------------------------------------------------------
template <typename T, int D, int SPLIT, bool ADD>
__global__ __launch_bounds__(256) void k_covar_pairs(
    GridT<T> g, const T* __restrict__ xa, const T* __restrict__ xb, int64_t t,
    const void* __restrict__ rt, const uint16_t* __restrict__ rt_lo, int kpad,
    const double* __restrict__ c0, const double* __restrict__ c1, const double* __restrict__ c2,
    const double* __restrict__ c3, T* __restrict__ cov, unsigned* __restrict__ status) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (p >= t) return;
  double wa[D][4], wb[D][4], dd[D][4];
  int64_t ba, bb;
  int ja_[D], jb_[D];
  bool ok = point_stencil_j<T, D>(g, xa + p * D, wa, dd, ja_, ba, false);
  ok = point_stencil_j<T, D>(g, xb + p * D, wb, dd, jb_, bb, false) && ok;
  constexpr int NA = Entries<D, ADD>::N;
  const bool two = kpad > WAVE;
  double ua0 = 0, ua1 = 0, ub0 = 0, ub1 = 0;
  for (int a = 0; a < NA; ++a) {
    double fa, fb;
    int64_t na, nb;
    stn_entry<T, D, ADD>(g, wa, ba, ja_, a, fa, na);
    stn_entry<T, D, ADD>(g, wb, bb, jb_, a, fb, nb);
    ua0 += fa * rt_load<T, SPLIT>(rt, rt_lo, na * kpad + lane);
    ub0 += fb * rt_load<T, SPLIT>(rt, rt_lo, nb * kpad + lane);
    if (two) {
      ua1 += fa * rt_load<T, SPLIT>(rt, rt_lo, na * kpad + lane + WAVE);
      ub1 += fb * rt_load<T, SPLIT>(rt, rt_lo, nb * kpad + lane + WAVE);
    }
  }
  const double uv = wave_sum(ua0 * ub0 + ua1 * ub1);
  if (lane == 0) {
    const double* cols[4] = {c0, c1, c2, c3};
    double pr = ADD ? 0.0 : 1.0;   // additive: sum of the axes' terms
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int ja = ja_[e], jb = jb_[e];
      double sacc = 0.0;
      for (int o = 0; o < 4; ++o)
        for (int q = 0; q < 4; ++q) {
          int lag = (ja + o) - (jb + q);
          lag = lag < 0 ? -lag : lag;
          sacc += wa[e][o] * wb[e][q] * cols[e][lag];
        }
      if (ADD) pr += sacc;
      else pr *= sacc;
    }
    if (ok) cov[p] = (T)(pr - uv);
    else {
      cov[p] = (T)NAN;
      atomicOr(status, SF_DOMAIN);
    }
  }
}

template <typename T>
love_status covar_pairs(const love_cache* c, const T* xa, const T* xb, int64_t t, T* cov,
                        hipStream_t s) {
  ProfScope ps("covar_pairs", s);
  if (t == 0) return LOVE_OK;
  GridT<T> g = make_grid<T>(c);
  dim3 grid((unsigned)cdiv(t, 4));
  const bool split = c->cfg.precision == LOVE_P_FP32_BF16SPLIT;
  const double* cc[4];
  for (int e = 0; e < 4; ++e) cc[e] = (const double*)(e < c->d ? c->toep.ax[e].c64 : nullptr);
#define LAUNCH_C(D, ADD)                                                                           \
  if (split)                                                                                       \
    k_covar_pairs<T, D, 1, ADD><<<grid, 256, 0, s>>>(g, xa, xb, t, c->rt, (const uint16_t*)c->rt_lo, \
                                                c->kpad, cc[0], cc[1], cc[2], cc[3], cov, c->status); \
  else                                                                                             \
    k_covar_pairs<T, D, 0, ADD><<<grid, 256, 0, s>>>(g, xa, xb, t, c->rt, nullptr, c->kpad, cc[0],  \
                                                cc[1], cc[2], cc[3], cov, c->status);
#define LAUNCH_CA(D)                                                                               \
  if (c->add) {                                                                                    \
    LAUNCH_C(D, true)                                                                              \
  } else {                                                                                         \
    LAUNCH_C(D, false)                                                                             \
  }
  switch (c->d) {
    case 1: LAUNCH_CA(1); break;
    case 2: LAUNCH_CA(2); break;
    case 3: LAUNCH_CA(3); break;
    case 4: LAUNCH_CA(4); break;
  }
#undef LAUNCH_CA
#undef LAUNCH_C
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}
// ----------------------------------------------------------------------------
// Predictive covariance block: cov[i, j] = k(xa_i, xb_j) for all pairs
// (Alg. 1 with w_i != w_j; eq. pred_covar_ski_fast):
//   cov = prod_e w_a,e^T T_e w_b,e  -  u_a . u_b,   u = Rt^T w (double).
//   k_covar_u      per point: u (double, kpad wide) and the stencil record
//                  [w (4 per axis) | base per axis | in-domain flag], 16 lanes
//                  per point as for the variances;
//   k_covar_block  32 x 32 pairs per block from LDS tiles of u.
// ----------------------------------------------------------------------------
template <int D>
struct CovRec {
  static constexpr int W = 0, J = 4 * D, OK = 5 * D, N = 5 * D + 1;   // doubles per point
};
template <typename T, int D, int SPLIT, int CPL, bool ADD>
__device__ inline void covar_u_body(const GridT<T>& g, const T* __restrict__ xs, int64_t t,
                                    const void* __restrict__ rt,
                                    const uint16_t* __restrict__ rt_lo, int kpad,
                                    double* __restrict__ U, double* __restrict__ rec) {
  const int lane = threadIdx.x & (WAVE - 1), sub = lane & (PLQ - 1);
  const int64_t p = (int64_t)blockIdx.x * PPB + threadIdx.x / PLQ;
  const bool live = p < t;
  const int64_t pc = live ? p : t - 1;
  double w[D][4], dw[D][4];
  int64_t base;
  int jb[D];
  const bool ok = point_stencil_j<T, D>(g, xs + pc * D, w, dw, jb, base, false);
  constexpr int NA = Entries<D, ADD>::N;
  double u[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) u[q] = 0.0;
#pragma unroll 4
  for (int a = 0; a < NA; ++a) {
    double wa;
    int64_t node;
    stn_entry<T, D, ADD>(g, w, base, jb, a, wa, node);
    double r[CPL];
    rt_row<T, SPLIT, CPL>(rt, rt_lo, node * kpad + sub * CPL, r);
#pragma unroll
    for (int q = 0; q < CPL; ++q) u[q] += wa * r[q];
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < CPL; ++q) U[p * kpad + sub * CPL + q] = u[q];
  if (sub == 0) {
    double* rp = rec + p * CovRec<D>::N;
#pragma unroll
    for (int e = 0; e < D; ++e) {
#pragma unroll
      for (int o = 0; o < 4; ++o) rp[CovRec<D>::W + 4 * e + o] = w[e][o];
      rp[CovRec<D>::J + e] = (double)jb[e];
    }
    rp[CovRec<D>::OK] = ok ? 1.0 : 0.0;
  }
}
template <typename T, int D, int SPLIT, bool ADD>
__global__ __launch_bounds__(256) void k_covar_u(GridT<T> g, const T* __restrict__ xs, int64_t t,
                                                 const void* __restrict__ rt,
                                                 const uint16_t* __restrict__ rt_lo, int kpad,
                                                 double* __restrict__ U, double* __restrict__ rec) {
  if (kpad > 64) covar_u_body<T, D, SPLIT, 128 / PLQ, ADD>(g, xs, t, rt, rt_lo, kpad, U, rec);
  else covar_u_body<T, D, SPLIT, 64 / PLQ, ADD>(g, xs, t, rt, rt_lo, kpad, U, rec);
}

constexpr int CB = 32;   // pairs per tile side
template <typename T, int D, bool ADD>
__global__ __launch_bounds__(256) void k_covar_block(
    const double* __restrict__ Ua, const double* __restrict__ ra, int64_t ta,
    const double* __restrict__ Ub, const double* __restrict__ rb, int64_t tb, int kpad,
    const Ctl* __restrict__ ctl, const double* __restrict__ c0, const double* __restrict__ c1,
    const double* __restrict__ c2, const double* __restrict__ c3, T* __restrict__ cov,
    unsigned* __restrict__ status) {
  __shared__ double A[CB][MAXK + 1], Bt[CB][MAXK + 1];
  __shared__ double RA[CB][CovRec<D>::N], RB[CB][CovRec<D>::N];
  const int keff = ctl->k_eff;
  const int64_t i0 = (int64_t)blockIdx.y * CB, j0 = (int64_t)blockIdx.x * CB;
  {
    // fixed-count unrolled loads, all issued before the LDS stores
    constexpr int NL = CB * MAXK / 256;
    double va[NL], vb[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx / MAXK, c = idx % MAXK;
      va[q] = (c < keff && i0 + r < ta) ? Ua[(i0 + r) * kpad + c] : 0.0;
      vb[q] = (c < keff && j0 + r < tb) ? Ub[(j0 + r) * kpad + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int idx = threadIdx.x + 256 * q;
      A[idx / MAXK][idx % MAXK] = va[q];
      Bt[idx / MAXK][idx % MAXK] = vb[q];
    }
  }
  for (int idx = threadIdx.x; idx < CB * CovRec<D>::N; idx += blockDim.x) {
    const int r = idx / CovRec<D>::N, c = idx - r * CovRec<D>::N;
    RA[r][c] = i0 + r < ta ? ra[(i0 + r) * CovRec<D>::N + c] : 0.0;
    RB[r][c] = j0 + r < tb ? rb[(j0 + r) * CovRec<D>::N + c] : 0.0;
  }
  __syncthreads();
  const double* cols[4] = {c0, c1, c2, c3};
  const int jj = threadIdx.x % CB;
  const int64_t j = j0 + jj;
  bool flag = false;
  for (int ii = threadIdx.x / CB; ii < CB; ii += blockDim.x / CB) {
    const int64_t i = i0 + ii;
    if (i >= ta || j >= tb) continue;
    double dot = 0.0;
    for (int c = 0; c < keff; ++c) dot += A[ii][c] * Bt[jj][c];
    double pr = ADD ? 0.0 : 1.0;   // additive: sum of the axes' terms
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int ja = (int)RA[ii][CovRec<D>::J + e], jb = (int)RB[jj][CovRec<D>::J + e];
      double se = 0.0;
#pragma unroll
      for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int lag = (ja + o) - (jb + q);
          lag = lag < 0 ? -lag : lag;
          se += RA[ii][CovRec<D>::W + 4 * e + o] * RB[jj][CovRec<D>::W + 4 * e + q] * cols[e][lag];
        }
      if (ADD) pr += se;
      else pr *= se;
    }
    const bool ok = RA[ii][CovRec<D>::OK] != 0.0 && RB[jj][CovRec<D>::OK] != 0.0;
    cov[i * tb + j] = ok ? (T)(pr - dot) : (T)NAN;
    flag = flag || !ok;
  }
  if (flag) atomicOr(status, SF_DOMAIN);
}

template <typename T>
love_status covar_block(const love_cache* c, const T* xa, int64_t ta, const T* xb, int64_t tb,
                        T* cov, hipStream_t s) {
  if (ta == 0 || tb == 0) return LOVE_OK;
  if (cdiv(ta, CB) > 65535) return LOVE_EINVAL;
  GridT<T> g = make_grid<T>(c);
  const int d = c->d, kpad = c->kpad, nrec = 5 * d + 1;
  double* U = nullptr;
  const size_t per = (size_t)kpad + nrec;
  U = (double*)ws_alloc(sizeof(double) * per * (size_t)(ta + tb), s);
  if (!U) return LOVE_ENOMEM;
  double* Ua = U;
  double* Ub = Ua + (size_t)kpad * ta;
  double* ra = Ub + (size_t)kpad * tb;
  double* rb = ra + (size_t)nrec * ta;
  const bool split = c->cfg.precision == LOVE_P_FP32_BF16SPLIT;
  const uint16_t* lo = (const uint16_t*)c->rt_lo;
  const double* cc[4];
  for (int e = 0; e < 4; ++e) cc[e] = (const double*)(e < d ? c->toep.ax[e].c64 : nullptr);
  dim3 grid((unsigned)cdiv(tb, CB), (unsigned)cdiv(ta, CB));
#define LAUNCH_CV(D, ADD)                                                                         \
  {                                                                                               \
    const unsigned na = (unsigned)cdiv(ta, PPB), nb = (unsigned)cdiv(tb, PPB);                     \
    if (split) {                                                                                  \
      tlaunch("covar_u", k_covar_u<T, D, 1, ADD>, na, 256, 0, s, g, xa, ta, c->rt, lo, kpad, Ua, ra); \
      tlaunch("covar_u", k_covar_u<T, D, 1, ADD>, nb, 256, 0, s, g, xb, tb, c->rt, lo, kpad, Ub, rb); \
    } else {                                                                                      \
      tlaunch("covar_u", k_covar_u<T, D, 0, ADD>, na, 256, 0, s, g, xa, ta, c->rt, lo, kpad, Ua, ra); \
      tlaunch("covar_u", k_covar_u<T, D, 0, ADD>, nb, 256, 0, s, g, xb, tb, c->rt, lo, kpad, Ub, rb); \
    }                                                                                             \
    tlaunch("covar_block", k_covar_block<T, D, ADD>, grid, 256, 0, s, (const double*)Ua,          \
            (const double*)ra, ta, (const double*)Ub, (const double*)rb, tb, kpad,                \
            (const Ctl*)c->ctl, cc[0], cc[1], cc[2], cc[3], cov, c->status);                      \
  }
#define LAUNCH_CVA(D)                                                                              \
  if (c->add) LAUNCH_CV(D, true) else LAUNCH_CV(D, false)
  switch (d) {
    case 1: LAUNCH_CVA(1); break;
    case 2: LAUNCH_CVA(2); break;
    case 3: LAUNCH_CVA(3); break;
    case 4: LAUNCH_CVA(4); break;
  }
#undef LAUNCH_CVA
#undef LAUNCH_CV
  ws_free(U, s);
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}
template love_status covar_block<float>(const love_cache*, const float*, int64_t, const float*, int64_t, float*, hipStream_t);
template love_status covar_block<double>(const love_cache*, const double*, int64_t, const double*, int64_t, double*, hipStream_t);

template love_status covar_pairs<float>(const love_cache*, const float*, const float*, int64_t, float*, hipStream_t);
template love_status covar_pairs<double>(const love_cache*, const double*, const double*, int64_t, double*, hipStream_t);

// ----------------------------------------------------------------------------
// Backward: d(sum g_mean*mean + g_var*var)/d x*.
//   d mean / dx_e = sum_a dW_a^e a[node_a]
//   d var  / dx_e = dp/dx_e - 2 u . v_e,  u = Rt^T w, v_e = Rt^T dw/dx_e
//   dp/dx_e = 2 (dw_e)^T T_e w_e * prod_{f != e} w_f^T T_f w_f
// Optional dRt = sum_i -2 g_var,i w(x*_i) u_i^T: this kernel writes each
// point's row H_i = -2 g_var,i u_i (float, kpad columns; zero for points
// outside the domain), k_grt_gather sums the rows per grid node.
// Lanes as in the predictive variances: 16 per point, lane sub holding the
// CPL = kpad / 16 consecutive columns from sub CPL of every stencil row.
// ----------------------------------------------------------------------------
template <typename T, int D, int SPLIT, int CPL, bool ADD>
__device__ inline void backward_body(const GridT<T>& g, const T* __restrict__ xs, int64_t t,
                                     const void* __restrict__ rt,
                                     const uint16_t* __restrict__ rt_lo, int kpad,
                                     const Ctl* __restrict__ ctl, const T* __restrict__ acache,
                                     const double* __restrict__ c4, const T* __restrict__ gm,
                                     const T* __restrict__ gv, T* __restrict__ gx,
                                     float* __restrict__ H, unsigned* __restrict__ status) {
  const int lane = threadIdx.x & (WAVE - 1), sub = lane & (PLQ - 1);
  const int64_t p = (int64_t)blockIdx.x * PPB + threadIdx.x / PLQ;
  const bool live = p < t;
  const int64_t pc = live ? p : t - 1;
  double w[D][4], dw[D][4];
  int64_t base;
  int jb[D];
  const bool ok = point_stencil_j<T, D>(g, xs + pc * D, w, dw, jb, base, true);
  constexpr int NA = Entries<D, ADD>::N;
  double u[CPL], v[D][CPL], dmu[D];
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    u[q] = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) v[e][q] = 0.0;
  }
#pragma unroll
  for (int e = 0; e < D; ++e) dmu[e] = 0.0;
  if constexpr (ADD) {
    // axis e's own four rows: w for u, dw for v_e (the other axes' blocks do
    // not depend on x_e)
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const int e = a >> 2, o = a & 3;
      const int64_t node = g.aoff[e] + jb[e] + o;
      double r[CPL];
      rt_row<T, SPLIT, CPL>(rt, rt_lo, node * kpad + sub * CPL, r);
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        u[q] += w[e][o] * r[q];
        v[e][q] += dw[e][o] * r[q];
      }
      if (a == sub && acache) dmu[e] += dw[e][o] * (double)acache[node];
    }
  }
  for (int a = 0; a < (ADD ? 0 : NA); ++a) {
    int o[D];
    int64_t node = base;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      o[e] = (a >> (2 * (D - 1 - e))) & 3;
      node += (int64_t)o[e] * g.nstride[e];
    }
    double wa = 1.0;
#pragma unroll
    for (int e = 0; e < D; ++e) wa *= w[e][o[e]];
    double r[CPL];
    rt_row<T, SPLIT, CPL>(rt, rt_lo, node * kpad + sub * CPL, r);
#pragma unroll
    for (int q = 0; q < CPL; ++q) u[q] += wa * r[q];
    const double av = ((a & (PLQ - 1)) == sub && acache) ? (double)acache[node] : 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      double dwa = 1.0;
#pragma unroll
      for (int f = 0; f < D; ++f) dwa *= (f == e) ? dw[f][o[f]] : w[f][o[f]];
#pragma unroll
      for (int q = 0; q < CPL; ++q) v[e][q] += dwa * r[q];
      dmu[e] += dwa * av;
    }
  }
  const double gmean = (gm && live) ? (double)gm[p] : 0.0;
  const double gvar = (gv && live) ? (double)gv[p] : 0.0;
  double qd[D], dq[D];
#pragma unroll
  for (int e = 0; e < D; ++e) {
    qd[e] = quad4(c4 + 4 * e, w[e], w[e]);
    dq[e] = 2.0 * quad4(c4 + 4 * e, dw[e], w[e]);
  }
#pragma unroll
  for (int e = 0; e < D; ++e) {
    double uv = 0.0;
#pragma unroll
    for (int q = 0; q < CPL; ++q) uv += u[q] * v[e][q];
    uv = group_sum(uv, PLQ);
    const double dm = group_sum(dmu[e], PLQ);
    if (sub == 0 && live) {
      double dp = dq[e];   // additive: the prior is a sum, so only axis e's term moves
#pragma unroll
      for (int f = 0; f < D; ++f)
        if (f != e && !ADD) dp *= qd[f];
      const double gval = gmean * dm + gvar * (dp - 2.0 * uv);
      gx[p * D + e] = ok ? (T)gval : (T)NAN;
    }
  }
  if (!ok && live && sub == 0) atomicOr(status, SF_DOMAIN);
  if (H && live) {
    const double f = ok ? -2.0 * gvar : 0.0;
#pragma unroll
    for (int q = 0; q < CPL; q += 4)
      *reinterpret_cast<float4*>(H + p * kpad + sub * CPL + q) =
          make_float4((float)(f * u[q]), (float)(f * u[q + 1]), (float)(f * u[q + 2]),
                      (float)(f * u[q + 3]));
  }
}

// dRt[node, :] += sum w_node(x*_i) H_i over the points i whose stencil holds
// the node: one wave per grid node, lane l summing columns l (and l + 64) in
// double over the cells around the node (stencil offsets ascending) and, in a
// cell, over its points in sorted order, so the result does not depend on
// scheduling.  order / cstart come from sort_points.
// With pscale, row i is taken as fac * pscale[i] * H_i (H then holds u_i).
template <typename T, int D, bool ADD, typename TH, typename TO>
__global__ __launch_bounds__(256) void k_grt_gather(GridT<T> g, const T* __restrict__ xs,
                                                    const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ cstart,
                                                    const TH* __restrict__ H, int kpad,
                                                    const Ctl* __restrict__ ctl,
                                                    TO* __restrict__ grt,
                                                    const double* __restrict__ pscale,
                                                    double fac) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t node = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
  if (node >= g.mtot) return;
  const bool two = kpad > WAVE;
  double acc0 = 0.0, acc1 = 0.0;
  if constexpr (ADD) {
    int e = 0;
#pragma unroll
    for (int f = 1; f < D; ++f)
      if (node >= g.aoff[f]) e = f;
    const int i = (int)(node - g.aoff[e]);
    for (int o = 0; o < 4; ++o) {
      const int cl = i - o;
      if (cl < 0 || cl >= g.cells[e]) continue;
      const int64_t key = g.acoff[e] + cl;
      for (uint32_t pos = cstart[key], en = cstart[key + 1]; pos < en; ++pos) {
        const int64_t pt = order[pos];
        T xe = xs[pt * D + e];
        if (!(xe == xe)) xe = g.lo[e];
        T sv;
        (void)stencil_at(g, e, xe, sv);
        double wv = (double)keys_weight_at<T>(o, sv);
        if (pscale) wv *= fac * pscale[pt];
        const TH* hr = H + pt * kpad;
        acc0 += wv * (double)hr[lane];
        if (two) acc1 += wv * (double)hr[lane + WAVE];
      }
    }
  } else {
    int ie[D];
    int64_t r = node;
#pragma unroll
    for (int e = D - 1; e >= 0; --e) {
      ie[e] = (int)(r % g.m[e]);
      r /= g.m[e];
    }
    for (int a = 0; a < (1 << (2 * D)); ++a) {
      int oe[D];
      int64_t cell = 0;
      bool valid = true;
#pragma unroll
      for (int e = 0; e < D; ++e) {
        oe[e] = (a >> (2 * (D - 1 - e))) & 3;
        const int cl = ie[e] - oe[e];
        valid = valid && cl >= 0 && cl < g.cells[e];
        cell += (int64_t)cl * g.cstride[e];
      }
      if (!valid) continue;
      for (uint32_t pos = cstart[cell], en = cstart[cell + 1]; pos < en; ++pos) {
        const int64_t pt = order[pos];
        double wv = 1.0;
#pragma unroll
        for (int e = 0; e < D; ++e) {
          T xe = xs[pt * D + e];
          if (!(xe == xe)) xe = g.lo[e];
          T sv;
          (void)stencil_at(g, e, xe, sv);
          wv *= (double)keys_weight_at<T>(oe[e], sv);
        }
        if (pscale) wv *= fac * pscale[pt];
        const TH* hr = H + pt * kpad;
        acc0 += wv * (double)hr[lane];
        if (two) acc1 += wv * (double)hr[lane + WAVE];
      }
    }
  }
  const int keff = ctl->k_eff;
  if (lane < keff) grt[node * keff + lane] += (TO)acc0;
  if (two && lane + WAVE < keff) grt[node * keff + lane + WAVE] += (TO)acc1;
}
template <typename T, int D, int SPLIT, bool ADD>
__global__ __launch_bounds__(256) void k_backward(GridT<T> g, const T* __restrict__ xs, int64_t t,
                                                  const void* __restrict__ rt,
                                                  const uint16_t* __restrict__ rt_lo, int kpad,
                                                  const Ctl* __restrict__ ctl,
                                                  const T* __restrict__ acache,
                                                  const double* __restrict__ c4,
                                                  const T* __restrict__ gm, const T* __restrict__ gv,
                                                  T* __restrict__ gx, float* __restrict__ H,
                                                  unsigned* __restrict__ status) {
  if (kpad > 64)
    backward_body<T, D, SPLIT, 128 / PLQ, ADD>(g, xs, t, rt, rt_lo, kpad, ctl, acache, c4, gm, gv,
                                               gx, H, status);
  else
    backward_body<T, D, SPLIT, 64 / PLQ, ADD>(g, xs, t, rt, rt_lo, kpad, ctl, acache, c4, gm, gv,
                                              gx, H, status);
}

template <typename T>
love_status backward(const love_cache* c, const T* xs, int64_t t, const T* gm, const T* gv, T* gx,
                     float* grt, hipStream_t s) {
  if (t == 0) return LOVE_OK;
  GridT<T> g = make_grid<T>(c);
  const unsigned nb = (unsigned)cdiv(t, PPB);
  const T* a = (c->cfg.flags & LOVE_FLAG_NO_MEAN) ? nullptr : (const T*)c->a;
  const bool split = c->cfg.precision == LOVE_P_FP32_BF16SPLIT;
  const Ctl* ctl = c->ctl;
  // dRt workspace: H (t x kpad float), the sorted point entries, cell starts
  float* H = nullptr;
  uint32_t *order = nullptr, *cst = nullptr;
  if (grt) {
    if (t >= (int64_t(1) << 31) / 4) return LOVE_EINVAL;
    const int64_t nv = c->add ? (int64_t)c->d * t : t;
    const size_t hbytes = sizeof(float) * (size_t)t * c->kpad;
    const size_t obytes = (sizeof(uint32_t) * (size_t)nv + 255) & ~size_t(255);
    char* buf = (char*)ws_alloc(hbytes + obytes + sizeof(uint32_t) * ((size_t)c->ctot + 1), s);
    if (!buf) return LOVE_ENOMEM;
    H = (float*)buf;
    order = (uint32_t*)(buf + hbytes);
    cst = (uint32_t*)(buf + hbytes + obytes);
  }
#define LAUNCH_B(D, ADD)                                                                          \
  if (split)                                                                                      \
    tlaunch("backward", k_backward<T, D, 1, ADD>, nb, 256, 0, s, g, xs, t, c->rt,                 \
            (const uint16_t*)c->rt_lo, c->kpad, ctl, a, (const double*)c->c4_dev, gm, gv, gx, H,   \
            c->status);                                                                           \
  else                                                                                            \
    tlaunch("backward", k_backward<T, D, 0, ADD>, nb, 256, 0, s, g, xs, t, c->rt,                 \
            (const uint16_t*)nullptr, c->kpad, ctl, a, (const double*)c->c4_dev, gm, gv, gx, H,    \
            c->status);
#define LAUNCH_BA(D)                                                                               \
  if (c->add) {                                                                                    \
    LAUNCH_B(D, true)                                                                              \
  } else {                                                                                         \
    LAUNCH_B(D, false)                                                                             \
  }
  switch (c->d) {
    case 1: LAUNCH_BA(1); break;
    case 2: LAUNCH_BA(2); break;
    case 3: LAUNCH_BA(3); break;
    case 4: LAUNCH_BA(4); break;
  }
#undef LAUNCH_BA
#undef LAUNCH_B
  if (grt) {
    love_status st = sort_points<T>(c, xs, t, order, cst, s);
    if (st == LOVE_OK) {
      const unsigned nbg = (unsigned)cdiv(g.mtot, 256 / WAVE);
#define LAUNCH_G(D)                                                                              \
  if (c->add)                                                                                    \
    tlaunch("grt_gather", k_grt_gather<T, D, true, float, float>, nbg, 256, 0, s, g, xs,         \
            (const uint32_t*)order, (const uint32_t*)cst, (const float*)H, c->kpad, ctl, grt,    \
            (const double*)nullptr, 0.0);                                                        \
  else                                                                                           \
    tlaunch("grt_gather", k_grt_gather<T, D, false, float, float>, nbg, 256, 0, s, g, xs,        \
            (const uint32_t*)order, (const uint32_t*)cst, (const float*)H, c->kpad, ctl, grt,    \
            (const double*)nullptr, 0.0);
      switch (c->d) {
        case 1: LAUNCH_G(1); break;
        case 2: LAUNCH_G(2); break;
        case 3: LAUNCH_G(3); break;
        case 4: LAUNCH_G(4); break;
      }
#undef LAUNCH_G
    }
    ws_free(H, s);
    if (st != LOVE_OK) return st;
  }
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}
template love_status backward<float>(const love_cache*, const float*, int64_t, const float*, const float*, float*, float*, hipStream_t);
template love_status backward<double>(const love_cache*, const double*, int64_t, const double*, const double*, double*, float*, hipStream_t);

// ----------------------------------------------------------------------------
// Posterior samples: out[i, j] = mu_i + f_i . z_j with f_i = S^T w(x*_i)
// (eq. sample, S from eq. pred_covar_ski_interp_form), in two launches:
//   k_sample_f   F = W_{X*} S (t x kspad, float) and mu, 16 lanes per point as
//                for the predictive variances (lane sub: columns sub CPL ..);
//   k_sample_mm  out = mu 1^T + F Z over 64-point x 64-sample tiles, F and Z
//                tiles in LDS, 4 x 4 outputs per thread; the number of
//                factor columns (k_chol) is read on the device.
// ----------------------------------------------------------------------------
template <typename T, int D, int CPL, bool ADD>
__device__ inline void sample_f_body(const GridT<T>& g, const T* __restrict__ xs, int64_t t,
                                     const float* __restrict__ S, int kspad,
                                     const T* __restrict__ acache, float* __restrict__ F,
                                     float* __restrict__ mu_out, unsigned* __restrict__ status,
                                     int64_t lb) {
  const int lane = threadIdx.x & (WAVE - 1), sub = lane & (PLQ - 1);
  const int64_t p = lb * PPB + threadIdx.x / PLQ;
  const bool live = p < t;
  const int64_t pc = live ? p : t - 1;
  double w[D][4], dw[D][4];
  int64_t base;
  int jb[D];
  const bool ok = point_stencil_j<T, D>(g, xs + pc * D, w, dw, jb, base, false);
  constexpr int NA = Entries<D, ADD>::N;
  double f[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) f[q] = 0.0;
  double mu = 0.0;
#pragma unroll 4
  for (int a = 0; a < NA; ++a) {
    double wa;
    int64_t node;
    stn_entry<T, D, ADD>(g, w, base, jb, a, wa, node);
    double r[CPL];
    rt_row<float, 0, CPL>(S, nullptr, node * kspad + sub * CPL, r);
#pragma unroll
    for (int q = 0; q < CPL; ++q) f[q] += wa * r[q];
    if ((a & (PLQ - 1)) == sub && acache) mu += wa * (double)acache[node];
  }
  mu = group_sum(mu, PLQ);
  if (!live) return;
#pragma unroll
  for (int q = 0; q < CPL; q += 4)
    *reinterpret_cast<float4*>(F + p * kspad + sub * CPL + q) =
        make_float4((float)f[q], (float)f[q + 1], (float)f[q + 2], (float)f[q + 3]);
  if (sub == 0) {
    mu_out[p] = ok ? (float)mu : NAN;
    if (!ok) atomicOr(status, SF_DOMAIN);
  }
}
template <typename T, int D, bool ADD>
__global__ __launch_bounds__(256) void k_sample_f(GridT<T> g, const T* __restrict__ xs, int64_t t,
                                                  const float* __restrict__ S, int kspad,
                                                  const T* __restrict__ acache,
                                                  float* __restrict__ F, float* __restrict__ mu,
                                                  unsigned* __restrict__ status) {
  if (kspad > 64)
    sample_f_body<T, D, 128 / PLQ, ADD>(g, xs, t, S, kspad, acache, F, mu, status, blockIdx.x);
  else sample_f_body<T, D, 64 / PLQ, ADD>(g, xs, t, S, kspad, acache, F, mu, status, blockIdx.x);
}

constexpr int SM_T = 64;   // points per output tile
constexpr int SM_J = 64;   // samples per output tile
typedef float f32x16 __attribute__((ext_vector_type(16)));
// out tile = mu 1^T + F_tile Z_tile on the matrix cores: wave w computes the
// 32 x 32 sub-tile (rows 32 (w / 2), columns 32 (w % 2)) with
// v_mfma_f32_32x32x2f32 over the k_chol factor columns, two per instruction
// (lane l supplies F[row l % 32][kk + l / 32] and Z[kk + l / 32][col l % 32];
// its 16 results are rows 8 (i / 4) + 4 (l / 32) + i % 4 of column l % 32).
// The tiles sit in LDS with zero padding past k_chol.
template <typename T>
__global__ __launch_bounds__(256) void k_sample_mm(const float* __restrict__ F,
                                                   const float* __restrict__ mu, int kspad,
                                                   const Ctl* ctl, const float* __restrict__ z,
                                                   int64_t ns, int64_t t, int64_t njt,
                                                   T* __restrict__ out) {
  __shared__ float Fl[SM_T][MAXK + 1];
  __shared__ float Zl[MAXK][SM_J];
  __shared__ float ml[SM_T];
  const int ks = ctl->k_chol;
  const int kk2 = (ks + 1) & ~1;   // k_chol rounded up to the MFMA depth (zero column)
  const int64_t p0 = (int64_t)blockIdx.x * SM_T;
  // tile loads: a fixed number per thread, all issued before any LDS store
  // (a loop with a run-time trip count waits for each load in turn)
  constexpr int NLD = SM_T * MAXK / 256;
  static_assert(SM_J * MAXK / 256 == NLD, "both tiles hold the same number of elements");
  {
    float v[NLD];
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx / MAXK, c = idx % MAXK;
      v[q] = (c < ks && p0 + r < t) ? F[(p0 + r) * kspad + c] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int idx = threadIdx.x + 256 * q;
      Fl[idx / MAXK][idx % MAXK] = v[q];
    }
  }
  if (threadIdx.x < SM_T) ml[threadIdx.x] = p0 + threadIdx.x < t ? mu[p0 + threadIdx.x] : 0.0f;
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int rw = 32 * (w >> 1), cw = 32 * (w & 1);
  const int li = lane & 31, lk = lane >> 5;
  for (int64_t jt = blockIdx.y; jt < njt; jt += gridDim.y) {
    const int64_t j0 = jt * SM_J;
    __syncthreads();
    {
      float v[NLD];
#pragma unroll
      for (int q = 0; q < NLD; ++q) {
        const int idx = threadIdx.x + 256 * q, c = idx / SM_J, jj = idx % SM_J;
        v[q] = (c < ks && j0 + jj < ns) ? z[(int64_t)c * ns + j0 + jj] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < NLD; ++q) {
        const int idx = threadIdx.x + 256 * q;
        Zl[idx / SM_J][idx % SM_J] = v[q];
      }
    }
    __syncthreads();
    f32x16 acc = {};
#pragma unroll 4
    for (int kk = 0; kk < kk2; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(Fl[rw + li][kk + lk], Zl[kk + lk][cw + li], acc,
                                                 0, 0, 0);
    const int64_t j = j0 + cw + li;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = rw + 8 * (i / 4) + 4 * lk + (i % 4);
      const int64_t p = p0 + r;
      if (p < t && j < ns) out[p * ns + j] = (T)(ml[r] + acc[i]);
    }
  }
}

template <typename T>
love_status sample(const love_cache* c, const T* xs, int64_t t, const float* z, int64_t ns, T* out,
                   hipStream_t s, float* scratch) {
  if (t == 0 || ns == 0) return LOVE_OK;
  GridT<T> g = make_grid<T>(c);
  const T* a = (c->cfg.flags & LOVE_FLAG_NO_MEAN) ? nullptr : (const T*)c->a;
  const int kspad = c->kspad;
  float* F = scratch;
  if (!F) F = (float*)ws_alloc(sizeof(float) * (size_t)t * (kspad + 1), s);
  if (!F) return LOVE_ENOMEM;
  float* mu = F + (size_t)t * kspad;
  const unsigned nbf = (unsigned)cdiv(t, PPB);
  switch (c->d) {
#define LAUNCH_SF(D)                                                                              \
  if (c->add)                                                                                     \
    tlaunch("sample_f", k_sample_f<T, D, true>, nbf, 256, 0, s, g, xs, t, (const float*)c->S,     \
            kspad, a, F, mu, c->status);                                                          \
  else                                                                                            \
    tlaunch("sample_f", k_sample_f<T, D, false>, nbf, 256, 0, s, g, xs, t, (const float*)c->S,    \
            kspad, a, F, mu, c->status);
    case 1: LAUNCH_SF(1); break;
    case 2: LAUNCH_SF(2); break;
    case 3: LAUNCH_SF(3); break;
    case 4: LAUNCH_SF(4); break;
#undef LAUNCH_SF
  }
  const int64_t njt = cdiv(ns, SM_J);
  dim3 grid((unsigned)cdiv(t, SM_T), (unsigned)std::min<int64_t>(njt, 65535));
  tlaunch("sample", k_sample_mm<T>, grid, 256, 0, s, (const float*)F, (const float*)mu, kspad,
          (const Ctl*)c->ctl_s, z, ns, t, njt, out);
  if (!scratch) ws_free(F, s);
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}
template love_status sample<float>(const love_cache*, const float*, int64_t, const float*, int64_t, float*, hipStream_t, float*);
template love_status sample<double>(const love_cache*, const double*, int64_t, const float*, int64_t, double*, hipStream_t, float*);

// ----------------------------------------------------------------------------
// Fixed device scratch of the sampling entry point that allocates nothing
// (love_sample_posterior_noalloc): F and mu of the sample path above.  Every
// device the library runs on holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: host code
// uses only the address hipGetSymbolAddress returns for the current device,
// looked up once per device and kept in scratch_dev.
// ----------------------------------------------------------------------------
static __device__ __align__(256) float scratch[LOVE_NOALLOC_SCRATCH_BYTES / sizeof(float)];

static std::mutex scratch_mu;
static std::vector<float*> scratch_dev;   // device ordinal -> address of its copy

static love_status scratch_of_current_device(float** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LOVE_EHIP;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if ((int)scratch_dev.size() <= dev) scratch_dev.resize(dev + 1, nullptr);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LOVE_EHIP;
    scratch_dev[dev] = (float*)p;
  }
  *out = scratch_dev[dev];
  return LOVE_OK;
}

template <typename T>
love_status sample_noalloc(const love_cache* c, const T* xs, int64_t t, const float* z, int64_t ns,
                           T* out, hipStream_t s) {
  const size_t need = sizeof(float) * (size_t)t * (size_t)(c->kspad + 1);
  if (need > (size_t)LOVE_NOALLOC_SCRATCH_BYTES) return LOVE_ELIMIT;
  float* F = nullptr;
  const love_status st = scratch_of_current_device(&F);
  if (st != LOVE_OK) return st;
  return sample<T>(c, xs, t, z, ns, out, s, F);
}
template love_status sample_noalloc<float>(const love_cache*, const float*, int64_t, const float*, int64_t, float*, hipStream_t);
template love_status sample_noalloc<double>(const love_cache*, const double*, int64_t, const float*, int64_t, double*, hipStream_t);


// Rt (m x kpad, stored precision) -> dst (m x keff, float)
template <typename T, int SPLIT>
__global__ void k_rt_export(int64_t m, const void* __restrict__ rt, const uint16_t* __restrict__ rt_lo,
                            int kpad, int keff, float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * keff) return;
  const int64_t u = i / keff, c = i % keff;
  dst[i] = (float)rt_load<T, SPLIT>(rt, rt_lo, u * kpad + c);
}

// Import: Rt (m x keff row-major, float or double) into the cache layout
// (m x kpad, zero columns past keff; bf16 hi + lo for the split), and the
// control blocks of an imported cache.
template <typename T, int SPLIT>
__global__ void k_rt_import(int64_t m, const float* __restrict__ src,
                            const double* __restrict__ src64, int keff, int kpad,
                            void* __restrict__ rt, uint16_t* __restrict__ rt_lo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * kpad) return;
  const int64_t u = i / kpad;
  const int c = (int)(i - u * kpad);
  if constexpr (SPLIT) {
    const float f = c < keff ? src[u * keff + c] : 0.0f;
    const uint16_t hi = f32_to_bf16_rne(f);
    ((uint16_t*)rt)[i] = hi;
    rt_lo[i] = f32_to_bf16_rne(f - bf16_to_f32(hi));
  } else if constexpr (sizeof(T) == 8) {
    ((double*)rt)[i] = c < keff ? src64[u * keff + c] : 0.0;
  } else {
    ((float*)rt)[i] = c < keff ? src[u * keff + c] : 0.0f;
  }
}
__global__ void k_import_ctl(Ctl* ctl, Ctl* ctl_s, double* ortho, int keff, int kchol) {
  Ctl z{};
  z.k_eff = keff;
  z.stop = 1;
  *ctl = z;
  Ctl zs{};
  zs.k_eff = kchol;
  zs.k_chol = kchol;
  zs.stop = 1;
  *ctl_s = zs;
  *ortho = NAN;
}
love_status rt_import(love_cache* c, const float* rt, const double* rt64, int keff, int kchol,
                      hipStream_t s) {
  const int64_t tot = c->m * c->kpad;
  dim3 grid((unsigned)cdiv(tot, 256));
  if (c->fp64)
    k_rt_import<double, 0><<<grid, 256, 0, s>>>(c->m, rt, rt64, keff, c->kpad, c->rt, nullptr);
  else if (c->cfg.precision == LOVE_P_FP32_BF16SPLIT)
    k_rt_import<float, 1><<<grid, 256, 0, s>>>(c->m, rt, rt64, keff, c->kpad, c->rt,
                                               (uint16_t*)c->rt_lo);
  else k_rt_import<float, 0><<<grid, 256, 0, s>>>(c->m, rt, rt64, keff, c->kpad, c->rt, nullptr);
  k_import_ctl<<<1, 1, 0, s>>>(c->ctl, c->ctl_s, c->ortho, keff, kchol);
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}

love_status rt_export_f32(const love_cache* c, float* dst, int keff, hipStream_t s) {
  if (keff <= 0) return LOVE_OK;
  const int64_t tot = c->m * keff;
  dim3 grid((unsigned)cdiv(tot, 256));
  if (c->fp64) k_rt_export<double, 0><<<grid, 256, 0, s>>>(c->m, c->rt, nullptr, c->kpad, keff, dst);
  else if (c->cfg.precision == LOVE_P_FP32_BF16SPLIT)
    k_rt_export<float, 1><<<grid, 256, 0, s>>>(c->m, c->rt, (const uint16_t*)c->rt_lo, c->kpad, keff, dst);
  else k_rt_export<float, 0><<<grid, 256, 0, s>>>(c->m, c->rt, nullptr, c->kpad, keff, dst);
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}

}  // namespace love

namespace love {

// ----------------------------------------------------------------------------
// Gradient of sum_i g_i var(x*_i) with respect to the hyper-parameters
// theta = (lengthscale_0 .. lengthscale_{d-1}, outputscale, sigma^2) through
// the cache.  Every solve Khat^{-1} in the derivative of
// var_i = w_i^T K w_i - w_i^T K W^T Khat^{-1} W K w_i is taken as the cached
// Lanczos solve Q L^{-T} L^{-1} Q^T (eq. lanczos_solve, T = L L^T), so
// z_i = Q L^{-T} u_i with u_i = Rt^T w_i, W^T z_i = B u_i (B = W^T Q L^{-T},
// Rt = K B), and
//   d/dtheta sum_i g_i var_i = sum_i g_i dp_i/dtheta + <dK/dtheta B, Y>_F
//                              + [theta = sigma^2] sum_i g_i ||L^{-T} u_i||^2,
//   Y = B M - 2 P,  M = sum_i g_i u_i u_i^T (k x k),  P = sum_i g_i w_i u_i^T.
// (||z_i||^2 = ||L^{-T} u_i||^2 takes Q^T Q = I.)  -2 P is the backward's
// d var / d Rt; dK/dtheta B is a Kronecker (or block) Toeplitz product with
// the differentiated axis column.  All sums are per-block partials added in
// a fixed order.
// ----------------------------------------------------------------------------
struct HyperPt {
  double t4[MAXD][4];   // first four entries of each unscaled axis column T_e
  double d4[MAXD][4];   // ... of d T_e / d lengthscale_e
  double s;             // outputscale
};

__device__ inline double quad4s(const double (&c)[4], const double (&w)[4]) {
  double q = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) q += w[a] * c[a > b ? a - b : b - a] * w[b];
  return q;
}

// per point: u (double, kpad columns) into U, g_i (0 outside the domain) into
// gw; per block: partial row of sum_i g_i dp_i/dtheta (d + 1 values)
template <typename T, int D, int SPLIT, int CPL, bool ADD>
__device__ inline void hyper_points_body(const GridT<T>& g, const T* __restrict__ xs, int64_t t,
                                         const void* __restrict__ rt,
                                         const uint16_t* __restrict__ rt_lo, int kpad,
                                         const T* __restrict__ gv, HyperPt hp,
                                         double* __restrict__ U, double* __restrict__ gw,
                                         double* __restrict__ dpp) {
  __shared__ double red[PPB][MAXD + 1];
  const int lane = threadIdx.x & (WAVE - 1), sub = lane & (PLQ - 1);
  const int pl = threadIdx.x / PLQ;
  const int64_t p = (int64_t)blockIdx.x * PPB + pl;
  const bool live = p < t;
  const int64_t pc = live ? p : t - 1;
  double w[D][4], dw[D][4];
  int64_t base;
  int jb[D];
  const bool ok = point_stencil_j<T, D>(g, xs + pc * D, w, dw, jb, base, false);
  constexpr int NA = Entries<D, ADD>::N;
  double u[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) u[q] = 0.0;
  for (int a = 0; a < NA; ++a) {
    double wa;
    int64_t node;
    stn_entry<T, D, ADD>(g, w, base, jb, a, wa, node);
    double r[CPL];
    rt_row<T, SPLIT, CPL>(rt, rt_lo, node * kpad + sub * CPL, r);
#pragma unroll
    for (int q = 0; q < CPL; ++q) u[q] += wa * r[q];
  }
  const double gi = (live && ok) ? (double)gv[p] : 0.0;
  if (live) {
#pragma unroll
    for (int q = 0; q < CPL; ++q) U[p * kpad + sub * CPL + q] = ok ? u[q] : 0.0;
    if (sub == 0) gw[p] = gi;
  }
  if (sub == 0) {
    double qd[D], dq[D];
#pragma unroll
    for (int e = 0; e < D; ++e) {
      qd[e] = quad4s(hp.t4[e], w[e]);
      dq[e] = quad4s(hp.d4[e], w[e]);
    }
#pragma unroll
    for (int e = 0; e < D; ++e) {
      double v = hp.s * dq[e];
      if (!ADD) {
#pragma unroll
        for (int f = 0; f < D; ++f)
          if (f != e) v *= qd[f];
      }
      red[pl][e] = gi * v;
    }
    double ps = ADD ? 0.0 : 1.0;
#pragma unroll
    for (int f = 0; f < D; ++f) ps = ADD ? ps + qd[f] : ps * qd[f];
    red[pl][D] = gi * ps;
  }
  __syncthreads();
  if (threadIdx.x <= D) {
    double s = 0.0;
    for (int q = 0; q < PPB; ++q) s += red[q][threadIdx.x];
    dpp[(int64_t)blockIdx.x * (MAXD + 1) + threadIdx.x] = s;
  }
}
template <typename T, int D, int SPLIT, bool ADD>
__global__ __launch_bounds__(256) void k_hyper_points(GridT<T> g, const T* __restrict__ xs,
                                                      int64_t t, const void* __restrict__ rt,
                                                      const uint16_t* __restrict__ rt_lo, int kpad,
                                                      const T* __restrict__ gv, HyperPt hp,
                                                      double* __restrict__ U,
                                                      double* __restrict__ gw,
                                                      double* __restrict__ dpp) {
  if (kpad > 64)
    hyper_points_body<T, D, SPLIT, 128 / PLQ, ADD>(g, xs, t, rt, rt_lo, kpad, gv, hp, U, gw, dpp);
  else
    hyper_points_body<T, D, SPLIT, 64 / PLQ, ADD>(g, xs, t, rt, rt_lo, kpad, gv, hp, U, gw, dpp);
}

// M partial of one chunk of HG_CHUNK points: Mp[chunk][a kpad + b] = sum g_i U_ia U_ib.
// Thread e holds entries e, e + 256, ..; HG_TILE points at a time in LDS.
constexpr int HG_CHUNK = 1024;
constexpr int HG_TILE = 32;
__global__ __launch_bounds__(256) void k_hyper_gram(const double* __restrict__ U,
                                                    const double* __restrict__ gw, int64_t t,
                                                    int kpad, double* __restrict__ Mp) {
  __shared__ double ut[HG_TILE][MAXK];
  __shared__ double gt[HG_TILE];
  constexpr int NE = MAXK * MAXK / 256;
  const int ne = kpad * kpad / 256;
  double acc[NE];
#pragma unroll
  for (int q = 0; q < NE; ++q) acc[q] = 0.0;
  const int64_t p0 = (int64_t)blockIdx.x * HG_CHUNK;
  const int64_t p1 = p0 + HG_CHUNK < t ? p0 + HG_CHUNK : t;
  for (int64_t pb = p0; pb < p1; pb += HG_TILE) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < HG_TILE * kpad; idx += 256) {
      const int r = idx / kpad, cl = idx - r * kpad;
      ut[r][cl] = pb + r < p1 ? U[(pb + r) * kpad + cl] : 0.0;
    }
    if (threadIdx.x < HG_TILE) gt[threadIdx.x] = pb + threadIdx.x < p1 ? gw[pb + threadIdx.x] : 0.0;
    __syncthreads();
    for (int r = 0; r < HG_TILE; ++r) {
      const double gr = gt[r];
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        if (q < ne) {
          const int e = threadIdx.x + 256 * q, a = e / kpad, b = e - a * kpad;
          acc[q] += gr * ut[r][a] * ut[r][b];
        }
      }
    }
  }
  for (int q = 0; q < ne; ++q)
    Mp[(int64_t)blockIdx.x * kpad * kpad + threadIdx.x + 256 * q] = acc[q];
}

// M[e] = sum over chunks of Mp[chunk][e] (chunk order)
__global__ void k_hyper_gram_sum(const double* __restrict__ Mp, int nch, int ne,
                                 double* __restrict__ M) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += Mp[(int64_t)c * ne + e];
  M[e] = s;
}

// Y[node, b] = sum_{a < keff} B[node, a] M[a, b] + P2[node, b] (b < keff; 0 beyond)
template <typename T>
__global__ void k_hyper_y(const T* __restrict__ B, const double* __restrict__ M,
                          const double* __restrict__ P2, const Ctl* __restrict__ ctl, int64_t m,
                          int kpad, double* __restrict__ Y) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * kpad) return;
  const int64_t node = idx / kpad;
  const int b = (int)(idx - node * kpad);
  const int keff = ctl->k_eff;
  double y = 0.0;
  if (b < keff) {
    for (int a = 0; a < keff; ++a) y += (double)B[node * kpad + a] * M[a * kpad + b];
    y += P2[node * keff + b];
  }
  Y[idx] = y;
}

// One axis of a Kronecker (or block) Toeplitz product on m x kpad rows:
// out[node, c] = sum_{|j - i| <= bw} col[|j - i|] in[node + (j - i) stride, c],
// i the node's index along the axis.  Product grids: axis e of the grid.
// Additive grids: only the rows of one block [lo_node, hi_node) (one axis's
// own 1-D grid, stride 1) are formed; the other rows are left as they are.
template <typename TI>
__global__ void k_hyper_axis(const TI* __restrict__ in, double* __restrict__ out, int64_t m,
                             int kpad, int64_t lo_node, int64_t hi_node, int64_t stride, int len,
                             const double* __restrict__ col, int bw) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * kpad) return;
  const int64_t node = idx / kpad;
  const int c = (int)(idx - node * kpad);
  if (node < lo_node || node >= hi_node) return;
  const int i = (int)(((node - lo_node) / stride) % len);
  const int j0 = i - bw > 0 ? i - bw : 0, j1 = i + bw < len - 1 ? i + bw : len - 1;
  double acc = 0.0;
  for (int jj = j0; jj <= j1; ++jj) {
    const int dd = jj > i ? jj - i : i - jj;
    acc += col[dd] * (double)in[(node + (int64_t)(jj - i) * stride) * kpad + c];
  }
  out[idx] = acc;
}

// per-block partials of <a, b> over len values
__global__ void k_hyper_dot(const double* __restrict__ a, const double* __restrict__ b,
                            int64_t len, double* __restrict__ part) {
  const int64_t i0 = (int64_t)blockIdx.x * 256 * 8 + threadIdx.x;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t i = i0 + 256 * q;
    if (i < len) s += a[i] * b[i];
  }
  s = wave_sum(s);
  __shared__ double ws[256 / WAVE];
  if ((threadIdx.x & (WAVE - 1)) == 0) ws[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 256 / WAVE; ++w) t += ws[w];
    part[blockIdx.x] = t;
  }
}

// The combine step, one block: the sums of the point and dot partials, and
// sum_i g_i ||L^{-T} u_i||^2 = sum_c x_c^T M x_c with x_c column c of L^{-1}
// (L from alpha, beta as in the build's Cholesky).  grad: d + 2 values.
__global__ __launch_bounds__(MAXK) void k_hyper_final(
    const double* __restrict__ dpp, int nbp, const double* __restrict__ dotp, int nbd,
    const double* __restrict__ alpha, const double* __restrict__ beta, const Ctl* __restrict__ ctl,
    const double* __restrict__ M, int kpad, double* __restrict__ X, int d, double s,
    double* __restrict__ grad) {
  __shared__ double ld[MAXK], ls[MAXK], qc[MAXK];
  const int k = ctl->k_eff, tid = threadIdx.x;
  if (tid == 0) {
    double prev = 0.0;
    for (int i = 0; i < k; ++i) {
      const double piv = alpha[i] - prev * prev;
      ld[i] = sqrt(piv);
      prev = (i + 1 < k) ? beta[i] / ld[i] : 0.0;
      ls[i] = prev;
    }
  }
  __syncthreads();
  // column tid of L^{-1}: x_tid = 1 / l_tid, x_i = -ls_{i-1} x_{i-1} / ld_i (i > tid)
  if (tid < k) {
    double x = 0.0;
    for (int i = 0; i < k; ++i) {
      x = i < tid ? 0.0 : (i == tid ? 1.0 / ld[i] : -ls[i - 1] * x / ld[i]);
      X[(int64_t)i * kpad + tid] = x;
    }
  }
  __syncthreads();
  double q = 0.0;
  if (tid < k) {
    for (int a = tid; a < k; ++a) {
      double y = 0.0;
      for (int b = tid; b < k; ++b) y += M[a * kpad + b] * X[(int64_t)b * kpad + tid];
      q += X[(int64_t)a * kpad + tid] * y;
    }
  }
  qc[tid] = tid < k ? q : 0.0;
  __syncthreads();
  if (tid == 0) {
    double noise = 0.0;
    for (int c = 0; c < k; ++c) noise += qc[c];
    for (int th = 0; th <= d; ++th) {
      double pt = 0.0, dt = 0.0;
      for (int b = 0; b < nbp; ++b) pt += dpp[(int64_t)b * (MAXD + 1) + th];
      for (int b = 0; b < nbd; ++b) dt += dotp[(int64_t)th * nbd + b];
      grad[th] = pt + (th < d ? s * dt : dt);
    }
    grad[d + 1] = noise;
  }
}

static double kernel_value(int kind, double r, double ell) {
  r = fabs(r);
  if (kind == LOVE_RBF) return exp(-0.5 * (r / ell) * (r / ell));
  const double z = sqrt(5.0) * r / ell;
  return (1.0 + z + z * z / 3.0) * exp(-z);
}
static double kernel_dell(int kind, double r, double ell) {
  r = fabs(r);
  if (kind == LOVE_RBF) return exp(-0.5 * (r / ell) * (r / ell)) * r * r / (ell * ell * ell);
  const double z = sqrt(5.0) * r / ell;
  return z * z * (1.0 + z) * exp(-z) / (3.0 * ell);
}
// largest lag whose coefficient still matters in double (|c| > 1e-17 max|c|)
static int band_of(const std::vector<double>& c) {
  double mx = 0.0;
  for (double v : c) mx = std::max(mx, fabs(v));
  int bw = (int)c.size() - 1;
  while (bw > 0 && !(fabs(c[bw]) > 1e-17 * mx)) --bw;
  return bw;
}

template <typename T>
love_status hyper_grad(const love_cache* c, const T* xs, int64_t t, const T* gv, double* grad,
                       hipStream_t s) {
  const int d = c->d, kpad = c->kpad;
  const int64_t m = c->m;
  const double os = c->cfg.outputscale;
  // host: unscaled axis columns and their lengthscale derivatives
  std::vector<double> cols;
  std::vector<int64_t> coff(2 * d);
  std::vector<int> bws(2 * d);
  HyperPt hp{};
  hp.s = os;
  for (int e = 0; e < d; ++e) {
    const int L = c->mdim[e];
    const double h = 1.0 / c->invh[e], ell = c->cfg.lengthscale[e];
    std::vector<double> tc(L), dc(L);
    for (int i = 0; i < L; ++i) {
      tc[i] = kernel_value(c->cfg.kernel, i * h, ell);
      dc[i] = kernel_dell(c->cfg.kernel, i * h, ell);
    }
    for (int a = 0; a < 4; ++a) {
      hp.t4[e][a] = a < L ? tc[a] : 0.0;
      hp.d4[e][a] = a < L ? dc[a] : 0.0;
    }
    coff[2 * e] = (int64_t)cols.size();
    bws[2 * e] = band_of(tc);
    cols.insert(cols.end(), tc.begin(), tc.end());
    coff[2 * e + 1] = (int64_t)cols.size();
    bws[2 * e + 1] = band_of(dc);
    cols.insert(cols.end(), dc.begin(), dc.end());
  }
  JobArena A;
  const size_t o_cols = A.add(cols);
  love_status st = A.upload(s);
  if (st != LOVE_OK) return st;
  const double* dcols = A.at<double>(o_cols);
  const int64_t tt = t > 0 ? t : 1;
  const int nbp = (int)cdiv(tt, PPB), nch = (int)cdiv(tt, HG_CHUNK);
  const int64_t mk = m * kpad;
  const int nbd = (int)cdiv(mk, 256 * 8);
  // scratch (doubles unless noted)
  const size_t n_u = (size_t)tt * kpad, n_g = tt, n_dpp = (size_t)nbp * (MAXD + 1),
               n_mp = (size_t)nch * kpad * kpad, n_m = (size_t)kpad * kpad,
               n_dot = (size_t)(d + 1) * nbd, n_x = (size_t)kpad * kpad;
  const size_t dbytes = sizeof(double) * (n_u + n_g + n_dpp + n_mp + n_m + 3 * (size_t)mk +
                                          n_dot + n_x);
  const size_t p2bytes = sizeof(double) * (size_t)mk;
  const int64_t nv = c->add ? (int64_t)d * tt : tt;
  const size_t obytes = (sizeof(uint32_t) * (size_t)nv + 255) & ~size_t(255);
  const size_t cbytes = sizeof(uint32_t) * ((size_t)c->ctot + 1);
  if (nv >= (int64_t(1) << 31)) {
    A.release(s);
    return LOVE_EINVAL;
  }
  char* buf = (char*)ws_alloc(dbytes + p2bytes + obytes + cbytes, s);
  if (!buf) {
    A.release(s);
    return LOVE_ENOMEM;
  }
  double* U = (double*)buf;
  double* gw = U + n_u;
  double* dpp = gw + n_g;
  double* Mp = dpp + n_dpp;
  double* M = Mp + n_mp;
  double* Y = M + n_m;
  double* V1 = Y + mk;
  double* V2 = V1 + mk;
  double* dotp = V2 + mk;
  double* X = dotp + n_dot;
  double* P2 = (double*)(buf + dbytes);
  uint32_t* order = (uint32_t*)(buf + dbytes + p2bytes);
  uint32_t* cst = (uint32_t*)(buf + dbytes + p2bytes + obytes);
  const Ctl* ctl = c->ctl;
  GridT<T> g = make_grid<T>(c);
  const bool split = c->cfg.precision == LOVE_P_FP32_BF16SPLIT;
  LOVE_HIP_TRY(hipMemsetAsync(P2, 0, sizeof(double) * (size_t)mk, s));
  if (t > 0) {
#define LAUNCH_HP(D, ADD)                                                                         \
  if (split)                                                                                      \
    tlaunch("hyper_points", k_hyper_points<T, D, 1, ADD>, nbp, 256, 0, s, g, xs, t, c->rt,        \
            (const uint16_t*)c->rt_lo, kpad, gv, hp, U, gw, dpp);                                 \
  else                                                                                            \
    tlaunch("hyper_points", k_hyper_points<T, D, 0, ADD>, nbp, 256, 0, s, g, xs, t, c->rt,        \
            (const uint16_t*)nullptr, kpad, gv, hp, U, gw, dpp);
#define LAUNCH_HPA(D)   \
  if (c->add) {         \
    LAUNCH_HP(D, true)  \
  } else {              \
    LAUNCH_HP(D, false) \
  }
    switch (d) {
      case 1: LAUNCH_HPA(1); break;
      case 2: LAUNCH_HPA(2); break;
      case 3: LAUNCH_HPA(3); break;
      case 4: LAUNCH_HPA(4); break;
    }
#undef LAUNCH_HPA
#undef LAUNCH_HP
    k_hyper_gram<<<nch, 256, 0, s>>>(U, gw, t, kpad, Mp);
    // -2 P = -2 sum_i g_i w_i u_i^T: the backward's deterministic per-node
    // gather over the cell-sorted points, here in double from U and g
    st = sort_points<T>(c, xs, t, order, cst, s);
    if (st != LOVE_OK) {
      ws_free(buf, s);
      A.release(s);
      return st;
    }
    const unsigned nbg = (unsigned)cdiv(m, 256 / WAVE);
#define LAUNCH_G(D)                                                                            \
  if (c->add)                                                                                  \
    k_grt_gather<T, D, true, double, double><<<nbg, 256, 0, s>>>(                              \
        g, xs, (const uint32_t*)order, (const uint32_t*)cst, (const double*)U, kpad, ctl, P2,  \
        (const double*)gw, -2.0);                                                              \
  else                                                                                         \
    k_grt_gather<T, D, false, double, double><<<nbg, 256, 0, s>>>(                             \
        g, xs, (const uint32_t*)order, (const uint32_t*)cst, (const double*)U, kpad, ctl, P2,  \
        (const double*)gw, -2.0);
    switch (d) {
      case 1: LAUNCH_G(1); break;
      case 2: LAUNCH_G(2); break;
      case 3: LAUNCH_G(3); break;
      case 4: LAUNCH_G(4); break;
    }
#undef LAUNCH_G
  } else {
    LOVE_HIP_TRY(hipMemsetAsync(dpp, 0, sizeof(double) * n_dpp, s));
    LOVE_HIP_TRY(hipMemsetAsync(Mp, 0, sizeof(double) * n_mp, s));
  }
  const int ne = kpad * kpad;
  k_hyper_gram_sum<<<(unsigned)cdiv(ne, 256), 256, 0, s>>>(Mp, nch, ne, M);
  const unsigned nbm = (unsigned)cdiv(mk, 256);
  k_hyper_y<T><<<nbm, 256, 0, s>>>((const T*)c->B, M, P2, ctl, m, kpad, Y);
  // <dK/dtheta B, Y> for theta = lengthscale_e (e < d) and the outputscale (e = d)
  for (int th = 0; th <= d; ++th) {
    if (c->add) {
      // block form: theta = lengthscale_e forms block e with d T_e; the
      // outputscale's K / s forms every block with its own T_f
      LOVE_HIP_TRY(hipMemsetAsync(V1, 0, sizeof(double) * (size_t)mk, s));
      for (int f = 0; f < d; ++f) {
        if (th < d && f != th) continue;
        const int use = th < d ? 2 * f + 1 : 2 * f;
        k_hyper_axis<T><<<nbm, 256, 0, s>>>((const T*)c->B, V1, m, kpad, c->aoff[f],
                                            c->aoff[f] + c->mdim[f], 1, c->mdim[f],
                                            dcols + coff[use], bws[use]);
      }
      k_hyper_dot<<<nbd, 256, 0, s>>>(V1, Y, mk, dotp + (size_t)th * nbd);
    } else {
      const double* src = nullptr;   // nullptr: read B
      double* dst = V1;
      int64_t stride = 1;
      std::vector<int64_t> strides(d);
      for (int f = d - 1; f >= 0; --f) {
        strides[f] = stride;
        stride *= c->mdim[f];
      }
      for (int f = 0; f < d; ++f) {
        const int use = (th == f) ? 2 * f + 1 : 2 * f;
        if (src)
          k_hyper_axis<double><<<nbm, 256, 0, s>>>(src, dst, m, kpad, 0, m, strides[f], c->mdim[f],
                                                   dcols + coff[use], bws[use]);
        else
          k_hyper_axis<T><<<nbm, 256, 0, s>>>((const T*)c->B, dst, m, kpad, 0, m, strides[f],
                                              c->mdim[f], dcols + coff[use], bws[use]);
        src = dst;
        dst = (dst == V1) ? V2 : V1;
      }
      k_hyper_dot<<<nbd, 256, 0, s>>>(src, Y, mk, dotp + (size_t)th * nbd);
    }
  }
  k_hyper_final<<<1, MAXK, 0, s>>>(dpp, nbp, dotp, nbd, c->alpha, c->beta, ctl, M, kpad, X, d, os,
                                   grad);
  ws_free(buf, s);
  A.release(s);
  return hipGetLastError() == hipSuccess ? LOVE_OK : LOVE_EHIP;
}
template love_status hyper_grad<float>(const love_cache*, const float*, int64_t, const float*, double*, hipStream_t);
template love_status hyper_grad<double>(const love_cache*, const double*, int64_t, const double*, double*, hipStream_t);

}  // namespace love
