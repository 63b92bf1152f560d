// The KISS-GP operator pieces (Sec. 2.3, eq. ski):
//   W^T v   (grid <- rows)   k_scatter: per-node deterministic gather over the
//                            cell-sorted rows, one wave per grid node
//   K g     (grid -> grid)   Toeplitz / Kronecker-of-Toeplitz product, one pass
//                            per axis; direct register-blocked product or the
//                            circulant-embedding FFT (fft.hip)
//   W u     (rows <- grid)   k_gather: 4^d-point stencil gather per row
// Interpolation weights are recomputed from x on the fly (4d bytes per row
// instead of a stored 20d-byte stencil).
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "internal.h"
#include "ops.h"
#include "toep_dev.h"

namespace love {

template <typename T>
GridT<T> make_grid(const love_cache* c) {
  GridT<T> g{};
  g.d = c->d;
  int64_t ns = 1, cs = 1;
  for (int e = MAXD - 1; e >= 0; --e) {
    if (e >= c->d) {
      g.m[e] = 1;
      g.cells[e] = 1;
      g.nstride[e] = 0;
      g.cstride[e] = 0;
      g.lo[e] = T(0);
      g.hi[e] = T(0);
      g.invh[e] = T(0);
      g.lo_f[e] = 0.f;
      g.invh_f[e] = 0.f;
      continue;
    }
    g.m[e] = c->mdim[e];
    g.cells[e] = c->mdim[e] - 3;
    g.nstride[e] = ns;
    g.cstride[e] = cs;
    ns *= g.m[e];
    cs *= g.cells[e];
    g.lo[e] = (T)c->lo[e];
    g.hi[e] = (T)c->hi[e];
    g.invh[e] = (T)c->invh[e];
    g.lo_f[e] = (float)c->lo[e];
    g.invh_f[e] = (float)c->invh[e];
  }
  g.mtot = ns;
  g.ctot = cs;
  g.cell_f = c->fp64 ? 0 : 1;
  if (c->add) {
    g.add = 1;
    g.mtot = c->m;
    g.ctot = c->ctot;
    for (int e = 0; e < MAXD; ++e) {
      g.aoff[e] = c->aoff[e];
      g.acoff[e] = c->acoff[e];
      g.nstride[e] = 0;
      g.cstride[e] = 0;
    }
    g.aperm = c->perm;
  }
  return g;
}
template GridT<float> make_grid<float>(const love_cache*);
template GridT<double> make_grid<double>(const love_cache*);

// ----------------------------------------------------------------------------
// W^T v: one wave per grid node u.  Rows touching u have cells c with
// c_e in [u_e - 3, u_e] on every axis; along the last axis those cells are
// contiguous, so the rows form 4^(D-1) contiguous runs of the sorted order.
// Lanes are split over the runs; each lane sums its rows, then the wave sums.
// mode bit 4: the gathered vector is v + ratio * v2 (CG direction p = z + ratio p),
// formed on the fly so W^T p is exact for the p the next kernel writes.
// ----------------------------------------------------------------------------
// Sum over rows r = r0, r0 + LPR, ... < re of w_node(x_r) * val_r for one
// lane: rows go in batches of four whose loads (global address space) are
// all issued before any weight is formed, so a lane walking many rows (d > 1)
// overlaps their latencies; rows past re add exact zeros, so the sum equals
// the row-by-row one.
template <typename T, int D, int LPR, bool COMB>
__device__ __forceinline__ T scatter_rows(const GridT<T>& g, const T* x, const T* v, const T* v2,
                                          T ratio, const int (&ue)[D], int32_t r0, int32_t re) {
  using GT = const __attribute__((address_space(1))) T;
  GT* gx = (GT*)x;
  GT* gv = (GT*)v;
  GT* gv2 = (GT*)v2;
  constexpr int UB = 4;
  T acc = T(0);
  for (int32_t rs = r0; rs < re; rs += UB * LPR) {
    T xr[UB][D], vr[UB], v2r[UB];
#pragma unroll
    for (int q = 0; q < UB; ++q) {
      const int64_t r = min(rs + q * LPR, re - 1);
#pragma unroll
      for (int e = 0; e < D; ++e) xr[q][e] = gx[r * D + e];
      vr[q] = gv[r];
      if constexpr (COMB) v2r[q] = gv2[r];
    }
#pragma unroll
    for (int q = 0; q < UB; ++q) {
      T w = T(1);
#pragma unroll
      for (int e = 0; e < D; ++e) {
        T s;
        const int jj = stencil_at(g, e, xr[q][e], s);
        w *= keys_weight_at(ue[e] - jj, s);
      }
      T val = vr[q];
      if constexpr (COMB) val = (T)(vr[q] + ratio * v2r[q]);
      acc += (rs + q * LPR < re) ? w * val : T(0);
    }
  }
  return acc;
}

// Additive composition: node ul of axis e gathers the rows of axis-e cells
// ul - 3 .. ul, listed (by row index) in g.aperm at positions [r0, re); a
// thread's positions go r0, r0 + ST, ... in batches of four whose loads go
// out first.
template <typename T, int D, bool COMB, int ST>
__device__ __forceinline__ T scatter_rows_add(const GridT<T>& g, int e, int ul, const T* x,
                                              const T* v, const T* v2, T ratio, int32_t r0,
                                              int32_t re) {
  using GT = const __attribute__((address_space(1))) T;
  using GI = const __attribute__((address_space(1))) int32_t;
  GT* gx = (GT*)x;
  GT* gv = (GT*)v;
  GT* gv2 = (GT*)v2;
  GI* gp = (GI*)g.aperm;
  constexpr int UB = 4;
  T acc = T(0);
  for (int32_t rs = r0; rs < re; rs += UB * ST) {
    int32_t rr[UB];
#pragma unroll
    for (int q = 0; q < UB; ++q) rr[q] = gp[min(rs + q * ST, re - 1)];
    T xr[UB], vr[UB], v2r[UB];
#pragma unroll
    for (int q = 0; q < UB; ++q) {
      xr[q] = gx[(int64_t)rr[q] * D + e];
      vr[q] = gv[rr[q]];
      if constexpr (COMB) v2r[q] = gv2[rr[q]];
    }
#pragma unroll
    for (int q = 0; q < UB; ++q) {
      T sq;
      const int jj = stencil_at(g, e, xr[q], sq);
      const T w = keys_weight_at(ul - jj, sq);
      T val = vr[q];
      if constexpr (COMB) val = (T)(vr[q] + ratio * v2r[q]);
      acc += (rs + q * ST < re) ? w * val : T(0);
    }
  }
  return acc;
}

// One block of 256 threads per stacked node u (a node's rows are those of
// four cells of its axis, ~4 n / m_e of them); thread sums, then the wave
// sums, then the four waves in order.  mode bits as for k_scatter.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_scatter_add(Tab tab, const ScatterJob<T>* __restrict__ jobs,
                                                     int j, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ScatterJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode)) return;
  const GridT<T>& g = J.g;
  const int64_t u = lb;
  if (u >= g.mtot) return;
  const bool comb = (mode & 4) && J.v2;
  const T ratio = comb ? (T)J.ctl->ratio : T(0);
  int e = 0;
#pragma unroll
  for (int q = 1; q < D; ++q) e = u >= g.aoff[q] ? q : e;
  const int ul = (int)(u - g.aoff[e]);
  const int cl = max(ul - 3, 0), ch = min(ul, g.cells[e] - 1);
  T acc = T(0);
  if (cl <= ch) {
    const int32_t rb = J.cell_start[g.acoff[e] + cl];
    const int32_t re = J.cell_start[g.acoff[e] + ch + 1];
    const T* v = J.v + (int64_t)j * J.v_js;
    const int32_t r0 = rb + (int32_t)threadIdx.x;
    if (comb) acc = scatter_rows_add<T, D, true, 256>(g, e, ul, J.x, v, J.v2, ratio, r0, re);
    else acc = scatter_rows_add<T, D, false, 256>(g, e, ul, J.x, v, J.v2, ratio, r0, re);
  }
  __shared__ T ws[256 / WAVE];
  acc = wave_sum(acc);
  if ((threadIdx.x & (WAVE - 1)) == 0) ws[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T tot = T(0);
#pragma unroll
    for (int w = 0; w < 256 / WAVE; ++w) tot += ws[w];
    J.out[(int64_t)j * J.out_js + u] = tot;
  }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_scatter(Tab tab, const ScatterJob<T>* __restrict__ jobs,
                                                 int j, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ScatterJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode) || J.cellp) return;   // cellp set: the two-stage kernels
  const GridT<T>& g = J.g;
  const T* __restrict__ x = J.x;
  const T* __restrict__ v = J.v + (int64_t)j * J.v_js;
  const T* __restrict__ v2 = J.v2;
  const bool comb = (mode & 4) && v2;
  const T ratio = comb ? (T)J.ctl->ratio : T(0);
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t u = (int64_t)lb * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (u >= g.mtot) return;
  constexpr int RUNS = 1 << (2 * (D - 1));
  constexpr int LPR = WAVE / RUNS;
  const int run = lane / LPR, sub = lane % LPR;
  int ue[D];
  {
    int64_t rem = u;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      ue[e] = (int)(rem / g.nstride[e]);
      rem -= (int64_t)ue[e] * g.nstride[e];
    }
  }
  bool ok = true;
  int64_t cbase = 0;
#pragma unroll
  for (int e = 0; e < D - 1; ++e) {
    const int o = (run >> (2 * (D - 2 - e))) & 3;
    const int ce = ue[e] - o;
    ok = ok && ce >= 0 && ce < g.cells[e];
    cbase += (int64_t)ce * g.cstride[e];
  }
  const int cl = max(ue[D - 1] - 3, 0);
  const int ch = min(ue[D - 1], g.cells[D - 1] - 1);
  ok = ok && cl <= ch;
  T acc = T(0);
  if (ok) {
    const int32_t rb = J.cell_start[cbase + cl];
    const int32_t re = J.cell_start[cbase + ch + 1];
    if (comb) acc = scatter_rows<T, D, LPR, true>(g, x, v, v2, ratio, ue, rb + sub, re);
    else acc = scatter_rows<T, D, LPR, false>(g, x, v, v2, ratio, ue, rb + sub, re);
  }
  acc = wave_sum(acc);
  if (lane == 0) J.out[(int64_t)j * J.out_js + u] = acc;
}

// ----------------------------------------------------------------------------
// W^T v in two stages for d >= 3, where a row touches 4^d >= 64 nodes and a
// cell holds few rows, so visiting every row once per node (above) repeats
// each row 4^d times.  Stage 1, one lane per stencil cell c: the cell's rows
// (contiguous in the sorted order) give the 4^d partial products
//   P[o][c] = sum over rows of val * prod_e w_e[o_e],
// stored offset-major so a wave writes consecutive cells.  Stage 2, one
// thread per node u: out[u] = sum over o of P[o][c(u - o)] for the cells that
// exist, o ascending.  Both summation orders are fixed: deterministic.
// ----------------------------------------------------------------------------
// Two stages for d >= 3, and for d <= 2 once cells hold 64 rows or more on
// average (then stage 1 takes one wave per cell and each row is read once,
// against four times by the one-wave-per-node kernel).
bool scatter_two_stage(const love_cache* c) {
  if (c->add) return false;   // additive: per-axis rows through perm, one wave per node
  return c->d >= 3 || c->n >= 64 * c->ctot;
}
int scatter_kinds(const std::vector<love_cache*>& cs) {
  int k = 0;
  for (auto* c : cs)
    k |= c->add ? SCATTER_ADDITIVE : scatter_two_stage(c) ? SCATTER_TWO_STAGE : SCATTER_NODES;
  return k;
}
// d >= 3: cells in tiles of TC^d, each tile's node partials over its
// (TC + 3)^d extended node box
template <int D>
struct TileShape {
  static constexpr int TC = D == 4 ? 4 : 6;   // cells per axis of a tile
  static constexpr int EXT = TC + 3;          // nodes per axis a tile's cells touch
  static constexpr int NCELL = D == 4 ? 256 : 216;
  static constexpr int NEXT = D == 4 ? 2401 : 729;
};
static int64_t scatter_tiles(const love_cache* c, int tc) {
  int64_t nt = 1;
  for (int e = 0; e < c->d; ++e) nt *= cdiv(c->mdim[e] - 3, tc);
  return nt;
}
size_t scatter_scratch_bytes(const love_cache* c, size_t elem) {
  if (!scatter_two_stage(c)) return 0;
  if (c->d == 4) return (size_t)scatter_tiles(c, TileShape<4>::TC) * TileShape<4>::NEXT * elem;
  if (c->d == 3) return (size_t)scatter_tiles(c, TileShape<3>::TC) * TileShape<3>::NEXT * elem;
  return ((size_t)1 << (2 * c->d)) * (size_t)c->ctot * elem;
}

// Stage 1 for heavy cells (d <= 2): one block of 256 threads per cell (a wave
// per cell left too few, too long waves for an even finish); threads stride
// its rows in batches (loads first), keep the 4^D partial products, and the
// block sums them: a fixed butterfly per wave, then the four waves in order.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_scatter_cells_wave(Tab tab,
                                                            const ScatterJob<T>* __restrict__ jobs,
                                                            int j, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ScatterJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode) || !J.cellp) return;
  const GridT<T>& g = J.g;
  const int64_t c = lb;
  if (c >= g.ctot) return;
  const int lane = threadIdx.x & (WAVE - 1);
  constexpr int NT = 256;
  using GT = const __attribute__((address_space(1))) T;
  GT* gx = (GT*)J.x;
  GT* gv = (GT*)(J.v + (int64_t)j * J.v_js);
  GT* gv2 = (GT*)J.v2;
  const bool comb = (mode & 4) && J.v2;
  const T ratio = comb ? (T)J.ctl->ratio : T(0);
  const int32_t r0 = J.cell_start[c], r1 = J.cell_start[c + 1];
  constexpr int NO = 1 << (2 * D);
  constexpr int UB = D == 1 ? 16 : 8;
  T cb[D];   // stencil base of the cell's rows (fraction = (x - lo) invh - c_e)
  {
    int64_t rem = c;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int64_t ce = rem / g.cstride[e];
      rem -= ce * g.cstride[e];
      cb[e] = (T)ce;
    }
  }
  T acc[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) acc[o] = T(0);
  for (int32_t rs = r0 + (int32_t)threadIdx.x; rs < r1; rs += UB * NT) {
    T xr[UB][D], vr[UB];
#pragma unroll
    for (int q = 0; q < UB; ++q) {
      const int64_t r = min(rs + q * NT, r1 - 1);
#pragma unroll
      for (int e = 0; e < D; ++e) xr[q][e] = gx[r * D + e];
      vr[q] = gv[r];
      if (comb) vr[q] = (T)(vr[q] + ratio * gv2[r]);
    }
#pragma unroll
    for (int q = 0; q < UB; ++q) {
      if (rs + q * NT >= r1) break;
      T w[D][4];
#pragma unroll
      for (int e = 0; e < D; ++e) keys_weights<T>((xr[q][e] - g.lo[e]) * g.invh[e] - cb[e], w[e]);
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        T prod = vr[q];
#pragma unroll
        for (int e = 0; e < D; ++e) prod *= w[e][(o >> (2 * (D - 1 - e))) & 3];
        acc[o] += prod;
      }
    }
  }
  __shared__ T ws[NT / WAVE][NO];
  const int w = threadIdx.x / WAVE;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const T sw = wave_sum(acc[o]);
    if (lane == 0) ws[w][o] = sw;
  }
  __syncthreads();
  if ((int)threadIdx.x < NO) {
    T tot = T(0);
#pragma unroll
    for (int q = 0; q < NT / WAVE; ++q) tot += ws[q][threadIdx.x];
    J.cellp[(int64_t)threadIdx.x * g.ctot + c] = tot;
  }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_scatter_cells(Tab tab,
                                                       const ScatterJob<T>* __restrict__ jobs,
                                                       int j, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ScatterJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode) || !J.cellp) return;
  const GridT<T>& g = J.g;
  const int64_t c = (int64_t)lb * 256 + threadIdx.x;
  if (c >= g.ctot) return;
  const T* __restrict__ x = J.x;
  const T* __restrict__ v = J.v + (int64_t)j * J.v_js;
  const T* __restrict__ v2 = J.v2;
  const bool comb = (mode & 4) && v2;
  const T ratio = comb ? (T)J.ctl->ratio : T(0);
  const int32_t r0 = J.cell_start[c], r1 = J.cell_start[c + 1];
  constexpr int NC = 1 << (2 * (D - 1));   // offsets per value of o_0
  T* __restrict__ P = J.cellp;
  const int64_t ctot = g.ctot;
  // the rows of cell c have stencil base c_e on every axis, so the fraction is
  // (x - lo) invh - c_e, the value stencil_at forms for them
  T cb[D];
  {
    int64_t rem = c;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int64_t ce = rem / g.cstride[e];
      rem -= ce * g.cstride[e];
      cb[e] = (T)ce;
    }
  }
#pragma unroll 1
  for (int o0 = 0; o0 < 4; ++o0) {
    T acc[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q] = T(0);
    for (int32_t r = r0; r < r1; ++r) {
      T w[D][4];
#pragma unroll
      for (int e = 0; e < D; ++e)
        keys_weights<T>((x[(int64_t)r * D + e] - g.lo[e]) * g.invh[e] - cb[e], w[e]);
      T val = v[r];
      if (comb) val = (T)(v[r] + ratio * v2[r]);
      const T a0 = val * w[0][o0];
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        T prod = a0;
#pragma unroll
        for (int e = 1; e < D; ++e) prod *= w[e][(q >> (2 * (D - 1 - e))) & 3];
        acc[q] += prod;
      }
    }
#pragma unroll
    for (int q = 0; q < NC; ++q) P[(int64_t)(o0 * NC + q) * ctot + c] = acc[q];
  }
}

// ----------------------------------------------------------------------------
// W^T v for d >= 3 by tiles: a block takes a tile of TC^d stencil cells and
// forms the tile's contribution to the (TC + 3)^d nodes those cells touch.
// The tile's rows (TC^(d-1) contiguous runs of the cell-sorted order) are
// staged in LDS once.  Then, for a chunk of OC stencil offsets at a time,
// one thread per cell forms P[o][c] = sum over its rows of
// val * prod_e w_e[o_e] into LDS, and each thread adds, for the pencils of
// box nodes along the last axis it owns, P of the cell u - o over the
// chunk's offsets (o ascending), in registers.  The box partials go out once
// per tile (a few MB instead of 4^d x cells values); k_scatter_halo adds,
// per node, the partials of the (at most 2 per axis) tiles whose boxes hold
// it, tiles in order.  Both orders are fixed: deterministic.
// ----------------------------------------------------------------------------
constexpr int ST_RMAX = 1024;   // rows of a tile staged in LDS (more: read from memory)
template <typename T, int D>
__global__ __launch_bounds__(256) void k_scatter_tiles(Tab tab,
                                                       const ScatterJob<T>* __restrict__ jobs,
                                                       int j, int mode) {
  using TS = TileShape<D>;
  constexpr int TC = TS::TC, EXT = TS::EXT, NCELL = TS::NCELL, NEXT = TS::NEXT;
  constexpr int NO = 1 << (2 * D);
  constexpr int OCMAX = 32768 / (NCELL * (int)sizeof(T));
  constexpr int OC = OCMAX >= 64 ? 64 : (OCMAX >= 32 ? 32 : 16);
  static_assert(OC <= NO && NO % OC == 0, "chunks tile the offsets");
  constexpr int NRUN = NCELL / TC;                 // runs of TC cells along the last axis
  constexpr int NPEN = NEXT / EXT;                 // pencils of EXT box nodes along it
  constexpr int PPT = (NPEN + 255) / 256;          // pencils per thread
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ScatterJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode) || !J.cellp) return;
  const GridT<T>& g = J.g;
  int nt[D];
  int64_t ntot = 1;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    nt[e] = (g.cells[e] + TC - 1) / TC;
    ntot *= nt[e];
  }
  const int64_t tile = lb;
  if (tile >= ntot) return;
  int t0[D];   // first cell of the tile per axis
  {
    int64_t rem = tile;
#pragma unroll
    for (int e = D - 1; e >= 0; --e) {
      t0[e] = (int)(rem % nt[e]) * TC;
      rem /= nt[e];
    }
  }
  __shared__ T Pl[OC][NCELL];
  __shared__ T xr[ST_RMAX][D + 1];   // staged rows: coordinates and value
  __shared__ int run_off[NRUN + 1];
  __shared__ int run_row[NRUN];      // first sorted row of each run
  const int tid = threadIdx.x;
  const int ncl = min(TC, g.cells[D - 1] - t0[D - 1]);   // cells of each run inside the grid
  const T* __restrict__ x = J.x;
  const T* __restrict__ v = J.v + (int64_t)j * J.v_js;
  const T* __restrict__ v2 = J.v2;
  const bool comb = (mode & 4) && v2;
  const T ratio = comb ? (T)J.ctl->ratio : T(0);
  // runs: run k = cells (k's first-axes cells, t0 .. t0 + ncl - 1 on the last axis)
  if (tid < NRUN) {
    int rem = tid;
    int64_t c0 = 0;
    bool in = true;
#pragma unroll
    for (int e = D - 2; e >= 0; --e) {
      const int ce = t0[e] + rem % TC;
      rem /= TC;
      in = in && ce < g.cells[e];
      c0 += (int64_t)ce * g.cstride[e];
    }
    c0 += t0[D - 1];
    const int a = in ? J.cell_start[c0] : 0, b = in ? J.cell_start[c0 + ncl] : 0;
    run_row[tid] = a;
    run_off[tid + 1] = b - a;
  }
  __syncthreads();
  if (tid == 0) {
    run_off[0] = 0;
    for (int k = 0; k < NRUN; ++k) run_off[k + 1] += run_off[k];
  }
  __syncthreads();
  const int nrow = run_off[NRUN];
  const bool staged = nrow <= ST_RMAX;
  if (staged) {
    for (int i = tid; i < nrow; i += 256) {
      int lo = 0, hi = NRUN - 1;   // run holding staged row i
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (run_off[mid] <= i) lo = mid;
        else hi = mid - 1;
      }
      const int64_t r = run_row[lo] + (i - run_off[lo]);
#pragma unroll
      for (int e = 0; e < D; ++e) xr[i][e] = x[r * D + e];
      xr[i][D] = comb ? (T)(v[r] + ratio * v2[r]) : v[r];
    }
  }
  // this thread's cell: its rows, staged positions (or sorted rows) [rb, re)
  int cl[D];
  int rb = 0, re = 0;
  int64_t gb = 0;
  if (tid < NCELL) {
    int rem = tid;
#pragma unroll
    for (int e = D - 1; e >= 0; --e) {
      cl[e] = rem % TC;
      rem /= TC;
    }
    const int k = tid / TC;   // run (the last axis is fastest)
    bool in = t0[D - 1] + cl[D - 1] < g.cells[D - 1];
    int64_t cidx = 0;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      in = in && t0[e] + cl[e] < g.cells[e];
      cidx += (int64_t)(t0[e] + cl[e]) * g.cstride[e];
    }
    if (in) {
      const int a = J.cell_start[cidx], b = J.cell_start[cidx + 1];
      gb = a;
      rb = a - run_row[k] + run_off[k];
      re = rb + (b - a);
    }
  }
  T cb[D];
#pragma unroll
  for (int e = 0; e < D; ++e) cb[e] = (T)(t0[e] + (tid < NCELL ? cl[e] : 0));
  // pencils owned: q -> pencil tid + 256 q, box coordinates of its first D-1 axes
  T pacc[PPT][EXT];
#pragma unroll
  for (int q = 0; q < PPT; ++q)
#pragma unroll
    for (int b = 0; b < EXT; ++b) pacc[q][b] = T(0);
  __syncthreads();
  for (int oc0 = 0; oc0 < NO; oc0 += OC) {
    // phase 1: this cell's P[o] for o in [oc0, oc0 + OC)
    if (tid < NCELL) {
      T acc[OC];
#pragma unroll
      for (int q = 0; q < OC; ++q) acc[q] = T(0);
      for (int i = rb; i < re; ++i) {
        T xv[D + 1];
        if (staged) {
#pragma unroll
          for (int e = 0; e <= D; ++e) xv[e] = xr[i][e];
        } else {
          const int64_t r = gb + (i - rb);
#pragma unroll
          for (int e = 0; e < D; ++e) xv[e] = x[r * D + e];
          xv[D] = comb ? (T)(v[r] + ratio * v2[r]) : v[r];
        }
        T w[D][4];
#pragma unroll
        for (int e = 0; e < D; ++e) keys_weights<T>((xv[e] - g.lo[e]) * g.invh[e] - cb[e], w[e]);
#pragma unroll
        for (int q = 0; q < OC; ++q) {
          const int o = oc0 + q;
          T prod = xv[D];
#pragma unroll
          for (int e = 0; e < D; ++e) prod *= w[e][(o >> (2 * (D - 1 - e))) & 3];
          acc[q] += prod;
        }
      }
#pragma unroll
      for (int q = 0; q < OC; ++q) Pl[q][tid] = acc[q];
    }
    __syncthreads();
    // phase 2: each owned pencil (box coordinates b_0 .. b_{D-2}, all EXT of
    // b_{D-1}) adds P[o][cell b - o]; the chunk fixes or ranges the leading
    // offset digits, the last digit runs over 0..3 (OC >= 16)
    int dlo[D - 1], dhi[D - 1];
#pragma unroll
    for (int e = 0; e < D - 1; ++e) {
      const int p4 = 1 << (2 * (D - 1 - e));
      if (OC >= 4 * p4) {
        dlo[e] = 0;
        dhi[e] = 3;
      } else if (OC >= p4) {
        dlo[e] = (oc0 / p4) & 3;
        dhi[e] = dlo[e] + OC / p4 - 1;
      } else {
        dlo[e] = dhi[e] = (oc0 / p4) & 3;
      }
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int pen = tid + 256 * q;
      if (pen >= NPEN) break;
      int bl[D - 1];
      {
        int rem = pen;
#pragma unroll
        for (int e = D - 2; e >= 0; --e) {
          bl[e] = rem % EXT;
          rem /= EXT;
        }
      }
      int lo[D - 1], hi[D - 1];
#pragma unroll
      for (int e = 0; e < D - 1; ++e) {
        lo[e] = max(dlo[e], bl[e] - TC + 1);
        hi[e] = min(dhi[e], bl[e]);
      }
      if constexpr (D == 4) {
        for (int d0 = lo[0]; d0 <= hi[0]; ++d0)
          for (int d1 = lo[1]; d1 <= hi[1]; ++d1)
            for (int d2 = lo[2]; d2 <= hi[2]; ++d2) {
              const int qo = d0 * 64 + d1 * 16 + d2 * 4 - oc0;
              const int cb3 = (((bl[0] - d0) * TC + (bl[1] - d1)) * TC + (bl[2] - d2)) * TC;
#pragma unroll
              for (int d3 = 0; d3 < 4; ++d3)
#pragma unroll
                for (int c3 = 0; c3 < TC; ++c3) pacc[q][c3 + d3] += Pl[qo + d3][cb3 + c3];
            }
      } else {
        for (int d0 = lo[0]; d0 <= hi[0]; ++d0)
          for (int d1 = lo[1]; d1 <= hi[1]; ++d1) {
            const int qo = d0 * 16 + d1 * 4 - oc0;
            const int cb2 = ((bl[0] - d0) * TC + (bl[1] - d1)) * TC;
#pragma unroll
            for (int d2 = 0; d2 < 4; ++d2)
#pragma unroll
              for (int c2 = 0; c2 < TC; ++c2) pacc[q][c2 + d2] += Pl[qo + d2][cb2 + c2];
          }
      }
    }
    __syncthreads();
  }
  T* __restrict__ NP = J.cellp + tile * NEXT;
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pen = tid + 256 * q;
    if (pen >= NPEN) break;
#pragma unroll
    for (int b = 0; b < EXT; ++b) NP[pen * EXT + b] = pacc[q][b];
  }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_scatter_halo(Tab tab,
                                                      const ScatterJob<T>* __restrict__ jobs,
                                                      int j, int mode) {
  using TS = TileShape<D>;
  constexpr int TC = TS::TC, EXT = TS::EXT, NEXT = TS::NEXT;
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ScatterJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode) || !J.cellp) return;
  const GridT<T>& g = J.g;
  const int64_t u = (int64_t)lb * 256 + threadIdx.x;
  if (u >= g.mtot) return;
  int ue[D], nt[D], tlo[D], thi[D];
  {
    int64_t rem = u;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      ue[e] = (int)(rem / g.nstride[e]);
      rem -= (int64_t)ue[e] * g.nstride[e];
    }
  }
#pragma unroll
  for (int e = 0; e < D; ++e) {
    nt[e] = (g.cells[e] + TC - 1) / TC;
    // tiles t with t TC <= ue < t TC + EXT
    int lo = ue[e] - EXT + 1 > 0 ? (ue[e] - EXT + 1 + TC - 1) / TC : 0;
    int hi = ue[e] / TC;
    hi = hi < nt[e] - 1 ? hi : nt[e] - 1;
    tlo[e] = lo;
    thi[e] = hi;
  }
  const T* __restrict__ NP = J.cellp;
  T acc = T(0);
  // up to 2^D tiles, in lexicographic order
  for (int a = 0; a < (1 << D); ++a) {
    int64_t tflat = 0;
    int bflat = 0;
    bool ok = true;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int te = tlo[e] + ((a >> (D - 1 - e)) & 1);
      ok = ok && te <= thi[e];
      tflat = tflat * nt[e] + te;
      bflat = bflat * EXT + (ue[e] - te * TC);
    }
    if (ok) acc += NP[tflat * NEXT + bflat];
  }
  J.out[(int64_t)j * J.out_js + u] = acc;
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_scatter_nodes(Tab tab,
                                                       const ScatterJob<T>* __restrict__ jobs,
                                                       int j, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ScatterJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode) || !J.cellp) return;
  const GridT<T>& g = J.g;
  const int64_t u = (int64_t)lb * 256 + threadIdx.x;
  if (u >= g.mtot) return;
  int ue[D];
  {
    int64_t rem = u;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      ue[e] = (int)(rem / g.nstride[e]);
      rem -= (int64_t)ue[e] * g.nstride[e];
    }
  }
  constexpr int NO = 1 << (2 * D);
  const T* __restrict__ P = J.cellp;
  const int64_t ctot = g.ctot;
  T acc = T(0);
#pragma unroll 16
  for (int o = 0; o < NO; ++o) {
    int64_t cidx = 0;
    bool ok = true;
#pragma unroll
    for (int e = 0; e < D; ++e) {
      const int ce = ue[e] - ((o >> (2 * (D - 1 - e))) & 3);
      ok = ok && ce >= 0 && ce < g.cells[e];
      cidx += (int64_t)ce * g.cstride[e];
    }
    acc += ok ? P[(int64_t)o * ctot + cidx] : T(0);
  }
  J.out[(int64_t)j * J.out_js + u] = acc;
}

// tab: cdiv(m, 4) blocks per GP (one wave per node).  A job with cellp set
// takes the two stages, the others the one-wave-per-node kernel; `kinds`
// (SCATTER_*) says which launches the batch needs, and each kernel skips the
// other kind's jobs.  The block-per-cell stage 1 (d <= 2) and the additive
// kernel (block per node) take 4 blocks per tab block (covering ctot < m and
// m); the lane-per-cell stage 1 (d >= 3) and stage 2 take cdiv(4 * blocks,
// 256) blocks per GP, which covers both nodes and cells.
template <typename T>
void launch_scatter(const Tab& tab, const ScatterJob<T>* jobs, int d, int j, int mode,
                    hipStream_t s, int kinds) {
  const unsigned nb = tab_blocks(tab);
  if (nb == 0) return;
  if (kinds & SCATTER_TWO_STAGE) {
    std::vector<int64_t> b(tab.G);
    for (int g = 0; g < tab.G; ++g) b[g] = cdiv(tab.off[g + 1] - tab.off[g], 64);
    const Tab t2 = make_tab(b);
    const unsigned n2 = tab_blocks(t2);
    // heavy-cell stage 1 (d <= 2): one block per cell; 4 blocks per node block
    // of the tab covers ctot < m cells
    std::vector<int64_t> bc(tab.G);
    for (int g = 0; g < tab.G; ++g) bc[g] = 4 * (tab.off[g + 1] - tab.off[g]);
    const Tab tc = make_tab(bc);
    const unsigned nc = tab_blocks(tc);
    switch (d) {
      case 1:
        tlaunch("scatter_cells", k_scatter_cells_wave<T, 1>, nc, 256, 0, s, tc, jobs, j, mode);
        tlaunch("scatter", k_scatter_nodes<T, 1>, n2, 256, 0, s, t2, jobs, j, mode);
        break;
      case 2:
        tlaunch("scatter_cells", k_scatter_cells_wave<T, 2>, nc, 256, 0, s, tc, jobs, j, mode);
        tlaunch("scatter", k_scatter_nodes<T, 2>, n2, 256, 0, s, t2, jobs, j, mode);
        break;
      case 3: {
        // tiles of 6^3 cells: at most cdiv(m, 64) per GP (ceil((m_e - 3) / 6) <= m_e / 4)
        std::vector<int64_t> bt(tab.G);
        for (int g = 0; g < tab.G; ++g) bt[g] = cdiv(4 * (tab.off[g + 1] - tab.off[g]), 64);
        const Tab tt = make_tab(bt);
        tlaunch("scatter_cells", k_scatter_tiles<T, 3>, tab_blocks(tt), 256, 0, s, tt, jobs, j,
                mode);
        tlaunch("scatter", k_scatter_halo<T, 3>, n2, 256, 0, s, t2, jobs, j, mode);
        break;
      }
      default:
        // tiles of 4^4 cells: at most cdiv(m, 256) per GP (ceil((m_e - 3) / 4) <= m_e / 4)
        tlaunch("scatter_cells", k_scatter_tiles<T, 4>, n2, 256, 0, s, t2, jobs, j, mode);
        tlaunch("scatter", k_scatter_halo<T, 4>, n2, 256, 0, s, t2, jobs, j, mode);
        break;
    }
  }
  if (kinds & SCATTER_ADDITIVE) {
    // a batch agrees on the composition: every job is additive; one block per node
    std::vector<int64_t> b(tab.G);
    for (int g = 0; g < tab.G; ++g) b[g] = 4 * (tab.off[g + 1] - tab.off[g]);
    const Tab ta = make_tab(b);
    const unsigned na = tab_blocks(ta);
    switch (d) {
      case 1: tlaunch("scatter", k_scatter_add<T, 1>, na, 256, 0, s, ta, jobs, j, mode); break;
      case 2: tlaunch("scatter", k_scatter_add<T, 2>, na, 256, 0, s, ta, jobs, j, mode); break;
      case 3: tlaunch("scatter", k_scatter_add<T, 3>, na, 256, 0, s, ta, jobs, j, mode); break;
      case 4: tlaunch("scatter", k_scatter_add<T, 4>, na, 256, 0, s, ta, jobs, j, mode); break;
    }
    return;
  }
  if (!(kinds & SCATTER_NODES) || d >= 3) return;
  switch (d) {
    case 1: tlaunch("scatter", k_scatter<T, 1>, nb, 256, 0, s, tab, jobs, j, mode); break;
    case 2: tlaunch("scatter", k_scatter<T, 2>, nb, 256, 0, s, tab, jobs, j, mode); break;
  }
}
template void launch_scatter<float>(const Tab&, const ScatterJob<float>*, int, int, int, hipStream_t,
                                    int);
template void launch_scatter<double>(const Tab&, const ScatterJob<double>*, int, int, int,
                                     hipStream_t, int);

// ----------------------------------------------------------------------------
// W u (+ sigma^2 v): GR sorted rows per thread (rows lb 256 GR + t + 256 q),
// all of whose x and v loads are issued before any stencil is formed.
// ----------------------------------------------------------------------------
constexpr int GR = 8;
template <typename T, int D>
__global__ __launch_bounds__(256) void k_gather(Tab tab, const GatherJob<T>* __restrict__ jobs,
                                                int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const GatherJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode)) return;
  const int64_t r0 = (int64_t)lb * 256 * GR + threadIdx.x;
  const T* __restrict__ x = J.x;
  const T* __restrict__ vs = J.vsig;
  T xr[GR][D], vv[GR];
#pragma unroll
  for (int q = 0; q < GR; ++q) {
    const int64_t r = min(r0 + 256 * q, J.n - 1);
#pragma unroll
    for (int e = 0; e < D; ++e) xr[q][e] = x[r * D + e];
    vv[q] = vs ? vs[r] : T(0);
  }
#pragma unroll
  for (int q = 0; q < GR; ++q) {
    const int64_t r = r0 + 256 * q;
    if (r >= J.n) break;
    J.out[r] = gather_row_vals<T, D>(J.g, xr[q], J.kg) + J.sigma2 * vv[q];
  }
}

// tab: cdiv(n, 256) blocks per GP; the kernel takes 256 GR rows per block.
template <typename T>
void launch_gather(const Tab& tab, const GatherJob<T>* jobs, int d, int mode, hipStream_t s) {
  if (tab_blocks(tab) == 0) return;
  std::vector<int64_t> b(tab.G);
  for (int g = 0; g < tab.G; ++g) b[g] = cdiv(tab.off[g + 1] - tab.off[g], GR);
  const Tab t2 = make_tab(b);
  const unsigned nb = tab_blocks(t2);
  switch (d) {
    case 1: tlaunch("gather", k_gather<T, 1>, nb, 256, 0, s, t2, jobs, mode); break;
    case 2: tlaunch("gather", k_gather<T, 2>, nb, 256, 0, s, t2, jobs, mode); break;
    case 3: tlaunch("gather", k_gather<T, 3>, nb, 256, 0, s, t2, jobs, mode); break;
    case 4: tlaunch("gather", k_gather<T, 4>, nb, 256, 0, s, t2, jobs, mode); break;
  }
}
template void launch_gather<float>(const Tab&, const GatherJob<float>*, int, int, hipStream_t);
template void launch_gather<double>(const Tab&, const GatherJob<double>*, int, int, hipStream_t);

template <typename TI, typename TO>
__global__ void k_convert(const TI* __restrict__ in, TO* __restrict__ out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (TO)in[i];
}
template <typename TI, typename TO>
void launch_convert(const TI* in, TO* out, int64_t n, hipStream_t s) {
  if (n > 0) k_convert<TI, TO><<<cdiv(n, 256), 256, 0, s>>>(in, out, n);
}
template void launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template void launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_convert<double, double>(const double*, double*, int64_t, hipStream_t);

// Direct Toeplitz product along a contiguous axis (long lines): toep_dev.h.
template <typename T>
__global__ __launch_bounds__(TB_WAVES * WAVE) void k_toep_band(Tab tab,
                                                               const ToepJob<T>* __restrict__ jobs,
                                                               int j, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ToepJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode)) return;
  toep_band_block<T>(J, lb, j);
}

template <typename T>
__global__ __launch_bounds__(TB_RED) void k_toep_reduce(Tab tab, const ToepJob<T>* __restrict__ jobs,
                                                        int j, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ToepJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode)) return;
  toep_reduce_block<T>(J, lb, j);
}

// Direct Toeplitz product for short / strided axes: a block owns 64
// consecutive lines (one per lane) and the whole axis (L <= TOEP_LINES_MAXL),
// staged in LDS as tile[j][lane]; wave w computes outputs i = w, w+4, ...
// L <= 256 keeps the double tile (256 x 64 x 8 B = 128 KB) inside the 160 KB LDS.
constexpr int TOEP_LINES_MAXL = 256;

template <typename T>
__global__ __launch_bounds__(256) void k_toep_lines(Tab tab, const ToepJob<T>* __restrict__ jobs,
                                                    int j, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ToepJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode)) return;
  extern __shared__ unsigned char smem_raw[];
  const int L = J.L;
  const int64_t inner = J.inner, nlines = J.outer * J.inner;
  T* tile = (T*)smem_raw;            // L x 64
  T* cl = tile + (int64_t)L * WAVE;  // L
  const T* in = J.in + (int64_t)j * J.in_js;
  const int64_t line0 = (int64_t)lb * WAVE;
  for (int idx = threadIdx.x; idx < L * WAVE; idx += 256) {
    const int i = idx / WAVE, ln = idx % WAVE;
    const int64_t line = line0 + ln;
    T v = T(0);
    if (line < nlines) {
      const int64_t o = line / inner, r = line % inner;
      v = in[o * L * inner + r + (int64_t)i * inner];
    }
    tile[idx] = v;
  }
  for (int i = threadIdx.x; i < L; i += 256) cl[i] = J.c[i];
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int64_t line = line0 + lane;
  if (line >= nlines) return;
  const int64_t o = line / inner, r = line % inner;
  T* dst = J.out + (int64_t)j * J.out_js + o * L * inner + r;
  for (int i = w; i < L; i += 4) {
    T acc = T(0);
    for (int q = 0; q < L; ++q) acc += cl[i > q ? i - q : q - i] * tile[q * WAVE + lane];
    dst[(int64_t)i * inner] = J.scale * acc;
  }
}

template <typename T>
void launch_fft_conv(const Tab& tab, const ToepJob<T>* jobs, size_t smem, int j, int mode,
                     hipStream_t s);

int64_t toeplitz_scratch_elems(const love_cache* c) { return (2 + TB_NSEG_MAX) * c->m; }

void toeplitz_set_attrs() {
  static bool done = false;
  if (done) return;
  done = true;
  (void)hipFuncSetAttribute((const void*)k_toep_lines<float>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
  (void)hipFuncSetAttribute((const void*)k_toep_lines<double>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
}

// Backend of one axis at working precision T: 0 band, 1 lines, 2 fft.
static int axis_backend(const ToepAxis& ax) {
  if (ax.mode == LOVE_TOEPLITZ_FFT) return 2;
  return (ax.inner == 1 && ax.L > TOEP_LINES_MAXL) ? 0 : 1;
}

template <typename T>
void toep_prepare(JobArena& A, ToepRun<T>& run, const std::vector<love_cache*>& cs,
                  const std::vector<const T*>& in, const std::vector<int64_t>& in_js,
                  const std::vector<T*>& out, const std::vector<int64_t>& out_js,
                  const std::vector<T*>& scratch, const std::vector<const Ctl*>& ctl) {
  const int G = (int)cs.size();
  const int d = cs[0]->d;
  const bool add = cs[0]->add;   // a batch agrees on the composition
  // One job: axis e of GP g at pass `step`, with its block counts per backend.
  // Products: axes applied last-to-first, intermediate results ping-pong
  // through the scratch halves.  Additive: axis e maps its own block of in to
  // the same block of out, with its own slice of the segment scratch.
  struct Counts {
    int64_t band = 0, red = 0, lines = 0, fft = 0;
    size_t smem_lines = 0, smem_fft = 0;
  };
  auto make_job = [&](int g, int e, int step, Counts& n) {
    const love_cache* c = cs[g];
    const ToepAxis& ax = c->toep.ax[e];
    ToepJob<T> J{};
    T* buf0 = scratch[g];
    T* buf1 = scratch[g] + c->m;
    const bool first = add || (e == d - 1), last = add || (e == 0);
    const int64_t off = add ? c->aoff[e] : 0;
    J.in = first ? in[g] + off : ((step - 1) % 2 == 0 ? buf0 : buf1);
    J.in_js = first ? in_js[g] : 0;
    J.out = last ? out[g] + off : (step % 2 == 0 ? buf0 : buf1);
    J.out_js = last ? out_js[g] : 0;
    J.c = (const T*)(sizeof(T) == 8 ? ax.c64 : ax.c32);
    J.spec = (const T*)(sizeof(T) == 8 ? ax.spec64 : ax.spec32);
    J.partial = scratch[g] + 2 * c->m + (int64_t)TB_NSEG_MAX * off;
    J.L = ax.L;
    J.bw = sizeof(T) == 8 ? ax.bw64 : ax.bw32;
    J.inner = ax.inner;
    J.outer = ax.outer;
    J.scale = T(1);
    J.ctl = ctl[g];
    const int be = axis_backend(ax);
    if (be == 0) {
      const int ntiles = (int)cdiv(ax.L, TB_OUT);
      const int band = std::min(ax.L, TB_OUT + 2 * J.bw);
      // segments: enough blocks to cover the chip (~512), each at least 256 inputs
      int nseg = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(512, ntiles * ax.outer),
                                                             cdiv(band, 256)));
      nseg = std::max(nseg, (int)cdiv(band, TB_SEG));
      nseg = std::min(nseg, TB_NSEG_MAX);
      J.ntiles = ntiles;
      J.nseg = nseg;
      J.seglen = (int)cdiv(band, nseg);
      n.band = (int64_t)ntiles * nseg * ax.outer;
      if (nseg > 1) n.red = cdiv((int64_t)ax.L * ax.outer, TB_RED);
    } else if (be == 1) {
      n.lines = cdiv(ax.outer * ax.inner, WAVE);
      n.smem_lines = sizeof(T) * ((size_t)ax.L * WAVE + ax.L);
    } else {
      int N = ax.fft_n, logN = 0;
      while ((1 << logN) < N) ++logN;
      J.N = N;
      J.logN = logN;
      n.fft = cdiv(ax.outer * ax.inner, 2);
      n.smem_fft = sizeof(T) * 2 * (size_t)N;
    }
    return J;
  };
  auto store = [&](int step, const std::vector<ToepJob<T>>& jobs, const std::vector<Counts>& n) {
    std::vector<int64_t> nband, nred, nlines, nfft;
    size_t sl = 0, sf = 0;
    for (const Counts& q : n) {
      nband.push_back(q.band);
      nred.push_back(q.red);
      nlines.push_back(q.lines);
      nfft.push_back(q.fft);
      sl = std::max(sl, q.smem_lines);
      sf = std::max(sf, q.smem_fft);
    }
    auto& A_ = run.ax[step];
    A_.jobs = A.add(jobs);
    A_.band = make_tab(nband);
    A_.reduce = make_tab(nred);
    A_.lines = make_tab(nlines);
    A_.fft = make_tab(nfft);
    A_.smem_lines = sl;
    A_.smem_fft = sf;
    A_.nseg0 = jobs.empty() ? 0 : jobs[0].nseg;
    A_.L0 = jobs.empty() ? 0 : jobs[0].L;
    A_.partial0 = jobs.empty() ? nullptr : jobs[0].partial;
  };
  if (add && (int64_t)G * d <= MAXG) {
    // additive: the d independent blocks of every GP in one pass (one launch
    // per backend), job g d + e
    run.d = 1;
    run.jpg = d;
    std::vector<ToepJob<T>> jobs(G * d);
    std::vector<Counts> n(G * d);
    for (int g = 0; g < G; ++g)
      for (int e = 0; e < d; ++e) jobs[g * d + e] = make_job(g, e, 0, n[g * d + e]);
    store(0, jobs, n);
    return;
  }
  run.d = d;
  run.jpg = 1;
  for (int e = d - 1, step = 0; e >= 0; --e, ++step) {
    std::vector<ToepJob<T>> jobs(G);
    std::vector<Counts> n(G);
    for (int g = 0; g < G; ++g) jobs[g] = make_job(g, e, step, n[g]);
    store(step, jobs, n);
  }
}

template <typename T>
void toep_run(const JobArena& A, const ToepRun<T>& run, int j, int mode, hipStream_t s) {
  ProfScope ps("toeplitz", s);
  for (int step = 0; step < run.d; ++step) {
    const auto& ax = run.ax[step];
    const ToepJob<T>* jobs = A.at<ToepJob<T>>(ax.jobs);
    if (tab_blocks(ax.band))
      tlaunch(sizeof(T) == 8 ? "toep_band64" : "toep_band", k_toep_band<T>, tab_blocks(ax.band),
              TB_WAVES * WAVE, 0, s, ax.band, jobs, j, mode);
    if (tab_blocks(ax.reduce))
      tlaunch(sizeof(T) == 8 ? "toep_reduce64" : "toep_reduce", k_toep_reduce<T>,
              tab_blocks(ax.reduce), TB_RED, 0, s, ax.reduce, jobs, j, mode);
    if (tab_blocks(ax.lines))
      k_toep_lines<T><<<tab_blocks(ax.lines), 256, ax.smem_lines, s>>>(ax.lines, jobs, j, mode);
    if (tab_blocks(ax.fft)) launch_fft_conv<T>(ax.fft, jobs, ax.smem_fft, j, mode, s);
  }
}

template void toep_prepare<float>(JobArena&, ToepRun<float>&, const std::vector<love_cache*>&,
                                  const std::vector<const float*>&, const std::vector<int64_t>&,
                                  const std::vector<float*>&, const std::vector<int64_t>&,
                                  const std::vector<float*>&, const std::vector<const Ctl*>&);
template void toep_prepare<double>(JobArena&, ToepRun<double>&, const std::vector<love_cache*>&,
                                   const std::vector<const double*>&, const std::vector<int64_t>&,
                                   const std::vector<double*>&, const std::vector<int64_t>&,
                                   const std::vector<double*>&, const std::vector<const Ctl*>&);
template void toep_run<float>(const JobArena&, const ToepRun<float>&, int, int, hipStream_t);
template void toep_run<double>(const JobArena&, const ToepRun<double>&, int, int, hipStream_t);

// ----------------------------------------------------------------------------
// Small helpers
// ----------------------------------------------------------------------------
template <typename T>
__global__ void k_fill_b(Tab tab, const FillJob<T>* __restrict__ jobs) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const FillJob<T>& J = jobs[gp];
  const int64_t i = (int64_t)lb * blockDim.x + threadIdx.x;
  if (i < J.n) J.p[i] = J.val;
}
template <typename T>
void launch_fill(const Tab& tab, const FillJob<T>* jobs, hipStream_t s) {
  if (tab_blocks(tab)) k_fill_b<T><<<tab_blocks(tab), 256, 0, s>>>(tab, jobs);
}
template void launch_fill<float>(const Tab&, const FillJob<float>*, hipStream_t);
template void launch_fill<double>(const Tab&, const FillJob<double>*, hipStream_t);

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill<T><<<cdiv(n, 256), 256, 0, s>>>(p, v, n);
}
template void launch_fill<float>(float*, float, int64_t, hipStream_t);
template void launch_fill<double>(double*, double, int64_t, hipStream_t);
template void launch_fill<unsigned>(unsigned*, unsigned, int64_t, hipStream_t);

template <typename T>
__global__ void k_permute(const T* __restrict__ in, T* __restrict__ out,
                          const int32_t* __restrict__ perm, int64_t n, int inverse) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (inverse) out[perm[p]] = in[p];   // sorted -> caller order
  else out[p] = in[perm[p]];           // caller -> sorted order
}
template <typename T>
void launch_permute(const T* in, T* out, const int32_t* perm, int64_t n, int inverse, hipStream_t s) {
  k_permute<T><<<cdiv(n, 256), 256, 0, s>>>(in, out, perm, n, inverse);
}
template void launch_permute<float>(const float*, float*, const int32_t*, int64_t, int, hipStream_t);
template void launch_permute<double>(const double*, double*, const int32_t*, int64_t, int, hipStream_t);

// ----------------------------------------------------------------------------
// Plan: first columns of the per-axis Toeplitz factors and the backend choice.
// ----------------------------------------------------------------------------
static double kern1d(int kind, double r, double ell) {
  r = std::fabs(r);
  if (kind == LOVE_MATERN52) {
    const double z = std::sqrt(5.0) * r / ell;
    return (1.0 + z + z * z / 3.0) * std::exp(-z);
  }
  const double q = r / ell;
  return std::exp(-0.5 * q * q);
}

love_status fft_plan_axis(love_cache* c, ToepAxis& ax, int e, const std::vector<double>& col);
int autotune_choose(love_cache* c, int e);

// The same columns evaluated on the device (no host-to-device copies in the
// build): c64 in double, c32 rounded from it, and c4 = the first four
// entries of every axis (1 for axes past d).
struct CoefAxis {
  double* c64;
  float* c32;
  int L;
  double h, ell, scale;
};
struct CoefJob {
  CoefAxis ax[MAXD];
  int d, kind;
  double* c4;
};
__device__ inline double kern1d_dev(int kind, double r, double ell) {
  r = fabs(r);
  if (kind == LOVE_MATERN52) {
    const double z = sqrt(5.0) * r / ell;
    return (1.0 + z + z * z / 3.0) * exp(-z);
  }
  const double q = r / ell;
  return exp(-0.5 * q * q);
}
__global__ void k_toep_coef(CoefJob J) {
  const int e = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J.d) {
    if (i < 4) J.c4[4 * e + i] = 1.0;
    return;
  }
  const CoefAxis& A = J.ax[e];
  if (i >= A.L) return;
  const double v = kern1d_dev(J.kind, i * A.h, A.ell) * A.scale;
  A.c64[i] = v;
  A.c32[i] = (float)v;
  if (i < 4) J.c4[4 * e + i] = v;
}

love_status toeplitz_plan(love_cache* c) {
  toeplitz_set_attrs();
  ToepPlan& p = c->toep;
  p.d = c->d;
  p.mtot = c->m;
  CoefJob cj{};
  cj.d = c->d;
  cj.kind = c->cfg.kernel;
  int maxL = 4;
  int64_t inner = 1;
  for (int e = c->d - 1; e >= 0; --e) {
    ToepAxis& ax = p.ax[e];
    ax.L = c->mdim[e];
    // additive: K is block diagonal, each axis one line of its own block, and
    // every block carries the outputscale
    ax.inner = c->add ? 1 : inner;
    ax.outer = c->add ? 1 : c->m / (inner * ax.L);
    inner *= ax.L;
    const double scale = (e == 0 || c->add) ? c->cfg.outputscale : 1.0;
    const double h = 1.0 / c->invh[e];
    std::vector<double> col(ax.L);
    for (int i = 0; i < ax.L; ++i) col[i] = kern1d(c->cfg.kernel, i * h, c->cfg.lengthscale[e]) * scale;
    for (int i = 0; i < 4; ++i) c->c4[e][i] = col[i];
    ax.c64 = dev_alloc(c, sizeof(double) * ax.L);
    ax.c32 = dev_alloc(c, sizeof(float) * ax.L);
    if (!ax.c64 || !ax.c32) return LOVE_ENOMEM;
    cj.ax[e] = CoefAxis{(double*)ax.c64, (float*)ax.c32, ax.L, h, c->cfg.lengthscale[e], scale};
    maxL = std::max(maxL, ax.L);
    int mode = c->cfg.toeplitz;
    if (mode == LOVE_TOEPLITZ_AUTO) mode = autotune_choose(c, e);
    ax.mode = mode;
    if (ax.mode == LOVE_TOEPLITZ_FFT) {
      love_status st = fft_plan_axis(c, ax, e, col);
      if (st != LOVE_OK) return st;
    }
    // band of coefficients that can matter at each working precision:
    // sum_{|d| > bw} |c_d| |g_j| <= L * thr * max|g|, with thr = eps * c_0 / L
    {
      auto band = [&](double eps) {
        const double thr = eps * std::fabs(col[0]) / (double)ax.L;
        int bw = ax.L - 1;
        while (bw > 0 && std::fabs(col[bw]) <= thr) --bw;
        return bw;
      };
      ax.bw32 = band(5.96e-8);
      ax.bw64 = band(1.12e-16);
    }
    if (ax.mode == LOVE_TOEPLITZ_DIRECT && ax.inner != 1 && ax.L > TOEP_LINES_MAXL)
      return LOVE_EUNSUPPORTED;  // long strided axis: use the FFT backend
    if (ax.mode == LOVE_TOEPLITZ_DIRECT && ax.inner == 1 && ax.L > TOEP_LINES_MAXL &&
        std::min(ax.L, TB_OUT + 2 * std::max(ax.bw32, ax.bw64)) > TB_NSEG_MAX * TB_SEG)
      return LOVE_EUNSUPPORTED;  // band wider than the segmented kernel covers: use the FFT
  }
  for (int e = 0; e < 4; ++e)
    if (e >= c->d)
      for (int i = 0; i < 4; ++i) c->c4[e][i] = 1.0;
  c->c4_dev = (double*)dev_alloc(c, sizeof(double) * 16);
  if (!c->c4_dev) return LOVE_ENOMEM;
  cj.c4 = c->c4_dev;
  k_toep_coef<<<dim3((unsigned)cdiv(maxL, 256), MAXD), 256, 0, c->stream>>>(cj);
  LOVE_HIP_TRY(hipGetLastError());
  return LOVE_OK;
}

}  // namespace love
