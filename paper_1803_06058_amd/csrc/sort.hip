// Interpolation setup: stable sort of the training rows by stencil cell.
//
// The cubic-interpolation matrix W (Sec. 2.3) is never stored.  Instead the
// rows are ordered by their stencil base cell so that (i) the rows touching a
// grid node form a few contiguous runs, which turns W^T v into a deterministic
// per-node gather (no floating-point atomics), and (ii) consecutive rows touch
// neighbouring grid nodes, so gathers from the grid stay in cache.
//
// Sort: least-significant-digit radix sort, 8-bit digits, stable (rank within
// a wave from ballots, across waves from per-wave digit counts), so the final
// order is (cell, original row) and does not depend on scheduling.  A batch of
// GPs is sorted at once: GP g's cells are keyed cell_off[g] + cell, so its
// rows land in one contiguous range, in the same order as a sort of its own.
#include "internal.h"

namespace love {

namespace {

constexpr int RS_BINS = 256;
constexpr int RS_BLOCK = 256;
constexpr int RS_TILE = 4096;

template <typename T>
struct SortJob {
  GridT<T> g;
  const T* x;                 // caller rows, n x d
  const T* y;
  T* xs;                      // sorted copies (cache)
  T* ys;
  int32_t* perm;
  int32_t* cell_start;        // ctot + 1
  int64_t n, row_off, ctot;
  uint32_t cell_off;
  unsigned* status;
};

template <typename T, int D>
__global__ void k_cells(Tab tab, const SortJob<T>* __restrict__ jobs, uint32_t* __restrict__ keys,
                        uint32_t* __restrict__ vals, uint32_t* __restrict__ count) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SortJob<T>& J = jobs[gp];
  const int64_t i = (int64_t)lb * blockDim.x + threadIdx.x;
  if (i >= J.n) return;
  const GridT<T>& g = J.g;
  unsigned bad = 0;
  int64_t cell = 0;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    T xe = J.x[i * D + e];
    if (!in_domain(xe, g.lo[e], g.hi[e])) bad |= SF_DOMAIN;
    if (!(xe == xe)) xe = g.lo[e];
    T s;
    int jj = stencil_at(g, e, xe, s);
    cell += (int64_t)jj * g.cstride[e];
  }
  T yi = J.y[i];
  if (!isfinite((double)yi)) bad |= SF_NONFINITE;
  if (bad) atomicOr(J.status, bad);
  const uint32_t key = J.cell_off + (uint32_t)cell;
  keys[J.row_off + i] = key;
  vals[J.row_off + i] = (uint32_t)(J.row_off + i);
  atomicAdd(&count[key], 1u);
}

__global__ void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                          uint32_t* __restrict__ hist, int nb) {
  __shared__ uint32_t cnt[RS_BINS];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int i = threadIdx.x; i < RS_TILE; i += RS_BLOCK) {
    int64_t idx = base + i;
    if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// In-place exclusive prefix sum of `len` uint32 values; one block of 1024.
// If total != nullptr the grand total is written there.
__global__ void k_scan_exclusive(uint32_t* __restrict__ data, int64_t len, uint32_t* total) {
  __shared__ uint32_t sums[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (len + 1023) / 1024;
  const int64_t b = t * chunk, e = (b + chunk < len) ? b + chunk : len;
  uint32_t s = 0;
  for (int64_t i = b; i < e; ++i) s += data[i];
  sums[t] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over 1024 partial sums
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = (t >= off) ? sums[t - off] : 0u;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  uint32_t run = (t == 0) ? 0u : sums[t - 1];
  for (int64_t i = b; i < e; ++i) {
    uint32_t v = data[i];
    data[i] = run;
    run += v;
  }
  if (total && t == 1023) *total = sums[1023];
}

__global__ void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                             uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n,
                             int shift, const uint32_t* __restrict__ hist, int nb) {
  __shared__ uint32_t base[RS_BINS];
  __shared__ uint32_t wcount[RS_BLOCK / WAVE][RS_BINS];
  const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
  base[t] = hist[(int64_t)t * nb + blockIdx.x];
  const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (WAVE - lane));
  const uint64_t above = (lane == WAVE - 1) ? 0ull : ((~0ull) << (lane + 1));
  for (int chunk = 0; chunk < RS_TILE; chunk += RS_BLOCK) {
#pragma unroll
    for (int q = 0; q < RS_BLOCK / WAVE; ++q) wcount[q][t] = 0u;
    __syncthreads();
    const int64_t idx = (int64_t)blockIdx.x * RS_TILE + chunk + t;
    const bool valid = idx < n;
    const uint32_t key = valid ? kin[idx] : 0u;
    const uint32_t dig = (key >> shift) & 255u;
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int bit = (dig >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      mask &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(mask & below);
    if (valid && (mask & above) == 0ull) wcount[w][dig] = (uint32_t)__popcll(mask);
    __syncthreads();
    if (valid) {
      uint32_t pre = 0;
      for (int q = 0; q < w; ++q) pre += wcount[q][dig];
      const uint32_t pos = base[dig] + pre + rank;
      kout[pos] = key;
      vout[pos] = vin[idx];
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int q = 0; q < RS_BLOCK / WAVE; ++q) add += wcount[q][t];
    base[t] += add;
    __syncthreads();
  }
}

// per GP: cell_start[c] = scan[cell_off + c] - row_off
template <typename T>
__global__ void k_cell_start(Tab tab, const SortJob<T>* __restrict__ jobs,
                             const uint32_t* __restrict__ scan) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SortJob<T>& J = jobs[gp];
  const int64_t c = (int64_t)lb * blockDim.x + threadIdx.x;
  if (c > J.ctot) return;
  J.cell_start[c] = (int32_t)((int64_t)scan[J.cell_off + c] - J.row_off);
}

template <typename T, int D>
__global__ void k_gather_sorted(Tab tab, const SortJob<T>* __restrict__ jobs,
                                const uint32_t* __restrict__ order) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SortJob<T>& J = jobs[gp];
  const int64_t p = (int64_t)lb * blockDim.x + threadIdx.x;
  if (p >= J.n) return;
  const int64_t i = (int64_t)order[J.row_off + p] - J.row_off;
#pragma unroll
  for (int e = 0; e < D; ++e) J.xs[p * D + e] = J.x[i * D + e];
  J.ys[p] = J.y[i];
  J.perm[p] = (int32_t)i;
}

template <typename T, int D>
love_status sort_impl(const std::vector<love_cache*>& cs, const std::vector<const T*>& xs,
                      const std::vector<const T*>& ys, hipStream_t s) {
  const int G = (int)cs.size();
  std::vector<SortJob<T>> jobs(G);
  std::vector<int64_t> brow(G), bcell(G);
  int64_t N = 0, K = 0;
  for (int g = 0; g < G; ++g) {
    love_cache* c = cs[g];
    SortJob<T> J{};
    J.g = make_grid<T>(c);
    J.x = xs[g];
    J.y = ys[g];
    J.xs = (T*)c->x;
    J.ys = (T*)c->y;
    J.perm = c->perm;
    J.cell_start = c->cell_start;
    J.n = c->n;
    J.row_off = N;
    J.ctot = c->ctot;
    J.cell_off = (uint32_t)K;
    J.status = c->status;
    jobs[g] = J;
    brow[g] = cdiv(c->n, 256);
    bcell[g] = cdiv(c->ctot + 1, 256);
    N += c->n;
    K += c->ctot;
  }
  if (N >= (int64_t(1) << 31) || K >= (int64_t(1) << 31)) return LOVE_EINVAL;
  JobArena A;
  const size_t jo = A.add(jobs);
  love_status st = A.upload(s);
  if (st != LOVE_OK) return st;
  const SortJob<T>* dj = A.at<SortJob<T>>(jo);
  const Tab trow = make_tab(brow), tcell = make_tab(bcell);
  // scratch: keys/vals ping-pong, histogram, counts (K + 1)
  const int nb = (int)cdiv(N, RS_TILE);
  uint32_t *k0, *v0, *k1, *v1, *hist, *cnt;
  size_t bytes = sizeof(uint32_t) * (4 * (size_t)N + (size_t)RS_BINS * nb + (size_t)K + 1);
  char* buf = nullptr;
  buf = (char*)ws_alloc(bytes, s);
  if (!buf) return LOVE_ENOMEM;
  k0 = (uint32_t*)buf;
  v0 = k0 + N;
  k1 = v0 + N;
  v1 = k1 + N;
  hist = v1 + N;
  cnt = hist + (size_t)RS_BINS * nb;
  LOVE_HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (K + 1), s));
  k_cells<T, D><<<tab_blocks(trow), 256, 0, s>>>(trow, dj, k0, v0, cnt);
  int bits = 1;
  while ((int64_t(1) << bits) < K) ++bits;
  const int passes = (bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    k_rs_hist<<<nb, RS_BLOCK, 0, s>>>(k0, N, shift, hist, nb);
    k_scan_exclusive<<<1, 1024, 0, s>>>(hist, (int64_t)RS_BINS * nb, nullptr);
    k_rs_scatter<<<nb, RS_BLOCK, 0, s>>>(k0, v0, k1, v1, N, shift, hist, nb);
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
  k_scan_exclusive<<<1, 1024, 0, s>>>(cnt, K + 1, nullptr);
  k_cell_start<T><<<tab_blocks(tcell), 256, 0, s>>>(tcell, dj, cnt);
  k_gather_sorted<T, D><<<tab_blocks(trow), 256, 0, s>>>(trow, dj, v0);
  ws_free(buf, s);
  A.release(s);
  LOVE_HIP_TRY(hipGetLastError());
  return LOVE_OK;
}

// ----------------------------------------------------------------------------
// Additive compositions: the rows stay in caller order; every (row, axis)
// pair is a virtual row keyed by its axis-e stencil cell (axis e's cells
// follow those of axis e - 1), so one stable sort lists, axis by axis, the
// rows of every cell.  A GP's virtual rows occupy [row_off, row_off + d n).
// ----------------------------------------------------------------------------
template <typename T, int D>
__global__ void k_cells_add(Tab tab, const SortJob<T>* __restrict__ jobs,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                            uint32_t* __restrict__ count) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SortJob<T>& J = jobs[gp];
  const int64_t i = (int64_t)lb * blockDim.x + threadIdx.x;
  if (i >= J.n) return;
  const GridT<T>& g = J.g;
  unsigned bad = 0;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    T xe = J.x[i * D + e];
    if (!in_domain(xe, g.lo[e], g.hi[e])) bad |= SF_DOMAIN;
    if (!(xe == xe)) xe = g.lo[e];
    T s;
    const int jj = stencil_at(g, e, xe, s);
    const uint32_t key = J.cell_off + (uint32_t)(g.acoff[e] + jj);
    const int64_t v = J.row_off + (int64_t)e * J.n + i;
    keys[v] = key;
    vals[v] = (uint32_t)i;
    atomicAdd(&count[key], 1u);
  }
  const T yi = J.y[i];
  if (!isfinite((double)yi)) bad |= SF_NONFINITE;
  if (bad) atomicOr(J.status, bad);
}

// rows copied in caller order; perm = the sorted virtual rows' row indices
template <typename T, int D>
__global__ void k_copy_add(Tab tab, const SortJob<T>* __restrict__ jobs,
                           const uint32_t* __restrict__ order) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const SortJob<T>& J = jobs[gp];
  const int64_t p = (int64_t)lb * blockDim.x + threadIdx.x;
  if (p >= J.n) return;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    J.xs[p * D + e] = J.x[p * D + e];
    J.perm[(int64_t)e * J.n + p] = (int32_t)order[J.row_off + (int64_t)e * J.n + p];
  }
  J.ys[p] = J.y[p];
}

template <typename T, int D>
love_status sort_add_impl(const std::vector<love_cache*>& cs, const std::vector<const T*>& xs,
                          const std::vector<const T*>& ys, hipStream_t s) {
  const int G = (int)cs.size();
  std::vector<SortJob<T>> jobs(G);
  std::vector<int64_t> brow(G), bcell(G);
  int64_t N = 0, K = 0;
  for (int g = 0; g < G; ++g) {
    love_cache* c = cs[g];
    SortJob<T> J{};
    J.g = make_grid<T>(c);
    J.x = xs[g];
    J.y = ys[g];
    J.xs = (T*)c->x;
    J.ys = (T*)c->y;
    J.perm = c->perm;
    J.cell_start = c->cell_start;
    J.n = c->n;
    J.row_off = N;
    J.ctot = c->ctot;
    J.cell_off = (uint32_t)K;
    J.status = c->status;
    jobs[g] = J;
    brow[g] = cdiv(c->n, 256);
    bcell[g] = cdiv(c->ctot + 1, 256);
    N += c->n * D;
    K += c->ctot;
  }
  if (N >= (int64_t(1) << 31) || K >= (int64_t(1) << 31)) return LOVE_EINVAL;
  JobArena A;
  const size_t jo = A.add(jobs);
  love_status st = A.upload(s);
  if (st != LOVE_OK) return st;
  const SortJob<T>* dj = A.at<SortJob<T>>(jo);
  const Tab trow = make_tab(brow), tcell = make_tab(bcell);
  const int nb = (int)cdiv(N, RS_TILE);
  uint32_t *k0, *v0, *k1, *v1, *hist, *cnt;
  size_t bytes = sizeof(uint32_t) * (4 * (size_t)N + (size_t)RS_BINS * nb + (size_t)K + 1);
  char* buf = nullptr;
  buf = (char*)ws_alloc(bytes, s);
  if (!buf) return LOVE_ENOMEM;
  k0 = (uint32_t*)buf;
  v0 = k0 + N;
  k1 = v0 + N;
  v1 = k1 + N;
  hist = v1 + N;
  cnt = hist + (size_t)RS_BINS * nb;
  LOVE_HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (K + 1), s));
  k_cells_add<T, D><<<tab_blocks(trow), 256, 0, s>>>(trow, dj, k0, v0, cnt);
  int bits = 1;
  while ((int64_t(1) << bits) < K) ++bits;
  const int passes = (bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    k_rs_hist<<<nb, RS_BLOCK, 0, s>>>(k0, N, shift, hist, nb);
    k_scan_exclusive<<<1, 1024, 0, s>>>(hist, (int64_t)RS_BINS * nb, nullptr);
    k_rs_scatter<<<nb, RS_BLOCK, 0, s>>>(k0, v0, k1, v1, N, shift, hist, nb);
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
  k_scan_exclusive<<<1, 1024, 0, s>>>(cnt, K + 1, nullptr);
  k_cell_start<T><<<tab_blocks(tcell), 256, 0, s>>>(tcell, dj, cnt);
  k_copy_add<T, D><<<tab_blocks(trow), 256, 0, s>>>(trow, dj, v0);
  ws_free(buf, s);
  A.release(s);
  LOVE_HIP_TRY(hipGetLastError());
  return LOVE_OK;
}

// ----------------------------------------------------------------------------
// Query points sorted by stencil cell (the backward's d var / d Rt gathers a
// grid node's contributions from the points of the cells around it).  Entry
// i < t is point i keyed by its flattened cell; for an additive composition
// entry e t + p is point p keyed by acoff[e] + its axis-e cell.  Stable, so
// the order is (cell, entry); order[pos] is the point of the pos-th entry.
// ----------------------------------------------------------------------------
template <typename T, int D, bool ADD>
__global__ void k_point_cells(GridT<T> g, const T* __restrict__ xs, int64_t t,
                              uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                              uint32_t* __restrict__ count) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= t) return;
  int64_t cell = 0;
#pragma unroll
  for (int e = 0; e < D; ++e) {
    T xe = xs[p * D + e];
    if (!(xe == xe)) xe = g.lo[e];
    T sv;
    const int j = stencil_at(g, e, xe, sv);
    if constexpr (ADD) {
      const uint32_t key = (uint32_t)(g.acoff[e] + j);
      keys[(int64_t)e * t + p] = key;
      vals[(int64_t)e * t + p] = (uint32_t)p;
      atomicAdd(&count[key], 1u);
    } else {
      cell += (int64_t)j * g.cstride[e];
    }
  }
  if constexpr (!ADD) {
    keys[p] = (uint32_t)cell;
    vals[p] = (uint32_t)p;
    atomicAdd(&count[cell], 1u);
  }
}

template <typename T, int D, bool ADD>
love_status sort_points_impl(const love_cache* c, const T* xs, int64_t t, uint32_t* order,
                             uint32_t* cstart, hipStream_t s) {
  const GridT<T> g = make_grid<T>(c);
  const int64_t N = ADD ? (int64_t)D * t : t, K = c->ctot;
  if (N >= (int64_t(1) << 31) || K >= (int64_t(1) << 31)) return LOVE_EINVAL;
  const int nb = (int)cdiv(N, RS_TILE);
  int bits = 1;
  while ((int64_t(1) << bits) < K) ++bits;
  const int passes = (bits + 7) / 8;
  const size_t bytes = sizeof(uint32_t) * (3 * (size_t)N + (size_t)RS_BINS * nb);
  uint32_t* buf = (uint32_t*)ws_alloc(bytes, s);
  if (!buf) return LOVE_ENOMEM;
  // values ping-pong between scratch and `order`, starting where the last
  // pass ends in `order`
  uint32_t *k0 = buf, *k1 = k0 + N, *vs = k1 + N, *hist = vs + N;
  uint32_t* v0 = (passes % 2) ? vs : order;
  uint32_t* v1 = (passes % 2) ? order : vs;
  LOVE_HIP_TRY(hipMemsetAsync(cstart, 0, sizeof(uint32_t) * (K + 1), s));
  k_point_cells<T, D, ADD><<<(unsigned)cdiv(t, 256), 256, 0, s>>>(g, xs, t, k0, v0, cstart);
  for (int q = 0; q < passes; ++q) {
    const int shift = 8 * q;
    k_rs_hist<<<nb, RS_BLOCK, 0, s>>>(k0, N, shift, hist, nb);
    k_scan_exclusive<<<1, 1024, 0, s>>>(hist, (int64_t)RS_BINS * nb, nullptr);
    k_rs_scatter<<<nb, RS_BLOCK, 0, s>>>(k0, v0, k1, v1, N, shift, hist, nb);
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
  k_scan_exclusive<<<1, 1024, 0, s>>>(cstart, K + 1, nullptr);
  ws_free(buf, s);
  LOVE_HIP_TRY(hipGetLastError());
  return LOVE_OK;
}

}  // namespace

template <typename T>
love_status sort_points(const love_cache* c, const T* xs, int64_t t, uint32_t* order,
                        uint32_t* cstart, hipStream_t s) {
#define SP_CASE(D)                                                              \
  case D:                                                                       \
    return c->add ? sort_points_impl<T, D, true>(c, xs, t, order, cstart, s)   \
                  : sort_points_impl<T, D, false>(c, xs, t, order, cstart, s);
  switch (c->d) {
    SP_CASE(1)
    SP_CASE(2)
    SP_CASE(3)
    SP_CASE(4)
  }
#undef SP_CASE
  return LOVE_EINVAL;
}
template love_status sort_points<float>(const love_cache*, const float*, int64_t, uint32_t*, uint32_t*, hipStream_t);
template love_status sort_points<double>(const love_cache*, const double*, int64_t, uint32_t*, uint32_t*, hipStream_t);

template <typename T>
love_status setup_sort(const std::vector<love_cache*>& cs, const std::vector<const T*>& xs,
                       const std::vector<const T*>& ys, hipStream_t s) {
  ProfScope ps("setup_sort", s);
  if (cs[0]->add) {
    switch (cs[0]->d) {
      case 1: return sort_add_impl<T, 1>(cs, xs, ys, s);
      case 2: return sort_add_impl<T, 2>(cs, xs, ys, s);
      case 3: return sort_add_impl<T, 3>(cs, xs, ys, s);
      case 4: return sort_add_impl<T, 4>(cs, xs, ys, s);
    }
    return LOVE_EINVAL;
  }
  switch (cs[0]->d) {
    case 1: return sort_impl<T, 1>(cs, xs, ys, s);
    case 2: return sort_impl<T, 2>(cs, xs, ys, s);
    case 3: return sort_impl<T, 3>(cs, xs, ys, s);
    case 4: return sort_impl<T, 4>(cs, xs, ys, s);
  }
  return LOVE_EINVAL;
}

template love_status setup_sort<float>(const std::vector<love_cache*>&, const std::vector<const float*>&, const std::vector<const float*>&, hipStream_t);
template love_status setup_sort<double>(const std::vector<love_cache*>&, const std::vector<const double*>&, const std::vector<const double*>&, hipStream_t);

}  // namespace love
