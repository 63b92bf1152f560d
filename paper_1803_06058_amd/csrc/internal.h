// Host-side internals of the LOVE library: the cache object, device buffers,
// Toeplitz plans, batched-launch helpers and the launchers implemented in the
// .hip translation units.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/love.h"
#include "common.h"
#include "jobs.h"

namespace love {

// ----------------------------------------------------------------------------
// Kernel timing (optional): event pairs around launches, keyed by name.
// ----------------------------------------------------------------------------
bool prof_on();
void prof_begin(const char* name, hipStream_t s);
void prof_end(const char* name, hipStream_t s);

// Kernel-level timing: when `name` is being timed, an event pair takes the
// launched kernel's own start and end timestamps (no extra stream packets).
bool prof_kernel_events(const char* name, hipEvent_t* start, hipEvent_t* stop);

// Launch `kernel` on `s`, timed under `name` when timing is on.
template <typename F, typename... Args>
inline void tlaunch(const char* name, F kernel, dim3 grid, dim3 block, uint32_t smem,
                    hipStream_t s, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (!prof_on() || !prof_kernel_events(name, &a, &b)) a = b = nullptr;
  hipExtLaunchKernelGGL(kernel, grid, block, smem, s, a, b, 0, args...);
}

struct ProfScope {
  const char* name;
  hipStream_t s;
  bool on;
  ProfScope(const char* n, hipStream_t st) : name(n), s(st), on(prof_on()) {
    if (on) prof_begin(name, s);
  }
  ~ProfScope() {
    if (on) prof_end(name, s);
  }
};

// ----------------------------------------------------------------------------
// Toeplitz / Kronecker-Toeplitz operator K_UU
// ----------------------------------------------------------------------------
struct ToepAxis {
  int mode = 1;          // 1 direct, 2 fft
  int L = 0;             // points along the axis (m_i)
  int64_t inner = 1;     // product of m over later axes
  int64_t outer = 1;     // product of m over earlier axes
  int fft_n = 0;         // complex FFT length (power of two) when mode == 2
  int bw32 = 0;          // coefficient band that matters in float  (|d| <= bw32)
  int bw64 = 0;          // ... and in double
  void* c32 = nullptr;   // float  first column (L), outputscale folded into axis 0
  void* c64 = nullptr;   // double first column (L)
  void* spec32 = nullptr;  // float  [circulant eigenvalues / N | twiddles], 2 N values
  void* spec64 = nullptr;  // double
};

struct ToepPlan {
  int d = 1;
  int64_t mtot = 0;
  ToepAxis ax[MAXD];
};

}  // namespace love

namespace love {
// Where the device memory of a library call comes from: the caller's
// love_allocator when one was given, else the device's stream-ordered pool
// (hipMallocAsync / hipFreeAsync).  A block is released on the stream that
// allocated it, after every stream that used it has been joined into that one.
struct MemSource {
  love_allocator a{};
  bool user = false;
};
void* mem_alloc(const MemSource& m, size_t bytes, hipStream_t s);
void mem_free(const MemSource& m, void* p, hipStream_t s);
// The memory source of the calling thread's current entry point (set by a
// MemScope there; the library's pool outside any scope).
const MemSource& cur_mem();
class MemScope {
 public:
  explicit MemScope(const MemSource& m);
  ~MemScope();
  MemScope(const MemScope&) = delete;
  MemScope& operator=(const MemScope&) = delete;

 private:
  const MemSource* prev_;
  MemSource mine_;
};
// Workspace of the current call: allocated and released on stream s.
inline void* ws_alloc(size_t bytes, hipStream_t s) { return mem_alloc(cur_mem(), bytes, s); }
inline void ws_free(void* p, hipStream_t s) {
  if (p) mem_free(cur_mem(), p, s);
}
}  // namespace love

struct love_cache {
  love_config cfg;
  love::MemSource mem;        // source of the cache's memory (kept for love_cache_free)
  bool fp64 = false;
  int d = 1;
  int64_t n = 0, m = 0;
  int64_t ldq = 0;            // n rounded up to the row-block size
  int k = 0, kpad = 0;        // Lanczos vectors the buffers hold; row stride of Rt
  int k1 = 0;                 // steps of the first Lanczos run (k unless restarts are allowed)
  // restart with a new probe (love_config.restart_*): rounds allowed, steps
  // per round, check groups; rounds taken and the last check's worst residual
  int restart_max = 0, restart_k = 0, restart_groups = 0;
  int restarts = 0;
  double solve_residual = NAN;
  int ks = 0, kspad = 0;      // sampler steps; row stride of S
  hipStream_t stream = nullptr;
  int device = 0;
  double tol_lanczos = 0.0;
  // geometry (double master copy)
  double lo[4], hi[4], invh[4];
  int mdim[4];
  // additive composition (LOVE_FLAG_ADDITIVE): the grid stacks the axes;
  // axis e's nodes start at aoff[e], its stencil cells at acoff[e]
  bool add = false;
  int64_t aoff[4] = {0, 0, 0, 0}, acoff[4] = {0, 0, 0, 0};
  // sorted training data
  void* x = nullptr;          // n x d, sorted by cell
  void* y = nullptr;          // n, sorted
  int32_t* perm = nullptr;    // sorted position -> caller row (additive: d x n, axis e's rows
                              // in order of their axis-e cell, caller order within a cell)
  int32_t* cell_start = nullptr;  // ctot + 1 (additive: positions in perm)
  int64_t ctot = 0;
  love::ToepPlan toep;
  double c4[4][4];            // first four entries of each axis column (outputscale in axis 0)
  double* c4_dev = nullptr;   // same, on device [4][4]
  // cache contents
  void* rt = nullptr;         // m x kpad (T) ; for bf16 split: hi plane (uint16)
  void* rt_lo = nullptr;      // bf16 split: lo plane (uint16)
  void* a = nullptr;          // m (T)
  void* B = nullptr;          // LOVE_FLAG_HYPER: m x kpad (T), W^T Q L^{-T} (Rt = K B)
  float* S = nullptr;         // m x kspad
  double* alpha = nullptr;    // k
  double* beta = nullptr;     // k
  love::Ctl* ctl = nullptr;   // device control block of the main Lanczos / CG
  love::Ctl* ctl_s = nullptr; // sampler Lanczos
  unsigned* status = nullptr; // device status word of queries (SF_* bits)
  double* ortho = nullptr;    // device: max |Q^T Q - I| of the Lanczos vectors
  // scratch for apply_khat
  void* v1 = nullptr;         // n
  void* v2 = nullptr;         // n
  void* g1 = nullptr;         // m
  void* g2 = nullptr;         // m
  void* tscr = nullptr;       // toeplitz_scratch_elems doubles: scratch of apply_khat / apply_kuu
  size_t bytes = 0;
  std::vector<void*> allocs;
  // one device block for the cache's buffers, handed out in order (dev_alloc)
  char* block = nullptr;
  size_t block_size = 0, block_used = 0;
  // k_eff and k_eff_sample as recorded on the host when a synchronous build or
  // an import finished (keff_known = 0: not yet read)
  int keff_known = 0;
  int32_t keff_h = 0, kseff_h = 0;
};

namespace love {

// allocation helper (tracks bytes): the next 256-byte aligned piece of the
// cache's device block, or a separate hipMalloc once the block is used up;
// returns nullptr on failure
void* dev_alloc(love_cache* c, size_t bytes);
// reserve the cache's device block (call before the first dev_alloc)
bool dev_reserve(love_cache* c, size_t bytes);
inline size_t dev_round(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) & ~size_t(255); }

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

#define LOVE_HIP_TRY(expr)                         \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return LOVE_EHIP;        \
  } while (0)

// ----------------------------------------------------------------------------
// Batched launches (host side)
// ----------------------------------------------------------------------------
// Work table from per-GP block counts (GP g: blocks[g] blocks, may be 0).
inline Tab make_tab(const std::vector<int64_t>& blocks) {
  Tab t{};
  t.G = (int)blocks.size();
  t.off[0] = 0;
  for (int g = 0; g < t.G; ++g) t.off[g + 1] = t.off[g] + (int)blocks[g];
  return t;
}
inline unsigned tab_blocks(const Tab& t) { return (unsigned)t.off[t.G]; }

// Job arrays of a build (or of one call), staged on the host and uploaded
// with one copy; device addresses are valid after upload().
class JobArena {
 public:
  template <class J>
  size_t add(const std::vector<J>& items) {
    const size_t off = (host_.size() + 63) & ~size_t(63);
    host_.resize(off + sizeof(J) * items.size());
    if (!items.empty()) std::memcpy(host_.data() + off, items.data(), sizeof(J) * items.size());
    return off;
  }
  love_status upload(hipStream_t s) {
    if (host_.empty()) return LOVE_OK;
    dev_ = (char*)ws_alloc(host_.size(), s);
    if (!dev_) return LOVE_ENOMEM;
    st_ = s;
    LOVE_HIP_TRY(hipMemcpyAsync(dev_, host_.data(), host_.size(), hipMemcpyHostToDevice, s));
    return LOVE_OK;
  }
  template <class J>
  const J* at(size_t off) const {
    return reinterpret_cast<const J*>(dev_ + off);
  }
  void release(hipStream_t s) {
    ws_free(dev_, s);
    dev_ = nullptr;
  }
  // A table not released by its owner (an error return) goes back on the
  // stream it was uploaded on, after the work queued there.
  ~JobArena() {
    if (dev_) ws_free(dev_, st_);
  }
  JobArena() = default;
  JobArena(const JobArena&) = delete;
  JobArena& operator=(const JobArena&) = delete;
  JobArena(JobArena&& o) noexcept : host_(std::move(o.host_)), dev_(o.dev_), st_(o.st_) {
    o.dev_ = nullptr;
  }
  JobArena& operator=(JobArena&& o) noexcept {
    if (this != &o) {
      if (dev_) ws_free(dev_, st_);
      host_ = std::move(o.host_);
      dev_ = o.dev_;
      st_ = o.st_;
      o.dev_ = nullptr;
    }
    return *this;
  }

 private:
  std::vector<char> host_;
  char* dev_ = nullptr;
  hipStream_t st_ = nullptr;
};

// A K_UU application prepared for G GPs (one entry per axis; each backend is
// launched once for the GPs that use it on that axis).
template <typename T>
struct ToepRun {
  struct Axis {
    size_t jobs = 0;
    Tab band{}, reduce{}, lines{}, fft{};
    size_t smem_lines = 0, smem_fft = 0;
    // the first job's banded segments (nseg0 > 1: partial0 holds nseg0 x L0
    // values that the segment sums add), for consumers that add them themselves
    int nseg0 = 0;
    int64_t L0 = 0;
    const void* partial0 = nullptr;
  };
  int d = 0;
  int jpg = 1;   // table entries (jobs) per GP: d when an additive batch runs in one pass
  Axis ax[MAXD];
};

// in/out per GP with per-step strides; scratch per GP holds
// toeplitz_scratch_elems(c) elements of T; ctl per GP (nullable).
template <typename T>
void toep_prepare(JobArena& A, ToepRun<T>& run, const std::vector<love_cache*>& cs,
                  const std::vector<const T*>& in, const std::vector<int64_t>& in_js,
                  const std::vector<T*>& out, const std::vector<int64_t>& out_js,
                  const std::vector<T*>& scratch, const std::vector<const Ctl*>& ctl);
template <typename T>
void toep_run(const JobArena& A, const ToepRun<T>& run, int j, int mode, hipStream_t s);

int64_t toeplitz_scratch_elems(const love_cache* c);
love_status toeplitz_plan(love_cache* c);
void toeplitz_set_attrs();

// --- setup (sort.hip) -------------------------------------------------------
// Query points xs (t x d) sorted by stencil cell: order[pos] (t entries, or
// d t for an additive composition, one per point and axis) is the point of
// the pos-th entry in (cell, entry) order and cstart[c] (ctot + 1) the first
// position of cell c (additive: axis e's cells from acoff[e]).
template <typename T>
love_status sort_points(const love_cache* c, const T* xs, int64_t t, uint32_t* order,
                        uint32_t* cstart, hipStream_t s);
// Sort the rows of every GP of the batch by stencil cell (one sort for all).
template <typename T>
love_status setup_sort(const std::vector<love_cache*>& cs, const std::vector<const T*>& xs,
                       const std::vector<const T*>& ys, hipStream_t s);

// --- operator pieces (mvm.hip) ---------------------------------------------
template <typename T>
GridT<T> make_grid(const love_cache* c);

// W^T v.  A GP takes two stages (per-cell partial products, then per-node
// sums) when scatter_two_stage(c); its job's cellp then holds
// scatter_scratch_bytes(c, sizeof(T)), and is null otherwise.  kinds: the
// SCATTER_* bits of the batch (scatter_kinds).
enum : int { SCATTER_NODES = 1, SCATTER_TWO_STAGE = 2, SCATTER_ADDITIVE = 4 };
template <typename T>
void launch_scatter(const Tab& tab, const ScatterJob<T>* jobs, int d, int j, int mode,
                    hipStream_t s, int kinds);
bool scatter_two_stage(const love_cache* c);
int scatter_kinds(const std::vector<love_cache*>& cs);
size_t scatter_scratch_bytes(const love_cache* c, size_t elem);   // 0 unless two stages
template <typename T>
void launch_gather(const Tab& tab, const GatherJob<T>* jobs, int d, int mode, hipStream_t s);
template <typename T>
void launch_fill(const Tab& tab, const FillJob<T>* jobs, hipStream_t s);
template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t s);
template <typename TI, typename TO>
void launch_convert(const TI* in, TO* out, int64_t n, hipStream_t s);
template <typename T>
void launch_permute(const T* in, T* out, const int32_t* perm, int64_t n, int inverse,
                    hipStream_t s);
// tables for one GP
inline Tab tab1(int64_t blocks) { return make_tab(std::vector<int64_t>{blocks}); }

// --- Lanczos / CG / sampler (lanczos.hip) -------------------------------------
// Lanczos, Rt and the mean cache for every GP of the batch (lock step, one
// launch per phase); the samplers run on `s_side` concurrently with the mean
// solve (nullptr: on `s`).
template <typename T>
love_status build_batch_lanczos(const std::vector<love_cache*>& cs, hipStream_t s,
                                hipStream_t s_side);

// --- grid-space mean solve (mean.hip) -----------------------------------------
// true when the cache's mean is solved in grid space (d >= 2, every axis at
// most SPEC_MAXM points, no flag asking for the data-space CG)
bool spectral_mean_applies(const love_cache* c);
// a = K W^T Khat^{-1} y for every GP of the batch, on a stream of its own
// beside the Lanczos (the solve needs only x, y and the grid).  start()
// enqueues the set-up and the first FIRST_CHUNK iterations without waiting;
// finish() checks convergence (the host waits on the solve's stream), runs
// further iterations as needed and stores a; the caller then joins the
// streams and calls merge() on the build stream, which writes cg_iters and the
// solve's status bits into each cache's control block.  x64 / y64: sorted
// training data in double; un: n doubles of scratch per GP; release() frees
// everything on the given stream.
class SpectralMean {
 public:
  static constexpr int FIRST_CHUNK = 16;
  love_status start(const std::vector<love_cache*>& cs, const std::vector<const double*>& x64,
                    const std::vector<const double*>& y64, const std::vector<double*>& un,
                    hipStream_t s);
  love_status finish();
  void merge(hipStream_t s);
  void release(hipStream_t s);

 private:
  void forward_passes(int src, int extra);
  void backward_passes(int dst, int last);
  void iterations(int count);
  hipStream_t s_ = nullptr;
  int G_ = 0, d_ = 0, it_ = 0, maxit_ = 0, kinds_ = 0;
  bool uploaded_ = false;
  std::vector<SpecJob> jobs_;
  std::vector<char*> mem_;
  std::vector<double*> cellp_;
  JobArena A_;
  const SpecJob* dj_ = nullptr;
  size_t o_j_ = 0, o_ga_ = 0, o_su_ = 0;
  Tab t_m_{}, t_n_{}, t_one_{}, t_nodes_{};
  int* dflag_ = nullptr;
};
// the non-blocking stream the grid-space mean solve runs on (one per device)
hipStream_t mean_stream();

// --- queries (query.hip) -----------------------------------------------------
template <typename T>
love_status predict_batch(const std::vector<const love_cache*>& cs,
                          const std::vector<const T*>& xs, const std::vector<int64_t>& ts,
                          const std::vector<T*>& means, const std::vector<T*>& vars,
                          hipStream_t s);

template <typename T>
love_status covar_block(const love_cache* c, const T* xa, int64_t ta, const T* xb, int64_t tb,
                        T* cov, hipStream_t s);

template <typename T>
love_status covar_pairs(const love_cache* c, const T* xa, const T* xb, int64_t t, T* cov,
                        hipStream_t s);

// scratch: t x (kspad + 1) floats for F and mu, or NULL to take them from the
// call's memory source
template <typename T>
love_status sample(const love_cache* c, const T* xs, int64_t t, const float* z, int64_t ns,
                   T* out, hipStream_t s, float* scratch = nullptr);
// The same on the device's fixed scratch array (no allocation); LOVE_ELIMIT
// when t x (kspad + 1) floats exceed it.  The current device must be the cache's.
template <typename T>
love_status sample_noalloc(const love_cache* c, const T* xs, int64_t t, const float* z,
                           int64_t ns, T* out, hipStream_t s);

template <typename T>
love_status backward(const love_cache* c, const T* xs, int64_t t, const T* gm, const T* gv,
                     T* gx, float* grt, hipStream_t s);

// d (sum g_var var) / d theta, theta = (lengthscales, outputscale, sigma^2)
// into grad (device, d + 2 doubles); needs the cache's B (LOVE_FLAG_HYPER)
template <typename T>
love_status hyper_grad(const love_cache* c, const T* xs, int64_t t, const T* gv, double* grad,
                       hipStream_t s);

love_status rt_export_f32(const love_cache* c, float* dst, int keff, hipStream_t s);
// imported Rt into the cache layout and the control blocks of an imported cache
love_status rt_import(love_cache* c, const float* rt, const double* rt64, int keff, int kchol,
                      hipStream_t s);

}  // namespace love
