// Host-side internals of the LOVE library: the cache object, device buffers,
// Toeplitz plans and the launchers implemented in the .hip translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/love.h"
#include "common.h"

namespace love {

// ----------------------------------------------------------------------------
// Kernel timing (optional): event pairs around launches, keyed by name.
// ----------------------------------------------------------------------------
bool prof_on();
void prof_begin(const char* name, hipStream_t s);
void prof_end(const char* name, hipStream_t s);

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
  int fft_single = 0;    // 1: real line packed into a half-length complex FFT
  int bw32 = 0;          // coefficient band that matters in float  (|d| <= bw32)
  int bw64 = 0;          // ... and in double
  void* c32 = nullptr;   // float  first column (L), outputscale folded into axis 0
  void* c64 = nullptr;   // double first column (L)
  void* spec32 = nullptr;  // float  circulant eigenvalues (fft_n [+1] reals)
  void* spec64 = nullptr;  // double
};

struct ToepPlan {
  int d = 1;
  int64_t mtot = 0;
  ToepAxis ax[MAXD];
};

// ----------------------------------------------------------------------------
// The cache
// ----------------------------------------------------------------------------
}  // namespace love

struct love_cache {
  love_config cfg;
  bool fp64 = false;
  int d = 1;
  int64_t n = 0, m = 0;
  int k = 0, kpad = 0;        // Lanczos steps requested; row stride of Rt
  int ks = 0, kspad = 0;      // sampler steps; row stride of S
  hipStream_t stream = nullptr;
  int device = 0;
  double tol_lanczos = 0.0;
  // geometry (double master copy)
  double lo[4], hi[4], invh[4];
  int mdim[4];
  // sorted training data
  void* x = nullptr;          // n x d, sorted by cell
  void* y = nullptr;          // n, sorted
  int32_t* perm = nullptr;    // sorted position -> caller row
  int32_t* cell_start = nullptr;  // ctot + 1
  int64_t ctot = 0;
  love::ToepPlan toep;
  double c4[4][4];            // first four entries of each axis column (outputscale in axis 0)
  double* c4_dev = nullptr;   // same, on device [4][4]
  // cache contents
  void* rt = nullptr;         // m x kpad (T) ; for bf16 split: hi plane (uint16)
  void* rt_lo = nullptr;      // bf16 split: lo plane (uint16)
  void* a = nullptr;          // m (T)
  float* S = nullptr;         // m x kspad
  double* alpha = nullptr;    // k
  double* beta = nullptr;     // k
  love::Ctl* ctl = nullptr;   // device control block of the main Lanczos / CG
  love::Ctl* ctl_s = nullptr; // sampler Lanczos
  unsigned* status = nullptr; // device status word of queries (SF_* bits)
  // scratch for apply_khat
  void* v1 = nullptr;         // n
  void* v2 = nullptr;         // n
  void* g1 = nullptr;         // m
  void* g2 = nullptr;         // m
  void* tscr = nullptr;       // 2 m (double-sized): Toeplitz scratch of apply_khat / apply_kuu
  size_t bytes = 0;
  std::vector<void*> allocs;
};

namespace love {

// allocation helper (tracks bytes); returns nullptr on failure
void* dev_alloc(love_cache* c, size_t bytes);

// --- setup (sort.hip) -------------------------------------------------------
template <typename T>
love_status setup_sort(love_cache* c, const T* x, const T* y, hipStream_t s);

// --- operator pieces (mvm.hip) ---------------------------------------------
template <typename T>
GridT<T> make_grid(const love_cache* c);

// `xsrc` (sorted coordinates in precision T) defaults to the cache's own copy
// g = W^T v; with ctl_mode bit 4, g = W^T (v + ctl->ratio * v2)
template <typename T>
void launch_scatter(const love_cache* c, const T* v, T* g, const T* v2, const Ctl* ctl,
                    int ctl_mode, hipStream_t s, const T* xsrc = nullptr);

template <typename T>
void launch_gather(const love_cache* c, const T* kg, const T* vsig, T sigma2, T* out,
                   const Ctl* ctl, hipStream_t s, const T* xsrc = nullptr);

template <typename TI, typename TO>
void launch_convert(const TI* in, TO* out, int64_t n, hipStream_t s);

// K_UU in -> out; `scratch` holds toeplitz_scratch_elems(c) elements of T
// (intermediate axis passes and per-segment partial sums).  Concurrent calls
// need distinct scratch.
int64_t toeplitz_scratch_elems(const love_cache* c);
template <typename T>
void toeplitz_apply(const love_cache* c, const T* in, T* out, T* scratch, const Ctl* ctl,
                    int ctl_mode, hipStream_t s);

love_status toeplitz_plan(love_cache* c);

// --- Lanczos / CG (lanczos.hip) ---------------------------------------------
// Lanczos, Rt, and (concurrently) the mean CG on `s` and the sampler on
// `s_side` (nullptr: everything on `s`).
template <typename T>
love_status build_lanczos_and_mean(love_cache* c, hipStream_t s, hipStream_t s_side);

// --- queries (query.hip) -----------------------------------------------------
template <typename T>
love_status predict(const love_cache* c, const T* xs, int64_t t, T* mean, T* var, hipStream_t s);

template <typename T>
love_status covar_pairs(const love_cache* c, const T* xa, const T* xb, int64_t t, T* cov,
                        hipStream_t s);

template <typename T>
love_status sample(const love_cache* c, const T* xs, int64_t t, const float* z, int64_t ns,
                   T* out, hipStream_t s);

template <typename T>
love_status backward(const love_cache* c, const T* xs, int64_t t, const T* gm, const T* gv,
                     T* gx, float* grt, hipStream_t s);

love_status rt_export_f32(const love_cache* c, float* dst, int keff, hipStream_t s);

// --- small helpers -------------------------------------------------------------
template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t s);

template <typename T>
void launch_permute(const T* in, T* out, const int32_t* perm, int64_t n, int inverse,
                    hipStream_t s);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

#define LOVE_HIP_TRY(expr)                         \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return LOVE_EHIP;        \
  } while (0)

}  // namespace love
