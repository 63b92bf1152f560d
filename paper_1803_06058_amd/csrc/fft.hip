// Circulant-embedding FFT backend for the Toeplitz factors of K_UU (Sec. 2.3:
// a regular grid makes K_UU Toeplitz, so K g costs O(m log m)), and the
// per-axis choice between it and the direct banded product.
//
// A symmetric Toeplitz matrix with first column c (length L) is the leading
// L x L block of the circulant C of size N >= 2L - 1 whose first column is
// [c_0, ..., c_{L-1}, 0, ..., 0, c_{L-1}, ..., c_1].  C = F^{-1} diag(lam) F with
// lam = F c_ext real and even, so for two real lines x1, x2 packed as
// z = x1 + i x2,  F^{-1}(lam * F z) = C x1 + i C x2: one complex FFT pair
// serves two lines and needs no post-processing.
//
// Kernel: one block per line pair, the whole length-N complex signal in LDS,
// iterative radix-2 decimation in time (bit-reversed load) for the forward
// transform, multiply by lam / N, decimation in frequency for the inverse
// (bit-reversed store).  Twiddles exp(-2 pi i k / N) and lam are tabulated on
// the host in double.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"
#include "ops.h"

namespace love {

constexpr int FFT_BLK = 256;

template <typename T>
struct Cx {
  T re, im;
};

__device__ inline unsigned bitrev(unsigned x, int bits) { return __brev(x) >> (32 - bits); }

template <typename T>
__global__ __launch_bounds__(FFT_BLK) void k_fft_conv(Tab tab, const ToepJob<T>* __restrict__ jobs,
                                                      int j, int mode) {
  int gp, lb;
  if (!tab_find(tab, blockIdx.x, gp, lb)) return;
  const ToepJob<T>& J = jobs[gp];
  if (ctl_skip(J.ctl, mode)) return;
  extern __shared__ unsigned char smem_raw[];
  const int N = J.N, logN = J.logN, L = J.L;
  const int64_t inner = J.inner, nlines = J.outer * J.inner;
  const T* __restrict__ lam = J.spec;
  const T* __restrict__ tw = J.spec + N;
  const T scale = J.scale;
  T* zr = (T*)smem_raw;        // N
  T* zi = zr + N;              // N
  const T* in = J.in + (int64_t)j * J.in_js;
  T* out = J.out + (int64_t)j * J.out_js;
  const int64_t l1 = 2 * (int64_t)lb, l2 = l1 + 1;
  const bool has2 = l2 < nlines;
  const int64_t o1 = l1 / inner, r1 = l1 % inner, o2 = l2 / inner, r2 = l2 % inner;
  const T* s1 = in + o1 * L * inner + r1;
  const T* s2 = in + o2 * L * inner + r2;
  for (int i = threadIdx.x; i < N; i += FFT_BLK) {
    const unsigned p = bitrev((unsigned)i, logN);
    zr[p] = i < L ? s1[(int64_t)i * inner] : T(0);
    zi[p] = (i < L && has2) ? s2[(int64_t)i * inner] : T(0);
  }
  __syncthreads();
  // forward, decimation in time
  for (int st = 1; st <= logN; ++st) {
    const int half = 1 << (st - 1);
    const int tstep = N >> st;   // twiddle index stride
    for (int b = threadIdx.x; b < N / 2; b += FFT_BLK) {
      const int grp = b >> (st - 1), jj = b & (half - 1);
      const int i1 = grp * 2 * half + jj, i2 = i1 + half;
      const T wr = tw[2 * (jj * tstep)], wi = tw[2 * (jj * tstep) + 1];
      const T xr = zr[i2], xi = zi[i2];
      const T tr = wr * xr - wi * xi, ti = wr * xi + wi * xr;
      const T ur = zr[i1], ui = zi[i1];
      zr[i1] = ur + tr;
      zi[i1] = ui + ti;
      zr[i2] = ur - tr;
      zi[i2] = ui - ti;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < N; i += FFT_BLK) {
    const T lv = lam[i];
    zr[i] *= lv;
    zi[i] *= lv;
  }
  __syncthreads();
  // inverse, decimation in frequency with conjugate twiddles
  for (int st = logN; st >= 1; --st) {
    const int half = 1 << (st - 1);
    const int tstep = N >> st;
    for (int b = threadIdx.x; b < N / 2; b += FFT_BLK) {
      const int grp = b >> (st - 1), jj = b & (half - 1);
      const int i1 = grp * 2 * half + jj, i2 = i1 + half;
      const T wr = tw[2 * (jj * tstep)], wi = -tw[2 * (jj * tstep) + 1];
      const T ur = zr[i1], ui = zi[i1], vr = zr[i2], vi = zi[i2];
      zr[i1] = ur + vr;
      zi[i1] = ui + vi;
      const T dr = ur - vr, di = ui - vi;
      zr[i2] = wr * dr - wi * di;
      zi[i2] = wr * di + wi * dr;
    }
    __syncthreads();
  }
  T* d1 = out + o1 * L * inner + r1;
  T* d2 = out + o2 * L * inner + r2;
  for (int i = threadIdx.x; i < L; i += FFT_BLK) {
    const unsigned p = bitrev((unsigned)i, logN);
    d1[(int64_t)i * inner] = scale * zr[p];
    if (has2) d2[(int64_t)i * inner] = scale * zi[p];
  }
}

template <typename T>
void launch_fft_conv(const Tab& tab, const ToepJob<T>* jobs, size_t smem, int j, int mode,
                     hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    attr = true;
    (void)hipFuncSetAttribute((const void*)k_fft_conv<float>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 2 * 16384 * 4);
    (void)hipFuncSetAttribute((const void*)k_fft_conv<double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 2 * 8192 * 8);
  }
  k_fft_conv<T><<<tab_blocks(tab), FFT_BLK, smem, s>>>(tab, jobs, j, mode);
}
template void launch_fft_conv<float>(const Tab&, const ToepJob<float>*, size_t, int, int, hipStream_t);
template void launch_fft_conv<double>(const Tab&, const ToepJob<double>*, size_t, int, int, hipStream_t);

// ----------------------------------------------------------------------------
// Host: tables
// ----------------------------------------------------------------------------
static int fft_max_n(bool dbl) { return dbl ? 8192 : 16384; }   // N complex values in LDS

// iterative radix-2 complex FFT in double (host, table building only)
static void host_fft(std::vector<std::complex<double>>& a) {
  const int n = (int)a.size();
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const double ang = -2.0 * M_PI / len;
    for (int i = 0; i < n; i += len)
      for (int j = 0; j < len / 2; ++j) {
        const std::complex<double> w(std::cos(ang * j), std::sin(ang * j));
        const std::complex<double> u = a[i + j], v = a[i + j + len / 2] * w;
        a[i + j] = u + v;
        a[i + j + len / 2] = u - v;
      }
  }
}

love_status fft_plan_axis(love_cache* c, ToepAxis& ax, int e, const std::vector<double>& col) {
  (void)e;
  int N = 1, logN = 0;
  while (N < 2 * ax.L - 1) {
    N <<= 1;
    ++logN;
  }
  // the double tables must fit in LDS too (sampler and mean run in double);
  // the autotuner never picks the FFT beyond that, an explicit request fails
  if (N > fft_max_n(true)) return LOVE_EUNSUPPORTED;
  std::vector<std::complex<double>> cext(N, 0.0);
  for (int i = 0; i < ax.L; ++i) cext[i] = col[i];
  for (int i = 1; i < ax.L; ++i) cext[N - i] = col[i];
  host_fft(cext);
  std::vector<double> lam64(N), tw64(N);
  std::vector<float> lam32(N), tw32(N);
  for (int i = 0; i < N; ++i) {
    lam64[i] = cext[i].real() / N;
    lam32[i] = (float)lam64[i];
  }
  for (int k = 0; k < N / 2; ++k) {
    tw64[2 * k] = std::cos(-2.0 * M_PI * k / N);
    tw64[2 * k + 1] = std::sin(-2.0 * M_PI * k / N);
    tw32[2 * k] = (float)tw64[2 * k];
    tw32[2 * k + 1] = (float)tw64[2 * k + 1];
  }
  ax.spec64 = dev_alloc(c, sizeof(double) * 2 * N);   // [lam | twiddles]
  ax.spec32 = dev_alloc(c, sizeof(float) * 2 * N);
  if (!ax.spec64 || !ax.spec32) return LOVE_ENOMEM;
  LOVE_HIP_TRY(hipMemcpy(ax.spec64, lam64.data(), sizeof(double) * N, hipMemcpyHostToDevice));
  LOVE_HIP_TRY(hipMemcpy((double*)ax.spec64 + N, tw64.data(), sizeof(double) * N, hipMemcpyHostToDevice));
  LOVE_HIP_TRY(hipMemcpy(ax.spec32, lam32.data(), sizeof(float) * N, hipMemcpyHostToDevice));
  LOVE_HIP_TRY(hipMemcpy((float*)ax.spec32 + N, tw32.data(), sizeof(float) * N, hipMemcpyHostToDevice));
  ax.fft_n = N;
  ax.mode = LOVE_TOEPLITZ_FFT;
  return LOVE_OK;
}

// ----------------------------------------------------------------------------
// Autotuner: per axis shape (L, lines), time the direct and the FFT backend
// on the device once per process (float, on a private stream) and keep the
// faster.  LOVE_AUTOTUNE=0 switches measuring off and uses a size rule.
// ----------------------------------------------------------------------------
// Time one axis backend: a one-GP, one-axis view of the cache.
static float time_axis(love_cache* c, const ToepAxis& ax, float* bin, float* bout, float* bscr,
                       hipStream_t s, hipEvent_t a, hipEvent_t b) {
  love_cache view = *c;
  view.d = 1;
  view.toep.d = 1;
  view.toep.ax[0] = ax;
  JobArena A;
  ToepRun<float> run;
  std::vector<love_cache*> cs{&view};
  toep_prepare<float>(A, run, cs, {bin}, {0}, {bout}, {0}, {bscr}, {nullptr});
  if (A.upload(s) != LOVE_OK) return 1e30f;
  float best = 1e30f;
  for (int rep = 0; rep < 4; ++rep) {
    (void)hipEventRecord(a, s);
    toep_run<float>(A, run, 0, 0, s);
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (rep > 0) best = std::min(best, ms);
  }
  A.release(s);
  (void)hipStreamSynchronize(s);
  return best;
}

static std::mutex g_tune_mu;
static std::map<std::tuple<int, int64_t, int64_t, int, int>, int> g_tune;

int autotune_choose(love_cache* c, int e) {
  ToepAxis ax = c->toep.ax[e];
  const char* env = std::getenv("LOVE_AUTOTUNE");
  const bool measure = !(env && env[0] == '0');
  int N = 1;
  while (N < 2 * ax.L - 1) N <<= 1;
  if (N > fft_max_n(true)) return LOVE_TOEPLITZ_DIRECT;
  const int64_t lines = ax.outer * ax.inner;
  if (ax.inner != 1 && ax.L > 256) return LOVE_TOEPLITZ_FFT;   // the direct kernel covers L <= 256 here
  if (!measure) return (ax.L >= 256 && lines >= 64) ? LOVE_TOEPLITZ_FFT : LOVE_TOEPLITZ_DIRECT;
  // temporary plans for both backends on this axis
  const double h = 1.0 / c->invh[e];
  std::vector<double> col(ax.L);
  for (int i = 0; i < ax.L; ++i)
    col[i] = std::exp(-0.5 * (i * h / c->cfg.lengthscale[e]) * (i * h / c->cfg.lengthscale[e]));
  if (c->cfg.kernel == LOVE_MATERN52)
    for (int i = 0; i < ax.L; ++i) {
      const double z = std::sqrt(5.0) * i * h / c->cfg.lengthscale[e];
      col[i] = (1.0 + z + z * z / 3.0) * std::exp(-z);
    }
  int bw = ax.L - 1;
  {
    const double thr = 5.96e-8 * std::fabs(col[0]) / (double)ax.L;
    while (bw > 0 && std::fabs(col[bw]) <= thr) --bw;
  }
  const auto key = std::make_tuple(ax.L, ax.inner, ax.outer, bw, (int)sizeof(float));
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  ToepAxis axd = ax, axf = ax;
  axd.mode = LOVE_TOEPLITZ_DIRECT;
  if (fft_plan_axis(c, axf, e, col) != LOVE_OK || axf.mode != LOVE_TOEPLITZ_FFT)
    return LOVE_TOEPLITZ_DIRECT;
  {
    axd.bw32 = axd.bw64 = bw;
    std::vector<float> c32(col.begin(), col.end());
    axd.c32 = dev_alloc(c, sizeof(float) * ax.L);
    if (!axd.c32) return LOVE_TOEPLITZ_DIRECT;
    if (hipMemcpy(axd.c32, c32.data(), sizeof(float) * ax.L, hipMemcpyHostToDevice) != hipSuccess)
      return LOVE_TOEPLITZ_DIRECT;
    axf.c32 = axd.c32;
  }
  hipStream_t s = nullptr;
  float *bin = nullptr, *bout = nullptr, *bscr = nullptr;
  const int64_t mt = c->m;
  int choice = LOVE_TOEPLITZ_DIRECT;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
      (bin = (float*)ws_alloc(sizeof(float) * mt, s)) != nullptr &&
      (bout = (float*)ws_alloc(sizeof(float) * mt, s)) != nullptr &&
      (bscr = (float*)ws_alloc(sizeof(float) * toeplitz_scratch_elems(c), s)) != nullptr) {
    (void)hipMemsetAsync(bin, 0, sizeof(float) * mt, s);
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    float best[2];
    best[0] = time_axis(c, axd, bin, bout, bscr, s, a, b);
    best[1] = time_axis(c, axf, bin, bout, bscr, s, a, b);
    choice = best[1] < best[0] ? LOVE_TOEPLITZ_FFT : LOVE_TOEPLITZ_DIRECT;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  if (s) {
    ws_free(bin, s);
    ws_free(bout, s);
    ws_free(bscr, s);
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = choice;
  return choice;
}

}  // namespace love
