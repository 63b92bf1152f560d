// Circulant-embedding FFT backend for the Toeplitz factors of K_UU and the
// per-axis backend choice.  (Filled in below; the direct backend is used
// until an axis selects the FFT.)
#include "internal.h"

namespace love {

love_status fft_plan_axis(love_cache* c, ToepAxis& ax, int e, const std::vector<double>& col) {
  (void)c; (void)e; (void)col;
  ax.mode = LOVE_TOEPLITZ_DIRECT;
  return LOVE_OK;
}

int autotune_choose(love_cache* c, int e) {
  (void)c; (void)e;
  return LOVE_TOEPLITZ_DIRECT;
}

template <typename T>
void fft_axis_apply(const love_cache* c, const ToepAxis& ax, const T* in, T* out, T scale,
                    const Ctl* ctl, int mode, hipStream_t s) {
  (void)c; (void)ax; (void)in; (void)out; (void)scale; (void)ctl; (void)mode; (void)s;
}
template void fft_axis_apply<float>(const love_cache*, const ToepAxis&, const float*, float*, float, const Ctl*, int, hipStream_t);
template void fft_axis_apply<double>(const love_cache*, const ToepAxis&, const double*, double*, double, const Ctl*, int, hipStream_t);

}  // namespace love
