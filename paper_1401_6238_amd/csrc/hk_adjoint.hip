// Elementwise step of the adjoint of the distinct-vector and BHHB products:
// the cotangent of mode 1, c = conj(v) + conj(phi) x_1, which enters every
// gradient linearly (see the distinct-vector adjoint in hk_api.cpp).
#include <hip/hip_runtime.h>

#include "hk_fft.hpp"
#include "hk_launch.hpp"

namespace hk {

// out[i] = (v ? conj(v[i]) : 0) + (phi ? conj(*phi) x[i] : 0), i < n.
template <typename T>
__global__ void __launch_bounds__(256) k_mode1_cotangent(cx<T> *out, const cx<T> *v, const cx<T> *phi,
                                                         const cx<T> *x, int64_t n) {
  const cx<T> ph = phi ? cconj(*phi) : czero<T>();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    cx<T> t = v ? cconj(v[i]) : czero<T>();
    if (phi) t = cfma(ph, x[i], t);
    out[i] = t;
  }
}

hipError_t launch_mode1_cotangent(bool dbl, void *out, const void *v, const void *phi, const void *x, int64_t n,
                                  hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  const dim3 grid((unsigned)(blocks < 4096 ? blocks : 4096));
  void *args[] = {&out, &v, &phi, &x, &n};
  const void *fn = dbl ? (const void *)&k_mode1_cotangent<double> : (const void *)&k_mode1_cotangent<float>;
  return launch_kernel(fn, grid, dim3(256), args, 0, st);
}

}  // namespace hk
