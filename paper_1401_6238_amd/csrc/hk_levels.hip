// Data movement of level-k block Hankel products (see hk_api.cpp): zero fill
// and the strided embedding of a compact k-dimensional array into a 1D vector
// (and back), for elements of 4, 8 or 16 bytes.
#include <hip/hip_runtime.h>

#include "hk_launch.hpp"

namespace hk {
namespace {

template <int ES>
struct Elem {
  uint32_t w[ES / 4];
};

template <int ES>
__global__ void __launch_bounds__(256) k_fill_zero(Elem<ES> *p, int64_t n) {
  Elem<ES> z;
#pragma unroll
  for (int i = 0; i < ES / 4; ++i) z.w[i] = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z;
}

// dir 0 (embed): emb[sum_t i_t stride_t] = compact[e];  dir 1 (extract): compact[e] = emb[...]
// for every compact linear index e = i_0 + ext_0 (i_1 + ext_1 (...)) < total.
template <int ES>
__global__ void __launch_bounds__(256) k_levels_copy(Elem<ES> *compact, Elem<ES> *emb, Levels lv, int64_t total,
                                                      int dir) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e, off = 0;
    for (int t = 0; t < lv.k; ++t) {
      const int64_t q = rem / lv.ext[t];
      off += (rem - q * lv.ext[t]) * lv.stride[t];
      rem = q;
    }
    if (dir == 0)
      emb[off] = compact[e];
    else
      compact[e] = emb[off];
  }
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

hipError_t launch_levels_fill(void *p, int64_t n, int es, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  void *args[] = {&p, &n};
  if (es == 4) return launch_kernel((void *)&k_fill_zero<4>, dim3(grid_for(n)), dim3(256), args, 0, st);
  if (es == 8) return launch_kernel((void *)&k_fill_zero<8>, dim3(grid_for(n)), dim3(256), args, 0, st);
  if (es == 16) return launch_kernel((void *)&k_fill_zero<16>, dim3(grid_for(n)), dim3(256), args, 0, st);
  return hipErrorInvalidValue;
}

hipError_t launch_levels_copy(void *compact, void *emb, const Levels &lv, int64_t total, int dir, int es,
                              hipStream_t st) {
  if (total <= 0) return hipSuccess;
  if (lv.k < 1 || lv.k > HK_MAX_LEVELS || (dir != 0 && dir != 1)) return hipErrorInvalidValue;
  Levels l = lv;
  void *args[] = {&compact, &emb, &l, &total, &dir};
  if (es == 4) return launch_kernel((void *)&k_levels_copy<4>, dim3(grid_for(total)), dim3(256), args, 0, st);
  if (es == 8) return launch_kernel((void *)&k_levels_copy<8>, dim3(grid_for(total)), dim3(256), args, 0, st);
  if (es == 16) return launch_kernel((void *)&k_levels_copy<16>, dim3(grid_for(total)), dim3(256), args, 0, st);
  return hipErrorInvalidValue;
}

}  // namespace hk
