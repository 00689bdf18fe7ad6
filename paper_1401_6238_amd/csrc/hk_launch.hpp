// Host-side interface between the C-ABI layer and the per-precision kernel
// translation units (hk_f32.hip, hk_f64.hip: power-of-two lengths and all
// column kernels; hk_f32_odd.hip, hk_f64_odd.hip: rows of lengths 3 * 2^k and
// 5 * 2^k).
#pragma once
#include <hip/hip_runtime.h>

#include "hk_common.hpp"

namespace hk {

// Template variants compiled for every power-of-two length 2^0 .. 2^12.
enum : int { MAX_LOGL = 12, ROW_MAXT = 256, COL_MAXT = 512 };

struct KernelLimits {
  int tps;         // lanes per sequence
  int seq_lds;     // LDS elements per row sequence
  int lds_raw;     // LDS elements one sequence's exchanges need (0: no exchange)
  int elem_bytes;  // bytes per complex element
  int row_maxt;    // most lanes of a plain row-kernel workgroup
};

// Every kernel launch goes through here.  While per-kernel profiling is on,
// the launch carries a start/stop event pair that the runtime timestamps at
// the dispatch's own begin and end (hipExtLaunchKernel), so the recorded
// duration is the kernel's execution, without event-packet overhead.
hipError_t launch_kernel(const void *fn, dim3 grid, dim3 block, void **args, size_t lds, hipStream_t st);
hipError_t launch_cooperative(const void *fn, dim3 grid, dim3 block, void **args, size_t lds, hipStream_t st);

#define HK_DECLARE_LAUNCHERS(SUFFIX)                                                                   \
  hipError_t init_tables_##SUFFIX(const double *tw4096_interleaved, const double *tw24_interleaved);   \
  bool limits_##SUFFIX(int logL, int E, KernelLimits *out);                                            \
  hipError_t launch_rows_##SUFFIX(int logL, int E, int rows_per_wg, dim3 grid, const Shape &sh,      \
                                  const Ptrs &p0, const Strides &str, int64_t count, hipStream_t st);   \
  hipError_t launch_batch_##SUFFIX(const BatchArgs &args, int grid, hipStream_t st);                  \
  hipError_t batch_resident_##SUFFIX(int *blocks_per_cu);                                           \
  hipError_t launch_copy_cols_##SUFFIX(void *out, const void *src, const int32_t *pairs,            \
                                       int64_t npairs, int64_t rows, bool complex_elems,             \
                                       hipStream_t st);                                              \
  hipError_t launch_alpha_##SUFFIX(const Shape &sh, const Ptrs &p0, const Strides &str, int64_t npart,       \
                                   int64_t count, hipStream_t st);                                     \
  void batch_geometry_##SUFFIX(int *blk, int *e_row, int *e_col, size_t *lds_bytes);                 \
  hipError_t launch_group_##SUFFIX(const BatchArgs &args, int kind, int logL, int odd, int ntasks,      \
                                   hipStream_t st);                                                 \
  hipError_t launch_cols_##SUFFIX(int logL, int E, int tw, int xcd, dim3 grid, const Shape &sh,         \
                                  const Ptrs &p0, const Strides &str, const ColJob *jobs, int njobs,    \
                                  hipStream_t st);

HK_DECLARE_LAUNCHERS(f32)
HK_DECLARE_LAUNCHERS(f64)

// Level-k block Hankel products (hk_levels.hip): zero fill of n elements of
// es bytes, and the strided embedding (dir 0) / extraction (dir 1) of a
// compact array of `total` elements.
hipError_t launch_levels_fill(void *p, int64_t n, int es, hipStream_t st);
hipError_t launch_levels_copy(void *compact, void *emb, const Levels &lv, int64_t total, int dir, int es,
                              hipStream_t st);

// Adjoint of the distinct-vector and BHHB products (hk_adjoint.hip):
// out[i] = (v ? conj(v[i]) : 0) + (phi ? conj(*phi) x[i] : 0), i < n complex
// elements of float (dbl = false) or double precision.
hipError_t launch_mode1_cotangent(bool dbl, void *out, const void *v, const void *phi, const void *x, int64_t n,
                                  hipStream_t st);

#define HK_DECLARE_ODD_LAUNCHERS(SUFFIX)                                                                  \
  hipError_t init_tables_odd_##SUFFIX(const double *tw4096_interleaved, const double *tw24_interleaved);  \
  bool limits_odd_##SUFFIX(int odd, int logL, int E, KernelLimits *out);                                \
  int odd_row_e_##SUFFIX();                                                                             \
  int group_rowb_tps_##SUFFIX(int odd, int logL);                                                       \
  bool odd_bwd_ok_##SUFFIX(int odd);                                                                    \
  hipError_t launch_rows_odd_##SUFFIX(int odd, int logL, int E, int rows_per_wg, dim3 grid, const Shape &sh, \
                                      const Ptrs &p0, const Strides &str, int64_t count, hipStream_t st);   \
  hipError_t launch_group_odd_##SUFFIX(const BatchArgs &args, int odd, int kind, int logL, int ntasks,     \
                                       hipStream_t st);                                                  \
  bool limits_r2c_##SUFFIX(int logL, int E, KernelLimits *out);                                         \
  int r2c_row_e_##SUFFIX();                                                                             \
  hipError_t launch_rows_r2c_##SUFFIX(int logL, int E, int rows_per_wg, dim3 grid, const Shape &sh,       \
                                      const Ptrs &p0, const Strides &str, int64_t count, hipStream_t st);   \
  hipError_t launch_group_r2c_##SUFFIX(const BatchArgs &args, int logL, int ntasks, hipStream_t st);       \
  bool limits_r2cp_##SUFFIX(int logL, int E, KernelLimits *out);                                        \
  hipError_t launch_rows_r2cp_##SUFFIX(int logL, int E, int groups_per_wg, dim3 grid, const Shape &sh,    \
                                       const Ptrs &p0, const Strides &str, int64_t count, hipStream_t st);  \
  hipError_t launch_group_r2cp_##SUFFIX(const BatchArgs &args, int logL, int ntasks, hipStream_t st);

HK_DECLARE_ODD_LAUNCHERS(f32)
HK_DECLARE_ODD_LAUNCHERS(f64)

}  // namespace hk
