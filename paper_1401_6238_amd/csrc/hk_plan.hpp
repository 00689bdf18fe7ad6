// Host-side planning of Hankel tensor-vector products: normalized problem
// descriptions, FFT layouts, schedules and the launch sequences of the plain
// (single-shape) path.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hankel.h"
#include "hk_common.hpp"
#include "hk_launch.hpp"

namespace hk {

// Largest 1D padded length handled by one workgroup.
enum : int { RES_MAX_LOG = 12 };

struct Status {
  hk_status_t code = HK_SUCCESS;
  std::string msg;
  bool ok() const { return code == HK_SUCCESS; }
};

Status fail(hk_status_t code, const std::string &msg);

// A product request after validation (pointers are device pointers).
struct Problem {
  hk_dtype_t dt = HK_C64;
  int prog = PROG_FWD;
  bool is_block = false;
  int m = 0;
  int64_t dims[HK_MAX_ORDER] = {0};
  int64_t bdims[HK_MAX_ORDER] = {0};
  const void *h = nullptr;
  const void *vec[HK_MAX_ORDER] = {nullptr};  // forward: vec[0] only for alpha
  // forward, multipass power-of-two 1D layouts: h / vec[q] (bit q) point to
  // spectra in row order instead of the vectors themselves
  bool h_spec = false;
  uint32_t spec_mask = 0;
  void *y = nullptr;
  void *alpha = nullptr;
  // adjoint (equal vectors): vec[1] = x
  const void *v = nullptr;
  const void *phi = nullptr;
  void *gx = nullptr;
  void *gh = nullptr;
  // forward variants (power-of-two complex layouts): conv = no generating
  // vector, output conj(x_1 * ... * x_m) over the generating grid; conj_y =
  // the vector output stored conjugated
  bool conv = false;
  bool conj_y = false;
};

// Launch parameters of one shape.
struct Sched {
  int E_row = 8;
  int rows_per_wg = 1;
  int E_col = 16;
  int tw = 8;
  int split = 0;  // multipass: logR - ceil(logN / 2) adjustment
  int xcd = 0;    // column passes: XCD-local tile numbering (1) or identity (0)
  int iters = 1;  // row pass: rows a workgroup's lane group transforms in turn, the
                  // next row's operands loading while the current one is transformed
};

struct Layout {
  bool resident = false;
  int odd = 1;       // 1D: transform length odd * 2^(logR + logC); BHHB: rows odd * 2^logR
  int odd_c = 1;     // BHHB: columns odd_c * 2^logC
  bool r2c = false;  // real inputs, resident: length 2^(logR + 1) real transforms
  int logR = 0, logC = 0;
  // length class of the schedule key: 1, 3, 5 = odd factor, 2 = real inputs;
  // BHHB grids add 16 * the column axis's odd factor when it has one
  int lclass() const { return (r2c ? 2 : odd) + (odd_c > 1 ? 16 * odd_c : 0); }
  bool block_odd() const { return odd > 1 || odd_c > 1; }
};

bool is_complex(hk_dtype_t dt);
size_t elem_bytes(hk_dtype_t dt);      // bytes of one stored element
size_t cplx_bytes(hk_dtype_t dt);      // bytes of one complex working element
int ceil_log2(int64_t v);

// Validation (host-side, before any enqueue).
Status validate_forward(const Problem &p);
Status validate_backward(const Problem &p);

// Shape construction.  `layout` decides the transform length (the smallest
// 2^k, 3 * 2^k or 5 * 2^k >= d_H with kernels; for real forward products
// with N <= 8192 a length-N real transform done as a length-N/2 complex one;
// powers of two only when allow_odd is false), resident vs multipass and the
// split.
// five: F5_AUTO takes the factor 5 in 1D lengths as the length policy says;
// F5_RESIDENT only for resident lengths (grouped plans); F5_NONE not at all
// (the plan autotuner's per-bucket alternative).
enum : int { F5_NONE = 0, F5_RESIDENT = 1, F5_AUTO = 2 };
Status layout_for(const Problem &p, int split, Layout *out, bool allow_odd = true, int64_t batch = 1,
                  int five = F5_AUTO);
// Process-wide transform-length policy (see hk_set_fft_lengths).
void set_length_policy(int policy);
int length_policy();
// Kernel limits of a layout's rows (odd factor and real-input aware).
bool layout_row_limits(hk_dtype_t dt, const Layout &lay, int E, KernelLimits *k);
// Row-kernel limits of a layout's row length (odd factor aware).
bool row_limits(hk_dtype_t dt, int odd, int logL, int E, KernelLimits *k);
Status build_shape(const Problem &p, const Layout &lay, const Sched &sc, Shape *sh, Ptrs *ptrs,
                   int op_src[MAXOPS]);

// Default schedule of a shape (overridden by the autotuner cache).
Sched default_sched(hk_dtype_t dt, const Layout &lay, int prog, int64_t batch);
// Clamp a schedule to what the kernels accept for this layout.
bool sched_valid(hk_dtype_t dt, const Layout &lay, const Sched &sc);

// Workspace bytes per instance for a shape (0 for resident).
size_t instance_ws_bytes(const Shape &sh, hk_dtype_t dt);
// Bytes one instance's passes read and write (the pass model; diagnostics).
int64_t pass_model_bytes(const Shape &sh, hk_dtype_t dt);

// Plain path: enqueue the product(s) of one shape; instance i uses the
// pointers p0 + i * str (byte strides).
Status launch_shape(hk_dtype_t dt, const Shape &sh, const Sched &sc, const Ptrs &p0, const Strides &str,
                    int64_t count, hipStream_t st);

// Device checks / one-time per-device setup (twiddle tables).
Status ensure_device();

// Schedule cache (autotuner).
bool sched_lookup(hk_dtype_t dt, int prog, int is_block, int odd, int logM, int logC_hint, int64_t batch,
                  Sched *sc);
void sched_store(hk_dtype_t dt, int prog, int is_block, int odd, int logM, int logC_hint, int64_t batch,
                 const Sched &sc);
Status sched_save(const char *path);
Status sched_load(const char *path, int *loaded);

// Thread-local launch counter.
void count_launch();

// Kernel timing (diagnostics): when enabled, every kernel the library
// enqueues carries a start/stop event pair timestamped at its dispatch's
// begin and end (launch_kernel), grouped by kind.
enum ProfKind : int { PK_RESIDENT = 0, PK_PASS_A = 1, PK_PASS_B = 2, PK_PASS_D = 3, PK_BATCH = 4, PK_COUNT = 5 };
bool prof_enabled();
void prof_before(hipStream_t st);
void prof_after(int kind, hipStream_t st);
Status prof_start();
Status prof_stop(double *ms, int64_t *counts);

}  // namespace hk
