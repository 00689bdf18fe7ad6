// Explicit instantiation and dispatch of the row kernels for transform
// lengths N = odd * 2^k (odd = 3, 5) in one precision.  Included by
// hk_f32_odd.hip / hk_f64_odd.hip with HK_REAL, HK_NS and HK_SUFFIX set; the
// column kernels (which take the odd factor at run time) come from the
// power-of-two unit.  A lane of these rows holds the same bins of all `odd`
// sequences (the operand being transformed and the running spectral product:
// 2 * odd * E complex values), so their elements per lane are low, 4 (8 for
// the grouped float factor-3 pass-B rows of up to 512 points), with up to
// 512 lanes per row; double precision has the factor 3 only (a
// factor-5 lane would not fit its registers).  The adjoint program keeps four
// spectra per lane and is built for float with the factor 3 only (the other
// variants spill to scratch); other adjoint shapes use power-of-two lengths.
#pragma once
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

// only the row and grouped kernels are needed here
#define HK_ROWS_ONLY
#include "hk_kernels.hpp"

namespace hk {
namespace HK_NS {

// elements per lane of the odd-factor rows (plain and batched)
constexpr int ODD_E = 4;
static_assert(ODD_E == BatchRowE<3>::value && ODD_E == BatchRowE<5>::value, "batched odd rows use ODD_E");
// lanes per workgroup of the plain odd-factor rows, and the longest row
constexpr int ODD_ROW_MAXT = 512;
constexpr int ODD_MAX_LOGL = 11;
constexpr bool HAS_ODD5 = sizeof(T) == 4;

constexpr bool has_bwd(int odd) { return sizeof(T) == 4 && odd == 3; }

// Resident instances and pass-B rows are separate kernels (k_rows_res,
// k_rows_pass): each path gets its own register allocation.
// Forward pass-B rows one per lane group (no rows in turn) run k_rows_pass1
// where it fits the registers and the streamed kernel spills: the float
// factor 5 (2-4 % faster) and the double factor 3 with rows of up to 256
// points (7-9 % faster; 1024-point rows measured 2-3 % slower).  The float
// factor-3 rows measured 1-2 % slower that way at three waves per SIMD and
// keep the streamed kernel.
template <int L, int ODD>
static void *row_fn(int prog, bool res, bool one_row) {
  if (prog == PROG_BWD) {
    if constexpr (has_bwd(ODD))
      return res ? (void *)&k_rows_res<L, ODD_E, ODD_ROW_MAXT, PROG_BWD, ODD>
                 : (void *)&k_rows_pass<L, ODD_E, ODD_ROW_MAXT, PROG_BWD, ODD>;
    return nullptr;
  }
  if (res) return (void *)&k_rows_res<L, ODD_E, ODD_ROW_MAXT, PROG_FWD, ODD>;
  if constexpr (ODD == 5 || (sizeof(T) == 8 && L <= 256))
    if (one_row) return (void *)&k_rows_pass1<L, ODD_E, ODD_ROW_MAXT, ODD>;
  return (void *)&k_rows_pass<L, ODD_E, ODD_ROW_MAXT, PROG_FWD, ODD>;
}

template <int ODD>
static void *pick_row(int logL, int prog, bool res, bool one_row) {
  switch (logL) {
    case 0: return row_fn<1, ODD>(prog, res, one_row);
    case 1: return row_fn<2, ODD>(prog, res, one_row);
    case 2: return row_fn<4, ODD>(prog, res, one_row);
    case 3: return row_fn<8, ODD>(prog, res, one_row);
    case 4: return row_fn<16, ODD>(prog, res, one_row);
    case 5: return row_fn<32, ODD>(prog, res, one_row);
    case 6: return row_fn<64, ODD>(prog, res, one_row);
    case 7: return row_fn<128, ODD>(prog, res, one_row);
    case 8: return row_fn<256, ODD>(prog, res, one_row);
    case 9: return row_fn<512, ODD>(prog, res, one_row);
    case 10: return row_fn<1024, ODD>(prog, res, one_row);
    case 11: return row_fn<2048, ODD>(prog, res, one_row);
  }
  return nullptr;
}

static void *row_kernel(int odd, int logL, int E, int prog, bool res, bool one_row) {
  if (E != ODD_E || logL < 0 || logL > ODD_MAX_LOGL) return nullptr;
  if (odd == 3) return pick_row<3>(logL, prog, res, one_row);
  if constexpr (HAS_ODD5)
    if (odd == 5) return pick_row<5>(logL, prog, res, one_row);
  return nullptr;
}

template <int L, int ODD>
static void *group_fn(int kind) {
  if (kind == GK_RES) return (void *)&k_group<L, GK_RES, ODD>;
  if (kind == GK_ROWB) return (void *)&k_group<L, GK_ROWB, ODD>;
  return nullptr;
}
template <int ODD>
static void *pick_group(int kind, int logL) {
  switch (logL) {
    case 0: return group_fn<1, ODD>(kind);
    case 1: return group_fn<2, ODD>(kind);
    case 2: return group_fn<4, ODD>(kind);
    case 3: return group_fn<8, ODD>(kind);
    case 4: return group_fn<16, ODD>(kind);
    case 5: return group_fn<32, ODD>(kind);
    case 6: return group_fn<64, ODD>(kind);
    case 7: return group_fn<128, ODD>(kind);
    case 8: return group_fn<256, ODD>(kind);
    case 9: return group_fn<512, ODD>(kind);
    case 10: return group_fn<1024, ODD>(kind);
    case 11: return group_fn<2048, ODD>(kind);
  }
  return nullptr;
}
static void *group_kernel(int odd, int kind, int logL) {
  if (logL < 0 || logL > ODD_MAX_LOGL) return nullptr;
  if (odd == 3) return pick_group<3>(kind, logL);
  if constexpr (HAS_ODD5)
    if (odd == 5) return pick_group<5>(kind, logL);
  return nullptr;
}

template <int L, int E = ODD_E>
static KernelLimits lim_of() {
  using S = FFTShape<L, E>;
  KernelLimits k;
  k.tps = S::TPS;
  k.seq_lds = S::ROW_SEQ;
  k.lds_raw = S::LDS;
  k.elem_bytes = (int)sizeof(cx<T>);
  k.row_maxt = ODD_ROW_MAXT;
  return k;
}
static KernelLimits lim_pick(int logL) {
  switch (logL) {
    case 0: return lim_of<1>();
    case 1: return lim_of<2>();
    case 2: return lim_of<4>();
    case 3: return lim_of<8>();
    case 4: return lim_of<16>();
    case 5: return lim_of<32>();
    case 6: return lim_of<64>();
    case 7: return lim_of<128>();
    case 8: return lim_of<256>();
    case 9: return lim_of<512>();
    case 10: return lim_of<1024>();
    default: return lim_of<2048>();
  }
}

// Real-input resident rows: R2C_E elements per lane, up to 512 lanes (rows up
// to 4096 in float, 2048 in double).
constexpr int R2C_MAXT = 512;
template <int L>
static KernelLimits lim_r2c() {
  using RB = RealRowBody<T, L, R2C_E>;
  KernelLimits k;
  k.tps = RB::TPS;
  k.seq_lds = RB::SEQ_LDS;
  k.lds_raw = RB::SEQ_LDS;
  k.elem_bytes = (int)sizeof(cx<T>);
  k.row_maxt = R2C_MAXT;
  return k;
}
#define HK_R2C_CASES(X) X(0, 1) X(1, 2) X(2, 4) X(3, 8) X(4, 16) X(5, 32) X(6, 64) X(7, 128) X(8, 256) \
  X(9, 512) X(10, 1024) X(11, 2048) X(12, 4096)
static bool r2c_pick(int logL, KernelLimits *k, void **row, void **group) {
  if ((1 << logL) / R2C_E > R2C_MAXT) return false;  // a row must fit one workgroup
  switch (logL) {
#define HK_R2C_CASE(lg, L)                                        \
  case lg:                                                        \
    if constexpr (L / R2C_E <= R2C_MAXT) {                        \
      *k = lim_r2c<L>();                                          \
      *row = (void *)&k_rows_r2c<L, R2C_E, R2C_MAXT>;             \
      *group = (void *)&k_group_r2c<L>;                           \
      return true;                                                \
    }                                                             \
    return false;
    HK_R2C_CASES(HK_R2C_CASE)
#undef HK_R2C_CASE
  }
  return false;
}

// Pass-B row pairs of multipass real-input transforms: R2C_E elements per
// lane, a row per lane group, two lane groups per pair (limits are per pair:
// tps = lanes of a pair, seq_lds = its LDS), at most 512 lanes per pair.
template <int L>
static KernelLimits lim_r2cp() {
  using PB = RealPairRowBody<T, L, R2C_E>;
  KernelLimits k;
  k.tps = 2 * PB::TPS;
  k.seq_lds = 2 * PB::SEQ_LDS;
  k.lds_raw = 2 * PB::SEQ_LDS;
  k.elem_bytes = (int)sizeof(cx<T>);
  k.row_maxt = R2C_MAXT;
  return k;
}
static bool r2cp_pick(int logL, KernelLimits *k, void **row, void **group) {
  if (2 * ((1 << logL) / R2C_E) > R2C_MAXT) return false;
  switch (logL) {
#define HK_R2CP_CASE(lg, L)                                          \
  case lg:                                                           \
    if constexpr (2 * (L / R2C_E) <= R2C_MAXT) {                     \
      *k = lim_r2cp<L>();                                            \
      *row = (void *)&k_rows_r2c_pairs<L, R2C_E, R2C_MAXT>;          \
      *group = (void *)&k_group_r2c_pairs<L>;                        \
      return true;                                                   \
    }                                                                \
    return false;
    HK_R2C_CASES(HK_R2CP_CASE)
#undef HK_R2CP_CASE
  }
  return false;
}

static std::mutex g_attr_mu;

static hipError_t ensure_lds(void *fn, size_t bytes) {
  static std::map<void *, size_t> done;
  if (bytes <= 65536) return hipSuccess;
  std::lock_guard<std::mutex> lk(g_attr_mu);
  auto it = done.find(fn);
  if (it != done.end() && it->second >= bytes) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done[fn] = bytes;
  return e;
}

}  // namespace HK_NS

#define HK_CAT2(a, b) a##b
#define HK_CAT(a, b) HK_CAT2(a, b)

// This unit's copy of the twiddle tables.
hipError_t HK_CAT(init_tables_odd_, HK_SUFFIX)(const double *tw4096, const double *tw24) {
  using namespace HK_NS;
  std::vector<cx<T>> a(4096), b(4096);
  for (int j = 0; j < 4096; ++j) {
    a[j].x = (T)tw4096[2 * j];
    a[j].y = (T)tw4096[2 * j + 1];
    b[j].x = (T)tw24[2 * j];
    b[j].y = (T)tw24[2 * j + 1];
  }
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_tw4096), a.data(), sizeof(cx<T>) * 4096, 0, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tw24), b.data(), sizeof(cx<T>) * 4096, 0, hipMemcpyHostToDevice);
}

bool HK_CAT(limits_odd_, HK_SUFFIX)(int odd, int logL, int E, KernelLimits *out) {
  using namespace HK_NS;
  if ((odd != 3 && !(odd == 5 && HAS_ODD5)) || E != ODD_E || logL < 0 || logL > ODD_MAX_LOGL) return false;
  *out = lim_pick(logL);
  return true;
}

int HK_CAT(odd_row_e_, HK_SUFFIX)() { return HK_NS::ODD_E; }

int HK_CAT(r2c_row_e_, HK_SUFFIX)() { return HK_NS::R2C_E; }

bool HK_CAT(odd_bwd_ok_, HK_SUFFIX)(int odd) { return HK_NS::has_bwd(odd); }

hipError_t HK_CAT(launch_rows_odd_, HK_SUFFIX)(int odd, int logL, int E, int rows_per_wg, dim3 grid,
                                               const Shape &sh, const Ptrs &p0, const Strides &str, int64_t count,
                                               hipStream_t st) {
  using namespace HK_NS;
  void *fn = row_kernel(odd, logL, E, sh.prog, sh.resident != 0, sh.row_iters <= 1);
  KernelLimits k;
  if (!fn || sh.odd != odd || !HK_CAT(limits_odd_, HK_SUFFIX)(odd, logL, E, &k)) return hipErrorInvalidValue;
  const int threads = rows_per_wg * k.tps;
  if (threads < 1 || threads > ODD_ROW_MAXT) return hipErrorInvalidValue;
  size_t lds = (size_t)rows_per_wg * k.seq_lds * sizeof(cx<T>);
  const size_t red = (size_t)threads * sizeof(cx<T>);
  if (lds < red) lds = red;
  hipError_t e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  Shape shc = sh;
  Ptrs pc = p0;
  Strides sc = str;
  int64_t cnt = count;
  void *args[] = {&shc, &pc, &sc, &cnt};
  return launch_kernel(fn, grid, dim3(threads), args, lds, st);
}

bool HK_CAT(limits_r2c_, HK_SUFFIX)(int logL, int E, KernelLimits *out) {
  using namespace HK_NS;
  void *r, *g;
  if (E != R2C_E) return false;
  return r2c_pick(logL, out, &r, &g);
}

hipError_t HK_CAT(launch_rows_r2c_, HK_SUFFIX)(int logL, int E, int rows_per_wg, dim3 grid, const Shape &sh,
                                               const Ptrs &p0, const Strides &str, int64_t count, hipStream_t st) {
  using namespace HK_NS;
  KernelLimits k;
  void *fn = nullptr, *g = nullptr;
  if (E != R2C_E || !sh.r2c || !r2c_pick(logL, &k, &fn, &g)) return hipErrorInvalidValue;
  const int threads = rows_per_wg * k.tps;
  if (threads < 1 || threads > R2C_MAXT) return hipErrorInvalidValue;
  size_t lds = (size_t)rows_per_wg * k.seq_lds * sizeof(cx<T>);
  lds = std::max(lds, (size_t)threads * sizeof(cx<T>));
  hipError_t e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  Shape shc = sh;
  Ptrs pc = p0;
  Strides sc = str;
  int64_t cnt = count;
  void *args[] = {&shc, &pc, &sc, &cnt};
  return launch_kernel(fn, grid, dim3(threads), args, lds, st);
}

hipError_t HK_CAT(launch_group_r2c_, HK_SUFFIX)(const BatchArgs &args, int logL, int ntasks, hipStream_t st) {
  using namespace HK_NS;
  if (ntasks <= 0) return hipSuccess;
  KernelLimits k;
  void *r = nullptr, *fn = nullptr;
  if (!r2c_pick(logL, &k, &r, &fn) || k.tps > BATCH_BLK) return hipErrorInvalidValue;
  const size_t lds = std::max((size_t)BATCH_BLK, (size_t)(BATCH_BLK / k.tps) * k.seq_lds) * sizeof(cx<T>);
  hipError_t e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  BatchArgs a = args;
  void *kargs[] = {&a};
  return launch_kernel(fn, dim3((unsigned)ntasks), dim3(BATCH_BLK), kargs, lds, st);
}

bool HK_CAT(limits_r2cp_, HK_SUFFIX)(int logL, int E, KernelLimits *out) {
  using namespace HK_NS;
  void *r, *g;
  if (E != R2C_E) return false;
  return r2cp_pick(logL, out, &r, &g);
}

hipError_t HK_CAT(launch_rows_r2cp_, HK_SUFFIX)(int logL, int E, int groups_per_wg, dim3 grid, const Shape &sh,
                                                const Ptrs &p0, const Strides &str, int64_t count, hipStream_t st) {
  using namespace HK_NS;
  KernelLimits k;
  void *fn = nullptr, *g = nullptr;
  if (E != R2C_E || !sh.r2c || sh.resident || !r2cp_pick(logL, &k, &fn, &g)) return hipErrorInvalidValue;
  const int threads = groups_per_wg * k.tps;
  if (threads < 1 || threads > R2C_MAXT) return hipErrorInvalidValue;
  size_t lds = (size_t)groups_per_wg * k.seq_lds * sizeof(cx<T>);
  lds = std::max(lds, (size_t)threads * sizeof(cx<T>));
  hipError_t e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  Shape shc = sh;
  Ptrs pc = p0;
  Strides sc = str;
  int64_t cnt = count;
  void *args[] = {&shc, &pc, &sc, &cnt};
  return launch_kernel(fn, grid, dim3(threads), args, lds, st);
}

hipError_t HK_CAT(launch_group_r2cp_, HK_SUFFIX)(const BatchArgs &args, int logL, int ntasks, hipStream_t st) {
  using namespace HK_NS;
  if (ntasks <= 0) return hipSuccess;
  KernelLimits k;
  void *r = nullptr, *fn = nullptr;
  if (!r2cp_pick(logL, &k, &r, &fn) || k.tps > BATCH_BLK) return hipErrorInvalidValue;
  const size_t lds = std::max((size_t)BATCH_BLK, (size_t)(BATCH_BLK / k.tps) * k.seq_lds) * sizeof(cx<T>);
  hipError_t e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  BatchArgs a = args;
  void *kargs[] = {&a};
  return launch_kernel(fn, dim3((unsigned)ntasks), dim3(BATCH_BLK), kargs, lds, st);
}

namespace HK_NS {
// Limits of the grouped pass-B rows (GroupRowbE elements per lane).
template <int L, int ODD>
static KernelLimits lim_rowb() {
  return lim_of<L, GroupRowbE<L, ODD>::value>();
}
template <int ODD>
static KernelLimits lim_rowb_pick(int logL) {
  switch (logL) {
    case 0: return lim_rowb<1, ODD>();
    case 1: return lim_rowb<2, ODD>();
    case 2: return lim_rowb<4, ODD>();
    case 3: return lim_rowb<8, ODD>();
    case 4: return lim_rowb<16, ODD>();
    case 5: return lim_rowb<32, ODD>();
    case 6: return lim_rowb<64, ODD>();
    case 7: return lim_rowb<128, ODD>();
    case 8: return lim_rowb<256, ODD>();
    case 9: return lim_rowb<512, ODD>();
    case 10: return lim_rowb<1024, ODD>();
    default: return lim_rowb<2048, ODD>();
  }
}
}  // namespace HK_NS

int HK_CAT(group_rowb_tps_, HK_SUFFIX)(int odd, int logL) {
  using namespace HK_NS;
  if (logL < 0 || logL > ODD_MAX_LOGL) return 0;
  return (odd == 5 ? lim_rowb_pick<5>(logL) : lim_rowb_pick<3>(logL)).tps;
}

hipError_t HK_CAT(launch_group_odd_, HK_SUFFIX)(const BatchArgs &args, int odd, int kind, int logL, int ntasks,
                                                hipStream_t st) {
  using namespace HK_NS;
  if (ntasks <= 0) return hipSuccess;
  void *fn = group_kernel(odd, kind, logL);
  KernelLimits k;
  if (!fn || !HK_CAT(limits_odd_, HK_SUFFIX)(odd, logL, ODD_E, &k)) return hipErrorInvalidValue;
  if (kind == GK_ROWB) k = odd == 5 ? lim_rowb_pick<5>(logL) : lim_rowb_pick<3>(logL);
  if (k.tps > BATCH_BLK) return hipErrorInvalidValue;
  const size_t lds = std::max((size_t)BATCH_BLK, (size_t)(BATCH_BLK / k.tps) * k.seq_lds) * sizeof(cx<T>);
  hipError_t e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  BatchArgs a = args;
  void *kargs[] = {&a};
  return launch_kernel(fn, dim3((unsigned)ntasks), dim3(BATCH_BLK), kargs, lds, st);
}

}  // namespace hk
