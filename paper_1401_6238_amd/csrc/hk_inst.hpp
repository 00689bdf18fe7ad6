// Explicit instantiation and dispatch of the kernels for one precision.
// Included by hk_f32.hip / hk_f64.hip with HK_REAL, HK_NS and HK_SUFFIX set.
#pragma once
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "hk_kernels.hpp"

namespace hk {
namespace HK_NS {

// Rows of 4 elements per lane take up to 512 lanes: fewer registers, more
// waves per SIMD, more LDS exchanges (the autotuner picks them where that
// pays, e.g. in batches); 8 and 16 elements per lane take up to ROW_MAXT.
constexpr int ROW_MAXT_E4 = 512;
constexpr int row_maxt(int E) { return E == 4 ? ROW_MAXT_E4 : ROW_MAXT; }

template <int L, int E>
static void *row_fn(int prog) {
  if (prog == PROG_BWD) return (void *)&k_rows<L, E, row_maxt(E), PROG_BWD>;
  if (prog == PROG_FWD_SPEC || prog == PROG_BWD_SPEC) {
    // spectra exist for the three-pass layouts only, whose rows have >= 2^7 points
    if constexpr (L >= 128) {
      if (prog == PROG_FWD_SPEC) return (void *)&k_rows<L, E, row_maxt(E), PROG_FWD_SPEC>;
      return (void *)&k_rows<L, E, row_maxt(E), PROG_BWD_SPEC>;
    }
    return nullptr;
  }
  return (void *)&k_rows<L, E, row_maxt(E), PROG_FWD>;
}
template <int L, int E>
static void *col_fn(int var) {
  if (var == CV_ODD) return (void *)&k_cols<L, E, COL_MAXT, CV_ODD>;
  if (var == CV_R2C) return (void *)&k_cols<L, E, COL_MAXT, CV_R2C>;
  if (var >= CV_BODD1) {
    // BHHB grids with odd factors: columns of 2^6 .. 2^11 points per sequence
    if constexpr (L >= 64 && L <= 2048) {
      if (var == CV_BODD1) return (void *)&k_cols<L, E, COL_MAXT, CV_BODD1>;
      if (var == CV_BODD3) return (void *)&k_cols<L, E, COL_MAXT, CV_BODD3>;
      return (void *)&k_cols<L, E, COL_MAXT, CV_BODD5>;
    }
    return nullptr;
  }
  return (void *)&k_cols<L, E, COL_MAXT, CV_POW2>;
}

template <int E>
static void *pick_row(int logL, int prog) {
  switch (logL) {
    case 0: return row_fn<1, E>(prog);
    case 1: return row_fn<2, E>(prog);
    case 2: return row_fn<4, E>(prog);
    case 3: return row_fn<8, E>(prog);
    case 4: return row_fn<16, E>(prog);
    case 5: return row_fn<32, E>(prog);
    case 6: return row_fn<64, E>(prog);
    case 7: return row_fn<128, E>(prog);
    case 8: return row_fn<256, E>(prog);
    case 9: return row_fn<512, E>(prog);
    case 10: return row_fn<1024, E>(prog);
    case 11: return row_fn<2048, E>(prog);
    case 12: return row_fn<4096, E>(prog);
  }
  return nullptr;
}
template <int E>
static void *pick_col(int logL, int var) {
  switch (logL) {
    case 0: return col_fn<1, E>(var);
    case 1: return col_fn<2, E>(var);
    case 2: return col_fn<4, E>(var);
    case 3: return col_fn<8, E>(var);
    case 4: return col_fn<16, E>(var);
    case 5: return col_fn<32, E>(var);
    case 6: return col_fn<64, E>(var);
    case 7: return col_fn<128, E>(var);
    case 8: return col_fn<256, E>(var);
    case 9: return col_fn<512, E>(var);
    case 10: return col_fn<1024, E>(var);
    case 11: return col_fn<2048, E>(var);
    case 12: return col_fn<4096, E>(var);
  }
  return nullptr;
}

static void *row_kernel(int logL, int E, int prog) {
  if (logL < 0 || logL > MAX_LOGL) return nullptr;
  if (E == 4) return logL <= 11 ? pick_row<4>(logL, prog) : nullptr;
  if (E == 8) return pick_row<8>(logL, prog);
  if (E == 16) return pick_row<16>(logL, prog);
  return nullptr;
}
static void *col_kernel(int logL, int E, int var) {
  if (logL < 0 || logL > MAX_LOGL) return nullptr;
  if (E == 8) return pick_col<8>(logL, var);
  if (E == 16) return pick_col<16>(logL, var);
  return nullptr;
}

template <int L, int E>
static KernelLimits lim_of() {
  using S = FFTShape<L, E>;
  KernelLimits k;
  k.tps = S::TPS;
  k.seq_lds = S::ROW_SEQ;
  k.lds_raw = S::LDS;
  k.elem_bytes = (int)sizeof(cx<T>);
  k.row_maxt = row_maxt(E);
  return k;
}

template <int E>
static KernelLimits lim_pick(int logL) {
  switch (logL) {
    case 0: return lim_of<1, E>();
    case 1: return lim_of<2, E>();
    case 2: return lim_of<4, E>();
    case 3: return lim_of<8, E>();
    case 4: return lim_of<16, E>();
    case 5: return lim_of<32, E>();
    case 6: return lim_of<64, E>();
    case 7: return lim_of<128, E>();
    case 8: return lim_of<256, E>();
    case 9: return lim_of<512, E>();
    case 10: return lim_of<1024, E>();
    case 11: return lim_of<2048, E>();
    default: return lim_of<4096, E>();
  }
}

// Column tasks of odd-factor transforms run in the ODD = 3 variant of the
// column group kernel (their odd factor is read from the shape), those of
// real-input transforms in the ODD = 2 one.
template <int L>
static void *group_fn(int kind, int var) {
  switch (kind) {
    case GK_RES: return var != CV_POW2 ? nullptr : (void *)&k_group<L, GK_RES>;
    case GK_ROWB: return var != CV_POW2 ? nullptr : (void *)&k_group<L, GK_ROWB>;
    case GK_COL:
      if (var == CV_ODD) return (void *)&k_group<L, GK_COL, 3>;
      if (var == CV_R2C) return (void *)&k_group<L, GK_COL, 2>;
      return (void *)&k_group<L, GK_COL>;
  }
  return nullptr;
}
static void *group_kernel(int kind, int logL, int var) {
  if (kind == GK_ALPHA) return (void *)&k_group<1, GK_ALPHA>;
  switch (logL) {
    case 0: return group_fn<1>(kind, var);
    case 1: return group_fn<2>(kind, var);
    case 2: return group_fn<4>(kind, var);
    case 3: return group_fn<8>(kind, var);
    case 4: return group_fn<16>(kind, var);
    case 5: return group_fn<32>(kind, var);
    case 6: return group_fn<64>(kind, var);
    case 7: return group_fn<128>(kind, var);
    case 8: return group_fn<256>(kind, var);
    case 9: return group_fn<512>(kind, var);
    case 10: return group_fn<1024>(kind, var);
    case 11: return group_fn<2048>(kind, var);
    case 12: return group_fn<4096>(kind, var);
  }
  return nullptr;
}

static std::mutex g_attr_mu;

static hipError_t ensure_lds(void *fn, size_t bytes) {
  // Raise a kernel's dynamic-LDS limit only when a launch needs more than
  // the value already set for it.
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

hipError_t HK_CAT(init_tables_, HK_SUFFIX)(const double *tw4096, const double *tw24) {
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

bool HK_CAT(limits_, HK_SUFFIX)(int logL, int E, KernelLimits *out) {
  using namespace HK_NS;
  if (logL < 0 || logL > MAX_LOGL) return false;
  if (E == 4 && logL <= 11) *out = lim_pick<4>(logL);
  else if (E == 8) *out = lim_pick<8>(logL);
  else if (E == 16) *out = lim_pick<16>(logL);
  else return false;
  return true;
}

hipError_t HK_CAT(launch_rows_, HK_SUFFIX)(int logL, int E, int rows_per_wg, dim3 grid, const Shape &sh,
                                           const Ptrs &p0, const Strides &str, int64_t count, hipStream_t st) {
  using namespace HK_NS;
  const bool spec = !sh.resident && shape_has_spec(sh);
  const int prog = !spec ? sh.prog : (sh.prog == PROG_FWD ? (int)PROG_FWD_SPEC : (int)PROG_BWD_SPEC);
  void *fn = row_kernel(logL, E, prog);
  KernelLimits k;
  if (!fn || !HK_CAT(limits_, HK_SUFFIX)(logL, E, &k)) return hipErrorInvalidValue;
  const int threads = rows_per_wg * k.tps;
  if (threads < 1 || threads > k.row_maxt) return hipErrorInvalidValue;
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

hipError_t HK_CAT(launch_cols_, HK_SUFFIX)(int logL, int E, int tw, int xcd, dim3 grid, const Shape &sh,
                                           const Ptrs &p0, const Strides &str, const ColJob *jobs, int njobs,
                                           hipStream_t st) {
  using namespace HK_NS;
  int var = sh.r2c ? CV_R2C : (sh.odd > 1 ? CV_ODD : CV_POW2);
  if (sh.is_block && (sh.odd > 1 || sh.odd_c > 1)) var = sh.odd_c == 5 ? CV_BODD5 : (sh.odd_c == 3 ? CV_BODD3 : CV_BODD1);
  void *fn = col_kernel(logL, E, var);
  KernelLimits k;
  if (!fn || !HK_CAT(limits_, HK_SUFFIX)(logL, E, &k)) return hipErrorInvalidValue;
  const int threads = tw * k.tps;
  if (threads < 1 || threads > COL_MAXT || njobs < 1 || njobs > MAXOPS) return hipErrorInvalidValue;
  size_t lds = (size_t)tw * k.lds_raw * sizeof(cx<T>);
  lds = std::max(lds, (size_t)threads * sizeof(cx<T>));  // room for the scalar reduction
  hipError_t e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  Shape shc = sh;
  Ptrs pc = p0;
  Strides sc = str;
  ColJobs cj;
  memset(&cj, 0, sizeof(cj));
  for (int i = 0; i < njobs; ++i) cj.j[i] = jobs[i];
  cj.n = njobs;
  cj.xcd = xcd ? 1 : 0;
  void *args[] = {&shc, &pc, &sc, &cj};
  return launch_kernel(fn, grid, dim3(threads), args, lds, st);
}

hipError_t HK_CAT(launch_alpha_, HK_SUFFIX)(const Shape &sh, const Ptrs &p0, const Strides &str, int64_t npart,
                                            int64_t count, hipStream_t st) {
  using namespace HK_NS;
  Shape shc = sh;
  Ptrs pc = p0;
  Strides sc = str;
  int64_t n = npart;
  void *args[] = {&shc, &pc, &sc, &n};
  return launch_kernel((void *)&k_alpha, dim3((unsigned)count), dim3(256), args, 0, st);
}

void HK_CAT(batch_geometry_, HK_SUFFIX)(int *blk, int *e_row, int *e_col, size_t *lds_bytes) {
  using namespace HK_NS;
  *blk = BATCH_BLK;
  *e_row = BATCH_E_ROW;
  *e_col = BATCH_E_COL;
  size_t mx = (size_t)BATCH_BLK;  // reduction scratch
  for (int l = 0; l <= MAX_LOGL; ++l) {
    KernelLimits kr, kc;
    HK_CAT(limits_, HK_SUFFIX)(l, BATCH_E_ROW, &kr);
    HK_CAT(limits_, HK_SUFFIX)(l, BATCH_E_COL, &kc);
    if (kr.tps <= BATCH_BLK) mx = std::max(mx, (size_t)(BATCH_BLK / kr.tps) * kr.seq_lds);
    if (kc.tps <= BATCH_BLK) {
      const int tw = BATCH_BLK / kc.tps;
      mx = std::max(mx, (size_t)tw * kc.lds_raw);
    }
  }
  *lds_bytes = mx * sizeof(cx<T>);
}

// LDS (elements) of one grouped launch: its own length's need, plus room for
// the workgroup reductions.
static size_t group_lds_elems(int kind, int logL) {
  using namespace HK_NS;
  size_t mx = (size_t)BATCH_BLK;
  if (kind == GK_RES || kind == GK_ROWB) {
    KernelLimits kr;
    HK_CAT(limits_, HK_SUFFIX)(logL, kind == GK_ROWB && logL <= 11 ? 4 : BATCH_E_ROW, &kr);
    if (kr.tps <= BATCH_BLK) mx = std::max(mx, (size_t)(BATCH_BLK / kr.tps) * kr.seq_lds);
  } else if (kind == GK_COL) {
    KernelLimits kc;
    HK_CAT(limits_, HK_SUFFIX)(logL, BATCH_E_COL, &kc);
    if (kc.tps <= BATCH_BLK) {
      const int tw = BATCH_BLK / kc.tps;
      mx = std::max(mx, (size_t)tw * kc.lds_raw);
    }
  }
  return mx;
}

hipError_t HK_CAT(launch_group_, HK_SUFFIX)(const BatchArgs &args, int kind, int logL, int odd, int ntasks,
                                            hipStream_t st) {
  using namespace HK_NS;
  if (ntasks <= 0) return hipSuccess;
  if (logL < 0 || logL > MAX_LOGL) return hipErrorInvalidValue;
  void *fn = group_kernel(kind, logL, odd == 2 ? CV_R2C : (odd > 1 ? CV_ODD : CV_POW2));
  if (!fn) return hipErrorInvalidValue;
  const size_t lds = group_lds_elems(kind, logL) * sizeof(cx<T>);
  hipError_t e = ensure_lds(fn, lds);
  if (e != hipSuccess) return e;
  BatchArgs a = args;
  void *kargs[] = {&a};
  return launch_kernel(fn, dim3((unsigned)ntasks), dim3(BATCH_BLK), kargs, lds, st);
}

hipError_t HK_CAT(batch_resident_, HK_SUFFIX)(int *blocks_per_cu) {
  using namespace HK_NS;
  int blk, er, ec;
  size_t lds;
  HK_CAT(batch_geometry_, HK_SUFFIX)(&blk, &er, &ec, &lds);
  hipError_t e = ensure_lds((void *)&k_batch, lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void *)&k_batch, blk, lds);
}

hipError_t HK_CAT(launch_batch_, HK_SUFFIX)(const BatchArgs &args, int grid, hipStream_t st) {
  using namespace HK_NS;
  // zero the control block with a kernel (not a memset node), so that graph
  // replays start from a clean queue
  BatchCtl *b = args.bctl;
  void *rargs[] = {&b};
  // not profiled: the event pair belongs to the batch kernel below
  hipError_t e = hipLaunchKernel((void *)&k_batch_reset, dim3(1), dim3(64), rargs, 0, st);
  if (e != hipSuccess) return e;
  int blk, er, ec;
  size_t lds;
  HK_CAT(batch_geometry_, HK_SUFFIX)(&blk, &er, &ec, &lds);
  e = ensure_lds((void *)&k_batch, lds);
  if (e != hipSuccess) return e;
  BatchArgs a = args;
  void *kargs[] = {&a};
  return launch_cooperative((void *)&k_batch, dim3((unsigned)grid), dim3(blk), kargs, lds, st);
}

hipError_t HK_CAT(launch_copy_cols_, HK_SUFFIX)(void *out, const void *src, const int32_t *pairs, int64_t npairs,
                                                int64_t rows, bool complex_elems, hipStream_t st) {
  using namespace HK_NS;
  const unsigned gx = (unsigned)std::min<int64_t>(64, (rows + 255) / 256);
  int64_t r = rows;
  for (int64_t p0 = 0; p0 < npairs; p0 += 65535) {
    const unsigned gy = (unsigned)std::min<int64_t>(65535, npairs - p0);
    const int32_t *pp = pairs + 2 * p0;
    hipError_t e;
    if (complex_elems) {
      cx<T> *o = (cx<T> *)out;
      const cx<T> *s = (const cx<T> *)src;
      void *args[] = {&o, &s, &pp, &r};
      e = launch_kernel((void *)&k_copy_cols<cx<T>>, dim3(gx, gy), dim3(256), args, 0, st);
    } else {
      T *o = (T *)out;
      const T *s = (const T *)src;
      void *args[] = {&o, &s, &pp, &r};
      e = launch_kernel((void *)&k_copy_cols<T>, dim3(gx, gy), dim3(256), args, 0, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace hk
