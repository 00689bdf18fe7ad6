// Kernels and their host-side launchers, instantiated once per real type by
// hk_f32.hip and hk_f64.hip (HK_REAL = float / double).
#pragma once
#include <hip/hip_runtime.h>

#include "hk_bodies.hpp"
#include "hk_launch.hpp"

#ifndef HK_REAL
#error "HK_REAL must be defined"
#endif

namespace hk {
namespace HK_NS {

using T = HK_REAL;

// Twiddle tables of this precision, filled once per device by init_tables():
// g_tw4096[j] = exp(-2 pi i j / 4096), g_tw24[j] = exp(-2 pi i j / 2^24).
static __device__ cx<T> g_tw4096[4096];
static __device__ cx<T> g_tw24[4096];

struct ColJobs {
  ColJob j[MAXOPS];
  int32_t n;
  int32_t xcd;  // 1: XCD-local tile numbering (xcd_local_tile)
};

// Rows of length L (ODD sequences each): resident instances
// (blockIdx.x * rows + rw) or pass-B rows of instance blockIdx.y.  PATH
// picks both at run time (sh.resident) or one of them at compile time.
enum : int { ROWS_ANY = 0, ROWS_RES = 1, ROWS_PASS = 2 };
template <int L, int E, int PROG, int ODD, int PATH>
__device__ __forceinline__ void rows_body(const Shape &sh, const Ptrs &p0, const Strides &str, int64_t count) {
  using RB = RowBody<T, L, E, ODD>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *smem = (cx<T> *)smem_raw;
  const int tid = threadIdx.x;
  const int rows = blockDim.x / RB::TPS;
  const int rw = tid / RB::TPS;
  const int t = tid % RB::TPS;
  cx<T> *lds = smem + rw * RB::SEQ_LDS;
  cx<T> *red = smem;  // reused for reductions after the transforms
  if constexpr (PATH != ROWS_PASS) {
    if (PATH == ROWS_RES || sh.resident) {
      const int64_t inst = (int64_t)blockIdx.x * rows + rw;
      const bool valid = inst < count;
      const PV P{&p0, &str, valid ? inst : 0, nullptr};
      if (PROG == PROG_BWD || PROG == PROG_BWD_SPEC) {
        RB::template run_bwd<PROG == PROG_BWD_SPEC>(sh, P, 0, valid, t, lds, true, g_tw24, g_tw4096);
        return;
      }
      const cx<T> part = RB::run_fwd(sh, P, 0, valid, t, lds, true, g_tw24, g_tw4096);
      if (sh.want_alpha) {
        const cx<T> tot = segment_sum(part, red, tid, RB::TPS);
        if (valid && t == 0) store_out<T>(P.alpha(), 0, tot, sh.real_out);
      }
      return;
    }
  }
  if constexpr (PATH != ROWS_RES) {
    const int64_t inst = blockIdx.y;
    const PV P{&p0, &str, inst, nullptr};
    // rows of this workgroup: (blockIdx.x * K + it) * rows + rw, it < K
    const int K = sh.row_iters > 1 ? sh.row_iters : 1;
    const int64_t row0 = (int64_t)blockIdx.x * K * rows + rw;
    if (PROG == PROG_BWD || PROG == PROG_BWD_SPEC) {
      RB::template run_bwd_rows<PROG == PROG_BWD_SPEC>(sh, P, row0, rows, K, t, lds, g_tw24, g_tw4096);
      return;
    }
    const cx<T> part =
        RB::template run_fwd_rows<PROG == PROG_FWD_SPEC>(sh, P, row0, rows, K, t, lds, g_tw24, g_tw4096);
    if (sh.want_alpha) {
      // One partial sum per workgroup; the next kernel in the stream (pass D
      // or the reduction kernel) adds them in index order.  No cross-workgroup
      // fence is needed: the kernel boundary makes them visible.
      const cx<T> tot = (blockDim.x & 63) == 0 ? block_sum(part, red, tid) : ragged_sum(part, red, tid, (int)blockDim.x);
      if (tid == 0) ws_partials<T>(sh, P)[blockIdx.x] = tot;
    }
  }
}

template <int L, int E, int MAXT, int PROG, int ODD = 1>
__global__ void __launch_bounds__(MAXT) k_rows(Shape sh, Ptrs p0, Strides str, int64_t count) {
  rows_body<L, E, PROG, ODD, ROWS_ANY>(sh, p0, str, count);
}
// The odd-factor rows come as two kernels, resident instances and pass-B
// rows: compiled as one kernel, both paths took the larger path's register
// count (float factor 3: up to 225 VGPRs against up to 163 for the resident
// rows alone; the factor-5 resident rows spilled to scratch).
template <int L, int E, int MAXT, int PROG, int ODD>
__global__ void __launch_bounds__(MAXT) k_rows_res(Shape sh, Ptrs p0, Strides str, int64_t count) {
  rows_body<L, E, PROG, ODD, ROWS_RES>(sh, p0, str, count);
}
template <int L, int E, int MAXT, int PROG, int ODD>
__global__ void __launch_bounds__(MAXT) k_rows_pass(Shape sh, Ptrs p0, Strides str, int64_t count) {
  rows_body<L, E, PROG, ODD, ROWS_PASS>(sh, p0, str, count);
}

// Pass-B rows one per lane group, without rows in turn (forward program):
// the float factor-5 and double factor-3 rows when a schedule takes one row
// per lane group.  Without the next row's operand in flight they spill less:
// none up to 256-point float and 64-point double rows, 8-72 bytes per lane
// beyond, against 12-248 for the streamed form.
template <int L, int E, int MAXT, int ODD>
__global__ void __launch_bounds__(MAXT) k_rows_pass1(Shape sh, Ptrs p0, Strides str, int64_t count) {
  using RB = RowBody<T, L, E, ODD>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *smem = (cx<T> *)smem_raw;
  const int tid = threadIdx.x;
  const int rows = blockDim.x / RB::TPS;
  const int rw = tid / RB::TPS;
  const int t = tid % RB::TPS;
  const PV P{&p0, &str, (int64_t)blockIdx.y, nullptr};
  const int64_t row = (int64_t)blockIdx.x * rows + rw;
  const bool valid = row < pass_rows(sh);
  const cx<T> part = RB::run_fwd(sh, P, row, valid, t, smem + rw * RB::SEQ_LDS, false, g_tw24, g_tw4096);
  if (sh.want_alpha) {
    const cx<T> tot = (blockDim.x & 63) == 0 ? block_sum(part, smem, tid) : ragged_sum(part, smem, tid, (int)blockDim.x);
    if (tid == 0) ws_partials<T>(sh, P)[blockIdx.x] = tot;
  }
}

// Real-input resident rows (RealRowBody): instance blockIdx.x * rows + rw.
template <int L, int E, int MAXT>
__global__ void __launch_bounds__(MAXT) k_rows_r2c(Shape sh, Ptrs p0, Strides str, int64_t count) {
  using RB = RealRowBody<T, L, E>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *smem = (cx<T> *)smem_raw;
  const int tid = threadIdx.x;
  const int rw = tid / RB::TPS;
  const int t = tid % RB::TPS;
  const int rows = blockDim.x / RB::TPS;
  const int64_t inst = (int64_t)blockIdx.x * rows + rw;
  const bool valid = inst < count;
  const PV P{&p0, &str, valid ? inst : 0, nullptr};
  const cx<T> part = RB::run_fwd(sh, P, valid, t, smem + rw * RB::SEQ_LDS, g_tw24, g_tw4096);
  if (sh.want_alpha) {
    const cx<T> tot = segment_sum(part, smem, tid, RB::TPS);
    if (valid && t == 0) store_out<T>(P.alpha(), 0, tot, sh.real_out);
  }
}

// Pass B of multipass real-input transforms (RealPairRowBody): row pairs
// blockIdx.x * pairs + pw of instance blockIdx.y, two lane groups each.
template <int L, int E, int MAXT>
__global__ void __launch_bounds__(MAXT) k_rows_r2c_pairs(Shape sh, Ptrs p0, Strides str, int64_t count) {
  using PB = RealPairRowBody<T, L, E>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *smem = (cx<T> *)smem_raw;
  const int tid = threadIdx.x;
  const int grp = tid / PB::TPS;
  const int t = tid % PB::TPS;
  const int pw = grp >> 1, g = grp & 1;
  const int pairs = blockDim.x / (2 * PB::TPS);
  const PV P{&p0, &str, (int64_t)blockIdx.y, nullptr};
  const int64_t npairs = ((int64_t)1 << sh.logC) / 2;
  const int64_t pi = (int64_t)blockIdx.x * pairs + pw;
  const bool valid = pi < npairs;
  const cx<T> part =
      PB::run_fwd(sh, P, valid ? pi : 0, g, valid, t, smem + pw * 2 * PB::SEQ_LDS, g_tw24, g_tw4096);
  if (sh.want_alpha) {
    const cx<T> tot = ragged_sum(part, smem, tid, (int)blockDim.x);
    if (tid == 0) ws_partials<T>(sh, P)[blockIdx.x] = tot;
  }
}

// Deterministic sum of the pass-B partial sums of one instance (count
// partials, fixed tree order) by one workgroup; lane 0 stores the scalar
// product.  `red` holds at least blockDim.x elements.
__device__ __forceinline__ void reduce_partials(const Shape &sh, const PV &P, int64_t count, cx<T> *red) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;  // a power of two
  const cx<T> *part = ws_partials<T>(sh, P);
  cx<T> v = czero<T>();
  for (int64_t i = tid; i < count; i += nthr) v = cadd(v, part[i]);
  const cx<T> tot = segment_sum(v, red, tid, nthr);
  if (tid == 0) store_out<T>(P.alpha(), 0, tot, sh.real_out);
}

#ifndef HK_ROWS_ONLY
// Scalar-only products: sums the pass-B partials (grid.x = instances).
__global__ void __launch_bounds__(256) k_alpha(Shape sh, Ptrs p0, Strides str, int64_t count) {
  __shared__ cx<T> red[256];
  const PV P{&p0, &str, (int64_t)blockIdx.x, nullptr};
  reduce_partials(sh, P, count, red);
}
#endif

// Workgroups are dealt to the eight XCDs round-robin by linear id.  The
// column passes renumber them so that each XCD runs one contiguous eighth of
// the column tiles of every (job, instance) slice: neighbouring tiles share
// 128-byte lines (a tile is TW elements wide), which then meet in the same
// L2 instead of being fetched and written back once per XCD, and every XCD
// gets the same share of each operand.  Slices are taken in order, so the
// tiles running at one time are close in memory.  A bijection of the grid
// whatever the hardware's actual dealing order; grids whose x extent is not
// a multiple of 8 keep the identity.
struct Tile3 {
  uint32_t x, y, z;
};
__device__ __forceinline__ Tile3 xcd_local_tile() {
  const uint32_t gx = gridDim.x, gy = gridDim.y;
  if (gx % 8 != 0) return Tile3{blockIdx.x, blockIdx.y, blockIdx.z};
  const uint32_t lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const uint32_t per = gx / 8, xcd = lin % 8, j = lin / 8;
  const uint32_t slice = j / per;
  return Tile3{xcd * per + j % per, slice % gy, slice / gy};
}

// Column-kernel variants: power-of-two complex transforms, odd factor 3 or 5
// (tiles over virtual columns), real inputs (real arrays as complex pairs).
enum ColVar : int { CV_POW2 = 0, CV_ODD = 1, CV_R2C = 2, CV_BODD1 = 3, CV_BODD3 = 4, CV_BODD5 = 5 };
// BHHB grids with odd factors: CV_BODD<k> tiles the row axis's odd * R
// virtual columns and carries the column axis's odd factor k (1: none).
constexpr int bodd_factor(int var) { return var == CV_BODD5 ? 5 : (var == CV_BODD3 ? 3 : 1); }
template <int L, int E, int MAXT, int VAR = CV_POW2>
__global__ void __launch_bounds__(MAXT) k_cols(Shape sh, Ptrs p0, Strides str, ColJobs jobs) {
  using CB = ColBody<T, L, E>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *smem = (cx<T> *)smem_raw;
  const Tile3 b = jobs.xcd ? xcd_local_tile() : Tile3{blockIdx.x, blockIdx.y, blockIdx.z};
  const ColJob &job = jobs.j[b.y];
  const int TW = blockDim.x / CB::TPS;
  const int64_t v0 = (int64_t)b.x * TW;  // first virtual column of the tile
  const PV P{&p0, &str, (int64_t)b.z, nullptr};
  if (job.kind == COL_D && job.npart > 0 && b.x == 0 && b.y == 0) {
    // the scalar product rides on the first pass-D workgroup
    reduce_partials(sh, P, job.npart, smem);
    __syncthreads();
  }
  if constexpr (VAR == CV_ODD) {
    // tiles over the odd * R virtual columns; a tile inside one sequence
    // whose storage columns are all pruned has nothing to do
    const int64_t R = (int64_t)1 << sh.logR;
    if (v0 >= (int64_t)sh.odd * R) return;
    if (TW <= R && (v0 & (R - 1)) >= job.ncols) return;
    CB::run_odd(sh, P, job, v0, TW, threadIdx.x, smem, g_tw24, g_tw4096);
  } else if constexpr (VAR >= CV_BODD1) {
    // tiles over the matrix rows that can be nonzero (pass A) or are kept (pass D)
    if (v0 >= job.ncols) return;
    CB::template run_block_odd<bodd_factor(VAR)>(sh, P, job, v0, TW, threadIdx.x, smem, g_tw4096);
  } else if constexpr (VAR == CV_R2C) {
    if (v0 >= job.ncols) return;
    CB::run_r2c(sh, P, job, v0, TW, threadIdx.x, smem, g_tw24, g_tw4096);
  } else {
    if (v0 >= job.ncols) return;
    CB::run(sh, P, job, v0, TW, threadIdx.x, smem, g_tw24, g_tw4096);
  }
}

}  // namespace HK_NS
}  // namespace hk

namespace hk {
namespace HK_NS {

// ---------------------------------------------------------------------------
// Batched task lists.  A plan's tasks form three phases: pass A column tiles
// and resident instances; pass B row blocks; scalar sums and pass D column
// tiles.  Tasks of one phase are independent; a phase reads only what
// earlier phases wrote.  Two schedules run them:
//  * grouped launches (k_group): per phase, one kernel per (kind, length,
//    odd factor); the stream orders the phases;
//  * one persistent launch (k_batch, power-of-two lengths only): resident
//    workgroups pull the tasks of a phase from a queue and meet in a
//    grid-wide barrier before the next phase.  The grid never exceeds the
//    workgroups the device can hold at once, and every barrier wait is
//    bounded: past the bound the error word is set and the kernel still
//    runs to its end.
// ---------------------------------------------------------------------------
enum : int { BATCH_BLK = 512, BATCH_E_ROW = 8, BATCH_E_COL = sizeof(T) == 4 ? 16 : 8 };
// Elements per lane of the batched row bodies: a lane of an odd-factor row
// holds ODD sequences, so it takes 4 to stay within registers.
template <int ODD>
struct BatchRowE {
  static constexpr int value = ODD > 1 ? 4 : BATCH_E_ROW;
};
// Elements per lane of the grouped pass-B rows: 4 up to 2048 points (fewer
// registers, more waves per SIMD; pass B of large batches is latency-bound at
// two waves), 8 beyond; the float factor-3 rows of 8-512 points take 8
// (radix-8 passes, half the LDS exchanges; 188-247 VGPRs, no scratch).  The
// persistent kernel keeps BATCH_E_ROW.
template <int L, int ODD>
struct GroupRowbE {
  static constexpr int value = (ODD == 3 && sizeof(T) == 4 && L >= 8 && L <= 512)
                                   ? 8
                                   : ((ODD > 1 || L <= 2048) ? 4 : BATCH_E_ROW);
};


template <int L, int ODD = 1>
__device__ __forceinline__ void batch_res_body(const BatchArgs &A, const Task &tk, cx<T> *smem, int tid) {
  using RB = RowBody<T, L, BatchRowE<ODD>::value, ODD>;
  const int rw = tid / RB::TPS;
  const int t = tid % RB::TPS;
  const bool valid = rw < tk.a;
  const int32_t inst = A.res_list[tk.inst + (valid ? rw : 0)];
  const Shape &sh = A.shapes[inst];
  const PV P{&A.ptrs[inst], nullptr, 0, nullptr};
  const cx<T> part = RB::run_fwd(sh, P, 0, valid, t, smem + rw * RB::SEQ_LDS, true, g_tw24, g_tw4096);
  if (sh.want_alpha) {
    const cx<T> tot = segment_sum(part, smem, tid, RB::TPS);
    if (valid && t == 0) store_out<T>(P.alpha(), 0, tot, sh.real_out);
  }
}

template <int L, int ODD = 1, int E = BatchRowE<ODD>::value>
__device__ __forceinline__ void batch_rowb_body(const BatchArgs &A, const Task &tk, const Shape &sh, const PV &P,
                                                cx<T> *smem, int tid) {
  using RB = RowBody<T, L, E, ODD>;
  const int rw = tid / RB::TPS;
  const int t = tid % RB::TPS;
  const int64_t row = (int64_t)tk.a + rw;
  const bool valid = row < ((int64_t)1 << sh.logC);
  const cx<T> part = RB::run_fwd(sh, P, row, valid, t, smem + rw * RB::SEQ_LDS, false, g_tw24, g_tw4096);
  if (sh.want_alpha) {  // partial sum of this task; a TASK_ALPHA adds them up
    const cx<T> tot = segment_sum(part, smem, tid, BATCH_BLK);
    if (tid == 0) ws_partials<T>(sh, P)[tk.b] = tot;
  }
}

template <int L, int VAR = CV_POW2>
__device__ __forceinline__ void batch_col_body(const Task &tk, const Shape &sh, const PV &P, cx<T> *smem, int tid) {
  using CB = ColBody<T, L, BATCH_E_COL>;
  constexpr int TW = BATCH_BLK / CB::TPS;
  ColJob job;
  if (tk.type == TASK_COLA) {
    job.kind = COL_A;
    job.op = tk.a;
    job.buf = sh.ops[tk.a].buf;
    job.conj_out = 0;
    job.ncols = sh.ops[tk.a].ncol_nz;
  } else {
    job.kind = COL_D;
    job.op = tk.a;
    job.buf = sh.ops[tk.a].buf;
    job.conj_out = (sh.prog == PROG_BWD && tk.a == 1) ? 1 : 0;
    const int64_t lim = tk.a == 0 ? sh.out_rows : sh.out1_len;
    // real outputs of a real-input transform are stored in pairs
    job.ncols = min(((int64_t)1 << sh.logR), VAR == CV_R2C ? (lim + 1) / 2 : lim);
  }
  // LDS sized by batch_geometry
  if constexpr (VAR == CV_ODD)
    CB::run_odd(sh, P, job, tk.b, TW, tid, smem, g_tw24, g_tw4096);
  else if constexpr (VAR == CV_R2C)
    CB::run_r2c(sh, P, job, tk.b, TW, tid, smem, g_tw24, g_tw4096);
  else
    CB::run(sh, P, job, tk.b, TW, tid, smem, g_tw24, g_tw4096);
}

#ifndef HK_ROWS_ONLY
// The persistent kernel calls the bodies out of line, so that its register
// allocation is the largest body's rather than the sum over the switch.
template <int L>
__device__ __noinline__ void batch_res(const BatchArgs &A, const Task &tk, cx<T> *smem, int tid) {
  batch_res_body<L>(A, tk, smem, tid);
}
template <int L>
__device__ __noinline__ void batch_rowb(const BatchArgs &A, const Task &tk, const Shape &sh, const PV &P,
                                           cx<T> *smem, int tid) {
  batch_rowb_body<L>(A, tk, sh, P, smem, tid);
}
template <int L>
__device__ __noinline__ void batch_col(const Task &tk, const Shape &sh, const PV &P, cx<T> *smem, int tid) {
  batch_col_body<L>(tk, sh, P, smem, tid);
}

#define HK_LSWITCH(logv, FN, ...)                  \
  switch (logv) {                                 \
    case 0: FN<1>(__VA_ARGS__); break;            \
    case 1: FN<2>(__VA_ARGS__); break;            \
    case 2: FN<4>(__VA_ARGS__); break;            \
    case 3: FN<8>(__VA_ARGS__); break;            \
    case 4: FN<16>(__VA_ARGS__); break;           \
    case 5: FN<32>(__VA_ARGS__); break;           \
    case 6: FN<64>(__VA_ARGS__); break;           \
    case 7: FN<128>(__VA_ARGS__); break;          \
    case 8: FN<256>(__VA_ARGS__); break;          \
    case 9: FN<512>(__VA_ARGS__); break;          \
    case 10: FN<1024>(__VA_ARGS__); break;        \
    case 11: FN<2048>(__VA_ARGS__); break;        \
    case 12: FN<4096>(__VA_ARGS__); break;        \
    default: break;                               \
  }

__device__ __forceinline__ void batch_task(const BatchArgs &A, const Task &tk, cx<T> *smem, int tid) {
  if (tk.type == TASK_RES) {
    const Shape &sh0 = A.shapes[A.res_list[tk.inst]];
    HK_LSWITCH(sh0.logR, batch_res, A, tk, smem, tid)
  } else {
    const Shape &sh = A.shapes[tk.inst];
    const PV P{&A.ptrs[tk.inst], nullptr, 0, A.ws_base};
    if (tk.type == TASK_ROWB) {
      HK_LSWITCH(sh.logR, batch_rowb, A, tk, sh, P, smem, tid)
    } else if (tk.type == TASK_ALPHA) {
      reduce_partials(sh, P, tk.nrowb, smem);
    } else {
      HK_LSWITCH(sh.logC, batch_col, tk, sh, P, smem, tid)
    }
  }
}

// Grid-wide barrier after phase ph: release this workgroup's stores, count
// the arrival, wait (bounded) for all gridDim.x workgroups, acquire.
__device__ __forceinline__ void batch_barrier(const BatchArgs &A, int ph, int tid) {
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    atomicAdd(&A.bctl->arrive[ph], 1u);
    uint32_t spins = 0;
    while (__hip_atomic_load(&A.bctl->arrive[ph], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > A.spin_limit ||
          __hip_atomic_load(&A.bctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        atomicOr(&A.bctl->error, 1u);
        break;
      }
    }
  }
  __syncthreads();
  __threadfence();  // acquire: observe the other workgroups' stores
}

__global__ void __launch_bounds__(BATCH_BLK) k_batch(BatchArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *smem = (cx<T> *)smem_raw;
  __shared__ int32_t s_task;
  const int tid = threadIdx.x;
  int32_t begin = 0;
  for (int ph = 0; ph < 3; ++ph) {
    const int32_t end = A.phase_end[ph];
    for (;;) {
      if (tid == 0) s_task = begin + (int32_t)atomicAdd(&A.bctl->next[ph], 1u);
      __syncthreads();
      const int32_t ti = s_task;
      __syncthreads();
      if (ti >= end) break;
      const Task tk = A.tasks[ti];
      batch_task(A, tk, smem, tid);
      __syncthreads();  // smem is reused by the next task
    }
    if (ph < 2) batch_barrier(A, ph, tid);
    begin = end;
  }
}
#endif  // HK_ROWS_ONLY

// Grouped launches: the tasks of one phase that share a kind, a transform
// length L and an odd factor run in one launch of a kernel specialised for
// them (one task per workgroup, A.order[A.begin + blockIdx.x]), so that each
// gets the registers and LDS of its own length instead of the largest one's.  Phases are
// ordered by the stream; no counters or waits are involved.
template <int L, int KIND, int ODD = 1>
__global__ void __launch_bounds__(BATCH_BLK) k_group(BatchArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *smem = (cx<T> *)smem_raw;
  const int tid = threadIdx.x;
  const int32_t ti = A.order[A.begin + (int32_t)blockIdx.x];
  const Task tk = A.tasks[ti];
  if constexpr (KIND == GK_RES) {
    batch_res_body<L, ODD>(A, tk, smem, tid);
  } else {
    const Shape &sh = A.shapes[tk.inst];
    const PV P{&A.ptrs[tk.inst], nullptr, 0, A.ws_base};
    if constexpr (KIND == GK_ROWB)
      batch_rowb_body<L, ODD, GroupRowbE<L, ODD>::value>(A, tk, sh, P, smem, tid);
    else if constexpr (KIND == GK_COL)
      batch_col_body<L, ODD == 2 ? CV_R2C : (ODD > 1 ? CV_ODD : CV_POW2)>(tk, sh, P, smem, tid);
    else
      reduce_partials(sh, P, tk.nrowb, smem);
  }
}

// Grouped real-input resident rows: task = up to BATCH_BLK / TPS instances.
// Elements per lane: 8 in float, 4 in double (8 would spill).
enum : int { R2C_E = sizeof(T) == 4 ? 8 : 4 };
template <int L>
__global__ void __launch_bounds__(BATCH_BLK) k_group_r2c(BatchArgs A) {
  using RB = RealRowBody<T, L, R2C_E>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *smem = (cx<T> *)smem_raw;
  const int tid = threadIdx.x;
  const Task tk = A.tasks[A.order[A.begin + (int32_t)blockIdx.x]];
  const int rw = tid / RB::TPS;
  const int t = tid % RB::TPS;
  const bool valid = rw < tk.a;
  const int32_t inst = A.res_list[tk.inst + (valid ? rw : 0)];
  const Shape &sh = A.shapes[inst];
  const PV P{&A.ptrs[inst], nullptr, 0, nullptr};
  const cx<T> part = RB::run_fwd(sh, P, valid, t, smem + rw * RB::SEQ_LDS, g_tw24, g_tw4096);
  if (sh.want_alpha) {
    const cx<T> tot = segment_sum(part, smem, tid, RB::TPS);
    if (valid && t == 0) store_out<T>(P.alpha(), 0, tot, sh.real_out);
  }
}

// Grouped pass-B row pairs of real-input transforms: pairs tk.a, tk.a + 1, ...
template <int L>
__global__ void __launch_bounds__(BATCH_BLK) k_group_r2c_pairs(BatchArgs A) {
  using PB = RealPairRowBody<T, L, R2C_E>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T> *smem = (cx<T> *)smem_raw;
  const int tid = threadIdx.x;
  const Task tk = A.tasks[A.order[A.begin + (int32_t)blockIdx.x]];
  const Shape &sh = A.shapes[tk.inst];
  const PV P{&A.ptrs[tk.inst], nullptr, 0, A.ws_base};
  const int grp = tid / PB::TPS;
  const int t = tid % PB::TPS;
  const int pw = grp >> 1, g = grp & 1;
  const int64_t pi = (int64_t)tk.a + pw;
  const bool valid = pi < ((int64_t)1 << sh.logC) / 2;
  const cx<T> part =
      PB::run_fwd(sh, P, valid ? pi : 0, g, valid, t, smem + pw * 2 * PB::SEQ_LDS, g_tw24, g_tw4096);
  if (sh.want_alpha) {  // partial sum of this task; a TASK_ALPHA adds them up
    const cx<T> tot = segment_sum(part, smem, tid, BATCH_BLK);
    if (tid == 0) ws_partials<T>(sh, P)[tk.b] = tot;
  }
}

// out[:, pairs[2k]] = src[:, pairs[2k + 1]] for column-major columns of
// `rows` elements of type V (tensor-matrix products: the symmetric
// completion, src = out, and the gather from the spectral path's staging).
template <typename V>
__global__ void __launch_bounds__(256) k_copy_cols(V *out, const V *src, const int32_t *pairs, int64_t rows) {
  const int64_t d = pairs[2 * blockIdx.y], s = pairs[2 * blockIdx.y + 1];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x)
    out[d * rows + i] = src[s * rows + i];
}

#ifndef HK_ROWS_ONLY
// Zeroes the persistent schedule's control block (a plain kernel rather than
// a memset node, so that graph replays stay exact).
__global__ void k_batch_reset(BatchCtl *bctl) {
  const int i = threadIdx.x;
  if (i < 3) {
    bctl->next[i] = 0;
    bctl->arrive[i] = 0;
  }
  if (i == 0) bctl->error = 0;
}
#endif

}  // namespace HK_NS
}  // namespace hk
