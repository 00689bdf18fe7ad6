// Descriptors shared by the host planner and the device kernels.
//
// A product (1D Hankel or BHHB, forward or adjoint) is described by a Shape
// (sizes, operand roles, FFT layout) plus per-instance pointers (Ptrs).  The
// 1D transform length is N = odd * M with odd in {1, 3, 5} and M a power of
// two.  For odd > 1 the cyclic group Z_N is handled as Z_odd x Z_M through
// the Chinese-remainder map n -> (n mod odd, n mod M) (Good-Thomas prime
// factor mapping, no twiddles between the two factors): the operands become
// `odd` sequences of length M, each transformed by the power-of-two passes
// below, and a length-odd DFT across the sequences, done in registers where
// a lane holds the same bins of all of them, completes the transform.  The
// products only need the transforms to diagonalize cyclic convolution, which
// holds for any group isomorphic to Z_N.  Each sequence of length M lives on
// a 2D "storage grid" of 2^logC rows of 2^logR contiguous elements:
//   * 1D, one workgroup per transform ("resident"): logC = 0, the row is the
//     whole padded vector of length N = 2^logR.
//   * 1D, multipass: N = 2^logR * 2^logC, element n at n1 + R n2 with
//     n = n1 + R n2 (four-step / Bailey decomposition; twiddles between the
//     column and row transforms).
//   * BHHB: the padded 2D grid itself, element (i, j) at i + R j; the 2D FFT
//     is a column FFT (along j) and a row FFT (along i), no twiddles.
// Pass A transforms columns of every input operand into workspace buffers;
// pass B does the row transforms, the pointwise spectral product and the row
// transform of the output; pass D does the output's column transform and the
// slice.  See hk_bodies.hpp for the index algebra.
#pragma once
#include <stdint.h>

namespace hk {

enum : int { MAXOPS = 10 };  // generating vector + up to 8 vectors + adjoint cotangent

enum Role : int32_t { ROLE_H = 0, ROLE_X = 1, ROLE_V = 2 };

enum OpFlag : int32_t {
  OPF_CONJ = 1,   // load conj(x)
  OPF_REAL = 2,   // source array is real
  OPF_ALPHA = 4,  // spectrum multiplies into the scalar product (x_1)
  // Multipass, power-of-two 1D rows only:
  OPF_SPEC = 8,         // the operand pointer holds the operand's spectrum in row order
                        // (no column pass; the row pass loads it as transformed)
  OPF_STORE_SPEC = 16,  // the row pass stores this operand's spectrum, in row order, to out1
};

enum Prog : int32_t { PROG_FWD = 0, PROG_BWD = 1 };

// Forward-program variants used by the adjoint of the distinct-vector and
// BHHB products (power-of-two complex layouts only):
enum ShapeFlag : int32_t {
  // no generating vector: the operands' spectra multiply from one, and the
  // output is fft(conj(z) / N) = conj(ifft(z)), i.e. the conjugate of the
  // operands' linear convolution (sliced to out_rows x out_cols)
  SHF_CONV = 1,
  SHF_CONJ_Y = 2,  // the vector output is stored conjugated
};
// Row-kernel variants (never a Shape's prog): the forward and adjoint
// programs built with stored-spectrum operands (OPF_SPEC, OPF_STORE_SPEC).
enum : int32_t { PROG_FWD_SPEC = 2, PROG_BWD_SPEC = 3 };

enum ColKind : int32_t { COL_A = 0, COL_D = 1 };

struct OpDesc {
  int32_t role;     // Role
  int32_t exp;      // multiplicity in the spectral product (ROLE_X)
  int32_t flags;    // OpFlag bits
  int32_t buf;      // multipass: workspace buffer that holds its column transform
  int64_t len;      // 1D: number of stored elements. BHHB: rows of the source matrix
  int64_t cols;     // BHHB: columns of the source matrix (1 for 1D)
  int64_t ncol_nz;  // multipass: storage columns that may be nonzero (rest are zero)
};

struct Shape {
  int32_t prog;        // Prog
  int32_t is_block;    // BHHB
  int32_t m;           // tensor order
  int32_t nops;        // operands in processing order (H first, scalar operand last)
  int32_t logR;        // contiguous (row) FFT length 2^logR
  int32_t logC;        // strided (column) FFT length 2^logC (0 for resident)
  int32_t resident;    // whole transform in one workgroup
  int32_t want_y;      // vector output (forward) / grad_h (adjoint)
  int32_t want_alpha;  // scalar output (forward)
  int32_t want_out1;   // adjoint: grad_x
  int32_t real_out;    // store only the real part
  int32_t rows_per_wg; // multipass row pass: rows per workgroup (side by side)
  int32_t row_iters;   // multipass row pass: rows each lane group handles in turn
  int32_t odd;         // odd factor of the 1D transform length (1, 3 or 5; 1 for BHHB)
  int32_t odd_inv;     // M^{-1} mod odd (0 when odd == 1)
  int32_t r2c;         // real inputs, resident: length-N real transforms as length-N/2
                       // complex ones (logR = log2(N/2)); forward program only
  int32_t fwd_flags;   // forward program variants (ShapeFlag bits)
  int32_t odd_c;       // BHHB: odd factor of the column (block-index) axis, 0 or 1 = none;
                       // the row axis takes `odd` (see hk_bodies.hpp, BHHB with odd factors)
  int32_t odd_c_inv;   // BHHB: C^{-1} mod odd_c (C = 2^logC)
  int64_t out_rows;    // output slice: 1D length / BHHB rows n_1; adjoint grad_h length
  int64_t out_cols;    // BHHB columns N_1 (1 for 1D)
  int64_t out1_len;    // adjoint grad_x length
  int64_t nbuf;        // multipass workspace buffers per instance
  int64_t partials;    // multipass: number of row-pass workgroups (alpha partial sums)
  int64_t ws_bytes;    // multipass workspace bytes per instance
  OpDesc ops[MAXOPS];
};

// True when a shape's row pass needs the PROG_FWD_SPEC kernels.
inline bool shape_has_spec(const Shape &sh) {
  for (int o = 0; o < sh.nops; ++o)
    if (sh.ops[o].flags & (OPF_SPEC | OPF_STORE_SPEC)) return true;
  return false;
}

struct Ptrs {
  const void *op[MAXOPS];
  void *y;           // forward vector output / adjoint grad_h
  void *alpha;       // forward scalar output
  void *out1;        // adjoint grad_x
  const void *phi;   // adjoint scalar cotangent (nullable)
  void *ws;          // instance workspace (multipass)
};

// Byte strides between consecutive instances of a strided batch (0 = shared).
// op[o] == OP_TABLE: the base pointer of operand o is a device array of
// per-instance pointers (stored-spectrum operands of the PROG_FWD_SPEC row
// kernels only).
constexpr int64_t OP_TABLE = INT64_MIN;
struct Strides {
  int64_t op[MAXOPS];
  int64_t y, alpha, out1, phi, ws;
};

struct ColJob {
  int32_t kind;   // COL_A: operand `op` -> buffer `buf`;  COL_D: buffer `buf` -> output `op` (0: y, 1: out1)
  int32_t op;
  int32_t buf;
  int32_t conj_out;
  int64_t ncols;  // storage columns to transform per sequence (pruned)
  int64_t npart;  // COL_D: pass-B partial sums to reduce into the scalar product (0: none)
};

// Persistent batched execution: task list entries.
enum TaskType : int32_t { TASK_RES = 0, TASK_COLA = 1, TASK_ROWB = 2, TASK_COLD = 3, TASK_ALPHA = 4 };

struct Task {
  int32_t type;
  int32_t inst;          // instance index (RES: first entry in the resident list)
  int32_t a;             // RES: number of instances; COLA: operand; COLD: output; ROWB: first row
  int32_t b;             // COLA/COLD: first column; ROWB: task index within the instance
  int32_t nrowb;         // ROWB / ALPHA: number of row tasks of the instance (scalar partials)
};

// Control block of the persistent schedule, zeroed before each run.
struct BatchCtl {
  uint32_t next[3];    // task queue head of each phase
  uint32_t arrive[3];  // workgroups that finished each phase (grid barrier)
  uint32_t error;      // nonzero: a barrier wait exceeded its bound
  uint32_t pad;
};

// Arguments of the batched (task-list) kernel.  Ptrs.ws of each instance is
// an offset from ws_base.
struct BatchArgs {
  const Task *tasks;
  const Shape *shapes;
  const Ptrs *ptrs;
  const int32_t *res_list;
  BatchCtl *bctl;
  char *ws_base;
  int32_t begin, end;      // grouped launches: range of `order` of this launch
  int32_t phase_end[3];    // persistent: tasks [phase_end[p-1], phase_end[p]) form phase p
  uint32_t spin_limit;     // bound on barrier polling iterations
  const int32_t *order;    // grouped launches: task indices sorted by (phase, kind, length)
};

// Level-k block Hankel products: a compact k-dimensional array (extents
// ext[0..k), column-major) and its embedding at strides stride[0..k) in a 1D
// vector (entry (i_0, ..., i_{k-1}) at sum_t i_t stride[t]).
enum : int { HK_MAX_LEVELS = 4 };
struct Levels {
  int32_t k;
  int32_t pad;
  int64_t ext[HK_MAX_LEVELS];
  int64_t stride[HK_MAX_LEVELS];
};

// Grouped launches: one specialised kernel per (task kind, transform length).
enum GroupKind : int { GK_RES = 0, GK_ROWB = 1, GK_COL = 2, GK_ALPHA = 3 };


}  // namespace hk
