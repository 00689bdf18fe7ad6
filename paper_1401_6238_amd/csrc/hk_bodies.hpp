// Workgroup bodies of the Hankel tensor-vector product on gfx950.
//
// Index algebra.  Let N = R * C (R = 2^logR contiguous "row" length, C =
// 2^logC "column" length) and store element n = n1 + R n2 at offset n.
// With n = n1 + R n2 and k = k2 + C k1 (Bailey's four-step decomposition):
//   X[k2 + C k1] = sum_n1 W_R^{n1 k1} W_N^{n1 k2} sum_n2 x[n1 + R n2] W_C^{n2 k2}.
// Pass A: for each column n1, a length-C FFT along n2, stored at n1 + R k2.
// Pass B: for each row k2, the twiddle W_N^{n1 k2} and a length-R FFT along
//         n1 give X[k2 + C k1] at offset k1 + R k2 ("transposed" spectral
//         order).  Every operand uses the same order, so the pointwise
//         spectral product is done here.  The input twiddles of row k2 are the
//         same numbers W_N^{pos k2}, pos = t + s TPS, as its output twiddles
//         below, so a row computes them once for all its operands and its
//         output, and pass A needs none.
//         The output transform y = fft(z) starts on the same row:
//           y[j1 + R j2] = sum_k2 W_C^{j2 k2} W_N^{j1 k2} sum_k1 z[k2 + C k1] W_R^{j1 k1},
//         i.e. a length-R FFT along k1, times W_N^{j1 k2}, stored at j1 + R k2.
// Pass D: for each column j1, a length-C FFT along k2 gives y[j1 + R j2] at
//         its natural offset; the slice keeps offsets < n_1.
// For BHHB the grid is the padded generating-matrix grid itself and the same
// three passes compute fft2 without twiddles.
// When N fits one workgroup (resident), the row body alone does everything.
//
// The generating vector needs ifft(h~); it is computed as
// conj(fft(conj(h~))) / N: operands with ROLE_H are conjugated on load and
// conjugated and scaled after their last transform.
#pragma once
#include "hk_common.hpp"
#include "hk_fft.hpp"

namespace hk {

// Pointers of one instance, read on demand from a base pointer set (the
// kernel argument, or a descriptor-table entry) and optional byte strides of
// a strided batch.  Reading fields through the base pointer (instead of
// copying the set into a private struct indexed at run time) keeps them out
// of scratch memory.
struct PV {
  const Ptrs *b;        // base pointer set
  const Strides *st;    // strides, or nullptr
  int64_t i;            // instance index within the strided batch
  char *ws_base;        // non-null: b->ws is an offset from ws_base
  __device__ __forceinline__ const char *adj(const void *p, int64_t s) const {
    return p ? (const char *)p + (st ? i * s : 0) : nullptr;
  }
  __device__ __forceinline__ const void *op(int o) const { return adj(b->op[o], st ? st->op[o] : 0); }
  __device__ __forceinline__ void *y() const { return (void *)adj(b->y, st ? st->y : 0); }
  __device__ __forceinline__ void *alpha() const { return (void *)adj(b->alpha, st ? st->alpha : 0); }
  __device__ __forceinline__ void *out1() const { return (void *)adj(b->out1, st ? st->out1 : 0); }
  __device__ __forceinline__ const void *phi() const { return adj(b->phi, st ? st->phi : 0); }
  __device__ __forceinline__ char *ws() const {
    return ws_base ? ws_base + (uintptr_t)b->ws : (char *)adj(b->ws, st ? st->ws : 0);
  }
};

// ---------------------------------------------------------------------------
// Memory access through raw buffer resources.  A resource covers
// [base, base + bytes); gfx9 range checking makes a load at an offset past
// the end return zero and drops such a store.  The zero padding of the
// operands, the output slice and the unused lanes of a tile therefore cost no
// compares or selects, and addresses are 32-bit byte offsets from one scalar
// base instead of 64-bit pointers per lane.  Every buffer here is below
// 2^31 bytes (at most 2^24 elements of 16 bytes), so OOB_OFF is out of range
// for all of them.
// ---------------------------------------------------------------------------
constexpr uint32_t OOB_OFF = 0x80000000u;
constexpr int BUF_WORD3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)
// Stores of whole 128-byte lines are non-temporal ("nt"): the pass outputs
// are read by the next kernel, mostly on another XCD, so keeping them in
// this XCD's L2 only delays the end of the kernel, which must write dirty
// lines back before the next launch can see them.  Streaming them out as
// they are produced shortened the column pass of the large single product
// from 10.3 to 8.9 us.  Narrower segments (column tiles of < 128 bytes) keep
// the default policy, so that L2 merges neighbouring tiles' halves of a line
// instead of memory doing partial-line writes.
constexpr int ST_NT = 2, ST_DEFAULT = 0;

// `base` and `bytes` must be the same on every lane of the wavefront (one
// instance per workgroup); they are moved to scalar registers explicitly so
// that the compiler need not prove it.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_buf(const void *base, int64_t bytes) {
  const int64_t nb = bytes < 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : bytes);
  const uint64_t b = (uint64_t)(uintptr_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  const int n = __builtin_amdgcn_readfirstlane((int)nb);
  return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), (short)0, n, BUF_WORD3);
}

template <typename T>
struct BufIO;
template <>
struct BufIO<float> {
  static __device__ __forceinline__ cx<float> ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return mk(__uint_as_float(v[0]), __uint_as_float(v[1]));
  }
  static __device__ __forceinline__ float ld1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  template <int POL = ST_NT>
  static __device__ __forceinline__ void st(cx<float> a, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    u2 v;
    v[0] = __float_as_uint(a.x);
    v[1] = __float_as_uint(a.y);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, POL);
  }
  template <int POL = ST_NT>
  static __device__ __forceinline__ void st1(float a, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(a), r, off, 0, POL);
  }
};
template <>
struct BufIO<double> {
  static __device__ __forceinline__ double u2d(unsigned lo, unsigned hi) {
    return __hiloint2double((int)hi, (int)lo);
  }
  static __device__ __forceinline__ cx<double> ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return mk(u2d(v[0], v[1]), u2d(v[2], v[3]));
  }
  static __device__ __forceinline__ double ld1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return u2d(v[0], v[1]);
  }
  template <int POL = ST_NT>
  static __device__ __forceinline__ void st(cx<double> a, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    u4 v;
    v[0] = (unsigned)__double2loint(a.x);
    v[1] = (unsigned)__double2hiint(a.x);
    v[2] = (unsigned)__double2loint(a.y);
    v[3] = (unsigned)__double2hiint(a.y);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, POL);
  }
  template <int POL = ST_NT>
  static __device__ __forceinline__ void st1(double a, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    u2 v;
    v[0] = (unsigned)__double2loint(a);
    v[1] = (unsigned)__double2hiint(a);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, POL);
  }
};

// Bytes of one stored element of an operand (OPF_REAL: real part only).
template <typename T>
__device__ __forceinline__ int elem_size(int flags) {
  return (flags & OPF_REAL) ? (int)sizeof(T) : (int)sizeof(cx<T>);
}

// a[s] = operand element at byte offset off[s] (zero past the resource's end),
// with the operand's REAL / CONJ conventions.  All EE loads issue back to back.
template <typename T, int EE>
__device__ __forceinline__ void bgather(cx<T> (&a)[EE], __amdgpu_buffer_rsrc_t r, const uint32_t (&off)[EE],
                                        int flags) {
  if (flags & OPF_REAL) {
    T v[EE];
#pragma unroll
    for (int s = 0; s < EE; ++s) v[s] = BufIO<T>::ld1(r, off[s]);
#pragma unroll
    for (int s = 0; s < EE; ++s) a[s] = mk(v[s], T(0));
  } else {
#pragma unroll
    for (int s = 0; s < EE; ++s) a[s] = BufIO<T>::ld(r, off[s]);
    if (flags & OPF_CONJ) {
#pragma unroll
      for (int s = 0; s < EE; ++s) a[s].y = -a[s].y;
    }
  }
}

// Stores v at byte offset off (dropped past the resource's end).
template <typename T, int POL = ST_NT>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, cx<T> v, int real_out) {
  if (real_out)
    BufIO<T>::template st1<POL>(v.x, r, off);
  else
    BufIO<T>::template st<POL>(v, r, off);
}

// Flat (64-bit per-lane address) access, for the resident rows of a
// workgroup that belong to different instances: a buffer resource must be
// uniform across the wave, per-lane bases would need a waterfall loop.
// Loads a[s] = src[idx[s]] where ok[s] and zero elsewhere, without branches:
// a slot that is not ok reads element 0 (every operand has at least one
// element) and is zeroed afterwards, so all EE loads issue back to back
// instead of each waiting behind a branch.
template <typename T, int EE>
__device__ __forceinline__ void gather(cx<T> (&a)[EE], const void *base, const int64_t (&idx)[EE],
                                       const bool (&ok)[EE], int flags) {
  if (flags & OPF_REAL) {
    const T *p = (const T *)base;
    T v[EE];
#pragma unroll
    for (int s = 0; s < EE; ++s) v[s] = p[ok[s] ? idx[s] : 0];
#pragma unroll
    for (int s = 0; s < EE; ++s) a[s] = mk(ok[s] ? v[s] : T(0), T(0));
  } else {
    const cx<T> *p = (const cx<T> *)base;
#pragma unroll
    for (int s = 0; s < EE; ++s) a[s] = p[ok[s] ? idx[s] : 0];
#pragma unroll
    for (int s = 0; s < EE; ++s) a[s] = ok[s] ? a[s] : czero<T>();
    if (flags & OPF_CONJ) {
#pragma unroll
      for (int s = 0; s < EE; ++s) a[s].y = -a[s].y;
    }
  }
}

template <typename T>
__device__ __forceinline__ void store_out(void *base, int64_t idx, cx<T> v, int real_out) {
  if (real_out)
    ((T *)base)[idx] = v.x;
  else
    ((cx<T> *)base)[idx] = v;
}

// Storage of one sequence and of a whole transform.  1D: a sequence has
// M = 2^(logR + logC) elements and the transform N = odd * M.  BHHB with odd
// factors: the grid (odd R) x (odd_c C) holds `odd` sequences along the row
// axis, each of odd_c C rows of R elements (after the column pass, row
// r = q_c C + k2 is bin k2 of the column transform's power-of-two axis and bin
// q_c of its odd axis), so M = odd_c R C.
__device__ __forceinline__ int oddc_of(const Shape &sh) { return sh.odd_c > 1 ? sh.odd_c : 1; }
__device__ __forceinline__ int64_t seq_len(const Shape &sh) { return (int64_t)oddc_of(sh) << (sh.logR + sh.logC); }
__device__ __forceinline__ int64_t fft_len(const Shape &sh) { return (int64_t)sh.odd * seq_len(sh); }
// Rows of the row pass: the storage grid's rows, odd_c C of them for BHHB.
__device__ __forceinline__ int64_t pass_rows(const Shape &sh) { return (int64_t)oddc_of(sh) << sh.logC; }
// BHHB grids with an odd row factor keep each workspace row (odd R elements)
// in natural order of the row index i: the column passes then read and
// write whole runs of consecutive i (the nonzero and the kept ones exactly),
// and the row pass gathers sequence q's position c from i = c + R tau.
__device__ __forceinline__ bool block_natural(const Shape &sh) { return sh.is_block && sh.odd > 1; }
// Elements of one workspace buffer and rows of the row pass for the
// power-of-two row bodies: 1D shapes 2^(logR + logC) and 2^logC; BHHB grids
// may have an odd column factor (odd_c 2^logC rows of 2^logR).  The 1D branch
// reads no odd factor, so the 1D hot loops are unchanged.
__device__ __forceinline__ int64_t pow2_grid_len(const Shape &sh) {
  return sh.is_block ? seq_len(sh) : ((int64_t)1 << (sh.logR + sh.logC));
}
__device__ __forceinline__ int64_t pow2_pass_rows(const Shape &sh) {
  return sh.is_block ? pass_rows(sh) : ((int64_t)1 << sh.logC);
}

// Multipass workspace: nbuf buffers of N elements (sequence q of a buffer at
// q * M), then the row pass's scalar partial sums.  ODDF: the shape may have
// an odd factor; the power-of-two bodies leave it out, so that their hot
// loops issue no extra scalar loads (whose waits also wait for LDS).
template <typename T, bool ODDF = false>
__device__ __forceinline__ cx<T> *ws_buf(const Shape &sh, const PV &P, int b) {
  if constexpr (ODDF) return (cx<T> *)P.ws() + (int64_t)b * fft_len(sh);
  if (sh.is_block) return (cx<T> *)P.ws() + (int64_t)b * seq_len(sh);
  return (cx<T> *)P.ws() + ((int64_t)b << (sh.logR + sh.logC));
}

template <typename T>
__device__ __forceinline__ cx<T> *ws_partials(const Shape &sh, const PV &P) {
  return (cx<T> *)P.ws() + sh.nbuf * fft_len(sh);
}

// Storage columns of output `which` (0: y / grad_h, 1: grad_x) that the
// output's column pass reads: the slice keeps positions < out_rows
// (< out1_len), and position p sits in storage column p mod R, so columns at
// or past that length (and past R) are never read.  Real outputs of
// real-input transforms are stored in pairs.  The row pass stores only these
// columns of its output rows.
__device__ __forceinline__ int64_t out_cols_read(const Shape &sh, int which) {
  const int64_t R = (int64_t)(sh.is_block && sh.odd > 1 ? sh.odd : 1) << sh.logR;
  const int64_t len = which == 0 ? (sh.r2c ? (sh.out_rows + 1) / 2 : sh.out_rows) : sh.out1_len;
  return len < R ? len : R;
}

// Chinese-remainder map of Z_N = Z_odd x Z_M: element (q, p) of the
// sequence grid is entry n = p + M tau of the length-N vector, with
// tau = ((q - p) M^{-1}) mod odd (then n = q mod odd and n = p mod M).
// tau[s] for the positions p0 + s * step (0 <= p0, step < 2^31); `odd` and
// `inv` = M^{-1} mod odd, constants where the caller's are.
template <int EE>
__device__ __forceinline__ void crt_tau(int (&tau)[EE], int q, uint32_t p0, uint32_t step, int odd, int inv) {
  const int pm = (int)(p0 % (uint32_t)odd);
  int t0 = ((q - pm + odd) * inv) % odd;
  const int d = (int)((step % (uint32_t)odd) * (uint32_t)inv % (uint32_t)odd);
#pragma unroll
  for (int s = 0; s < EE; ++s) {
    tau[s] = t0;
    t0 -= d;
    t0 += t0 < 0 ? odd : 0;
  }
}

// Tree sum over the lanes [seg*S, seg*S + S) of the workgroup (S a power of
// two, segments aligned); the result is valid in the first lane of each
// segment.  Fixed order, so results are bitwise reproducible.
template <typename T>
__device__ __forceinline__ cx<T> segment_sum(cx<T> v, cx<T> *red, int tid, int S) {
  __syncthreads();
  red[tid] = v;
  for (int s = S >> 1; s > 0; s >>= 1) {
    __syncthreads();
    const int t = tid & (S - 1);
    if (t < s) red[tid] = cadd(red[tid], red[tid + s]);
  }
  __syncthreads();
  return red[tid];
}

// Sum over a workgroup of n lanes, any n, valid in thread 0: a tree over the
// LDS that folds lanes [s, 2s) onto [0, s) for s = the halves of the next
// power of two (fixed order, bitwise reproducible).  red holds n values.
template <typename T>
__device__ __forceinline__ cx<T> ragged_sum(cx<T> v, cx<T> *red, int tid, int n) {
  __syncthreads();
  red[tid] = v;
  int s = 1;
  while (s < n) s <<= 1;
  for (s >>= 1; s > 0; s >>= 1) {
    __syncthreads();
    if (tid < s && tid + s < n) red[tid] = cadd(red[tid], red[tid + s]);
  }
  __syncthreads();
  return red[0];
}

// Sum over the whole workgroup (blockDim.x a multiple of 64), valid in
// thread 0: each wavefront folds its lanes with cross-lane shuffles (a fixed
// butterfly order), then thread 0 adds the wavefronts' sums in index order.
// Bitwise reproducible, two workgroup barriers.
template <typename T>
__device__ __forceinline__ cx<T> block_sum(cx<T> v, cx<T> *red, int tid) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    v.x += __shfl_xor(v.x, d, 64);
    v.y += __shfl_xor(v.y, d, 64);
  }
  __syncthreads();  // the transforms' last LDS reads are done
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  cx<T> tot = czero<T>();
  if (tid == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot = cadd(tot, red[w]);
  return tot;
}

// ---------------------------------------------------------------------------
// Row body: one sequence of length L per row; TPS lanes per row.  With ODD > 1
// a row stands for the same row of the ODD sequences of the Z_odd x Z_M grid,
// all held by the row's lanes (slot s of sequence q in h[q][s]).
// resident = true : the row is a whole 1D instance (load inputs with padding,
//                   store the sliced outputs).
// resident = false: pass B row `row` of a multipass instance.
// Returns this lane's contribution to the scalar product (forward program).
// ---------------------------------------------------------------------------
template <typename T, int L, int E, int ODD = 1>
struct RowBody {
  using S = FFTShape<L, E>;
  static constexpr int EE = S::EE;
  static constexpr int TPS = S::TPS;
  static constexpr int SEQ_LDS = S::ROW_SEQ;
  // A row's TPS lanes are consecutive, so a row of at most 64 lanes lives in
  // one wavefront and its exchanges need no workgroup barrier.
  static constexpr bool WAVE = TPS <= 64;
  using Seqs = cx<T>[ODD][EE];

  static __device__ __forceinline__ void fft(cx<T> (&a)[EE], int t, cx<T> *lds, const StageTw<T, L, E> &tw) {
    fft_seq<T, L, E, WAVE>(a, t, lds, tw);
  }

  // Length-ODD DFT across the sequences, bin by bin (the odd axis of the
  // transform).
  static __device__ __forceinline__ void odd_dft(Seqs &h) {
    if constexpr (ODD > 1) {
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        cx<T> v[ODD];
#pragma unroll
        for (int q = 0; q < ODD; ++q) v[q] = h[q][s];
        dft_odd<T, ODD>(v);
#pragma unroll
        for (int q = 0; q < ODD; ++q) h[q][s] = v[q];
      }
    }
  }

  // Vector entries of slots s of sequence q of a resident row: positions
  // t + s TPS of the length-L sequence, mapped to Z_N.
  static __device__ __forceinline__ void res_index(int64_t (&idx)[EE], int q, int t) {
    int tau[EE];
    if constexpr (ODD > 1) {
      constexpr int inv = (L % ODD == 1) ? 1 : (ODD == 3 ? 2 : ((L % 5 == 2) ? 3 : ((L % 5 == 3) ? 2 : 4)));
      crt_tau<EE>(tau, q, (uint32_t)t, (uint32_t)TPS, ODD, inv);
    }
#pragma unroll
    for (int s = 0; s < EE; ++s) idx[s] = t + s * TPS + (ODD > 1 ? (int64_t)L * tau[s] : 0);
  }

  // Power-of-two rows (ODD == 1): one sequence per row.  SPEC: the row
  // kernel variant for shapes with stored spectra (OPF_SPEC operands).
  template <bool SPEC = false>
  static __device__ __forceinline__ void load(cx<T> (&a)[EE], const Shape &sh, const PV &P, int o,
                                              int64_t row, bool valid_row, int t, bool resident) {
    const OpDesc &od = sh.ops[o];
    uint32_t off[EE];
    if (resident) {
      // the rows of a workgroup may be different instances: flat loads
      int64_t idx[EE];
      bool ok[EE];
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        idx[s] = t + s * TPS;
        ok[s] = valid_row && idx[s] < od.len;
      }
      gather<T, EE>(a, P.op(o), idx, ok, od.flags);
    } else {
      // row `row` of the operand's column transform; its columns past
      // ncol_nz were never written and read as zero.  A stored spectrum
      // (OPF_SPEC) is read whole from the operand pointer.
      const int64_t N = pow2_grid_len(sh);
      const uint32_t rbase = (uint32_t)(row * L * (int64_t)sizeof(cx<T>));
      if constexpr (SPEC) {
        const bool spec = (od.flags & OPF_SPEC) != 0;
        const void *src = (const void *)ws_buf<T>(sh, P, od.buf);
        if (spec) src = (P.st && P.st->op[o] == OP_TABLE) ? ((const void *const *)P.b->op[o])[P.i] : P.op(o);
        const auto r = make_buf(src, N * (int64_t)sizeof(cx<T>));
        const int64_t ncol = spec ? (int64_t)L : od.ncol_nz;
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          const int i = t + s * TPS;
          off[s] = (valid_row && i < ncol) ? rbase + (uint32_t)(i * (int)sizeof(cx<T>)) : OOB_OFF;
        }
        bgather<T, EE>(a, r, off, 0);
      } else {
        const auto r = make_buf(ws_buf<T>(sh, P, od.buf), N * (int64_t)sizeof(cx<T>));
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          const int i = t + s * TPS;
          off[s] = (valid_row && i < od.ncol_nz) ? rbase + (uint32_t)(i * (int)sizeof(cx<T>)) : OOB_OFF;
        }
        bgather<T, EE>(a, r, off, 0);
      }
    }
  }

  // Spectrum row `row` (natural order within the row) to out1: element k_c
  // of row k_r is bin k_r + C k_c of the length-N transform.
  static __device__ __forceinline__ void store_spec(const cx<T> (&a)[EE], const Shape &sh, const PV &P, int64_t row,
                                                    bool valid_row, int t) {
    if (!valid_row) return;
    const int64_t N = (int64_t)1 << (sh.logR + sh.logC);
    const auto r = make_buf(P.out1(), N * (int64_t)sizeof(cx<T>));
    const uint32_t rbase = (uint32_t)(row * L * (int64_t)sizeof(cx<T>));
#pragma unroll
    for (int s = 0; s < EE; ++s) BufIO<T>::st(a[s], r, rbase + (uint32_t)((t + s * TPS) * (int)sizeof(cx<T>)));
  }

  // Stores output `which` (0: y / grad_h, 1: grad_x) of this row.
  static __device__ __forceinline__ void store(const cx<T> (&a)[EE], const Shape &sh, const PV &P,
                                               int which, int64_t row, bool valid_row, int t,
                                               bool resident, const cx<T> (&w)[EE]) {
    if (!valid_row) return;
    if (resident) {
      void *dst = which == 0 ? P.y() : P.out1();
      const int64_t lim = which == 0 ? sh.out_rows : sh.out1_len;
      const bool cj = which == 1 ? sh.prog == PROG_BWD : (sh.fwd_flags & SHF_CONJ_Y) != 0;
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const int pos = t + s * TPS;
        if (pos < lim) store_out<T>(dst, pos, cj ? cconj(a[s]) : a[s], sh.real_out);
      }
    } else {
      const int64_t N = pow2_grid_len(sh);
      const auto r = make_buf(ws_buf<T>(sh, P, sh.ops[which].buf), N * (int64_t)sizeof(cx<T>));
      const uint32_t rbase = (uint32_t)(row * L * (int64_t)sizeof(cx<T>));
      // columns the output's column pass never reads are not stored
      const int keep = (int)out_cols_read(sh, which);
      uint32_t off[EE];
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const int pos = t + s * TPS;
        off[s] = pos < keep ? rbase + (uint32_t)(pos * (int)sizeof(cx<T>)) : OOB_OFF;
      }
      if (!sh.is_block) {
        // four-step twiddles W_N^{pos * row}, pos = t + s TPS (from twiddles())
#pragma unroll
        for (int s = 0; s < EE; ++s) BufIO<T>::st(cmul(a[s], w[s]), r, off[s]);
      } else {
#pragma unroll
        for (int s = 0; s < EE; ++s) BufIO<T>::st(a[s], r, off[s]);
      }
    }
  }

  // Pass-B rows of a 1D instance: w[s] = W_N^{(t + s TPS) row}, used on the
  // loaded operands (pass A's twiddle) and on the stored output.
  static __device__ __forceinline__ bool twiddles(cx<T> (&w)[EE], const Shape &sh, int64_t row, int t,
                                                  bool resident, const cx<T> *tw24, const cx<T> *tw4096) {
    const bool on = !resident && !sh.is_block;
    if (on) slot_twiddles<T, EE>(w, row, t, TPS, sh.logR + sh.logC, tw24, tw4096);
    return on;
  }
  static __device__ __forceinline__ void twiddle_in(cx<T> (&a)[EE], const cx<T> (&w)[EE], bool on) {
    if (on) {
#pragma unroll
      for (int s = 0; s < EE; ++s) a[s] = cmul(a[s], w[s]);
    }
  }

  // Forward program: z = h^ prod_p x^_p^{e_p}; y = fft(z); alpha = sum z x^_1.
  static __device__ __forceinline__ cx<T> run_fwd(const Shape &sh, const PV &P, int64_t row, bool valid_row,
                                                  int t, cx<T> *lds, bool resident, const cx<T> *tw24,
                                                  const cx<T> *tw4096) {
    if constexpr (ODD > 1) {
      return run_fwd_odd(sh, P, row, 0, 1, valid_row, t, lds, resident, tw24, tw4096);
    } else {
    const T invN = T(1) / T((int64_t)1 << (sh.logR + sh.logC));
    const bool conv = (sh.fwd_flags & SHF_CONV) != 0;
    cx<T> a[EE], nx[EE], acc[EE];
    cx<T> part = czero<T>();
#pragma unroll
    for (int s = 0; s < EE; ++s) acc[s] = mk(conv ? T(1) : T(0), T(0));
    load(a, sh, P, 0, row, valid_row, t, resident);
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    cx<T> w[EE];
    const bool tw_on = twiddles(w, sh, row, t, resident, tw24, tw4096);
    for (int o = 0; o < sh.nops; ++o) {
      // the next operand's loads are in flight while this one is transformed
      if (o + 1 < sh.nops) load(nx, sh, P, o + 1, row, valid_row, t, resident);
      twiddle_in(a, w, tw_on);
      fft(a, t, lds, stw);
      const OpDesc &od = sh.ops[o];
      if (od.role == ROLE_H) {
#pragma unroll
        for (int s = 0; s < EE; ++s) acc[s] = cscale(cconj(a[s]), invN);
      } else {
        for (int e = 0; e < od.exp; ++e) {
#pragma unroll
          for (int s = 0; s < EE; ++s) acc[s] = cmul(acc[s], a[s]);
        }
        if (od.flags & OPF_ALPHA) {
#pragma unroll
          for (int s = 0; s < EE; ++s) part = cfma(acc[s], a[s], part);
        }
      }
#pragma unroll
      for (int s = 0; s < EE; ++s) a[s] = nx[s];
    }
    if (sh.want_y) {
      if (conv) {
#pragma unroll
        for (int s = 0; s < EE; ++s) acc[s] = cscale(cconj(acc[s]), invN);
      }
      fft(acc, t, lds, stw);
      store(acc, sh, P, 0, row, valid_row, t, resident, w);
    }
    return part;
    }
  }

  // Pass B, forward program, over K rows row0, row0 + rstride, ... handled in
  // turn by this lane group: while a row's last operand is transformed, the
  // first operand of the next row is already loading, so the memory traffic
  // of one row overlaps the arithmetic of the previous one.  Returns the lane's
  // share of the scalar product over its rows.
  // SPEC: operands may be stored spectra (OPF_SPEC: no twiddle, transform or
  // conjugation) and the spectrum of an operand may be stored (OPF_STORE_SPEC).
  template <bool SPEC = false>
  static __device__ __forceinline__ cx<T> run_fwd_rows(const Shape &sh, const PV &P, int64_t row0, int rstride,
                                                       int K, int t, cx<T> *lds, const cx<T> *tw24,
                                                       const cx<T> *tw4096) {
    if constexpr (ODD > 1) {
      return run_fwd_odd(sh, P, row0, rstride, K, true, t, lds, false, tw24, tw4096);
    } else {
    const int64_t C = pow2_pass_rows(sh);
    const T invN = T(1) / T(pow2_grid_len(sh));
    const bool conv = (sh.fwd_flags & SHF_CONV) != 0;
    cx<T> a[EE], nx[EE], acc[EE], w[EE];
    cx<T> part = czero<T>();
    int64_t row = row0;
    bool valid = row < C;
    // The (row, operand) items in processing order stream through two
    // register sets: `a` holds the item being transformed and `nx` the next
    // one, in flight.  The first two loads go out before the twiddle set-up,
    // whose table reads would otherwise delay the second.
    int nit = 0, nop = 0;  // the next item to load
    auto load_item = [&](cx<T>(&dst)[EE]) {
      if (nit < K) {
        const int64_t r = row0 + (int64_t)nit * rstride;
        load<SPEC>(dst, sh, P, nop, r, r < C, t, false);
      }
      if (++nop == sh.nops) {
        nop = 0;
        ++nit;
      }
    };
    load_item(a);
    load_item(nx);
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    for (int it = 0; it < K; ++it) {
      const bool tw_on = twiddles(w, sh, row, t, false, tw24, tw4096);
      const int64_t nrow = row + rstride;
      const bool nvalid = (it + 1 < K) && nrow < C;
#pragma unroll
      for (int s = 0; s < EE; ++s) acc[s] = mk(conv ? T(1) : T(0), T(0));
      for (int o = 0; o < sh.nops; ++o) {
        const OpDesc &od = sh.ops[o];
        if constexpr (SPEC) {
          const bool spec = (od.flags & OPF_SPEC) != 0;
          if (!spec) {
            twiddle_in(a, w, tw_on);
            fft(a, t, lds, stw);
          }
          if (od.role == ROLE_H) {
            if (spec) {
#pragma unroll
              for (int s = 0; s < EE; ++s) acc[s] = a[s];
            } else {
#pragma unroll
              for (int s = 0; s < EE; ++s) acc[s] = cscale(cconj(a[s]), invN);
            }
            if (od.flags & OPF_STORE_SPEC) store_spec(acc, sh, P, row, valid, t);
          } else {
            if (od.flags & OPF_STORE_SPEC) store_spec(a, sh, P, row, valid, t);
            for (int e = 0; e < od.exp; ++e) {
#pragma unroll
              for (int s = 0; s < EE; ++s) acc[s] = cmul(acc[s], a[s]);
            }
            if (od.flags & OPF_ALPHA) {
#pragma unroll
              for (int s = 0; s < EE; ++s) part = cfma(acc[s], a[s], part);
            }
          }
        } else {
        twiddle_in(a, w, tw_on);
        fft(a, t, lds, stw);
        if (od.role == ROLE_H) {
#pragma unroll
          for (int s = 0; s < EE; ++s) acc[s] = cscale(cconj(a[s]), invN);
        } else {
          for (int e = 0; e < od.exp; ++e) {
#pragma unroll
            for (int s = 0; s < EE; ++s) acc[s] = cmul(acc[s], a[s]);
          }
          if (od.flags & OPF_ALPHA) {
#pragma unroll
            for (int s = 0; s < EE; ++s) part = cfma(acc[s], a[s], part);
          }
        }
        }
#pragma unroll
        for (int s = 0; s < EE; ++s) a[s] = nx[s];
        load_item(nx);
      }
      if (sh.want_y) {
        if (conv) {
#pragma unroll
          for (int s = 0; s < EE; ++s) acc[s] = cscale(cconj(acc[s]), invN);
        }
        fft(acc, t, lds, stw);
        store(acc, sh, P, 0, row, valid, t, false, w);
      }
      row = nrow;
      valid = nvalid;
    }
    return part;
    }
  }

  // Adjoint of g = H x^{m-1}, f = H x^m (equal vectors).  Operands in order:
  // X, then optionally V (cotangent of g, conjugated on load), then H when
  // grad_x is requested.
  // SPEC: x (operand 0) may be a stored spectrum (OPF_SPEC): loaded as
  // transformed, no twiddle or transform.
  template <bool SPEC = false>
  static __device__ __forceinline__ void run_bwd(const Shape &sh, const PV &P, int64_t row, bool valid_row,
                                                 int t, cx<T> *lds, bool resident, const cx<T> *tw24,
                                                 const cx<T> *tw4096) {
    if constexpr (ODD > 1) {
      run_bwd_odd(sh, P, row, valid_row, t, lds, resident, tw24, tw4096);
      return;
    }
    const T invN = T(1) / T((int64_t)1 << (sh.logR + sh.logC));
    cx<T> a[EE], gq[EE];
    cx<T> phc = czero<T>();  // conj(phi)
    if (P.phi()) phc = cconj(*(const cx<T> *)P.phi());
    const T m1 = T(sh.m - 1), m0 = T(sh.m);
    StageTw<T, L, E> stw;
    cx<T> w[EE];
    bool tw_on;
    {
      cx<T> xs[EE], p1[EE], vs[EE];
      load<SPEC>(xs, sh, P, 0, row, valid_row, t, resident);
      stw.init(t, tw4096);
      tw_on = twiddles(w, sh, row, t, resident, tw24, tw4096);
      if constexpr (SPEC) {
        if (!(sh.ops[0].flags & OPF_SPEC)) {
          twiddle_in(xs, w, tw_on);
          fft(xs, t, lds, stw);
        }
      } else {
        twiddle_in(xs, w, tw_on);
        fft(xs, t, lds, stw);
      }
#pragma unroll
      for (int s = 0; s < EE; ++s) p1[s] = mk(T(1), T(0));
      for (int e = 0; e < sh.m - 2; ++e) {
#pragma unroll
        for (int s = 0; s < EE; ++s) p1[s] = cmul(p1[s], xs[s]);
      }
      const bool has_v = sh.nops > 1 && sh.ops[1].role == ROLE_V;
      if (has_v) {
        load(vs, sh, P, 1, row, valid_row, t, resident);
        twiddle_in(vs, w, tw_on);
        fft(vs, t, lds, stw);
      } else {
#pragma unroll
        for (int s = 0; s < EE; ++s) vs[s] = czero<T>();
      }
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        // grad_x spectrum factor: x^{m-2} ((m-1) V + m conj(phi) x)
        gq[s] = cmul(p1[s], cadd(cscale(vs[s], m1), cscale(cmul(phc, xs[s]), m0)));
        // grad_h spectrum: conj(x^{m-1} (V + conj(phi) x)) / N, transformed forward
        a[s] = cscale(cconj(cmul(cmul(p1[s], xs[s]), cfma(phc, xs[s], vs[s]))), invN);
      }
    }
    if (sh.want_y) {
      fft(a, t, lds, stw);
      store(a, sh, P, 0, row, valid_row, t, resident, w);
    }
    if (sh.want_out1) {
      load(a, sh, P, sh.nops - 1, row, valid_row, t, resident);  // H
      twiddle_in(a, w, tw_on);
      fft(a, t, lds, stw);
#pragma unroll
      for (int s = 0; s < EE; ++s) a[s] = cmul(cscale(cconj(a[s]), invN), gq[s]);
      fft(a, t, lds, stw);
      store(a, sh, P, 1, row, valid_row, t, resident, w);
    }
  }

  // Pass B of the adjoint over K rows row0, row0 + rstride, ... in turn
  // (power-of-two rows): the operands of a row (X, V, H) are all in flight
  // before its first transform, and the next row's X and V load while this
  // row's outputs are transformed and stored, its H once this row's H has
  // been used.  Same arithmetic as run_bwd.
  template <bool SPEC = false>
  static __device__ __forceinline__ void run_bwd_rows(const Shape &sh, const PV &P, int64_t row0, int rstride,
                                                      int K, int t, cx<T> *lds, const cx<T> *tw24,
                                                      const cx<T> *tw4096) {
    if constexpr (ODD > 1) {
      for (int it = 0; it < K; ++it) {
        const int64_t row = row0 + (int64_t)it * rstride;
        run_bwd_odd(sh, P, row, row < pass_rows(sh), t, lds, false, tw24, tw4096);
      }
    } else if constexpr (sizeof(T) == 8 && EE >= 16) {
      // double rows of 16 elements per lane: five live operand sets would
      // spill (over 1 KB per lane); one row at a time, operands in turn
      for (int it = 0; it < K; ++it) {
        const int64_t row = row0 + (int64_t)it * rstride;
        run_bwd<SPEC>(sh, P, row, row < ((int64_t)1 << sh.logC), t, lds, false, tw24, tw4096);
      }
    } else {
    const int64_t C = (int64_t)1 << sh.logC;
    const T invN = T(1) / T((int64_t)1 << (sh.logR + sh.logC));
    cx<T> phc = czero<T>();  // conj(phi)
    if (P.phi()) phc = cconj(*(const cx<T> *)P.phi());
    const T m1 = T(sh.m - 1), m0 = T(sh.m);
    const bool has_v = sh.nops > 1 && sh.ops[1].role == ROLE_V;
    const bool x_spec = SPEC && (sh.ops[0].flags & OPF_SPEC) != 0;
    const int oh = sh.nops - 1;  // H, present when grad_x is requested
    cx<T> xs[EE], vs[EE], hs[EE], a[EE], gq[EE], w[EE];
    int64_t row = row0;
    bool valid = row < C;
    load<SPEC>(xs, sh, P, 0, row, valid, t, false);
    if (has_v) load(vs, sh, P, 1, row, valid, t, false);
    if (sh.want_out1) load(hs, sh, P, oh, row, valid, t, false);
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    for (int it = 0; it < K; ++it) {
      const bool tw_on = twiddles(w, sh, row, t, false, tw24, tw4096);
      const int64_t nrow = row + rstride;
      const bool more = it + 1 < K;
      const bool nvalid = more && nrow < C;
      if (!x_spec) {
        twiddle_in(xs, w, tw_on);
        fft(xs, t, lds, stw);
      }
      if (has_v) {
        twiddle_in(vs, w, tw_on);
        fft(vs, t, lds, stw);
      } else {
#pragma unroll
        for (int s = 0; s < EE; ++s) vs[s] = czero<T>();
      }
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        cx<T> p1 = mk(T(1), T(0));
        for (int e = 0; e < sh.m - 2; ++e) p1 = cmul(p1, xs[s]);
        // grad_x spectrum factor: x^{m-2} ((m-1) V + m conj(phi) x)
        gq[s] = cmul(p1, cadd(cscale(vs[s], m1), cscale(cmul(phc, xs[s]), m0)));
        // grad_h spectrum: conj(x^{m-1} (V + conj(phi) x)) / N, transformed forward
        a[s] = cscale(cconj(cmul(cmul(p1, xs[s]), cfma(phc, xs[s], vs[s]))), invN);
      }
      // X and V of this row are used up: the next row's are loaded now
      if (more) {
        load<SPEC>(xs, sh, P, 0, nrow, nvalid, t, false);
        if (has_v) load(vs, sh, P, 1, nrow, nvalid, t, false);
      }
      if (sh.want_y) {
        fft(a, t, lds, stw);
        store(a, sh, P, 0, row, valid, t, false, w);
      }
      if (sh.want_out1) {
        twiddle_in(hs, w, tw_on);
        fft(hs, t, lds, stw);
#pragma unroll
        for (int s = 0; s < EE; ++s) a[s] = cmul(cscale(cconj(hs[s]), invN), gq[s]);
        if (more) load(hs, sh, P, oh, nrow, nvalid, t, false);
        fft(a, t, lds, stw);
        store(a, sh, P, 1, row, valid, t, false, w);
      }
      row = nrow;
      valid = nvalid;
    }
    }
  }

  // ---- Odd-factor rows (ODD > 1): the same row of ODD sequences. ----

  static __device__ __forceinline__ void load_seq(cx<T> (&a)[EE], const Shape &sh, const PV &P, int o,
                                                  int64_t row, bool valid_row, int t, bool resident, int q) {
    const OpDesc &od = sh.ops[o];
    uint32_t off[EE];
    if (resident) {
      // the rows of a workgroup may be different instances: flat loads
      int64_t idx[EE];
      bool ok[EE];
      res_index(idx, q, t);
#pragma unroll
      for (int s = 0; s < EE; ++s) ok[s] = valid_row && idx[s] < od.len;
      gather<T, EE>(a, P.op(o), idx, ok, od.flags);
    } else if (sh.is_block) {
      // BHHB: row `row` of the column transform in natural order of i;
      // sequence q's position c is entry i = c + L tau; entries at or past
      // ncol_nz (the operand's rows) were never written and read as zero
      int tau[EE];
      crt_tau<EE>(tau, q, (uint32_t)t, (uint32_t)TPS, ODD, sh.odd_inv);
      const auto r = make_buf(ws_buf<T, true>(sh, P, od.buf), fft_len(sh) * (int64_t)sizeof(cx<T>));
      const uint32_t rbase = (uint32_t)(row * (ODD * L) * (int64_t)sizeof(cx<T>));
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const int i = t + s * TPS + L * tau[s];
        off[s] = (valid_row && i < od.ncol_nz) ? rbase + (uint32_t)(i * (int)sizeof(cx<T>)) : OOB_OFF;
      }
      bgather<T, EE>(a, r, off, 0);
    } else {
      // row `row` of sequence q of the operand's column transform; its
      // columns past ncol_nz were never written and read as zero
      const int64_t M = seq_len(sh);
      const auto r = make_buf(ws_buf<T, true>(sh, P, od.buf), ODD * M * (int64_t)sizeof(cx<T>));
      const uint32_t rbase = (uint32_t)((q * M + row * L) * (int64_t)sizeof(cx<T>));
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const int i = t + s * TPS;
        off[s] = (valid_row && i < od.ncol_nz) ? rbase + (uint32_t)(i * (int)sizeof(cx<T>)) : OOB_OFF;
      }
      bgather<T, EE>(a, r, off, 0);
    }
  }

  // Stores sequence q of output `which` (0: y / grad_h, 1: grad_x) of this row.
  static __device__ __forceinline__ void store_seq(const cx<T> (&a)[EE], const Shape &sh, const PV &P,
                                                   int which, int64_t row, bool valid_row, int t,
                                                   bool resident, const cx<T> (&w)[EE], int q) {
    if (!valid_row) return;
    if (resident) {
      void *dst = which == 0 ? P.y() : P.out1();
      const int64_t lim = which == 0 ? sh.out_rows : sh.out1_len;
      const bool cj = which == 1 ? sh.prog == PROG_BWD : (sh.fwd_flags & SHF_CONJ_Y) != 0;
      int64_t idx[EE];
      res_index(idx, q, t);
#pragma unroll
      for (int s = 0; s < EE; ++s)
        if (idx[s] < lim) store_out<T>(dst, idx[s], cj ? cconj(a[s]) : a[s], sh.real_out);
    } else if (sh.is_block) {
      // BHHB: natural order of i; only the entries the output's column pass
      // reads (i < out_rows) are stored
      int tau[EE];
      crt_tau<EE>(tau, q, (uint32_t)t, (uint32_t)TPS, ODD, sh.odd_inv);
      const auto r = make_buf(ws_buf<T, true>(sh, P, sh.ops[which].buf), fft_len(sh) * (int64_t)sizeof(cx<T>));
      const uint32_t rbase = (uint32_t)(row * (ODD * L) * (int64_t)sizeof(cx<T>));
      const int keep = (int)out_cols_read(sh, which);
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const int i = t + s * TPS + L * tau[s];
        BufIO<T>::template st<ST_DEFAULT>(a[s], r, i < keep ? rbase + (uint32_t)(i * (int)sizeof(cx<T>)) : OOB_OFF);
      }
    } else {
      const int64_t M = seq_len(sh);
      const auto r = make_buf(ws_buf<T, true>(sh, P, sh.ops[which].buf), ODD * M * (int64_t)sizeof(cx<T>));
      const uint32_t rbase = (uint32_t)((q * M + row * L) * (int64_t)sizeof(cx<T>));
      // columns the output's column pass never reads are not stored
      const int keep = (int)out_cols_read(sh, which);
      uint32_t off[EE];
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const int pos = t + s * TPS;
        off[s] = pos < keep ? rbase + (uint32_t)(pos * (int)sizeof(cx<T>)) : OOB_OFF;
      }
      if (!sh.is_block) {
        // four-step twiddles W_M^{pos * row}, pos = t + s TPS (from twiddles())
#pragma unroll
        for (int s = 0; s < EE; ++s) BufIO<T>::st(cmul(a[s], w[s]), r, off[s]);
      } else {
#pragma unroll
        for (int s = 0; s < EE; ++s) BufIO<T>::st(a[s], r, off[s]);
      }
    }
  }

  // Spectrum of operand o on this row: its ODD sequences loaded (each next
  // one in flight while the current one is transformed), transformed along
  // the power-of-two axis, then across the sequences.
  static __device__ __forceinline__ void spectrum(Seqs &h, const Shape &sh, const PV &P, int o, int64_t row,
                                                  bool valid_row, int t, cx<T> *lds, bool resident,
                                                  const StageTw<T, L, E> &stw, const cx<T> (&w)[EE], bool tw_on) {
    cx<T> nx[EE];
    load_seq(nx, sh, P, o, row, valid_row, t, resident, 0);
#pragma unroll
    for (int q = 0; q < ODD; ++q) {
#pragma unroll
      for (int s = 0; s < EE; ++s) h[q][s] = nx[s];
      if (q + 1 < ODD) load_seq(nx, sh, P, o, row, valid_row, t, resident, q + 1);
      twiddle_in(h[q], w, tw_on);
      fft(h[q], t, lds, stw);
    }
    odd_dft(h);
  }

  // Spectral product step of the forward program for operand o with
  // spectrum h: the generating vector's ifft starts acc, vectors multiply in
  // with their multiplicity, the scalar operand's spectrum closes alpha.
  static __device__ __forceinline__ void combine_fwd(Seqs &acc, const Seqs &h, const OpDesc &od, T invN,
                                                     cx<T> &part) {
    if (od.role == ROLE_H) {
#pragma unroll
      for (int q = 0; q < ODD; ++q)
#pragma unroll
        for (int s = 0; s < EE; ++s) acc[q][s] = cscale(cconj(h[q][s]), invN);
    } else {
      for (int e = 0; e < od.exp; ++e) {
#pragma unroll
        for (int q = 0; q < ODD; ++q)
#pragma unroll
          for (int s = 0; s < EE; ++s) acc[q][s] = cmul(acc[q][s], h[q][s]);
      }
      if (od.flags & OPF_ALPHA) {
#pragma unroll
        for (int q = 0; q < ODD; ++q)
#pragma unroll
          for (int s = 0; s < EE; ++s) part = cfma(acc[q][s], h[q][s], part);
      }
    }
  }

  // Output transform y = fft(z) of the row (odd axis, then each sequence)
  // and its store.
  static __device__ __forceinline__ void output(Seqs &acc, const Shape &sh, const PV &P, int which, int64_t row,
                                                bool valid_row, int t, cx<T> *lds, bool resident,
                                                const StageTw<T, L, E> &stw, const cx<T> (&w)[EE]) {
    odd_dft(acc);
#pragma unroll
    for (int q = 0; q < ODD; ++q) {
      fft(acc[q], t, lds, stw);
      store_seq(acc[q], sh, P, which, row, valid_row, t, resident, w, q);
    }
  }

  // Forward program of odd-factor rows over K rows row0, row0 + rstride, ...
  // handled in turn by this lane group (K = 1 for resident rows).  The loads run one sequence
  // ahead of the transforms: while a sequence is transformed the next one
  // (of this operand, the next operand or the next row's first operand) is
  // already loading, so the memory traffic of a row overlaps the arithmetic.
  // Returns the lane's share of the scalar product over its rows.
  static __device__ __forceinline__ cx<T> run_fwd_odd(const Shape &sh, const PV &P, int64_t row0, int rstride,
                                                      int K, bool valid0, int t, cx<T> *lds, bool resident,
                                                       const cx<T> *tw24, const cx<T> *tw4096) {
    const int64_t C = pass_rows(sh);
    const T invN = T(1) / T(fft_len(sh));
    // SHF_CONV: no generating vector; the product of the spectra starts at 1
    // and the output is conj(ifft(prod)), formed as fft(conj(prod) / N)
    const bool conv = (sh.fwd_flags & SHF_CONV) != 0;
    cx<T> nx[EE], w[EE];
    Seqs h, acc;
    cx<T> part = czero<T>();
    int64_t row = row0;
    bool valid = resident ? valid0 : row < C;
    load_seq(nx, sh, P, 0, row, valid, t, resident, 0);
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    for (int it = 0; it < K; ++it) {
      const bool tw_on = twiddles(w, sh, row, t, resident, tw24, tw4096);
      const int64_t nrow = row + rstride;
      const bool nvalid = (it + 1 < K) && nrow < C;
#pragma unroll
      for (int q = 0; q < ODD; ++q)
#pragma unroll
        for (int s = 0; s < EE; ++s) acc[q][s] = mk(conv ? T(1) : T(0), T(0));
      for (int o = 0; o < sh.nops; ++o) {
#pragma unroll
        for (int q = 0; q < ODD; ++q) {
#pragma unroll
          for (int s = 0; s < EE; ++s) h[q][s] = nx[s];
          if (q + 1 < ODD)
            load_seq(nx, sh, P, o, row, valid, t, resident, q + 1);
          else if (o + 1 < sh.nops)
            load_seq(nx, sh, P, o + 1, row, valid, t, resident, 0);
          else if (it + 1 < K)
            load_seq(nx, sh, P, 0, nrow, nvalid, t, resident, 0);
          twiddle_in(h[q], w, tw_on);
          fft(h[q], t, lds, stw);
        }
        odd_dft(h);
        combine_fwd(acc, h, sh.ops[o], invN, part);
      }
      if (sh.want_y) {
        if (conv) {
#pragma unroll
          for (int q = 0; q < ODD; ++q)
#pragma unroll
            for (int s = 0; s < EE; ++s) acc[q][s] = cscale(cconj(acc[q][s]), invN);
        }
        output(acc, sh, P, 0, row, valid, t, lds, resident, stw, w);
      }
      row = nrow;
      valid = nvalid;
    }
    return part;
  }

  // Adjoint of odd-factor rows (see run_bwd).
  static __device__ __forceinline__ void run_bwd_odd(const Shape &sh, const PV &P, int64_t row, bool valid_row,
                                                 int t, cx<T> *lds, bool resident, const cx<T> *tw24,
                                                 const cx<T> *tw4096) {
    const T invN = T(1) / T((int64_t)ODD << (sh.logR + sh.logC));
    // Two spectra are live at a time: a (X's, then the grad_h spectrum, then
    // H's) and gq (V's, then the grad_x factor), updated in place.
    Seqs a, gq;
    cx<T> phc = czero<T>();  // conj(phi)
    if (P.phi()) phc = cconj(*(const cx<T> *)P.phi());
    const T m1 = T(sh.m - 1), m0 = T(sh.m);
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    cx<T> w[EE];
    const bool tw_on = twiddles(w, sh, row, t, resident, tw24, tw4096);
    spectrum(a, sh, P, 0, row, valid_row, t, lds, resident, stw, w, tw_on);
    const bool has_v = sh.nops > 1 && sh.ops[1].role == ROLE_V;
    if (has_v) {
      spectrum(gq, sh, P, 1, row, valid_row, t, lds, resident, stw, w, tw_on);
    } else {
#pragma unroll
      for (int q = 0; q < ODD; ++q)
#pragma unroll
        for (int s = 0; s < EE; ++s) gq[q][s] = czero<T>();
    }
#pragma unroll
    for (int q = 0; q < ODD; ++q)
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const cx<T> x = a[q][s], v = gq[q][s];
        cx<T> p1 = mk(T(1), T(0));  // x^{m-2}
        for (int e = 0; e < sh.m - 2; ++e) p1 = cmul(p1, x);
        // grad_x spectrum factor: x^{m-2} ((m-1) V + m conj(phi) x)
        gq[q][s] = cmul(p1, cadd(cscale(v, m1), cscale(cmul(phc, x), m0)));
        // grad_h spectrum: conj(x^{m-1} (V + conj(phi) x)) / N, transformed forward
        a[q][s] = cscale(cconj(cmul(cmul(p1, x), cfma(phc, x, v))), invN);
      }
    if (sh.want_y) output(a, sh, P, 0, row, valid_row, t, lds, resident, stw, w);
    if (sh.want_out1) {
      spectrum(a, sh, P, sh.nops - 1, row, valid_row, t, lds, resident, stw, w, tw_on);  // H
#pragma unroll
      for (int q = 0; q < ODD; ++q)
#pragma unroll
        for (int s = 0; s < EE; ++s) a[q][s] = cmul(cscale(cconj(a[q][s]), invN), gq[q][s]);
      output(a, sh, P, 1, row, valid_row, t, lds, resident, stw, w);
    }
  }
};

// ---------------------------------------------------------------------------
// Real-input rows (forward program, resident): the zero-padded real vectors of
// length N = 2L are read as L complex pairs z_j = v_{2j} + i v_{2j+1}, so one
// length-L transform Z per operand gives its length-N real transform
//   V_k = (Z_k + conj Z_{L-k}) / 2 - i W_N^k (Z_k - conj Z_{L-k}) / 2,  k < L,
//   V_L = Re Z_0 - Im Z_0,
// the other half being conj(V_{N-k}) (Hermitian).  The spectral product runs
// on bins 0..L.  Its transform y = fft(z^) is real and comes out packed,
// y_{2j} + i y_{2j+1} = FFT_L(Q)_j with
//   Q_k = (z^_k + conj z^_{L-k}) + i W_N^k (z^_k - conj z^_{L-k}),
// and alpha = t_0 + t_L + 2 Re sum_{0<k<L} t_k over the half spectrum.  The
// mirror bins L - k sit on other lanes; they pass through the row's LDS.
// Published method: the half-length complex FFT for real data (two real
// sequences packed into one complex transform, then split by symmetry).
// ---------------------------------------------------------------------------
template <typename T, int L, int E>
struct RealRowBody {
  using S = FFTShape<L, E>;
  static constexpr int EE = S::EE;
  static constexpr int TPS = S::TPS;
  static constexpr int SEQ_LDS = S::ROW_SEQ > L ? S::ROW_SEQ : L;
  static constexpr bool WAVE = TPS <= 64;

  // z_j for the lane's slots j = t + s TPS, real entries past `len` zero
  static __device__ __forceinline__ void load(cx<T> (&a)[EE], const void *src, int64_t len, bool valid, int t) {
    const T *p = (const T *)src;
    T re[EE], im[EE];
#pragma unroll
    for (int s = 0; s < EE; ++s) {
      const int64_t j2 = 2 * (int64_t)(t + s * TPS);
      const bool ok0 = valid && j2 < len, ok1 = valid && j2 + 1 < len;
      re[s] = p[ok0 ? j2 : 0];
      im[s] = p[ok1 ? j2 + 1 : 0];
      re[s] = ok0 ? re[s] : T(0);
      im[s] = ok1 ? im[s] : T(0);
    }
#pragma unroll
    for (int s = 0; s < EE; ++s) a[s] = mk(re[s], im[s]);
  }

  // m[s] = a at the mirror bin (L - j) mod L of the lane's slot j
  static __device__ __forceinline__ void mirror(cx<T> (&m)[EE], const cx<T> (&a)[EE], int t, cx<T> *lds) {
    seq_sync<WAVE>();
#pragma unroll
    for (int s = 0; s < EE; ++s) lds[t + s * TPS] = a[s];
    seq_sync<WAVE>();
#pragma unroll
    for (int s = 0; s < EE; ++s) m[s] = lds[(L - (t + s * TPS)) & (L - 1)];
  }

  static __device__ __forceinline__ cx<T> run_fwd(const Shape &sh, const PV &P, bool valid, int t, cx<T> *lds,
                                                  const cx<T> *tw24, const cx<T> *tw4096) {
    constexpr int LOGN = S::LOGL + 1;
    const T invN = T(1) / T(2 * L);
    cx<T> a[EE], nx[EE], acc[EE], w[EE], m[EE];
    cx<T> accn = czero<T>();  // bin L (real for real inputs)
    T part = T(0);
    slot_twiddles<T, EE>(w, 1, t, TPS, LOGN, tw24, tw4096);  // W_N^j
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    load(a, P.op(0), sh.ops[0].len, valid, t);
#pragma unroll
    for (int s = 0; s < EE; ++s) acc[s] = czero<T>();
    for (int o = 0; o < sh.nops; ++o) {
      if (o + 1 < sh.nops) load(nx, P.op(o + 1), sh.ops[o + 1].len, valid, t);
      fft_seq<T, L, E, WAVE>(a, t, lds, stw);
      mirror(m, a, t, lds);
      const T vn = a[0].x - a[0].y;  // V_L (meaningful on the lane with slot j = 0)
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const cx<T> zm = cconj(m[s]);
        const cx<T> sp = cadd(a[s], zm), df = csub(a[s], zm);
        // (sp - i w df) / 2
        const cx<T> wd = cmul(w[s], df);
        a[s] = mk(T(0.5) * (sp.x + wd.y), T(0.5) * (sp.y - wd.x));
      }
      const OpDesc &od = sh.ops[o];
      if (od.role == ROLE_H) {
#pragma unroll
        for (int s = 0; s < EE; ++s) acc[s] = cscale(cconj(a[s]), invN);
        accn = mk(vn * invN, T(0));
      } else {
        for (int e = 0; e < od.exp; ++e) {
#pragma unroll
          for (int s = 0; s < EE; ++s) acc[s] = cmul(acc[s], a[s]);
          accn.x *= vn;
        }
        if (od.flags & OPF_ALPHA) {
#pragma unroll
          for (int s = 0; s < EE; ++s) {
            const T tre = acc[s].x * a[s].x - acc[s].y * a[s].y;  // Re(acc V)
            part += (t + s * TPS == 0) ? tre : T(2) * tre;
          }
          if (t == 0) part += accn.x * vn;
        }
      }
#pragma unroll
      for (int s = 0; s < EE; ++s) a[s] = nx[s];
    }
    if (sh.want_y) {
      mirror(m, acc, t, lds);
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const cx<T> zm = cconj((t + s * TPS == 0) ? accn : m[s]);
        const cx<T> sp = cadd(acc[s], zm), df = csub(acc[s], zm);
        const cx<T> wd = cmul(w[s], df);
        acc[s] = mk(sp.x - wd.y, sp.y + wd.x);  // sp + i w df
      }
      fft_seq<T, L, E, WAVE>(acc, t, lds, stw);
      if (valid) {
        T *dst = (T *)P.y();
        const int64_t lim = sh.out_rows;
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          const int64_t j2 = 2 * (int64_t)(t + s * TPS);
          if (j2 < lim) dst[j2] = acc[s].x;
          if (j2 + 1 < lim) dst[j2 + 1] = acc[s].y;
        }
      }
    }
    return mk(part, T(0));
  }
};

// ---------------------------------------------------------------------------
// Column body: TW columns of length L (one sequence each), TPS lanes per
// column, lane l -> column l % TW, position-lane l / TW (so that a wave
// reads TW contiguous elements of several rows at once).  Columns are
// numbered across the ODD sequences of a transform ("virtual" column
// v = q R + c: storage column c of sequence q); a job transforms the first
// job.ncols storage columns of every sequence.
// ---------------------------------------------------------------------------
template <typename T, int L, int E>
struct ColBody {
  using S = FFTShape<L, E>;
  static constexpr int EE = S::EE;
  static constexpr int TPS = S::TPS;

  // Byte offsets of the lane's slots in a length-N vector: positions
  // p_s = c + R (t + s TPS) of sequence q, mapped to Z_N.
  static __device__ __forceinline__ void vec_offsets(uint32_t (&off)[EE], const Shape &sh, int q, int64_t c,
                                                     int64_t R, int t, int es) {
    if (sh.odd > 1) {
      int tau[EE];
      crt_tau<EE>(tau, q, (uint32_t)(c + R * t), (uint32_t)(R * TPS), sh.odd, sh.odd_inv);
      const int64_t M = seq_len(sh);
#pragma unroll
      for (int s = 0; s < EE; ++s) off[s] = (uint32_t)((c + R * (t + s * TPS) + M * tau[s]) * es);
    } else {
#pragma unroll
      for (int s = 0; s < EE; ++s) off[s] = (uint32_t)((c + R * (t + s * TPS)) * es);
    }
  }

  // Power-of-two transforms (odd == 1).
  static __device__ __forceinline__ void run(const Shape &sh, const PV &P, const ColJob &job, int64_t c0,
                                             int TW, int tid, cx<T> *lds, const cx<T> *tw24,
                                             const cx<T> *tw4096) {
    const int cw = tid % TW;
    const int t = tid / TW;
    const int64_t c = c0 + cw;
    const bool cvalid = c < job.ncols;
    const int64_t R = (int64_t)1 << sh.logR;
    cx<T> a[EE];
    uint32_t off[EE];
    constexpr int CB = (int)sizeof(cx<T>);
    const int64_t N = (int64_t)1 << (sh.logR + sh.logC);
    if (job.kind == COL_A) {
      const OpDesc &od = sh.ops[job.op];
      const int es = elem_size<T>(od.flags);
      if (!sh.is_block) {
        // element c + R k of the padded operand; past its end reads zero
        const auto r = make_buf(P.op(job.op), od.len * es);
#pragma unroll
        for (int s = 0; s < EE; ++s) off[s] = (uint32_t)((c + R * (t + s * TPS)) * es);
        bgather<T, EE>(a, r, off, od.flags);
      } else {
        // generating matrix (len rows x cols columns, column-major): row c,
        // column k; rows past len are zero padding (k past cols falls past
        // the end of the resource)
        const auto r = make_buf(P.op(job.op), od.len * od.cols * es);
        const bool crow = c < od.len;
#pragma unroll
        for (int s = 0; s < EE; ++s) off[s] = crow ? (uint32_t)((c + od.len * (t + s * TPS)) * es) : OOB_OFF;
        bgather<T, EE>(a, r, off, od.flags);
      }
    } else {
      const auto r = make_buf(ws_buf<T>(sh, P, job.buf), N * CB);
#pragma unroll
      for (int s = 0; s < EE; ++s) off[s] = (uint32_t)((c + R * (t + s * TPS)) * CB);
      bgather<T, EE>(a, r, off, 0);
    }
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    // TW interleaved columns: element i of column cw at lds[(sw(i) << log2 TW) + cw]
    fft_seq<T, L, E>(a, t, lds + cw, stw, __builtin_ctz((unsigned)TW));
    if (!cvalid) return;
    // a row segment of the tile is TW elements: whole lines stream out
    // (non-temporal), narrower ones merge in L2
    if (TW * CB >= 128)
      store_tile<ST_NT>(a, sh, P, job, c, R, t, N);
    else
      store_tile<ST_DEFAULT>(a, sh, P, job, c, R, t, N);
  }

  template <int POL>
  static __device__ __forceinline__ void store_tile(const cx<T> (&a)[EE], const Shape &sh, const PV &P,
                                                    const ColJob &job, int64_t c, int64_t R, int t, int64_t N) {
    constexpr int CB = (int)sizeof(cx<T>);
    if (job.kind == COL_A) {
      const auto r = make_buf(ws_buf<T>(sh, P, job.buf), N * CB);
#pragma unroll
      for (int s = 0; s < EE; ++s) BufIO<T>::template st<POL>(a[s], r, off_ws(c, R, t + s * TPS));
    } else {
      void *dst = job.op == 0 ? P.y() : P.out1();
      const int es = sh.real_out ? (int)sizeof(T) : CB;
      if (!sh.is_block) {
        // the slice [0, lim) is the resource: later positions are dropped
        const int64_t lim = job.op == 0 ? sh.out_rows : sh.out1_len;
        const auto r = make_buf(dst, lim * es);
#pragma unroll
        for (int s = 0; s < EE; ++s)
          bstore<T, POL>(r, (uint32_t)((c + R * (t + s * TPS)) * es), job.conj_out ? cconj(a[s]) : a[s],
                         sh.real_out);
      } else if (c < sh.out_rows) {
        // out_rows x out_cols corner, column-major; columns past out_cols fall
        // past the end of the resource
        const auto r = make_buf(dst, sh.out_rows * sh.out_cols * es);
#pragma unroll
        for (int s = 0; s < EE; ++s)
          bstore<T, POL>(r, (uint32_t)((c + sh.out_rows * (t + s * TPS)) * es), job.conj_out ? cconj(a[s]) : a[s],
                         sh.real_out);
      }
    }
  }

  static __device__ __forceinline__ uint32_t off_ws(int64_t c, int64_t R, int k) {
    return (uint32_t)((c + R * k) * (int64_t)sizeof(cx<T>));
  }

  // Odd-factor transforms: virtual column v0 + lane column of the odd * R.
  static __device__ __forceinline__ void run_odd(const Shape &sh, const PV &P, const ColJob &job, int64_t v0,
                                                 int TW, int tid, cx<T> *lds, const cx<T> *tw24,
                                             const cx<T> *tw4096) {
    const int cw = tid % TW;
    const int t = tid / TW;
    const int64_t v = v0 + cw;
    const int q = sh.odd > 1 ? (int)(v >> sh.logR) : 0;
    const int64_t R = (int64_t)1 << sh.logR;
    const int64_t c = sh.odd > 1 ? (v & (R - 1)) : v;
    const bool cvalid = c < job.ncols && q < sh.odd;
    cx<T> a[EE];
    uint32_t off[EE];
    constexpr int CB = (int)sizeof(cx<T>);
    const int64_t M = seq_len(sh);
    const int64_t N = fft_len(sh);
    if (job.kind == COL_A) {
      const OpDesc &od = sh.ops[job.op];
      const int es = elem_size<T>(od.flags);
      if (!sh.is_block) {
        // entry c + R k of the padded operand (sequence q of it); past its
        // end reads zero
        const auto r = make_buf(P.op(job.op), od.len * es);
        vec_offsets(off, sh, q, c, R, t, es);
        bgather<T, EE>(a, r, off, od.flags);
      } else {
        // generating matrix (len rows x cols columns, column-major): row c,
        // column k; rows past len are zero padding (k past cols falls past
        // the end of the resource)
        const auto r = make_buf(P.op(job.op), od.len * od.cols * es);
        const bool crow = c < od.len;
#pragma unroll
        for (int s = 0; s < EE; ++s) off[s] = crow ? (uint32_t)((c + od.len * (t + s * TPS)) * es) : OOB_OFF;
        bgather<T, EE>(a, r, off, od.flags);
      }
    } else {
      const auto r = make_buf(ws_buf<T, true>(sh, P, job.buf), N * CB);
#pragma unroll
      for (int s = 0; s < EE; ++s) off[s] = (uint32_t)((q * M + c + R * (t + s * TPS)) * CB);
      bgather<T, EE>(a, r, off, 0);
    }
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    // TW interleaved columns: element i of column cw at lds[(sw(i) << log2 TW) + cw]
    fft_seq<T, L, E>(a, t, lds + cw, stw, __builtin_ctz((unsigned)TW));
    if (!cvalid) return;
    // a row segment of the tile is TW elements: whole lines stream out
    // (non-temporal), narrower ones merge in L2
    if (TW * CB >= 128)
      store_tile_odd<ST_NT>(a, sh, P, job, q, c, R, t);
    else
      store_tile_odd<ST_DEFAULT>(a, sh, P, job, q, c, R, t);
  }

  template <int POL>
  static __device__ __forceinline__ void store_tile_odd(const cx<T> (&a)[EE], const Shape &sh, const PV &P,
                                                        const ColJob &job, int q, int64_t c, int64_t R, int t) {
    constexpr int CB = (int)sizeof(cx<T>);
    if (job.kind == COL_A) {
      const int64_t M = seq_len(sh);
      const auto r = make_buf(ws_buf<T, true>(sh, P, job.buf), fft_len(sh) * CB);
#pragma unroll
      for (int s = 0; s < EE; ++s)
        BufIO<T>::template st<POL>(a[s], r, (uint32_t)((q * M + c + R * (t + s * TPS)) * CB));
    } else {
      void *dst = job.op == 0 ? P.y() : P.out1();
      const int es = sh.real_out ? (int)sizeof(T) : CB;
      if (!sh.is_block) {
        // the slice [0, lim) is the resource: later entries are dropped
        const int64_t lim = job.op == 0 ? sh.out_rows : sh.out1_len;
        const auto r = make_buf(dst, lim * es);
        uint32_t off[EE];
        vec_offsets(off, sh, q, c, R, t, es);
#pragma unroll
        for (int s = 0; s < EE; ++s)
          bstore<T, POL>(r, off[s], job.conj_out ? cconj(a[s]) : a[s], sh.real_out);
      } else if (c < sh.out_rows) {
        // out_rows x out_cols corner, column-major; columns past out_cols fall
        // past the end of the resource
        const auto r = make_buf(dst, sh.out_rows * sh.out_cols * es);
#pragma unroll
        for (int s = 0; s < EE; ++s)
          bstore<T, POL>(r, (uint32_t)((c + sh.out_rows * (t + s * TPS)) * es), job.conj_out ? cconj(a[s]) : a[s],
                         sh.real_out);
      }
    }
  }

  // BHHB grids with odd factors: rows odd * R (row axis i), columns
  // ODDC * C (column axis j), each axis through its own Chinese-remainder
  // map (i <-> (i mod odd, i mod R), j <-> (j mod ODDC, j mod C)).  The
  // workspace keeps i in natural order (the row pass applies the row axis's
  // map), so a tile is TW consecutive matrix rows i and only rows that can be
  // nonzero (pass A) or are kept (pass D) are transformed.  The ODDC column
  // sequences (index q_c) of a row are held side by side in the lane (slot s
  // of sequence q_c at position t + s TPS), each transformed along the
  // power-of-two axis, and a length-ODDC DFT across them per bin completes
  // the column axis (after the power-of-two transforms in the inputs' pass,
  // before them in the output's: the two factors commute).  Workspace row
  // r = q_c C + k2 holds bin k2 of the power-of-two axis, bin q_c of the odd one.
  template <int ODDC>
  static __device__ __forceinline__ void run_block_odd(const Shape &sh, const PV &P, const ColJob &job, int64_t v0,
                                                       int TW, int tid, cx<T> *lds, const cx<T> *tw4096) {
    const int cw = tid % TW;
    const int t = tid / TW;
    const int64_t i = v0 + cw;  // matrix row
    const bool cvalid = i < job.ncols;
    const int64_t C = (int64_t)1 << sh.logC;
    const int64_t W = (int64_t)(sh.odd > 1 ? sh.odd : 1) << sh.logR;  // workspace row length
    constexpr int CB = (int)sizeof(cx<T>);
    cx<T> a[ODDC][EE];
    if (job.kind == COL_A) {
      // generating matrix / vec(X_p): len rows x cols columns, column-major;
      // columns past cols fall past the end of the resource
      const OpDesc &od = sh.ops[job.op];
      const int es = elem_size<T>(od.flags);
      const auto r = make_buf(P.op(job.op), od.len * od.cols * es);
#pragma unroll
      for (int qc = 0; qc < ODDC; ++qc) {
        int tau[EE];
        if constexpr (ODDC > 1) crt_tau<EE>(tau, qc, (uint32_t)t, (uint32_t)TPS, ODDC, sh.odd_c_inv);
        uint32_t off[EE];
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          const int64_t j = t + s * TPS + (ODDC > 1 ? C * tau[s] : 0);
          off[s] = cvalid ? (uint32_t)((i + od.len * j) * es) : OOB_OFF;
        }
        bgather<T, EE>(a[qc], r, off, od.flags);
      }
    } else {
      const auto r = make_buf(ws_buf<T, true>(sh, P, job.buf), fft_len(sh) * CB);
#pragma unroll
      for (int qc = 0; qc < ODDC; ++qc) {
        uint32_t off[EE];
#pragma unroll
        for (int s = 0; s < EE; ++s)
          off[s] = cvalid ? (uint32_t)(((qc * C + t + s * TPS) * W + i) * CB) : OOB_OFF;
        bgather<T, EE>(a[qc], r, off, 0);
      }
    }
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    auto odd_axis = [&]() {
      if constexpr (ODDC > 1) {
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          cx<T> w[ODDC];
#pragma unroll
          for (int qc = 0; qc < ODDC; ++qc) w[qc] = a[qc][s];
          dft_odd<T, ODDC>(w);
#pragma unroll
          for (int qc = 0; qc < ODDC; ++qc) a[qc][s] = w[qc];
        }
      }
    };
    if (job.kind == COL_D) odd_axis();
    // TW interleaved columns: element k of column cw at lds[(sw(k) << log2 TW) + cw]
#pragma unroll
    for (int qc = 0; qc < ODDC; ++qc) fft_seq<T, L, E>(a[qc], t, lds + cw, stw, __builtin_ctz((unsigned)TW));
    if (job.kind == COL_A) odd_axis();
    if (!cvalid) return;
    if (job.kind == COL_A) {
      const auto r = make_buf(ws_buf<T, true>(sh, P, job.buf), fft_len(sh) * CB);
#pragma unroll
      for (int qc = 0; qc < ODDC; ++qc)
#pragma unroll
        for (int s = 0; s < EE; ++s)
          BufIO<T>::template st<ST_DEFAULT>(a[qc][s], r, (uint32_t)(((qc * C + t + s * TPS) * W + i) * CB));
    } else {
      // out_rows x out_cols corner of the output grid, column-major; columns
      // past out_cols fall past the end of the resource
      void *dst = job.op == 0 ? P.y() : P.out1();
      const int eo = sh.real_out ? (int)sizeof(T) : CB;
      const auto r = make_buf(dst, sh.out_rows * sh.out_cols * eo);
#pragma unroll
      for (int qc = 0; qc < ODDC; ++qc) {
        int tau[EE];
        if constexpr (ODDC > 1) crt_tau<EE>(tau, qc, (uint32_t)t, (uint32_t)TPS, ODDC, sh.odd_c_inv);
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          const int64_t j = t + s * TPS + (ODDC > 1 ? C * tau[s] : 0);
          bstore<T, ST_DEFAULT>(r, (uint32_t)((i + sh.out_rows * j) * eo), job.conj_out ? cconj(a[qc][s]) : a[qc][s],
                                sh.real_out);
        }
      }
    }
  }

  // Real-input transforms of length 2 * 2^(logR + logC): operands and output
  // are real arrays read and written as complex pairs (entry e = c + R k of
  // the complex view is real entries 2e and 2e + 1, each range-checked on its
  // own, so padding and the slice need no compares).
  static __device__ __forceinline__ void run_r2c(const Shape &sh, const PV &P, const ColJob &job, int64_t c0,
                                                 int TW, int tid, cx<T> *lds, const cx<T> *tw24,
                                                 const cx<T> *tw4096) {
    const int cw = tid % TW;
    const int t = tid / TW;
    const int64_t c = c0 + cw;
    const bool cvalid = c < job.ncols;
    const int64_t R = (int64_t)1 << sh.logR;
    const int64_t N = (int64_t)1 << (sh.logR + sh.logC);
    constexpr int CB = (int)sizeof(cx<T>), TB = (int)sizeof(T);
    cx<T> a[EE];
    if (job.kind == COL_A) {
      const auto r = make_buf(P.op(job.op), sh.ops[job.op].len * TB);
      T re[EE], im[EE];
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const uint32_t off = (uint32_t)(2 * (c + R * (t + s * TPS)) * TB);
        re[s] = BufIO<T>::ld1(r, off);
        im[s] = BufIO<T>::ld1(r, off + TB);
      }
#pragma unroll
      for (int s = 0; s < EE; ++s) a[s] = mk(re[s], im[s]);
    } else {
      const auto r = make_buf(ws_buf<T>(sh, P, job.buf), N * CB);
      uint32_t off[EE];
#pragma unroll
      for (int s = 0; s < EE; ++s) off[s] = (uint32_t)((c + R * (t + s * TPS)) * CB);
      bgather<T, EE>(a, r, off, 0);
    }
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    fft_seq<T, L, E>(a, t, lds + cw, stw, __builtin_ctz((unsigned)TW));
    if (!cvalid) return;
    if (job.kind == COL_A) {
      const auto r = make_buf(ws_buf<T>(sh, P, job.buf), N * CB);
#pragma unroll
      for (int s = 0; s < EE; ++s) BufIO<T>::template st<ST_DEFAULT>(a[s], r, off_ws(c, R, t + s * TPS));
    } else {
      const auto r = make_buf(job.op == 0 ? P.y() : P.out1(), sh.out_rows * TB);
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const uint32_t off = (uint32_t)(2 * (c + R * (t + s * TPS)) * TB);
        BufIO<T>::template st1<ST_DEFAULT>(a[s].x, r, off);
        BufIO<T>::template st1<ST_DEFAULT>(a[s].y, r, off + TB);
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Pass B of multipass real-input transforms (complex length N' = R C, real
// length N = 2 N').  Bin k of row r sits at position k1 with k = r + C k1; its
// mirror N' - k is in row C - r at position R - 1 - k1, and for rows 0 and
// C / 2 in the same row at positions -k1 mod R and R - 1 - k1.  Two lane
// groups of one workgroup take the row pair (p, C - p), or (0, C / 2) for
// p = 0, one row each, and find every mirror bin of the real transform's split
// and of the output's packing (see RealRowBody) in the pair's LDS.
// ---------------------------------------------------------------------------
template <typename T, int L, int E>
struct RealPairRowBody {
  using S = FFTShape<L, E>;
  using RB = RowBody<T, L, E, 1>;
  static constexpr int EE = S::EE;
  static constexpr int TPS = S::TPS;  // lanes per row; a pair takes 2 TPS
  static constexpr int SEQ_LDS = S::ROW_SEQ > L ? S::ROW_SEQ : L;  // per row; a pair takes 2 SEQ_LDS
  static constexpr bool WAVE = TPS <= 64;

  // W_N^{r + C (t + s TPS)}, N = 2 R C
  static __device__ __forceinline__ void split_tw(cx<T> (&w)[EE], const Shape &sh, int64_t r, int t,
                                                  const cx<T> *tw24, const cx<T> *tw4096) {
    const int logN = sh.logR + sh.logC + 1;
    slot_twiddles<T, EE>(w, (int64_t)1 << sh.logC, t, TPS, logN, tw24, tw4096);
    const cx<T> wr = twiddle_big<T>(r, logN, tw24, tw4096);
#pragma unroll
    for (int s = 0; s < EE; ++s) w[s] = cmul(w[s], wr);
  }

  // m[s] = the mirror of this row's slot s: from the partner row at R - 1 - k1,
  // or, for the rows 0 and C / 2 (self), from this row.  The barriers span the
  // workgroup: the partner row is another lane group, and the next transform
  // writes this row's LDS only after the partner has read it.
  static __device__ __forceinline__ void mirror(cx<T> (&m)[EE], const cx<T> (&a)[EE], bool self, int g, int t,
                                                cx<T> *mine, const cx<T> *partner) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < EE; ++s) mine[t + s * TPS] = a[s];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < EE; ++s) {
      const int k1 = t + s * TPS;
      const int rev = L - 1 - k1;
      m[s] = (self ? (const cx<T> *)mine : partner)[(self && g == 0) ? ((L - k1) & (L - 1)) : rev];
    }
    __syncthreads();
  }

  // Forward program on row g of pair p; returns the lane's share of alpha.
  static __device__ __forceinline__ cx<T> run_fwd(const Shape &sh, const PV &P, int64_t p, int g, bool valid, int t,
                                                  cx<T> *lds_pair, const cx<T> *tw24, const cx<T> *tw4096) {
    const int64_t C = (int64_t)1 << sh.logC;
    const bool self = p == 0;
    const int64_t r = g == 0 ? p : (self ? C / 2 : C - p);
    cx<T> *mine = lds_pair + g * SEQ_LDS;
    const cx<T> *partner = lds_pair + (1 - g) * SEQ_LDS;
    const T invN = T(1) / T((int64_t)2 << (sh.logR + sh.logC));
    const bool lane0 = self && g == 0 && t == 0;  // holds bin 0 (row 0, position 0) and the bin N'
    cx<T> a[EE], nx[EE], m[EE], acc[EE], w4[EE], wu[EE];
    cx<T> accn = czero<T>();
    T part = T(0);
    RB::twiddles(w4, sh, r, t, false, tw24, tw4096);
    split_tw(wu, sh, r, t, tw24, tw4096);
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
#pragma unroll
    for (int s = 0; s < EE; ++s) acc[s] = czero<T>();
    RB::load(a, sh, P, 0, r, valid, t, false);
    for (int o = 0; o < sh.nops; ++o) {
      if (o + 1 < sh.nops) RB::load(nx, sh, P, o + 1, r, valid, t, false);
      RB::twiddle_in(a, w4, true);
      RB::fft(a, t, mine, stw);
      const T vn = a[0].x - a[0].y;  // bin N' (on lane0)
      mirror(m, a, self, g, t, mine, partner);
#pragma unroll
      for (int s = 0; s < EE; ++s) {  // V = (Z + conj Zm) / 2 - i w (Z - conj Zm) / 2
        const cx<T> zm = cconj(m[s]);
        const cx<T> sp = cadd(a[s], zm), df = csub(a[s], zm);
        const cx<T> wd = cmul(wu[s], df);
        a[s] = mk(T(0.5) * (sp.x + wd.y), T(0.5) * (sp.y - wd.x));
      }
      const OpDesc &od = sh.ops[o];
      if (od.role == ROLE_H) {
#pragma unroll
        for (int s = 0; s < EE; ++s) acc[s] = cscale(cconj(a[s]), invN);
        accn = mk(vn * invN, T(0));
      } else {
        for (int e = 0; e < od.exp; ++e) {
#pragma unroll
          for (int s = 0; s < EE; ++s) acc[s] = cmul(acc[s], a[s]);
          accn.x *= vn;
        }
        if (od.flags & OPF_ALPHA) {
#pragma unroll
          for (int s = 0; s < EE; ++s) {
            const T tr = acc[s].x * a[s].x - acc[s].y * a[s].y;
            part += (lane0 && s == 0) ? tr : T(2) * tr;  // bin 0 counts once
          }
          if (lane0) part += accn.x * vn;
        }
      }
#pragma unroll
      for (int s = 0; s < EE; ++s) a[s] = nx[s];
    }
    if (sh.want_y) {
      mirror(m, acc, self, g, t, mine, partner);
      if (lane0) m[0] = accn;  // the mirror of bin 0 is bin N'
#pragma unroll
      for (int s = 0; s < EE; ++s) {  // Q = (z + conj zm) + i w (z - conj zm)
        const cx<T> zm = cconj(m[s]);
        const cx<T> sp = cadd(acc[s], zm), df = csub(acc[s], zm);
        const cx<T> wd = cmul(wu[s], df);
        acc[s] = mk(sp.x - wd.y, sp.y + wd.x);
      }
      RB::fft(acc, t, mine, stw);
      RB::store(acc, sh, P, 0, r, valid, t, false, w4);
    }
    return mk(part, T(0));
  }
};

}  // namespace hk
