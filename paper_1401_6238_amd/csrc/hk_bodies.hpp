// Workgroup bodies of the Hankel tensor-vector product on gfx950.
//
// Index algebra.  Let N = R * C (R = 2^logR contiguous "row" length, C =
// 2^logC "column" length) and store element n = n1 + R n2 at offset n.
// With n = n1 + R n2 and k = k2 + C k1 (Bailey's four-step decomposition):
//   X[k2 + C k1] = sum_n1 W_R^{n1 k1} W_N^{n1 k2} sum_n2 x[n1 + R n2] W_C^{n2 k2}.
// Pass A: for each column n1, a length-C FFT along n2, times W_N^{n1 k2},
//         stored at n1 + R k2.
// Pass B: for each row k2, a length-R FFT along n1 gives X[k2 + C k1] at
//         offset k1 + R k2 ("transposed" spectral order).  Every operand uses
//         the same order, so the pointwise spectral product is done here.
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

template <typename T>
__device__ __forceinline__ cx<T> load_op(const void *base, int64_t idx, int flags) {
  if (flags & OPF_REAL) {
    const T v = ((const T *)base)[idx];
    return mk(v, T(0));
  }
  cx<T> v = ((const cx<T> *)base)[idx];
  if (flags & OPF_CONJ) v.y = -v.y;
  return v;
}

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

template <typename T>
__device__ __forceinline__ cx<T> *ws_buf(const Shape &sh, const PV &P, int b) {
  const int64_t N = (int64_t)1 << (sh.logR + sh.logC);
  return (cx<T> *)P.ws() + (int64_t)b * N;
}

template <typename T>
__device__ __forceinline__ cx<T> *ws_partials(const Shape &sh, const PV &P) {
  const int64_t N = (int64_t)1 << (sh.logR + sh.logC);
  return (cx<T> *)P.ws() + sh.nbuf * N;
}

template <typename T>
__device__ __forceinline__ uint32_t *ws_counter(const Shape &sh, const PV &P) {
  return (uint32_t *)(ws_partials<T>(sh, P) + sh.partials);
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

// ---------------------------------------------------------------------------
// Row body: one sequence of length L per row; TPS lanes per row.
// resident = true : the row is a whole 1D instance (load inputs with padding,
//                   store the sliced outputs).
// resident = false: pass B row `row` of a multipass instance.
// Returns this lane's contribution to the scalar product (forward program).
// ---------------------------------------------------------------------------
template <typename T, int L, int E>
struct RowBody {
  using S = FFTShape<L, E>;
  static constexpr int EE = S::EE;
  static constexpr int TPS = S::TPS;
  static constexpr int SEQ_LDS = S::ROW_SEQ;
  // A row's TPS lanes are consecutive, so a row of at most 64 lanes lives in
  // one wavefront and its exchanges need no workgroup barrier.
  static constexpr bool WAVE = TPS <= 64;

  static __device__ __forceinline__ void fft(cx<T> (&a)[EE], int t, cx<T> *lds, const StageTw<T, L, E> &tw) {
    fft_seq<T, L, E, WAVE>(a, t, lds, tw);
  }

  static __device__ __forceinline__ void load(cx<T> (&a)[EE], const Shape &sh, const PV &P, int o,
                                              int64_t row, bool valid_row, int t, bool resident) {
    const OpDesc &od = sh.ops[o];
    int64_t idx[EE];
    bool ok[EE];
    if (resident) {
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        idx[s] = t + s * TPS;
        ok[s] = valid_row && idx[s] < od.len;
      }
      gather<T, EE>(a, P.op(o), idx, ok, od.flags);
    } else {
      const cx<T> *src = ws_buf<T>(sh, P, od.buf) + (valid_row ? row : 0) * L;
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        idx[s] = t + s * TPS;
        ok[s] = valid_row && idx[s] < od.ncol_nz;
      }
      gather<T, EE>(a, src, idx, ok, 0);
    }
  }

  // Stores output `which` (0: y / grad_h, 1: grad_x) of this row.
  static __device__ __forceinline__ void store(const cx<T> (&a)[EE], const Shape &sh, const PV &P,
                                               int which, int64_t row, bool valid_row, int t,
                                               bool resident, const cx<T> *tw24, const cx<T> *tw4096) {
    if (!valid_row) return;
    if (resident) {
      void *dst = which == 0 ? P.y() : P.out1();
      const int64_t lim = which == 0 ? sh.out_rows : sh.out1_len;
      const bool cj = (sh.prog == PROG_BWD) && which == 1;
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        const int pos = t + s * TPS;
        if (pos < lim) store_out<T>(dst, pos, cj ? cconj(a[s]) : a[s], sh.real_out);
      }
    } else {
      cx<T> *dst = ws_buf<T>(sh, P, sh.ops[which].buf) + row * L;
      if (!sh.is_block) {
        // four-step twiddles W_N^{pos * row}, pos = t + s TPS
        cx<T> w[EE];
        slot_twiddles<T, EE>(w, row, t, TPS, sh.logR + sh.logC, tw24, tw4096);
#pragma unroll
        for (int s = 0; s < EE; ++s) dst[t + s * TPS] = cmul(a[s], w[s]);
      } else {
#pragma unroll
        for (int s = 0; s < EE; ++s) dst[t + s * TPS] = a[s];
      }
    }
  }

  // Forward program: z = h^ prod_p x^_p^{e_p}; y = fft(z); alpha = sum z x^_1.
  static __device__ __forceinline__ cx<T> run_fwd(const Shape &sh, const PV &P, int64_t row, bool valid_row,
                                                  int t, cx<T> *lds, bool resident, const cx<T> *tw24,
                                                  const cx<T> *tw4096) {
    const T invN = T(1) / T((int64_t)1 << (sh.logR + sh.logC));
    cx<T> a[EE], nx[EE], acc[EE];
    cx<T> part = czero<T>();
#pragma unroll
    for (int s = 0; s < EE; ++s) acc[s] = czero<T>();
    load(a, sh, P, 0, row, valid_row, t, resident);
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    for (int o = 0; o < sh.nops; ++o) {
      // the next operand's loads are in flight while this one is transformed
      if (o + 1 < sh.nops) load(nx, sh, P, o + 1, row, valid_row, t, resident);
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
      fft(acc, t, lds, stw);
      store(acc, sh, P, 0, row, valid_row, t, resident, tw24, tw4096);
    }
    return part;
  }

  // Adjoint of g = H x^{m-1}, f = H x^m (equal vectors).  Operands in order:
  // X, then optionally V (cotangent of g, conjugated on load), then H when
  // grad_x is requested.
  static __device__ __forceinline__ void run_bwd(const Shape &sh, const PV &P, int64_t row, bool valid_row,
                                                 int t, cx<T> *lds, bool resident, const cx<T> *tw24,
                                                 const cx<T> *tw4096) {
    const T invN = T(1) / T((int64_t)1 << (sh.logR + sh.logC));
    cx<T> a[EE], gq[EE];
    cx<T> phc = czero<T>();  // conj(phi)
    if (P.phi()) phc = cconj(*(const cx<T> *)P.phi());
    const T m1 = T(sh.m - 1), m0 = T(sh.m);
    StageTw<T, L, E> stw;
    {
      cx<T> xs[EE], p1[EE], vs[EE];
      load(xs, sh, P, 0, row, valid_row, t, resident);
      stw.init(t, tw4096);
      fft(xs, t, lds, stw);
#pragma unroll
      for (int s = 0; s < EE; ++s) p1[s] = mk(T(1), T(0));
      for (int e = 0; e < sh.m - 2; ++e) {
#pragma unroll
        for (int s = 0; s < EE; ++s) p1[s] = cmul(p1[s], xs[s]);
      }
      const bool has_v = sh.nops > 1 && sh.ops[1].role == ROLE_V;
      if (has_v) {
        load(vs, sh, P, 1, row, valid_row, t, resident);
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
      store(a, sh, P, 0, row, valid_row, t, resident, tw24, tw4096);
    }
    if (sh.want_out1) {
      load(a, sh, P, sh.nops - 1, row, valid_row, t, resident);  // H
      fft(a, t, lds, stw);
#pragma unroll
      for (int s = 0; s < EE; ++s) a[s] = cmul(cscale(cconj(a[s]), invN), gq[s]);
      fft(a, t, lds, stw);
      store(a, sh, P, 1, row, valid_row, t, resident, tw24, tw4096);
    }
  }
};

// ---------------------------------------------------------------------------
// Column body: TW columns of length L (one sequence each), TPS lanes per
// column, lane l -> column l % TW, position-lane l / TW (so that a wave
// reads TW contiguous elements of several rows at once).
// ---------------------------------------------------------------------------
template <typename T, int L, int E>
struct ColBody {
  using S = FFTShape<L, E>;
  static constexpr int EE = S::EE;
  static constexpr int TPS = S::TPS;

  static __device__ __forceinline__ void run(const Shape &sh, const PV &P, const ColJob &job, int64_t c0,
                                             int TW, int tid, cx<T> *lds, const cx<T> *tw24,
                                             const cx<T> *tw4096) {
    const int cw = tid % TW;
    const int t = tid / TW;
    const int64_t c = c0 + cw;
    const bool cvalid = c < job.ncols;
    const int64_t R = (int64_t)1 << sh.logR;
    cx<T> a[EE];
    int64_t idx[EE];
    bool ok[EE];
    if (job.kind == COL_A) {
      const OpDesc &od = sh.ops[job.op];
      if (!sh.is_block) {
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          idx[s] = c + R * (t + s * TPS);
          ok[s] = cvalid && idx[s] < od.len;
        }
      } else {
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          const int64_t r = t + s * TPS;
          idx[s] = c + od.len * r;
          ok[s] = cvalid && c < od.len && r < od.cols;
        }
      }
      gather<T, EE>(a, P.op(job.op), idx, ok, od.flags);
    } else {
#pragma unroll
      for (int s = 0; s < EE; ++s) {
        idx[s] = c + R * (t + s * TPS);
        ok[s] = cvalid;
      }
      gather<T, EE>(a, ws_buf<T>(sh, P, job.buf), idx, ok, 0);
    }
    StageTw<T, L, E> stw;
    stw.init(t, tw4096);
    // pass A's four-step twiddles W_N^{c k}, k = t + s TPS: their table loads
    // are issued before the transform so that they overlap it
    cx<T> wst[EE];
    const bool twid = job.kind == COL_A && !sh.is_block;
    if (twid) slot_twiddles<T, EE>(wst, c, t, TPS, sh.logR + sh.logC, tw24, tw4096);
    // TW interleaved columns: element i of column cw at lds[(sw(i) << log2 TW) + cw]
    fft_seq<T, L, E>(a, t, lds + cw, stw, __builtin_ctz((unsigned)TW));
    if (!cvalid) return;
    if (job.kind == COL_A) {
      cx<T> *dst = ws_buf<T>(sh, P, job.buf);
      if (twid) {
#pragma unroll
        for (int s = 0; s < EE; ++s) dst[c + R * (t + s * TPS)] = cmul(a[s], wst[s]);
      } else {
#pragma unroll
        for (int s = 0; s < EE; ++s) dst[c + R * (t + s * TPS)] = a[s];
      }
    } else {
      void *dst = job.op == 0 ? P.y() : P.out1();
      if (!sh.is_block) {
        const int64_t lim = job.op == 0 ? sh.out_rows : sh.out1_len;
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          const int64_t pos = c + R * (t + s * TPS);
          if (pos < lim) store_out<T>(dst, pos, job.conj_out ? cconj(a[s]) : a[s], sh.real_out);
        }
      } else if (c < sh.out_rows) {
#pragma unroll
        for (int s = 0; s < EE; ++s) {
          const int64_t k = t + s * TPS;
          if (k < sh.out_cols) store_out<T>(dst, c + sh.out_rows * k, job.conj_out ? cconj(a[s]) : a[s], sh.real_out);
        }
      }
    }
  }
};

}  // namespace hk
