// Device building blocks: complex arithmetic, in-register DFTs (powers of
// two up to 32, and the odd sizes 3 and 5) and a workgroup-level Stockham FFT
// for power-of-two lengths on gfx950.
//
// Transform convention (the paper's Matlab-type fft, Section 2.1):
//   X_k = sum_j x_j exp(-2 pi i j k / L).
// Only the forward transform is implemented; the inverse used for the
// generating vector, ifft(v) = conj(fft(conj(v))) / L, is obtained by
// conjugating on load and store.
//
// Layout contract of fft_seq<T, L, E>: a sequence of length L is owned by
// TPS = L / E consecutive lanes; lane t holds elements t + s*TPS in register
// slot s (s < E) before the call and the transform's outputs t + s*TPS after
// it, so consecutive transforms and pointwise products chain in registers.
// Internally the transform is a Stockham autosort sequence of radix-E passes
// (last pass radix L / E^(P-1)); consecutive passes exchange data through a
// padded LDS buffer private to the sequence.  The in-register radix-R DFTs
// (R <= 32) are radix-2 decimation-in-frequency networks with compile-time
// twiddles.  Published methods: Cooley-Tukey (1965) radix-2 DIF, Stockham
// autosort formulation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) {
  return mk(a.x + b.x, a.y + b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) {
  return mk(a.x - b.x, a.y - b.y);
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
template <typename T>
__device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {  // a*b + c
  return mk(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) {
  return mk(a.x, -a.y);
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) {
  return mk(a.x * s, a.y * s);
}
template <typename T>
__device__ __forceinline__ cx<T> czero() {
  return mk(T(0), T(0));
}

__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }
__host__ __device__ constexpr int ipowc(int b, int e) { return e == 0 ? 1 : b * ipowc(b, e - 1); }
__host__ __device__ constexpr int bitrevc(int v, int bits) {
  return bits == 0 ? 0 : ((v & 1) << (bits - 1)) | bitrevc(v >> 1, bits - 1);
}

// cos(2 pi k / 32) for k = 0..8 (sin follows by symmetry).
__host__ __device__ constexpr double cos32_base(int k) {
  return k == 0   ? 1.0
         : k == 1 ? 0.980785280403230449126182236134
         : k == 2 ? 0.923879532511286756128183189397
         : k == 3 ? 0.831469612302545237078788377618
         : k == 4 ? 0.707106781186547524400844362105
         : k == 5 ? 0.555570233019602224742830813949
         : k == 6 ? 0.382683432365089771728459984030
         : k == 7 ? 0.195090322016128267848284868477
                  : 0.0;
}
// cos / sin of 2 pi k / 32 for k in [0, 16).
__host__ __device__ constexpr double cos32(int k) { return k <= 8 ? cos32_base(k) : -cos32_base(16 - k); }
__host__ __device__ constexpr double sin32(int k) { return k <= 8 ? cos32_base(8 - k) : cos32_base(k - 8); }

// a * exp(-2 pi i k / 32), k a compile-time constant after unrolling (k < 16).
template <typename T>
__device__ __forceinline__ cx<T> twmul32(cx<T> a, int k) {
  if (k == 0) return a;
  if (k == 8) return mk(a.y, -a.x);  // * (-i)
  if (k == 4) {
    const T c = T(0.707106781186547524400844362105);
    return mk((a.x + a.y) * c, (a.y - a.x) * c);
  }
  if (k == 12) {
    const T c = T(0.707106781186547524400844362105);
    return mk((a.y - a.x) * c, -(a.x + a.y) * c);
  }
  const T cr = T(cos32(k));
  const T si = T(sin32(k));
  return mk(fma(a.x, cr, a.y * si), fma(a.y, cr, -(a.x * si)));
}

// In-register forward DFT of size R (natural order in and out), R <= 32.
template <typename T, int R>
__device__ __forceinline__ void dft(cx<T> (&v)[R]) {
  static_assert(R >= 1 && R <= 32 && (R & (R - 1)) == 0, "radix");
  if constexpr (R > 1) {
#pragma unroll
    for (int s = R / 2; s >= 1; s >>= 1) {
#pragma unroll
      for (int g = 0; g < R; g += 2 * s) {
#pragma unroll
        for (int j = 0; j < s; ++j) {
          const cx<T> u = v[g + j];
          const cx<T> w = v[g + j + s];
          v[g + j] = cadd(u, w);
          v[g + j + s] = twmul32(csub(u, w), j * (32 / (2 * s)));
        }
      }
    }
    constexpr int bits = ilog2c(R);
    cx<T> o[R];
#pragma unroll
    for (int k = 0; k < R; ++k) o[k] = v[bitrevc(k, bits)];
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = o[k];
  }
}

// In-register forward DFT of odd size Q in {1, 3, 5}, natural order:
// X_k = sum_a v_a exp(-2 pi i a k / Q).  Written from the definition with the
// symmetric pairs v_a +- v_{Q-a}, so that each output needs one real
// constant per pair (Winograd-style short DFTs).
template <typename T, int Q>
__device__ __forceinline__ void dft_odd(cx<T> (&v)[Q]) {
  static_assert(Q == 1 || Q == 3 || Q == 5, "odd factor");
  if constexpr (Q == 3) {
    const T c = T(0.866025403784438646763723170753);  // sin(2 pi / 3)
    const cx<T> s = cadd(v[1], v[2]);
    const cx<T> d = csub(v[1], v[2]);
    const cx<T> m = mk(v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y);
    // -i sin(2 pi / 3) d
    const cx<T> r = mk(c * d.y, -c * d.x);
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  } else if constexpr (Q == 5) {
    const T c1 = T(0.309016994374947424102293417183);   // cos(2 pi / 5)
    const T c2 = T(-0.809016994374947424102293417183);  // cos(4 pi / 5)
    const T s1 = T(0.951056516295153572116439333379);   // sin(2 pi / 5)
    const T s2 = T(0.587785252292473129168705954639);   // sin(4 pi / 5)
    const cx<T> a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const cx<T> a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    // real-weighted sums of the pairs
    const cx<T> m1 = mk(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
    const cx<T> m2 = mk(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
    // odd parts: u1 = s1 b1 + s2 b2, u2 = s2 b1 - s1 b2; outputs take -i u
    const cx<T> u1 = mk(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
    const cx<T> u2 = mk(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
    const cx<T> r1 = mk(u1.y, -u1.x);
    const cx<T> r2 = mk(u2.y, -u2.x);
    v[0] = mk(v[0].x + a1.x + a2.x, v[0].y + a1.y + a2.y);
    v[1] = cadd(m1, r1);
    v[4] = csub(m1, r1);
    v[2] = cadd(m2, r2);
    v[3] = csub(m2, r2);
  }
}

// Static layout of a length-L transform with (at most) E elements per lane.
template <int L, int E>
struct FFTShape {
  static_assert(L >= 1 && (L & (L - 1)) == 0, "L must be a power of two");
  static_assert(E >= 1 && E <= 32 && (E & (E - 1)) == 0, "E must be a power of two <= 32");
  static constexpr int EE = E < L ? E : L;  // elements per lane
  static constexpr int TPS = L / EE;        // lanes per sequence
  static constexpr int LOGL = ilog2c(L);
  static constexpr int LOGE = ilog2c(EE);
  static constexpr int P = LOGL == 0 ? 0 : (LOGL + LOGE - 1) / LOGE;  // Stockham passes
  static constexpr int LOG_LAST = LOGL - LOGE * (P > 0 ? P - 1 : 0);
  // LDS elements one sequence's exchanges need (no padding: see sw()).
  static constexpr int LDS = P > 1 ? L : 0;
  // Row sequences placed side by side in one wavefront (TPS < 32) are
  // offset by TPS elements so that their lanes fall on different banks.
  static constexpr int ROW_SEQ = P > 1 ? L + (TPS < 32 ? TPS : 0) : 0;
  static __host__ __device__ constexpr int radix(int p) { return p < P - 1 ? EE : (1 << LOG_LAST); }
  static __host__ __device__ constexpr int nbf(int p) { return EE / radix(p); }  // butterflies per lane
  // offset of pass p's twiddles in a lane's precomputed set (passes 1..P-1)
  static __host__ __device__ constexpr int tw_off(int p) {
    int o = 0;
    for (int i = 1; i < p; ++i) o += nbf(i) * (radix(i) - 1);
    return o;
  }
  static constexpr int TWN = tw_off(P) > 0 ? tw_off(P) : 1;
  // LDS slot of element i: the low five index bits are XORed with the bits
  // above log2(EE).  Reads (consecutive i across lanes) stay a permutation of
  // aligned 32-element blocks, and the strided writes of the first pass
  // (i = EE b + r) land on distinct 8-byte slots, so every exchange of 32
  // lanes touches 32 distinct slots: no bank conflicts, no padding.
  static constexpr int SWM = (L < 32 ? L : 32) - 1;
  static __device__ __forceinline__ int sw(int i) { return i ^ ((i >> LOGE) & SWM); }
};

// Register array holding one lane's share of a length-L sequence.
template <typename T, int L, int E>
using Regs = cx<T>[FFTShape<L, E>::EE];

// Synchronization between the LDS write and read halves of an exchange.
// WAVE = true when every lane of a sequence sits in the same wavefront (the
// sequence's TPS lanes are consecutive and TPS divides 64): LDS operations of
// one wave execute in order, so ordering the compiler's memory operations is
// enough.  Otherwise a workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void seq_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// exp(-2 pi i r k / (Ns R)) for r = 1..R-1 from the log2(R) table entries
// W^{k 2^j}: each power is a product of at most log2(R) table values, so the
// error stays within a few ulp while the lane issues log2(R) loads instead of
// R - 1.
template <typename T, int R>
__device__ __forceinline__ void stage_twiddles(cx<T> (&w)[R], int k, int step, const cx<T> *__restrict__ tw4096) {
  constexpr int LR = ilog2c(R);
  cx<T> base[LR > 0 ? LR : 1];
#pragma unroll
  for (int j = 0; j < LR; ++j) base[j] = tw4096[((k << j) * step) & 4095];
  w[0] = mk(T(1), T(0));
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const int rest = r & (r - 1);       // r without its lowest set bit
    const int lb = ilog2c(r & (-r));    // index of that bit
    w[r] = rest == 0 ? base[lb] : cmul(w[rest], base[lb]);
  }
}

// A lane's twiddles for every pass p >= 1 of a length-L transform.  They
// depend only on the lane, so a kernel computes them once (their table loads
// overlap the first data loads) and reuses them for all its transforms.
template <typename T, int L, int E>
struct StageTw {
  using S = FFTShape<L, E>;
  cx<T> w[S::TWN];

  template <int p>
  __device__ __forceinline__ void init_pass(int t, const cx<T> *__restrict__ tw4096) {
    if constexpr (p < S::P) {
      constexpr int R = S::radix(p);
      constexpr int Ns = ipowc(S::EE, p);
      constexpr int step = 4096 / (Ns * R);
#pragma unroll
      for (int q = 0; q < S::nbf(p); ++q) {
        cx<T> tmp[R];
        stage_twiddles<T, R>(tmp, (t + q * S::TPS) & (Ns - 1), step, tw4096);
#pragma unroll
        for (int r = 1; r < R; ++r) w[S::tw_off(p) + q * (R - 1) + r - 1] = tmp[r];
      }
      init_pass<p + 1>(t, tw4096);
    }
  }
  __device__ __forceinline__ void init(int t, const cx<T> *__restrict__ tw4096) { init_pass<1>(t, tw4096); }
};

// One Stockham pass.  Slot (q, r) of lane t holds input b + r*(L/R) with
// butterfly b = t + q*TPS; span Ns = EE^p; outputs go to
// (b - k) R + k + r Ns, k = b mod Ns.  With PRE the twiddles come from the
// lane's precomputed set, otherwise from the table.
//
// LDS layout: element i of the sequence sits at lds[sw(i) << ls]; ls = 0 for
// a row sequence, log2(TW) for a column tile whose TW columns are
// interleaved (lds already offset by the lane's column).
template <typename T, int L, int E, bool WAVE, bool PRE, int p>
__device__ __forceinline__ void fft_pass(Regs<T, L, E> &a, int t, cx<T> *lds, int ls,
                                         const cx<T> *__restrict__ tw4096, const StageTw<T, L, E> &pre) {
  using S = FFTShape<L, E>;
  constexpr int EE = S::EE;
  constexpr int TPS = S::TPS;
  constexpr int R = S::radix(p);
  constexpr int B = EE / R;
  constexpr int Ns = ipowc(EE, p);
  constexpr bool last = (p == S::P - 1);
  if constexpr (p > 0) {
    seq_sync<WAVE>();
#pragma unroll
    for (int q = 0; q < B; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) a[q + r * B] = lds[S::sw(t + q * TPS + r * (L / R)) << ls];
  }
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int b = t + q * TPS;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[q + r * B];
    if constexpr (p > 0) {
      if constexpr (PRE) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], pre.w[S::tw_off(p) + q * (R - 1) + r - 1]);
      } else {
        const int k = b & (Ns - 1);
        constexpr int step = 4096 / (Ns * R);
        cx<T> w[R];
        stage_twiddles<T, R>(w, k, step, tw4096);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
      }
    }
    dft<T, R>(v);
#pragma unroll
    for (int r = 0; r < R; ++r) a[q + r * B] = v[r];
  }
  if constexpr (!last) {
    seq_sync<WAVE>();
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int b = t + q * TPS;
      const int k = b & (Ns - 1);
      const int base = (b - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[S::sw(base + r * Ns) << ls] = a[q + r * B];
    }
    fft_pass<T, L, E, WAVE, PRE, p + 1>(a, t, lds, ls, tw4096, pre);
  }
}

// Forward FFT of one length-L sequence held in registers (see file comment).
// Every lane of the workgroup must call this (it contains barriers when the
// transform needs more than one pass and WAVE is false).
template <typename T, int L, int E, bool WAVE = false>
__device__ __forceinline__ void fft_seq(Regs<T, L, E> &a, int t, cx<T> *lds,
                                        const cx<T> *__restrict__ tw4096, int ls = 0) {
  StageTw<T, L, E> none;
  if constexpr (FFTShape<L, E>::P > 0) fft_pass<T, L, E, WAVE, false, 0>(a, t, lds, ls, tw4096, none);
}

// Same, with the lane's precomputed twiddles.
template <typename T, int L, int E, bool WAVE = false>
__device__ __forceinline__ void fft_seq(Regs<T, L, E> &a, int t, cx<T> *lds, const StageTw<T, L, E> &pre,
                                        int ls = 0) {
  if constexpr (FFTShape<L, E>::P > 0) fft_pass<T, L, E, WAVE, true, 0>(a, t, lds, ls, nullptr, pre);
}


// exp(-2 pi i e / 2^logN) for 0 <= e < 2^logN <= 2^24 from two 4096-entry
// tables: tw24[j] = exp(-2 pi i j / 2^24), tw4096[j] = exp(-2 pi i j / 4096).
template <typename T>
__device__ __forceinline__ cx<T> twiddle_big(int64_t e, int logN, const cx<T> *__restrict__ tw24,
                                             const cx<T> *__restrict__ tw4096) {
  const uint32_t bidx = (uint32_t)(e << (24 - logN));
  // tw24[0] is exactly 1, so the product is exact when the low part vanishes.
  return cmul(tw24[bidx & 4095u], tw4096[bidx >> 12]);
}

// Twiddles W_N^{u (t + s TPS)} for the EE slots s of a lane: one table product
// for the lane's base exponent u t, log2(EE) for the steps u TPS 2^j, and
// at most log2(EE) products per slot.
template <typename T, int EE>
__device__ __forceinline__ void slot_twiddles(cx<T> (&w)[EE], int64_t u, int t, int TPS, int logN,
                                              const cx<T> *__restrict__ tw24, const cx<T> *__restrict__ tw4096) {
  constexpr int LE = ilog2c(EE);
  const int64_t Nm = ((int64_t)1 << logN) - 1;
  cx<T> st[LE > 0 ? LE : 1];
#pragma unroll
  for (int j = 0; j < LE; ++j) st[j] = twiddle_big<T>((u * ((int64_t)TPS << j)) & Nm, logN, tw24, tw4096);
  cx<T> pw[EE];
  pw[0] = mk(T(1), T(0));
#pragma unroll
  for (int s = 1; s < EE; ++s) {
    const int rest = s & (s - 1);       // s without its lowest set bit
    const int lb = ilog2c(s & (-s));    // index of that bit
    pw[s] = rest == 0 ? st[lb] : cmul(pw[rest], st[lb]);
  }
  const cx<T> b0 = twiddle_big<T>((u * t) & Nm, logN, tw24, tw4096);
#pragma unroll
  for (int s = 0; s < EE; ++s) w[s] = s == 0 ? b0 : cmul(b0, pw[s]);
}

}  // namespace hk
