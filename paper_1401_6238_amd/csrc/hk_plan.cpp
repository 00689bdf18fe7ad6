// Planning and launch sequencing of the plain (single-shape) path.
#include "hk_plan.hpp"

#include <hip/hip_ext.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>

namespace hk {

static thread_local int tl_launches = 0;
void count_launch() { ++tl_launches; }
int launches_and_reset() {
  const int v = tl_launches;
  tl_launches = 0;
  return v;
}

Status fail(hk_status_t code, const std::string &msg) {
  Status s;
  s.code = code;
  s.msg = msg;
  return s;
}

bool is_complex(hk_dtype_t dt) { return dt == HK_C64 || dt == HK_C128; }
size_t elem_bytes(hk_dtype_t dt) {
  switch (dt) {
    case HK_C64: return 8;
    case HK_C128: return 16;
    case HK_F32: return 4;
    case HK_F64: return 8;
  }
  return 0;
}
size_t cplx_bytes(hk_dtype_t dt) { return (dt == HK_C128 || dt == HK_F64) ? 16 : 8; }
static bool is_double(hk_dtype_t dt) { return dt == HK_C128 || dt == HK_F64; }

int ceil_log2(int64_t v) {
  int l = 0;
  while (((int64_t)1 << l) < v) ++l;
  return l;
}

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
static Status check_common(const Problem &p) {
  if (p.dt < HK_C64 || p.dt > HK_F64) return fail(HK_ERR_INVALID_VALUE, "unknown dtype");
  if (p.m < 2 || p.m > HK_MAX_ORDER) return fail(HK_ERR_INVALID_VALUE, "order m must be in [2, 8]");
  for (int q = 0; q < p.m; ++q) {
    if (p.dims[q] < 1) return fail(HK_ERR_INVALID_VALUE, "every dimension must be >= 1");
    if (p.dims[q] > ((int64_t)1 << 40)) return fail(HK_ERR_SIZE_LIMIT, "dimension too large");
    if (p.is_block) {
      if (p.bdims[q] < 1) return fail(HK_ERR_INVALID_VALUE, "every block count must be >= 1");
      if (p.bdims[q] > ((int64_t)1 << 40)) return fail(HK_ERR_SIZE_LIMIT, "block count too large");
    }
  }
  return Status();
}

Status validate_forward(const Problem &p) {
  Status s = check_common(p);
  if (!s.ok()) return s;
  if (!p.y && !p.alpha) return fail(HK_ERR_NULL_POINTER, "neither y nor alpha requested");
  if ((p.conv || p.conj_y) && !is_complex(p.dt))
    return fail(HK_ERR_NOT_SUPPORTED, "the adjoint is implemented for complex dtypes");
  if (p.conv) {
    if (!p.y || p.alpha) return fail(HK_ERR_INVALID_VALUE, "the convolution program has a vector output only");
    if (!p.vec[0]) return fail(HK_ERR_NULL_POINTER, "vector 1 is NULL");
  } else if (!p.h) {
    return fail(HK_ERR_NULL_POINTER, "generating vector/matrix is NULL");
  }
  for (int q = 1; q < p.m; ++q)
    if (!p.vec[q]) return fail(HK_ERR_NULL_POINTER, "vector " + std::to_string(q + 1) + " is NULL");
  if (p.alpha && !p.vec[0]) return fail(HK_ERR_NULL_POINTER, "alpha requested but vector 1 is NULL");
  const size_t a = elem_bytes(p.dt);
  if ((p.h && !aligned(p.h, a)) || (p.y && !aligned(p.y, a)) || (p.alpha && !aligned(p.alpha, a)))
    return fail(HK_ERR_MISALIGNED, "pointer not aligned to the element size");
  for (int q = 0; q < p.m; ++q)
    if (p.vec[q] && !aligned(p.vec[q], a)) return fail(HK_ERR_MISALIGNED, "vector not aligned to the element size");
  Layout lay;
  return layout_for(p, 0, &lay);
}

Status validate_backward(const Problem &p) {
  Status s = check_common(p);
  if (!s.ok()) return s;
  if (!is_complex(p.dt)) return fail(HK_ERR_NOT_SUPPORTED, "the adjoint is implemented for complex dtypes");
  if (!p.gx && !p.gh) return fail(HK_ERR_NULL_POINTER, "neither grad_x nor grad_h requested");
  if (!p.h || !p.vec[1]) return fail(HK_ERR_NULL_POINTER, "h or x is NULL");
  const size_t a = elem_bytes(p.dt);
  const void *ps[] = {p.h, p.vec[1], p.v, p.phi, p.gx, p.gh};
  for (const void *q : ps)
    if (q && !aligned(q, a)) return fail(HK_ERR_MISALIGNED, "pointer not aligned to the element size");
  Layout lay;
  return layout_for(p, 0, &lay);
}

// ---------------------------------------------------------------------------
// Layout
// ---------------------------------------------------------------------------
bool row_limits(hk_dtype_t dt, int odd, int logL, int E, KernelLimits *k) {
  if (odd == 1) return is_double(dt) ? limits_f64(logL, E, k) : limits_f32(logL, E, k);
  return is_double(dt) ? limits_odd_f64(odd, logL, E, k) : limits_odd_f32(odd, logL, E, k);
}

static int odd_row_e(hk_dtype_t dt) { return is_double(dt) ? odd_row_e_f64() : odd_row_e_f32(); }

// Real-input rows: elements per lane and limits.
static int r2c_row_e(hk_dtype_t dt) { return is_double(dt) ? r2c_row_e_f64() : r2c_row_e_f32(); }
static bool r2c_limits(hk_dtype_t dt, int logL, int E, KernelLimits *k) {
  return is_double(dt) ? limits_r2c_f64(logL, E, k) : limits_r2c_f32(logL, E, k);
}

// Pass-B row pairs of multipass real-input transforms: as many elements per
// lane as the resident real-input rows.
static bool r2cp_limits(hk_dtype_t dt, int logL, int E, KernelLimits *k) {
  return is_double(dt) ? limits_r2cp_f64(logL, E, k) : limits_r2cp_f32(logL, E, k);
}

bool layout_row_limits(hk_dtype_t dt, const Layout &lay, int E, KernelLimits *k) {
  if (lay.r2c) return lay.resident ? r2c_limits(dt, lay.logR, E, k) : r2cp_limits(dt, lay.logR, E, k);
  return row_limits(dt, lay.odd, lay.logR, E, k);
}

// Longest row (log2) the row kernels of odd factor `odd` handle in this
// precision and program (-1: none).
static int odd_max_logl(hk_dtype_t dt, int odd, int prog) {
  if (prog == PROG_BWD && !(is_double(dt) ? odd_bwd_ok_f64(odd) : odd_bwd_ok_f32(odd))) return -1;
  KernelLimits k;
  int best = -1;
  for (int l = 0; l <= MAX_LOGL; ++l)
    if (row_limits(dt, odd, l, odd_row_e(dt), &k)) best = l;
  return best;
}

// Split of a power-of-two sequence of length 2^logM into rows of 2^logR and
// columns of 2^logC: logR = ceil(logM / 2) + split, clamped so that rows are
// at most 2^maxR and columns at most 2^MAX_LOGL.
static bool split_of(int logM, int split, int maxR, int *logR, int *logC) {
  int r = (logM + 1) / 2 + split;
  r = std::max<int>(logM - MAX_LOGL, std::min<int>(maxR, r));
  if (r < 0 || r > maxR || logM - r > MAX_LOGL || logM - r < 0) return false;
  *logR = r;
  *logC = logM - r;
  return true;
}

// Process-wide transform-length policy (hk_set_fft_lengths).  Odd-factor
// lengths save bytes but give each lane group `odd` sequences in turn: they
// pay off where there is enough work to fill the device (measured: single
// products gain from N ~ 2^18 on, batches of many small ones do), and cost
// latency below.  HK_LENGTHS_AUTO therefore takes them when batch * (the
// power-of-two length) >= 2^18; real inputs take their half-length transform
// under every policy but HK_LENGTHS_POW2.  The three-pass factor-5 rows hold
// five sequences per lane group: under HK_LENGTHS_AUTO they are taken where
// batch * N >= 2^22 (measured on strided batches: from there on 8-20 %
// faster than the next length, below it 4-46 % slower), and in grouped plans
// not at all (F5_RESIDENT).
static std::atomic<int> g_length_policy{HK_LENGTHS_AUTO};
void set_length_policy(int policy) { g_length_policy.store(policy); }
int length_policy() { return g_length_policy.load(); }
constexpr int64_t kOddWorkMin = (int64_t)1 << 18;
constexpr int64_t kFiveWorkMin = (int64_t)1 << 22;

Status layout_for(const Problem &p, int split, Layout *out, bool allow_odd, int64_t batch, int five) {
  const int policy = g_length_policy.load();
  const bool allow_r2c = allow_odd && policy != HK_LENGTHS_POW2;
  if (policy == HK_LENGTHS_POW2) allow_odd = false;
  if (allow_odd && policy == HK_LENGTHS_AUTO) {
    int64_t dh = 1 - p.m, dc = 1 - p.m;
    for (int q = 0; q < p.m; ++q) {
      dh += p.dims[q];
      dc += p.bdims[q];
    }
    int64_t n2 = (int64_t)1 << std::max(0, ceil_log2(dh));
    if (p.is_block) n2 <<= std::max(0, ceil_log2(dc));
    if (std::max<int64_t>(1, batch) * n2 < kOddWorkMin) allow_odd = false;
  }
  Layout lay;
  if (!p.is_block) {
    int64_t dh = 1 - p.m;
    for (int q = 0; q < p.m; ++q) dh += p.dims[q];
    if (ceil_log2(dh) > HK_MAX_FFT_LOG2) return fail(HK_ERR_SIZE_LIMIT, "padded length exceeds 2^24");
    // Real forward products: a length-N real transform (N = 2^k >= max(d_H, 2))
    // as a length-N/2 complex one, in one workgroup or in three passes whose
    // row pass takes mirrored row pairs.
    if (allow_r2c && p.prog == PROG_FWD && !is_complex(p.dt)) {
      const int logN = std::max(1, ceil_log2(dh));
      KernelLimits k;
      if (r2c_limits(p.dt, logN - 1, r2c_row_e(p.dt), &k)) {
        lay.r2c = true;
        lay.resident = true;
        lay.logR = logN - 1;
        lay.logC = 0;
        *out = lay;
        return Status();
      }
      int maxR = -1;
      for (int l = 0; l <= MAX_LOGL; ++l)
        if (r2cp_limits(p.dt, l, r2c_row_e(p.dt), &k)) maxR = l;
      Layout c;
      if (maxR >= 0 && split_of(logN - 1, split, maxR, &c.logR, &c.logC) && c.logC >= 1) {
        c.r2c = true;
        c.resident = false;
        *out = c;
        return Status();
      }
    }
    // The smallest N = odd * 2^logM >= d_H among the lengths with kernels.
    int64_t bestN = -1;
    for (int odd : {1, 3, 5}) {
      if (odd == 5 && five == F5_NONE) continue;
      const int omax = odd == 1 ? MAX_LOGL : (allow_odd ? odd_max_logl(p.dt, odd, p.prog) : -1);
      if (omax < 0) continue;
      int logM = 0;
      while (((int64_t)odd << logM) < dh) ++logM;
      const int64_t N = (int64_t)odd << logM;
      if (N > ((int64_t)1 << HK_MAX_FFT_LOG2)) continue;
      if (bestN >= 0 && N >= bestN) continue;
      Layout c;
      c.odd = odd;
      const int res_max = odd == 1 ? RES_MAX_LOG : omax;
      if (logM <= res_max) {
        c.resident = true;
        c.logR = logM;
        c.logC = 0;
      } else if (odd == 5 && policy == HK_LENGTHS_AUTO &&
                 (five != F5_AUTO || std::max<int64_t>(1, batch) * N < kFiveWorkMin)) {
        // three-pass factor-5 rows (five sequences per lane group) pay only
        // with enough work; in grouped plans they measured slower
        continue;
      } else if (!split_of(logM, split, omax, &c.logR, &c.logC)) {
        continue;
      }
      lay = c;
      bestN = N;
    }
    if (bestN < 0) return fail(HK_ERR_SIZE_LIMIT, "no transform length with kernels for this d_H");
  } else {
    int64_t rows = 1 - p.m, cols = 1 - p.m;
    for (int q = 0; q < p.m; ++q) {
      rows += p.dims[q];
      cols += p.bdims[q];
    }
    lay.logR = ceil_log2(rows);
    lay.logC = ceil_log2(cols);
    if (lay.logR > MAX_LOGL || lay.logC > MAX_LOGL)
      return fail(HK_ERR_SIZE_LIMIT, "padded BHHB grid exceeds 4096 along an axis");
    lay.resident = false;
    if (allow_odd && is_complex(p.dt)) {
      // Each axis is the shortest of 2^k, 3 * 2^k and 5 * 2^k with kernels.
      // The passes' bytes scale with the column axis only (pass A writes,
      // pass B reads and writes, pass D reads columns of that length; the row
      // pass loads and stores only a row's nonzero and kept entries); the row
      // axis sets the row transforms' arithmetic.  An odd column factor needs
      // column kernels of 2^6 .. 2^11 points per sequence; it combines with
      // either kind of row.  (Measured on the 64-tensor batch with 512 blocks
      // of 512: rows of 3 * 512 took 30.1 us per tensor, power-of-two rows of
      // 2048 over the same columns 34.4 us, so the row axis is not lengthened
      // to a power of two either.)
      auto axis = [&](int64_t ext, int odd, int *logp) {
        int l = 0;
        while (((int64_t)odd << l) < ext) ++l;
        *logp = l;
        return (int64_t)odd << l;
      };
      int64_t nc_best = (int64_t)1 << lay.logC;
      for (int ocol : {3, 5}) {
        int lc = 0;
        const int64_t nc = axis(cols, ocol, &lc);
        if (lc < 6 || lc > 11) continue;
        if (nc < nc_best) {
          nc_best = nc;
          lay.odd_c = ocol;
          lay.logC = lc;
        }
      }
      const int64_t nr_pow2 = (int64_t)1 << lay.logR;
      int64_t nr_odd = -1;
      int orow_best = 1, lr_best = lay.logR;
      for (int orow : {3, 5}) {
        int lr = 0;
        const int64_t nr = axis(rows, orow, &lr);
        if (lr > odd_max_logl(p.dt, orow, p.prog)) continue;
        // factor-5 rows: with enough work only, as in 1D (measured on strided
        // batches: from batch * grid >= 2^22 on 2-24 % faster, below 5-15 % slower)
        if (orow == 5 && policy == HK_LENGTHS_AUTO &&
            (five != F5_AUTO || std::max<int64_t>(1, batch) * nr * nc_best < kFiveWorkMin))
          continue;
        if (nr_odd < 0 || nr < nr_odd) {
          nr_odd = nr;
          orow_best = orow;
          lr_best = lr;
        }
      }
      if (nr_odd > 0 && nr_odd < nr_pow2) {
        lay.odd = orow_best;
        lay.logR = lr_best;
      }
    }
  }
  *out = lay;
  return Status();
}

// ---------------------------------------------------------------------------
// Shape
// ---------------------------------------------------------------------------
Status build_shape(const Problem &p, const Layout &lay, const Sched &sc, Shape *shp, Ptrs *ptrs,
                   int op_src[MAXOPS]) {
  Shape sh;
  memset(&sh, 0, sizeof(sh));
  Ptrs P;
  memset(&P, 0, sizeof(P));
  sh.prog = p.prog;
  sh.is_block = p.is_block ? 1 : 0;
  sh.m = p.m;
  sh.logR = lay.logR;
  sh.logC = lay.logC;
  sh.resident = lay.resident ? 1 : 0;
  sh.r2c = lay.r2c ? 1 : 0;
  sh.odd = lay.odd;
  sh.odd_inv = 0;
  // the Chinese-remainder maps need the power-of-two part's inverse modulo
  // the odd factor: M = R C in 1D, R (rows) and C (columns) for BHHB
  auto inv_mod = [](int64_t pow2, int odd) {
    const int r = (int)(pow2 % odd);
    for (int v = 1; v < odd; ++v)
      if ((r * v) % odd == 1) return v;
    return 0;
  };
  if (lay.odd > 1) sh.odd_inv = inv_mod((int64_t)1 << (p.is_block ? lay.logR : lay.logR + lay.logC), lay.odd);
  sh.odd_c = lay.odd_c;
  sh.odd_c_inv = lay.odd_c > 1 ? inv_mod((int64_t)1 << lay.logC, lay.odd_c) : 0;
  sh.real_out = is_complex(p.dt) ? 0 : 1;
  const int real_flag = is_complex(p.dt) ? 0 : OPF_REAL;
  const int64_t R = (int64_t)1 << lay.logR;
  int64_t hrows = 1 - p.m, hcols = 1 - p.m;
  for (int q = 0; q < p.m; ++q) {
    hrows += p.dims[q];
    hcols += p.bdims[q];
  }
  auto add_op = [&](int role, int exp, int flags, int64_t len, int64_t cols, const void *ptr, int src) {
    OpDesc &od = sh.ops[sh.nops];
    od.role = role;
    od.exp = exp;
    od.flags = flags;
    od.len = len;
    od.cols = cols;
    od.buf = sh.nops;
    // storage columns that may be nonzero (real inputs: pairs of entries;
    // BHHB grids with an odd row factor: rows of the natural-order workspace)
    const int64_t rw = (p.is_block && lay.odd > 1) ? (int64_t)lay.odd * R : R;
    od.ncol_nz = std::min<int64_t>(rw, lay.r2c ? (len + 1) / 2 : len);
    P.op[sh.nops] = ptr;
    if (op_src) op_src[sh.nops] = src;
    ++sh.nops;
  };
  if (p.prog == PROG_FWD && p.conv) {
    // conj(x_1 * ... * x_m) on the generating grid: every vector an operand
    // (identical ones merged into powers), no generating vector, no scalar
    sh.want_y = 1;
    sh.fwd_flags = SHF_CONV;
    struct G {
      const void *ptr;
      int64_t n, nb;
      int exp, src;
    };
    std::vector<G> groups;
    for (int q = 0; q < p.m; ++q) {
      bool found = false;
      for (auto &g : groups)
        if (g.ptr == p.vec[q] && g.n == p.dims[q] && g.nb == (p.is_block ? p.bdims[q] : 1)) {
          g.exp++;
          found = true;
          break;
        }
      if (!found) groups.push_back({p.vec[q], p.dims[q], p.is_block ? p.bdims[q] : 1, 1, q});
    }
    for (const G &g : groups) add_op(ROLE_X, g.exp, 0, g.n, g.nb, g.ptr, g.src);
    sh.out_rows = hrows;
    sh.out_cols = p.is_block ? hcols : 1;
    P.y = p.y;
  } else if (p.prog == PROG_FWD) {
    sh.want_y = p.y ? 1 : 0;
    sh.want_alpha = p.alpha ? 1 : 0;
    sh.fwd_flags = p.conj_y ? SHF_CONJ_Y : 0;
    add_op(ROLE_H, 1, p.h_spec ? OPF_SPEC : (OPF_CONJ | real_flag), p.is_block ? hrows : hrows,
           p.is_block ? hcols : 1, p.h, -1);
    // Group identical vectors of modes 2..m (same pointer, shape and kind).
    struct G {
      const void *ptr;
      int64_t n, nb;
      int exp;
      int src;
      bool spec;
    };
    auto is_spec = [&](int q) { return ((p.spec_mask >> q) & 1u) != 0; };
    std::vector<G> groups;
    for (int q = 1; q < p.m; ++q) {
      bool found = false;
      for (auto &g : groups)
        if (g.ptr == p.vec[q] && g.n == p.dims[q] && g.nb == (p.is_block ? p.bdims[q] : 1) && g.spec == is_spec(q)) {
          g.exp++;
          found = true;
          break;
        }
      if (!found) groups.push_back({p.vec[q], p.dims[q], p.is_block ? p.bdims[q] : 1, 1, q, is_spec(q)});
    }
    int alpha_group = -1;
    if (p.alpha) {
      for (size_t i = 0; i < groups.size(); ++i)
        if (groups[i].ptr == p.vec[0] && groups[i].n == p.dims[0] &&
            groups[i].nb == (p.is_block ? p.bdims[0] : 1) && groups[i].spec == is_spec(0))
          alpha_group = (int)i;
      if (alpha_group < 0) {
        groups.push_back({p.vec[0], p.dims[0], p.is_block ? p.bdims[0] : 1, 0, 0, is_spec(0)});
        alpha_group = (int)groups.size() - 1;
      }
      std::swap(groups[alpha_group], groups.back());  // scalar operand is processed last
      alpha_group = (int)groups.size() - 1;
    }
    for (size_t i = 0; i < groups.size(); ++i) {
      // a stored spectrum is complex whatever the dtype
      const int flags = (groups[i].spec ? OPF_SPEC : real_flag) | ((int)i == alpha_group ? OPF_ALPHA : 0);
      add_op(ROLE_X, groups[i].exp, flags, groups[i].n, groups[i].nb, groups[i].ptr, groups[i].src);
    }
    sh.out_rows = p.dims[0];
    sh.out_cols = p.is_block ? p.bdims[0] : 1;
    P.y = p.y;
    P.alpha = p.alpha;
  } else {
    // Adjoint of the equal-vector products: X, [V], [H].
    const int64_t n = p.dims[0];
    sh.want_y = p.gh ? 1 : 0;
    sh.want_out1 = p.gx ? 1 : 0;
    // x may be given by its stored spectrum (spec_mask bit 1)
    add_op(ROLE_X, 0, (p.spec_mask & 2u) ? OPF_SPEC : 0, n, 1, p.vec[1], 1);
    if (p.v) add_op(ROLE_V, 0, OPF_CONJ, n, 1, p.v, -2);
    if (p.gx) add_op(ROLE_H, 1, OPF_CONJ, hrows, 1, p.h, -1);
    sh.out_rows = hrows;  // grad_h length d_H
    sh.out_cols = 1;
    sh.out1_len = n;      // grad_x length
    P.y = p.gh;
    P.out1 = p.gx;
    P.phi = p.phi;
  }
  if (!lay.resident) {
    // The workspace size does not depend on the schedule: partial sums are
    // reserved for the largest possible number of row-pass workgroups.
    sh.rows_per_wg = sc.rows_per_wg;
    sh.row_iters = sc.iters;
    sh.nbuf = sh.nops;
    // (adjoint shapes keep one buffer per operand: grad_h and grad_x leave the
    // row pass in the buffers of operands 0 and 1)
    if (p.prog == PROG_FWD && (p.h_spec || p.spec_mask)) {
      // Spectrum operands need no buffer: the others take buffers 0, 1, ...;
      // the output row goes to buffer 0 (operand 0's), in place of a row the
      // row pass has already read, or to a buffer of its own.
      int nb = 0;
      for (int o = 0; o < sh.nops; ++o)
        if (!(sh.ops[o].flags & OPF_SPEC)) sh.ops[o].buf = nb++;
      for (int o = 0; o < sh.nops; ++o)
        if (sh.ops[o].flags & OPF_SPEC) sh.ops[o].buf = 0;
      sh.nbuf = std::max(1, nb);
    }
    sh.partials = (int64_t)1 << MAX_LOGL;
    const size_t eb = cplx_bytes(p.dt);
    const size_t bytes =
        (size_t)sh.nbuf * ((size_t)lay.odd * lay.odd_c << (lay.logR + lay.logC)) * eb + (size_t)sh.partials * eb;
    sh.ws_bytes = (int64_t)((bytes + 255) & ~(size_t)255);
  }
  *shp = sh;
  *ptrs = P;
  return Status();
}

size_t instance_ws_bytes(const Shape &sh, hk_dtype_t) { return sh.resident ? 0 : (size_t)sh.ws_bytes; }

// Bytes the passes of one instance read and write as built: pass A reads each
// operand and writes the storage columns that can be nonzero; pass B reads
// those columns and writes the output columns the last pass reads; pass D
// reads them back and writes the slice.  Resident instances move their
// inputs and outputs once.
int64_t pass_model_bytes(const Shape &sh, hk_dtype_t dt) {
  const int64_t s = (int64_t)cplx_bytes(dt);
  const int64_t es_out = sh.real_out ? s / 2 : s;
  int64_t in = 0;
  for (int o = 0; o < sh.nops; ++o) {
    const OpDesc &od = sh.ops[o];
    if (!(od.flags & OPF_SPEC)) in += od.len * od.cols * ((od.flags & OPF_REAL) ? s / 2 : s);
  }
  int64_t out = 0;
  if (sh.want_y) out += sh.out_rows * sh.out_cols * es_out;
  if (sh.want_alpha) out += es_out;
  if (sh.prog == PROG_BWD && sh.want_out1) out += sh.out1_len * es_out;
  if (sh.resident) return in + out;
  const int64_t C = (int64_t)1 << sh.logC;
  // columns of one workspace row and rows per column: 1D, `odd` sequences of
  // R x C; BHHB, natural rows of odd R over odd_c C
  const bool nat = sh.is_block;
  const int64_t R = (int64_t)(nat ? sh.odd : 1) << sh.logR;
  const int64_t seq = (nat ? (int64_t)(sh.odd_c > 1 ? sh.odd_c : 1) : (int64_t)sh.odd) * C;
  int64_t a_write = 0, b_read = 0;
  for (int o = 0; o < sh.nops; ++o) {
    const OpDesc &od = sh.ops[o];
    if (od.flags & OPF_SPEC) {
      b_read += R * seq * s;
    } else {
      a_write += od.ncol_nz * seq * s;
      b_read += od.ncol_nz * seq * s;
    }
  }
  int64_t b_write = 0;
  if (sh.want_y) b_write += std::min<int64_t>(R, sh.r2c ? (sh.out_rows + 1) / 2 : sh.out_rows) * seq * s;
  if (sh.prog == PROG_BWD && sh.want_out1) b_write += std::min<int64_t>(R, sh.out1_len) * seq * s;
  return (in + a_write) + (b_read + b_write) + (b_write + out);
}

// ---------------------------------------------------------------------------
// Schedules
// ---------------------------------------------------------------------------
static bool lim(hk_dtype_t dt, int logL, int E, KernelLimits *k) {
  return is_double(dt) ? limits_f64(logL, E, k) : limits_f32(logL, E, k);
}

bool sched_valid(hk_dtype_t dt, const Layout &lay, const Sched &sc) {
  KernelLimits kr, kc;
  if (!layout_row_limits(dt, lay, sc.E_row, &kr)) return false;
  if (sc.rows_per_wg < 1 || sc.rows_per_wg * kr.tps > kr.row_maxt) return false;
  const size_t row_lds = std::max((size_t)sc.rows_per_wg * kr.seq_lds, (size_t)sc.rows_per_wg * kr.tps) * kr.elem_bytes;
  if (row_lds > 160 * 1024) return false;
  if (sc.iters != 1 && (lay.resident || lay.r2c || (sc.iters != 2 && sc.iters != 4))) return false;
  if (!lay.resident) {
    if (sc.E_col != 8 && sc.E_col != 16) return false;  // the column kernels built
    if (!lim(dt, lay.logC, sc.E_col, &kc)) return false;
    // column tiles interleave TW columns in the LDS by log2(TW): powers of two only
    if (sc.tw < 1 || (sc.tw & (sc.tw - 1)) != 0 || sc.tw * kc.tps > COL_MAXT) return false;
    if ((size_t)sc.tw * kc.lds_raw * kc.elem_bytes > 160 * 1024) return false;
  }
  return true;
}

Sched default_sched(hk_dtype_t dt, const Layout &lay, int prog, int64_t batch) {
  Sched sc;
  const bool dbl = is_double(dt);
  sc.E_row = lay.r2c ? r2c_row_e(dt) : (lay.odd > 1 ? odd_row_e(dt) : 8);
  sc.E_col = (dbl || lay.odd_c > 1) ? 8 : 16;
  KernelLimits kr, kc;
  layout_row_limits(dt, lay, sc.E_row, &kr);
  if (lay.odd == 1 && !lay.r2c && kr.tps > ROW_MAXT) {  // 4096-point rows need 16 elements per lane
    sc.E_row = 16;
    lim(dt, lay.logR, sc.E_row, &kr);
  }
  if (lay.resident) {
    // One instance per row; pack rows up to 256 lanes when batched.
    const int max_rows = std::max(1, std::min((int)ROW_MAXT, kr.row_maxt) / kr.tps);
    sc.rows_per_wg = (int)std::max<int64_t>(1, std::min<int64_t>(max_rows, batch));
  } else {
    sc.rows_per_wg = std::max(1, std::min(std::min((int)ROW_MAXT, kr.row_maxt) / kr.tps, 1 << lay.logC));
    lim(dt, lay.logC, sc.E_col, &kc);
    const int want_tw = dbl ? 8 : 16;  // 128-byte row segments
    int tw = std::max(1, std::min(want_tw, COL_MAXT / kc.tps));
    while (tw > 1 && (size_t)tw * kc.lds_raw * kc.elem_bytes > 144 * 1024) tw >>= 1;
    sc.tw = tw;
  }
  (void)prog;
  return sc;
}

// ---------------------------------------------------------------------------
// Launch sequences
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Kernel timing with HIP events (diagnostics)
// ---------------------------------------------------------------------------
struct ProfState {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  std::vector<int> kinds;
  size_t used = 0;
  bool armed = false;  // prof_before handed out pool[used] for the next launch
};
static ProfState g_prof;
static std::mutex g_prof_mu;

bool prof_enabled() { return g_prof.on; }

void prof_before(hipStream_t) {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (g_prof.used == g_prof.pool.size()) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
    g_prof.pool.push_back({a, b});
    g_prof.kinds.push_back(-1);
  }
  g_prof.armed = true;
}

void prof_after(int kind, hipStream_t) {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (g_prof.used >= g_prof.pool.size()) return;
  if (g_prof.armed) return;  // the launch did not take the events (failed)
  g_prof.kinds[g_prof.used] = kind;
  ++g_prof.used;
}

hipError_t launch_kernel(const void *fn, dim3 grid, dim3 block, void **args, size_t lds, hipStream_t st) {
  hipEvent_t a = nullptr, b = nullptr;
  if (g_prof.on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (g_prof.armed && g_prof.used < g_prof.pool.size()) {
      a = g_prof.pool[g_prof.used].first;
      b = g_prof.pool[g_prof.used].second;
      g_prof.armed = false;
    }
  }
  if (a) return hipExtLaunchKernel(fn, grid, block, args, lds, st, a, b, 0);
  return hipLaunchKernel(fn, grid, block, args, lds, st);
}

// The persistent kernel's grid-wide barriers need every workgroup resident at
// once: a cooperative launch makes the runtime check that (and fail instead of
// starting a grid that cannot be co-resident).  Launches recorded into a
// graph, and launches timed by the profiling events, are plain launches of
// the same occupancy-sized grid.
hipError_t launch_cooperative(const void *fn, dim3 grid, dim3 block, void **args, size_t lds, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return e;
  bool timed = false;
  if (g_prof.on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    timed = g_prof.armed && g_prof.used < g_prof.pool.size();
  }
  if (cs != hipStreamCaptureStatusNone || timed) return launch_kernel(fn, grid, block, args, lds, st);
  return hipLaunchCooperativeKernel(fn, grid, block, args, (unsigned int)lds, st);
}

Status prof_start() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.on = true;
  g_prof.used = 0;
  g_prof.armed = false;
  return Status();
}

Status prof_stop(double *ms, int64_t *counts) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.on = false;
  for (int k = 0; k < PK_COUNT; ++k) {
    ms[k] = 0;
    counts[k] = 0;
  }
  for (size_t i = 0; i < g_prof.used; ++i) {
    hipError_t e = hipEventSynchronize(g_prof.pool[i].second);
    if (e != hipSuccess) return fail(HK_ERR_HIP, std::string("profile event: ") + hipGetErrorString(e));
    float t = 0;
    e = hipEventElapsedTime(&t, g_prof.pool[i].first, g_prof.pool[i].second);
    if (e != hipSuccess) return fail(HK_ERR_HIP, std::string("profile elapsed: ") + hipGetErrorString(e));
    const int k = g_prof.kinds[i];
    if (k >= 0 && k < PK_COUNT) {
      ms[k] += t;
      counts[k] += 1;
    }
  }
  g_prof.used = 0;
  return Status();
}

static hipError_t rows(hk_dtype_t dt, int logL, int E, int rpw, dim3 g, const Shape &sh, const Ptrs &p0,
                       const Strides &str, int64_t cnt, hipStream_t st) {
  count_launch();
  prof_before(st);
  hipError_t e;
  if (sh.r2c && sh.resident)
    e = is_double(dt) ? launch_rows_r2c_f64(logL, E, rpw, g, sh, p0, str, cnt, st)
                      : launch_rows_r2c_f32(logL, E, rpw, g, sh, p0, str, cnt, st);
  else if (sh.r2c)
    e = is_double(dt) ? launch_rows_r2cp_f64(logL, E, rpw, g, sh, p0, str, cnt, st)
                      : launch_rows_r2cp_f32(logL, E, rpw, g, sh, p0, str, cnt, st);
  else if (sh.odd > 1)
    e = is_double(dt) ? launch_rows_odd_f64(sh.odd, logL, E, rpw, g, sh, p0, str, cnt, st)
                      : launch_rows_odd_f32(sh.odd, logL, E, rpw, g, sh, p0, str, cnt, st);
  else
    e = is_double(dt) ? launch_rows_f64(logL, E, rpw, g, sh, p0, str, cnt, st)
                      : launch_rows_f32(logL, E, rpw, g, sh, p0, str, cnt, st);
  prof_after(sh.resident ? PK_RESIDENT : PK_PASS_B, st);
  return e;
}
static hipError_t cols(hk_dtype_t dt, int logL, int E, int tw, int xcd, dim3 g, const Shape &sh, const Ptrs &p0,
                       const Strides &str, const ColJob *jobs, int nj, hipStream_t st) {
  count_launch();
  prof_before(st);
  const hipError_t e = is_double(dt) ? launch_cols_f64(logL, E, tw, xcd, g, sh, p0, str, jobs, nj, st)
                                     : launch_cols_f32(logL, E, tw, xcd, g, sh, p0, str, jobs, nj, st);
  prof_after(jobs[0].kind == COL_A ? PK_PASS_A : PK_PASS_D, st);
  return e;
}

static Status hip_fail(hipError_t e, const char *what) {
  return fail(HK_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

Status launch_shape(hk_dtype_t dt, const Shape &sh, const Sched &sc, const Ptrs &p0, const Strides &str,
                    int64_t count, hipStream_t st) {
  if (count < 1) return Status();
  if (count > 65535 && !sh.resident) return fail(HK_ERR_SIZE_LIMIT, "batch too large for one launch");
  hipError_t e;
  if (sh.resident) {
    const int64_t blocks = (count + sc.rows_per_wg - 1) / sc.rows_per_wg;
    if (blocks > 0x7fffffff) return fail(HK_ERR_SIZE_LIMIT, "batch too large");
    e = rows(dt, sh.logR, sc.E_row, sc.rows_per_wg, dim3((unsigned)blocks), sh, p0, str, count, st);
    if (e != hipSuccess) return hip_fail(e, "resident launch");
    return Status();
  }
  const int64_t R = (int64_t)1 << sh.logR;
  const int64_t C = (int64_t)1 << sh.logC;
  // Pass A: column transforms of every operand not given as a spectrum.
  ColJob ja[MAXOPS];
  memset(ja, 0, sizeof(ja));
  int64_t max_cols = 0;
  int na = 0;
  for (int o = 0; o < sh.nops; ++o) {
    if (sh.ops[o].flags & OPF_SPEC) continue;
    ja[na].kind = COL_A;
    ja[na].op = o;
    ja[na].buf = sh.ops[o].buf;
    ja[na].conj_out = 0;
    ja[na].ncols = sh.ops[o].ncol_nz;
    max_cols = std::max(max_cols, ja[na].ncols);
    ++na;
  }
  // BHHB grids with an odd row factor: the column passes tile the natural rows
  const bool nat = sh.is_block && sh.odd > 1;
  if (na > 0) {
    // tiles over the storage columns of every sequence (virtual columns)
    const int64_t vcols_a = (sh.odd > 1 && !nat) ? sh.odd * R : max_cols;
    dim3 ga((unsigned)((vcols_a + sc.tw - 1) / sc.tw), (unsigned)na, (unsigned)count);
    e = cols(dt, sh.logC, sc.E_col, sc.tw, sc.xcd, ga, sh, p0, str, ja, na, st);
    if (e != hipSuccess) return hip_fail(e, "pass A launch");
  }
  // Pass B: row transforms, spectral product, row transform of the output
  // (real inputs: C / 2 mirrored row pairs).
  const int64_t rows_wg = (int64_t)sc.rows_per_wg * sc.iters;  // rows (pairs) per workgroup
  const int64_t brows = sh.r2c ? C / 2 : C * (sh.odd_c > 1 ? sh.odd_c : 1);
  dim3 gb((unsigned)((brows + rows_wg - 1) / rows_wg), (unsigned)count);
  e = rows(dt, sh.logR, sc.E_row, sc.rows_per_wg, gb, sh, p0, str, count, st);
  if (e != hipSuccess) return hip_fail(e, "pass B launch");
  // Pass D: column transforms of the outputs and the slice; its first
  // workgroup also sums pass B's scalar partials.
  const int64_t npart = (sh.prog == PROG_FWD && sh.want_alpha) ? (brows + rows_wg - 1) / rows_wg : 0;
  ColJob jd[2];
  memset(jd, 0, sizeof(jd));
  int nd = 0;
  int64_t dcols = 0;
  if (sh.want_y) {
    jd[nd].kind = COL_D;
    jd[nd].op = 0;
    jd[nd].buf = sh.ops[0].buf;
    jd[nd].conj_out = (sh.prog == PROG_FWD && (sh.fwd_flags & SHF_CONJ_Y)) ? 1 : 0;
    jd[nd].npart = npart;
    // real outputs of real-input transforms are stored in pairs
    jd[nd].ncols = std::min<int64_t>(nat ? sh.odd * R : R, sh.r2c ? (sh.out_rows + 1) / 2 : sh.out_rows);
    dcols = std::max(dcols, jd[nd].ncols);
    ++nd;
  }
  if (sh.prog == PROG_BWD && sh.want_out1) {
    jd[nd].kind = COL_D;
    jd[nd].op = 1;
    jd[nd].buf = sh.ops[1].buf;
    jd[nd].conj_out = 1;
    jd[nd].ncols = std::min<int64_t>(R, sh.out1_len);
    dcols = std::max(dcols, jd[nd].ncols);
    ++nd;
  }
  if (nd > 0) {
    const int64_t vcols_d = (sh.odd > 1 && !nat) ? sh.odd * R : dcols;
    dim3 gd((unsigned)((vcols_d + sc.tw - 1) / sc.tw), (unsigned)nd, (unsigned)count);
    e = cols(dt, sh.logC, sc.E_col, sc.tw, sc.xcd, gd, sh, p0, str, jd, nd, st);
    if (e != hipSuccess) return hip_fail(e, "pass D launch");
  } else if (npart > 0) {
    count_launch();
    prof_before(st);
    e = is_double(dt) ? launch_alpha_f64(sh, p0, str, npart, count, st) : launch_alpha_f32(sh, p0, str, npart, count, st);
    prof_after(PK_PASS_D, st);
    if (e != hipSuccess) return hip_fail(e, "scalar reduction launch");
  }
  return Status();
}

// ---------------------------------------------------------------------------
// Device setup
// ---------------------------------------------------------------------------
static void twiddle_tables(std::vector<double> &t4096, std::vector<double> &t24) {
  t4096.resize(8192);
  t24.resize(8192);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int j = 0; j < 4096; ++j) {
    const long double a = two_pi * ((long double)j / 4096.0L);
    t4096[2 * j] = (double)cosl(a);
    t4096[2 * j + 1] = (double)-sinl(a);
    const long double b = two_pi * ((long double)j / 16777216.0L);
    t24[2 * j] = (double)cosl(b);
    t24[2 * j + 1] = (double)-sinl(b);
  }
  // Exact values at the quarter points.
  t4096[0] = 1.0;
  t4096[1] = 0.0;
  t4096[2 * 1024] = 0.0;
  t4096[2 * 1024 + 1] = -1.0;
  t4096[2 * 2048] = -1.0;
  t4096[2 * 2048 + 1] = 0.0;
  t4096[2 * 3072] = 0.0;
  t4096[2 * 3072 + 1] = 1.0;
  t24[0] = 1.0;
  t24[1] = 0.0;
}

Status ensure_device() {
  static std::mutex mu;
  static std::map<int, int> state;  // device -> 1 ok, -1 not gfx950
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(mu);
  auto it = state.find(dev);
  if (it != state.end()) {
    if (it->second == 1) return Status();
    return fail(HK_ERR_DEVICE, "current device is not gfx950");
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    state[dev] = -1;
    return fail(HK_ERR_DEVICE, std::string("current device is ") + prop.gcnArchName + ", not gfx950");
  }
  std::vector<double> a, b;
  twiddle_tables(a, b);
  e = init_tables_f32(a.data(), b.data());
  if (e == hipSuccess) e = init_tables_f64(a.data(), b.data());
  if (e == hipSuccess) e = init_tables_odd_f32(a.data(), b.data());
  if (e == hipSuccess) e = init_tables_odd_f64(a.data(), b.data());
  if (e != hipSuccess) return hip_fail(e, "twiddle table upload");
  state[dev] = 1;
  return Status();
}

// ---------------------------------------------------------------------------
// Schedule cache
// ---------------------------------------------------------------------------
using SchedKey = std::tuple<int, int, int, int, int, int, int>;
static std::mutex g_sched_mu;
static std::map<SchedKey, Sched> g_sched;

static int batch_class(int64_t b) { return b <= 1 ? 0 : (b < 16 ? 1 : 2); }

bool sched_lookup(hk_dtype_t dt, int prog, int is_block, int odd, int logM, int logC_hint, int64_t batch,
                  Sched *sc) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  auto it = g_sched.find(SchedKey((int)dt, prog, is_block, odd, logM, logC_hint, batch_class(batch)));
  if (it == g_sched.end()) return false;
  *sc = it->second;
  return true;
}

void sched_store(hk_dtype_t dt, int prog, int is_block, int odd, int logM, int logC_hint, int64_t batch,
                 const Sched &sc) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  g_sched[SchedKey((int)dt, prog, is_block, odd, logM, logC_hint, batch_class(batch))] = sc;
}

// Text database, one schedule per line:
//   dtype prog is_block lclass logM logC_hint batch_class : E_row rows_per_wg E_col tw split xcd iters
// (lclass = the odd factor 1, 3 or 5 of the transform length, or 2 for real
// inputs transformed at half length; logM = log2 of its power-of-two part;
// xcd and iters may be omitted: 0 and 1).  Lines with six key fields (no odd factor)
// are read as odd = 1.  '#' starts a comment line.
static const char *kDbHeader =
    "# hankel schedule database v4: dt prog blk odd logM logC bclass : E_row rows E_col tw split xcd iters\n";

Status sched_save(const char *path) {
  if (!path) return fail(HK_ERR_NULL_POINTER, "path is NULL");
  std::lock_guard<std::mutex> lk(g_sched_mu);
  FILE *f = fopen(path, "w");
  if (!f) return fail(HK_ERR_INVALID_VALUE, std::string("cannot open ") + path + " for writing");
  fputs(kDbHeader, f);
  for (const auto &kv : g_sched) {
    const SchedKey &k = kv.first;
    const Sched &s = kv.second;
    fprintf(f, "%d %d %d %d %d %d %d : %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
            std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), s.E_row, s.rows_per_wg, s.E_col, s.tw,
            s.split, s.xcd, s.iters);
  }
  const bool ok = fclose(f) == 0;
  return ok ? Status() : fail(HK_ERR_INVALID_VALUE, std::string("error writing ") + path);
}

// Length classes of the schedule key (Layout::lclass): 1, 2 (real), 3, 5,
// and for BHHB grids the row factor plus 16 times an odd column factor.
static bool lclass_ok(int c) {
  const int base = c % 16, col = c / 16;
  return (base == 1 || base == 2 || base == 3 || base == 5) && (col == 0 || col == 3 || col == 5);
}

Status sched_load(const char *path, int *loaded) {
  if (!path) return fail(HK_ERR_NULL_POINTER, "path is NULL");
  FILE *f = fopen(path, "r");
  if (!f) return fail(HK_ERR_INVALID_VALUE, std::string("cannot open ") + path);
  std::map<SchedKey, Sched> add;
  char line[256];
  int lineno = 0;
  Status st;
  while (fgets(line, sizeof(line), f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    char *colon = strchr(line, ':');
    int k[7] = {0, 0, 0, 1, 0, 0, 0}, v[7] = {0, 0, 0, 0, 0, 0, 1};
    int nk = -1, nv = -1;
    if (colon) {
      *colon = 0;
      int t[8];
      nk = sscanf(line, "%d %d %d %d %d %d %d %d", &t[0], &t[1], &t[2], &t[3], &t[4], &t[5], &t[6], &t[7]);
      if (nk == 7) {
        for (int i = 0; i < 7; ++i) k[i] = t[i];
      } else if (nk == 6) {  // no odd factor: power-of-two length
        k[0] = t[0];
        k[1] = t[1];
        k[2] = t[2];
        k[3] = 1;
        k[4] = t[3];
        k[5] = t[4];
        k[6] = t[5];
      }
      int extra = 0;
      nv = sscanf(colon + 1, "%d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &extra);
    }
    if ((nk != 6 && nk != 7) || nv < 5 || nv > 7) {
      st = fail(HK_ERR_INVALID_VALUE, std::string(path) + ": malformed line " + std::to_string(lineno));
      break;
    }
    const bool key_ok = k[0] >= HK_C64 && k[0] <= HK_F64 && (k[1] == PROG_FWD || k[1] == PROG_BWD) &&
                        (k[2] == 0 || k[2] == 1) && lclass_ok(k[3]) && k[4] >= 0 &&
                        k[4] <= HK_MAX_FFT_LOG2 && k[5] >= -1 && k[5] <= HK_MAX_FFT_LOG2 && k[6] >= 0 && k[6] <= 2;
    Sched s;
    s.E_row = v[0];
    s.rows_per_wg = v[1];
    s.E_col = v[2];
    s.tw = v[3];
    s.split = v[4];
    s.xcd = v[5];
    s.iters = v[6];
    // entries are re-checked against the kernel limits when used (sched_valid)
    const bool val_ok = (s.E_row == 4 || s.E_row == 8 || s.E_row == 16) && (s.E_col == 8 || s.E_col == 16) &&
                        s.rows_per_wg >= 1 && s.rows_per_wg <= 64 && s.tw >= 1 && s.tw <= 64 &&
                        (s.tw & (s.tw - 1)) == 0 && s.split >= -4 &&
                        s.split <= 4 && (s.xcd == 0 || s.xcd == 1) && (s.iters == 1 || s.iters == 2 || s.iters == 4);
    if (!key_ok || !val_ok) {
      st = fail(HK_ERR_INVALID_VALUE, std::string(path) + ": value out of range on line " + std::to_string(lineno));
      break;
    }
    add[SchedKey(k[0], k[1], k[2], k[3], k[4], k[5], k[6])] = s;
  }
  fclose(f);
  if (!st.ok()) return st;
  std::lock_guard<std::mutex> lk(g_sched_mu);
  for (const auto &kv : add) g_sched[kv.first] = kv.second;
  if (loaded) *loaded = (int)add.size();
  return Status();
}

}  // namespace hk
