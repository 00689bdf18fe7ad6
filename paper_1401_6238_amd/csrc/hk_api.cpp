// C ABI of the fast Hankel tensor-vector product (see include/hankel.h).
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "hk_batch.hpp"
#include "hk_plan.hpp"

using namespace hk;

namespace hk {
int launches_and_reset();
}

static thread_local std::string tl_err;
static thread_local int tl_last_launches = 0;

static hk_status_t finish(const Status &s) {
  tl_last_launches = launches_and_reset();
  if (!s.ok()) tl_err = s.msg;
  return s.code;
}

namespace hk {
hk_status_t api_finish(const Status &s) { return finish(s); }
}  // namespace hk

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static Status check_ws(size_t need, const void *ws, size_t ws_bytes) {
  if (need == 0) return Status();
  if (!ws) return fail(HK_ERR_WORKSPACE, "workspace pointer is NULL but " + std::to_string(need) + " bytes are needed");
  if (ws_bytes < need)
    return fail(HK_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes is smaller than the " +
                                      std::to_string(need) + " bytes needed");
  if (((uintptr_t)ws) % 256 != 0) return fail(HK_ERR_MISALIGNED, "workspace must be 256-byte aligned");
  return Status();
}

// Picks the schedule (autotuned if cached, else the default) and builds the shape.
static Status prepare(const Problem &p, int64_t batch, Shape *sh, Ptrs *P, Sched *sc) {
  Layout lay;
  Status s = layout_for(p, 0, &lay, true, batch);
  if (!s.ok()) return s;
  Sched sch;
  const int logM = lay.logR + lay.logC;
  if (sched_lookup(p.dt, p.prog, p.is_block ? 1 : 0, lay.lclass(), logM, p.is_block ? lay.logC : -1, batch, &sch)) {
    Layout l2;
    if (layout_for(p, sch.split, &l2, true, batch).ok() && l2.lclass() == lay.lclass() && sched_valid(p.dt, l2, sch))
      lay = l2;
    else
      sch = default_sched(p.dt, lay, p.prog, batch);
  } else {
    sch = default_sched(p.dt, lay, p.prog, batch);
  }
  if (!sched_valid(p.dt, lay, sch)) return fail(HK_ERR_NOT_SUPPORTED, "no valid schedule for this shape");
  s = build_shape(p, lay, sch, sh, P, nullptr);
  if (!s.ok()) return s;
  *sc = sch;
  return Status();
}

static Status ws_size(const Problem &p, int64_t batch, size_t *bytes) {
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = prepare(p, batch, &sh, &P, &sc);
  if (!s.ok()) return s;
  *bytes = instance_ws_bytes(sh, p.dt) * (size_t)batch;
  return Status();
}

static Status run_one(const Problem &p, void *ws, size_t ws_bytes, hipStream_t st) {
  // host-side checks first: argument errors never need the device
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = prepare(p, 1, &sh, &P, &sc);
  if (!s.ok()) return s;
  s = check_ws(instance_ws_bytes(sh, p.dt), ws, ws_bytes);
  if (!s.ok()) return s;
  s = ensure_device();
  if (!s.ok()) return s;
  P.ws = ws;
  Strides str;
  memset(&str, 0, sizeof(str));
  return launch_shape(p.dt, sh, sc, P, str, 1, st);
}

static Problem tvp_problem(hk_dtype_t dt, const void *h, int m, int64_t n, const void *x, void *y, void *alpha) {
  Problem p;
  p.dt = dt;
  p.prog = PROG_FWD;
  p.m = m;
  for (int q = 0; q < m && q < HK_MAX_ORDER; ++q) {
    p.dims[q] = n;
    p.vec[q] = x;
  }
  if (!alpha) p.vec[0] = x;  // unused for the vector product; keeps grouping uniform
  p.h = h;
  p.y = y;
  p.alpha = alpha;
  return p;
}

static Status mode_problem(hk_dtype_t dt, const void *h, int m, const int64_t *dims, const void *const *vectors,
                           void *y, void *alpha, Problem *out) {
  if (!dims) return fail(HK_ERR_NULL_POINTER, "dims is NULL");
  if (!vectors) return fail(HK_ERR_NULL_POINTER, "vectors is NULL");
  if (m < 2 || m > HK_MAX_ORDER) return fail(HK_ERR_INVALID_VALUE, "order m must be in [2, 8]");
  Problem p;
  p.dt = dt;
  p.prog = PROG_FWD;
  p.m = m;
  for (int q = 0; q < m; ++q) {
    p.dims[q] = dims[q];
    p.vec[q] = vectors[q];
  }
  if (!alpha) p.vec[0] = nullptr;
  p.h = h;
  p.y = y;
  p.alpha = alpha;
  *out = p;
  return Status();
}

static Status block_problem(hk_dtype_t dt, const void *H, int m, const int64_t *inner, const int64_t *blocks,
                            const void *const *vectors, void *y, void *alpha, Problem *out) {
  if (!inner || !blocks) return fail(HK_ERR_NULL_POINTER, "inner_dims or block_dims is NULL");
  Status s = mode_problem(dt, H, m, inner, vectors, y, alpha, out);
  if (!s.ok()) return s;
  out->is_block = true;
  for (int q = 0; q < m; ++q) out->bdims[q] = blocks[q];
  return Status();
}

static Problem bwd_problem(hk_dtype_t dt, const void *h, int m, int64_t n, const void *x, const void *gy,
                           const void *ga, void *gx, void *gh) {
  Problem p;
  p.dt = dt;
  p.prog = PROG_BWD;
  p.m = m;
  for (int q = 0; q < m && q < HK_MAX_ORDER; ++q) p.dims[q] = n;
  p.h = h;
  p.vec[1] = x;
  p.v = gy;
  p.phi = ga;
  p.gx = gx;
  p.gh = gh;
  return p;
}

// ---------------------------------------------------------------------------
// Level-k block Hankel tensors (Section 2.2: block Hankel tensors whose blocks
// are level-(k-1) block Hankel tensors; k = 2 is the BHHB tensor).  With the
// generating tensor G stored column-major, its entry (i_0, ..., i_{k-1}) sits
// at sum_t i_t S_t, S_t = d_0 ... d_{t-1}.  Each X_p is embedded at the same
// strides; along level t the indices of a product add up to at most d_t - 1,
// so no sum carries into the next level, and the level-k product is exactly
// the 1D Hankel product with generating vector G (prod_t d_t entries, which is
// sum_p L_p - m + 1) and the embedded vectors (L_p = 1 + sum_t (n_p^(t) - 1)
// S_t entries), whose output is read back at the same strides (a Kronecker
// substitution).  One 1D transform of length >= prod_t d_t takes the place of
// the k-dimensional one of the paper's procedure (the multi-dimensional FFT
// on the grid prod_t 2^ceil(log2 d_t)), with the same result.
// ---------------------------------------------------------------------------
struct LevelsRun {
  int k = 0, m = 0;
  int64_t S[HK_MAX_LEVELS] = {0};
  int64_t L[HK_MAX_ORDER] = {0};
  int src[HK_MAX_ORDER] = {0};     // first mode with the same vector (pointer and sizes)
  bool need[HK_MAX_ORDER] = {false};
  size_t off_vec[HK_MAX_ORDER] = {0}, off_y = 0, ws1d = 0, total = 0;
  Problem p1;                     // the 1D problem, with workspace placeholders
};

static Status levels_setup(hk_dtype_t dt, const void *G, int m, int k, const int64_t *dims,
                           const void *const *vectors, bool want_y, bool want_alpha, LevelsRun *r) {
  if (m < 2 || m > HK_MAX_ORDER) return fail(HK_ERR_INVALID_VALUE, "order m must be in [2, 8]");
  if (k < 1 || k > HK_MAX_LEVELS) return fail(HK_ERR_INVALID_VALUE, "levels k must be in [1, 4]");
  if (!dims) return fail(HK_ERR_NULL_POINTER, "dims is NULL");
  if (!vectors) return fail(HK_ERR_NULL_POINTER, "vectors is NULL");
  if (!want_y && !want_alpha) return fail(HK_ERR_NULL_POINTER, "neither y nor alpha requested");
  if (dt < HK_C64 || dt > HK_F64) return fail(HK_ERR_INVALID_VALUE, "unknown dtype");
  for (int i = 0; i < k * m; ++i)
    if (dims[i] < 1) return fail(HK_ERR_INVALID_VALUE, "every size must be >= 1");
  r->k = k;
  r->m = m;
  int64_t prod = 1;
  for (int t = 0; t < k; ++t) {
    int64_t d = 1 - m;
    for (int p = 0; p < m; ++p) {
      if (dims[t * m + p] > ((int64_t)1 << HK_MAX_FFT_LOG2)) return fail(HK_ERR_SIZE_LIMIT, "size too large");
      d += dims[t * m + p];
    }
    r->S[t] = prod;
    if (d > ((int64_t)1 << HK_MAX_FFT_LOG2) || prod > (((int64_t)1 << HK_MAX_FFT_LOG2) / d))
      return fail(HK_ERR_SIZE_LIMIT, "generating tensor exceeds 2^24 entries");
    prod *= d;
  }
  for (int p = 0; p < m; ++p) {
    r->L[p] = 1;
    for (int t = 0; t < k; ++t) r->L[p] += (dims[t * m + p] - 1) * r->S[t];
    r->need[p] = p > 0 || want_alpha;
    if (r->need[p] && !vectors[p])
      return fail(HK_ERR_NULL_POINTER, "vector " + std::to_string(p + 1) + " is NULL");
    r->src[p] = p;
    for (int q = 0; q < p; ++q) {
      if (!r->need[q] || vectors[q] != vectors[p]) continue;
      bool same = true;
      for (int t = 0; t < k; ++t) same = same && dims[t * m + q] == dims[t * m + p];
      if (same) {
        r->src[p] = r->src[q];
        break;
      }
    }
  }
  // the 1D problem; placeholders stand for the workspace pointers
  Problem &q = r->p1;
  q = Problem();
  q.dt = dt;
  q.prog = PROG_FWD;
  q.m = m;
  q.h = G ? G : (const void *)256;
  for (int p = 0; p < m; ++p) {
    q.dims[p] = r->L[p];
    q.vec[p] = r->need[p] ? (const void *)(uintptr_t)(256 * (1 + r->src[p])) : nullptr;
  }
  q.y = want_y ? (void *)256 : nullptr;
  q.alpha = want_alpha ? (void *)256 : nullptr;
  Status s = validate_forward(q);
  if (!s.ok()) return s;
  Shape sh;
  Ptrs P;
  Sched sc;
  s = prepare(q, 1, &sh, &P, &sc);
  if (!s.ok()) return s;
  const size_t es = elem_bytes(dt);
  size_t off = (instance_ws_bytes(sh, dt) + 255) & ~(size_t)255;
  r->ws1d = off;
  if (k > 1) {
    for (int p = 0; p < m; ++p) {
      if (!r->need[p] || r->src[p] != p) continue;
      r->off_vec[p] = off;
      off += ((size_t)r->L[p] * es + 255) & ~(size_t)255;
    }
    if (want_y) {
      r->off_y = off;
      off += ((size_t)r->L[0] * es + 255) & ~(size_t)255;
    }
  }
  r->total = off;
  return Status();
}

extern "C" {

int hk_version(void) { return 10000; }

const char *hk_status_string(hk_status_t s) {
  switch (s) {
    case HK_SUCCESS: return "success";
    case HK_ERR_INVALID_VALUE: return "invalid value";
    case HK_ERR_NULL_POINTER: return "null pointer";
    case HK_ERR_MISALIGNED: return "misaligned pointer";
    case HK_ERR_WORKSPACE: return "workspace too small";
    case HK_ERR_SIZE_LIMIT: return "size limit exceeded";
    case HK_ERR_DEVICE: return "unsupported device";
    case HK_ERR_HIP: return "HIP runtime error";
    case HK_ERR_DEVICE_FAULT: return "device-side error reported";
    case HK_ERR_NOT_SUPPORTED: return "not supported";
  }
  return "unknown status";
}

const char *hk_last_error(void) { return tl_err.c_str(); }

int hk_last_launch_count(void) { return tl_last_launches; }

hk_status_t hk_set_fft_lengths(int policy) {
  if (policy != HK_LENGTHS_AUTO && policy != HK_LENGTHS_SMALLEST && policy != HK_LENGTHS_POW2)
    return finish(fail(HK_ERR_INVALID_VALUE, "unknown length policy"));
  set_length_policy(policy);
  return finish(Status());
}

int hk_get_fft_lengths(void) { return length_policy(); }

hk_status_t hk_fft_layout(int64_t d_h, int64_t *n_fft, int64_t *n_row, int64_t *n_col) {
  if (!n_fft || !n_row || !n_col) return finish(fail(HK_ERR_NULL_POINTER, "output pointer is NULL"));
  if (d_h < 1) return finish(fail(HK_ERR_INVALID_VALUE, "d_h must be >= 1"));
  Problem p;
  p.m = 2;
  p.dims[0] = d_h;
  p.dims[1] = 1;
  Layout lay;
  Status s = layout_for(p, 0, &lay);
  if (!s.ok()) return finish(s);
  *n_fft = (int64_t)lay.odd << (lay.logR + lay.logC);
  *n_row = (int64_t)1 << lay.logR;
  *n_col = (int64_t)1 << lay.logC;
  return finish(Status());
}

// ---------------------------------------------------------------------------
hk_status_t hankel_tvp_workspace_size(hk_dtype_t dt, int m, int64_t n, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  Problem p = tvp_problem(dt, (const void *)16, m, n, (const void *)16, (void *)16, nullptr);
  Status s = validate_forward(p);
  if (!s.ok()) return finish(s);
  return finish(ws_size(p, 1, bytes));
}

hk_status_t hankel_tvp(hk_dtype_t dt, const void *h, int m, int64_t n, const void *x, void *y, void *alpha, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
  Problem p = tvp_problem(dt, h, m, n, x, y, alpha);
  Status s = validate_forward(p);
  if (!s.ok()) return finish(s);
  return finish(run_one(p, ws, ws_bytes, stream));
}

hk_status_t hankel_mode_products_workspace_size(hk_dtype_t dt, int m, const int64_t *dims, const void *const *vectors,
                                                int want_y, int want_alpha, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  Problem p;
  Status s = mode_problem(dt, (const void *)16, m, dims, vectors, want_y ? (void *)16 : nullptr,
                          want_alpha ? (void *)16 : nullptr, &p);
  if (!s.ok()) return finish(s);
  s = validate_forward(p);
  if (!s.ok()) return finish(s);
  return finish(ws_size(p, 1, bytes));
}

hk_status_t hankel_mode_products(hk_dtype_t dt, const void *h, int m, const int64_t *dims, const void *const *vectors,
                                 void *y, void *alpha, void *ws, size_t ws_bytes, hipStream_t stream) {
  Problem p;
  Status s = mode_problem(dt, h, m, dims, vectors, y, alpha, &p);
  if (!s.ok()) return finish(s);
  s = validate_forward(p);
  if (!s.ok()) return finish(s);
  return finish(run_one(p, ws, ws_bytes, stream));
}

// ---------------------------------------------------------------------------
// Spectral form.  The fast product is a pointwise product of spectra,
// h^ = ifft(pad_N h) and x^_p = fft(pad_N x_p) on one transform length N
// (Section 3, the procedures for the mode products and the scalar).  A
// spectrum computed once serves every product that shares the operand.
// Spectra use the power-of-two three-pass layout with a fixed split (row
// length R = 2^(ceil(log2(N) / 2) + 1) from N = 2^16 on, the split the tuned
// schedules of large transforms use, else 2^ceil(log2(N) / 2); C = N / R
// rows), so that spectra made by separate calls combine; element r R + c
// holds bin r + C c.
// ---------------------------------------------------------------------------
static Status spectral_problem(hk_dtype_t dt, int m, const int64_t *dims, Problem *out) {
  if (dt < HK_C64 || dt > HK_F64) return fail(HK_ERR_INVALID_VALUE, "unknown dtype");
  if (m < 2 || m > HK_MAX_ORDER) return fail(HK_ERR_INVALID_VALUE, "order m must be in [2, 8]");
  if (!dims) return fail(HK_ERR_NULL_POINTER, "dims is NULL");
  Problem p;
  p.dt = dt;
  p.prog = PROG_FWD;
  p.m = m;
  for (int q = 0; q < m; ++q) {
    if (dims[q] < 1) return fail(HK_ERR_INVALID_VALUE, "every dimension must be >= 1");
    if (dims[q] > ((int64_t)1 << 40)) return fail(HK_ERR_SIZE_LIMIT, "dimension too large");
    p.dims[q] = dims[q];
  }
  *out = p;
  return Status();
}

static Status spectral_setup(const Problem &p, Layout *lay, Sched *sc, int64_t batch = 1) {
  int64_t dh = 1 - p.m;
  for (int q = 0; q < p.m; ++q) dh += p.dims[q];
  int logN = 0;
  while (((int64_t)1 << logN) < dh) ++logN;
  const int split = logN >= 16 ? 1 : 0;
  Status s = layout_for(p, split, lay, /*allow_odd=*/false, 1);
  if (!s.ok()) return s;
  if (lay->resident || lay->odd != 1 || lay->r2c)
    return fail(HK_ERR_NOT_SUPPORTED, "spectra need the three-pass layout: d_H above 4096");
  Sched sch;
  const int logM = lay->logR + lay->logC;
  // the cached schedule of this shape, moved to the spectral split when it was
  // tuned for another (its row and column parameters still fit the batch)
  bool have = sched_lookup(p.dt, p.prog, 0, lay->lclass(), logM, -1, batch, &sch);
  if (have) {
    sch.split = split;
    have = sched_valid(p.dt, *lay, sch);
  }
  if (have)
    *sc = sch;
  else {
    *sc = default_sched(p.dt, *lay, p.prog, batch);
    sc->split = split;
  }
  if (!sched_valid(p.dt, *lay, *sc)) return fail(HK_ERR_NOT_SUPPORTED, "no valid schedule for this shape");
  return Status();
}

// The spectrum program: the column pass of one operand (h for which = -1,
// the vector of mode `which` otherwise), its row transform stored to `spec`
// in row order, no product.
static Status spectrum_prepare(hk_dtype_t dt, int m, const int64_t *dims, int which, const void *src, void *spec,
                               Shape *sh, Ptrs *P, Sched *sc) {
  Problem p;
  Status s = spectral_problem(dt, m, dims, &p);
  if (!s.ok()) return s;
  if (which < -1 || which >= m) return fail(HK_ERR_INVALID_VALUE, "which must be -1 (h) or a mode in [0, m)");
  Layout lay;
  s = spectral_setup(p, &lay, sc);
  if (!s.ok()) return s;
  const void *dummy = (const void *)256;
  p.h = dummy;
  for (int q = 0; q < m; ++q) p.vec[q] = dummy;
  p.y = (void *)256;
  Shape b;
  Ptrs bp;
  s = build_shape(p, lay, *sc, &b, &bp, nullptr);
  if (!s.ok()) return s;
  OpDesc od = b.ops[0];  // h: conjugated on load, conjugated and scaled by 1/N after the row transform
  if (which >= 0) {
    od.role = ROLE_X;
    od.exp = 0;
    od.flags = is_complex(dt) ? 0 : OPF_REAL;
    od.len = dims[which];
    od.cols = 1;
    od.ncol_nz = std::min<int64_t>((int64_t)1 << lay.logR, dims[which]);
  }
  od.flags |= OPF_STORE_SPEC;
  od.buf = 0;
  b.ops[0] = od;
  b.nops = 1;
  b.want_y = 0;
  b.want_alpha = 0;
  b.nbuf = 1;
  const size_t eb = cplx_bytes(dt);
  b.ws_bytes = (int64_t)(((((size_t)1 << (lay.logR + lay.logC)) + (size_t)b.partials) * eb + 255) & ~(size_t)255);
  memset(&bp, 0, sizeof(bp));
  bp.op[0] = src;
  bp.out1 = spec;
  *sh = b;
  *P = bp;
  return Status();
}

hk_status_t hankel_spectrum_layout(hk_dtype_t dt, int m, const int64_t *dims, int64_t *n_fft, int64_t *row_len) {
  if (!n_fft || !row_len) return finish(fail(HK_ERR_NULL_POINTER, "n_fft or row_len is NULL"));
  Problem p;
  Status s = spectral_problem(dt, m, dims, &p);
  if (!s.ok()) return finish(s);
  Layout lay;
  Sched sc;
  s = spectral_setup(p, &lay, &sc);
  if (!s.ok()) return finish(s);
  *n_fft = (int64_t)1 << (lay.logR + lay.logC);
  *row_len = (int64_t)1 << lay.logR;
  return finish(Status());
}

hk_status_t hankel_spectrum_workspace_size(hk_dtype_t dt, int m, const int64_t *dims, int which, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = spectrum_prepare(dt, m, dims, which, nullptr, nullptr, &sh, &P, &sc);
  if (!s.ok()) return finish(s);
  *bytes = instance_ws_bytes(sh, dt);
  return finish(Status());
}

hk_status_t hankel_spectrum(hk_dtype_t dt, int m, const int64_t *dims, int which, const void *src, void *spec,
                            void *ws, size_t ws_bytes, hipStream_t stream) {
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = spectrum_prepare(dt, m, dims, which, src, spec, &sh, &P, &sc);
  if (!s.ok()) return finish(s);
  if (!src || !spec) return finish(fail(HK_ERR_NULL_POINTER, "src or spec is NULL"));
  if (!aligned(src, elem_bytes(dt)) || !aligned(spec, cplx_bytes(dt)))
    return finish(fail(HK_ERR_MISALIGNED, "pointer not aligned to the element size"));
  s = check_ws(instance_ws_bytes(sh, dt), ws, ws_bytes);
  if (!s.ok()) return finish(s);
  s = ensure_device();
  if (!s.ok()) return finish(s);
  P.ws = ws;
  Strides str;
  memset(&str, 0, sizeof(str));
  return finish(launch_shape(dt, sh, sc, P, str, 1, stream));
}

// Mode products with h given by its spectrum and each vector by itself or by
// its spectrum (specs[q] non-NULL).
static Status spectral_products_problem(hk_dtype_t dt, const void *h_spec, int m, const int64_t *dims,
                                        const void *const *vectors, const void *const *specs, void *y, void *alpha,
                                        Problem *out) {
  Problem p;
  Status s = spectral_problem(dt, m, dims, &p);
  if (!s.ok()) return s;
  p.h = h_spec;
  p.h_spec = true;
  for (int q = 0; q < m; ++q) {
    if (q == 0 && !alpha) continue;
    if (specs && specs[q]) {
      p.vec[q] = specs[q];
      p.spec_mask |= 1u << q;
    } else if (vectors) {
      p.vec[q] = vectors[q];
    }
  }
  p.y = y;
  p.alpha = alpha;
  s = validate_forward(p);
  if (!s.ok()) return s;
  *out = p;
  return Status();
}

static Status spectral_products_prepare(const Problem &p, Shape *sh, Ptrs *P, Sched *sc, int64_t batch = 1) {
  Layout lay;
  Status s = spectral_setup(p, &lay, sc, batch);
  if (!s.ok()) return s;
  return build_shape(p, lay, *sc, sh, P, nullptr);
}

hk_status_t hankel_mode_products_spectral_workspace_size(hk_dtype_t dt, int m, const int64_t *dims,
                                                         const void *const *vectors, const void *const *specs,
                                                         int want_y, int want_alpha, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  Problem p;
  Status s = spectral_products_problem(dt, (const void *)256, m, dims, vectors, specs,
                                       want_y ? (void *)256 : nullptr, want_alpha ? (void *)256 : nullptr, &p);
  if (!s.ok()) return finish(s);
  Shape sh;
  Ptrs P;
  Sched sc;
  s = spectral_products_prepare(p, &sh, &P, &sc);
  if (!s.ok()) return finish(s);
  *bytes = instance_ws_bytes(sh, dt);
  return finish(Status());
}

hk_status_t hankel_mode_products_spectral(hk_dtype_t dt, const void *h_spec, int m, const int64_t *dims,
                                          const void *const *vectors, const void *const *specs, void *y,
                                          void *alpha, void *ws, size_t ws_bytes, hipStream_t stream) {
  Problem p;
  Status s = spectral_products_problem(dt, h_spec, m, dims, vectors, specs, y, alpha, &p);
  if (!s.ok()) return finish(s);
  Shape sh;
  Ptrs P;
  Sched sc;
  s = spectral_products_prepare(p, &sh, &P, &sc);
  if (!s.ok()) return finish(s);
  s = check_ws(instance_ws_bytes(sh, dt), ws, ws_bytes);
  if (!s.ok()) return finish(s);
  s = ensure_device();
  if (!s.ok()) return finish(s);
  P.ws = ws;
  Strides str;
  memset(&str, 0, sizeof(str));
  return finish(launch_shape(dt, sh, sc, P, str, 1, stream));
}

// Strided batch of equal-vector products sharing one stored h^: operand 0 is
// the spectrum (stride 0), operand 1 the vector x (one transform, power m - 1).
static Status spectral_batch_problem(hk_dtype_t dt, const void *h_spec, int m, int64_t n, const void *x, void *y,
                                     void *alpha, Problem *p) {
  if (m < 2 || m > HK_MAX_ORDER) return fail(HK_ERR_INVALID_VALUE, "order m must be in [2, 8]");
  int64_t dims[HK_MAX_ORDER];
  const void *vecs[HK_MAX_ORDER];
  for (int q = 0; q < m; ++q) {
    dims[q] = n;
    vecs[q] = x;
  }
  return spectral_products_problem(dt, h_spec, m, dims, vecs, nullptr, y, alpha, p);
}

hk_status_t hankel_tvp_spectral_strided_batched_workspace_size(hk_dtype_t dt, int m, int64_t n, int64_t batch,
                                                               size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  if (batch < 0) return finish(fail(HK_ERR_INVALID_VALUE, "batch must be >= 0"));
  Problem p;
  Status s = spectral_batch_problem(dt, (const void *)256, m, n, (const void *)256, (void *)256, (void *)256, &p);
  if (!s.ok()) return finish(s);
  Shape sh;
  Ptrs P;
  Sched sc;
  s = spectral_products_prepare(p, &sh, &P, &sc, std::max<int64_t>(1, batch));
  if (!s.ok()) return finish(s);
  *bytes = instance_ws_bytes(sh, dt) * (size_t)batch;
  return finish(Status());
}

hk_status_t hankel_tvp_spectral_strided_batched(hk_dtype_t dt, const void *h_spec, int m, int64_t n, const void *x,
                                                int64_t x_stride, void *y, int64_t y_stride, void *alpha,
                                                int64_t batch, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (batch < 0) return finish(fail(HK_ERR_INVALID_VALUE, "batch must be >= 0"));
  Problem p;
  Status s = spectral_batch_problem(dt, h_spec, m, n, x, y, alpha, &p);
  if (!s.ok()) return finish(s);
  if (batch == 0) return finish(Status());
  Shape sh;
  Ptrs P;
  Sched sc;
  s = spectral_products_prepare(p, &sh, &P, &sc, batch);
  if (!s.ok()) return finish(s);
  const size_t per = instance_ws_bytes(sh, dt);
  s = check_ws(per * (size_t)batch, ws, ws_bytes);
  if (!s.ok()) return finish(s);
  s = ensure_device();
  if (!s.ok()) return finish(s);
  if (sh.nops != 2 || !(sh.ops[0].flags & OPF_SPEC))
    return finish(fail(HK_ERR_NOT_SUPPORTED, "unexpected operand layout"));
  const int64_t eb = (int64_t)elem_bytes(dt);
  Strides str;
  memset(&str, 0, sizeof(str));
  str.op[1] = x_stride * eb;  // operand 0, the stored h^, is shared
  str.y = y_stride * eb;
  str.alpha = eb;
  str.ws = (int64_t)per;
  P.ws = ws;
  return finish(launch_shape(dt, sh, sc, P, str, batch, stream));
}

// Adjoint of the equal-vector products with x given by its stored spectrum
// (the forward's x^, from hankel_spectrum on the same shape): the column
// pass of x and its row transform are skipped.
static Status backward_spectral_prepare(const Problem &p, Shape *sh, Ptrs *P, Sched *sc, int64_t batch = 1) {
  Status s = validate_backward(p);
  if (!s.ok()) return s;
  Layout lay;
  s = spectral_setup(p, &lay, sc, batch);
  if (!s.ok()) return s;
  return build_shape(p, lay, *sc, sh, P, nullptr);
}

hk_status_t hankel_tvp_backward_spectral_workspace_size(hk_dtype_t dt, int m, int64_t n, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  Problem p = bwd_problem(dt, (const void *)256, m, n, (const void *)256, (const void *)256, (const void *)256,
                          (void *)256, (void *)256);
  p.spec_mask = 2u;
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = backward_spectral_prepare(p, &sh, &P, &sc);
  if (!s.ok()) return finish(s);
  *bytes = instance_ws_bytes(sh, dt);
  return finish(Status());
}

hk_status_t hankel_tvp_backward_spectral(hk_dtype_t dt, const void *h, int m, int64_t n, const void *x_spec,
                                         const void *grad_y, const void *grad_alpha, void *grad_x, void *grad_h,
                                         void *ws, size_t ws_bytes, hipStream_t stream) {
  Problem p = bwd_problem(dt, h, m, n, x_spec, grad_y, grad_alpha, grad_x, grad_h);
  p.spec_mask = 2u;
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = backward_spectral_prepare(p, &sh, &P, &sc);
  if (!s.ok()) return finish(s);
  if (!(sh.ops[0].flags & OPF_SPEC)) return finish(fail(HK_ERR_NOT_SUPPORTED, "unexpected operand layout"));
  s = check_ws(instance_ws_bytes(sh, dt), ws, ws_bytes);
  if (!s.ok()) return finish(s);
  s = ensure_device();
  if (!s.ok()) return finish(s);
  P.ws = ws;
  Strides str;
  memset(&str, 0, sizeof(str));
  return finish(launch_shape(dt, sh, sc, P, str, 1, stream));
}

// Forward equal-vector products that also store x^ = fft(pad_N x) in the row
// order of hankel_spectrum (the shape's spectral layout), to be reused by the
// adjoint (hankel_tvp_backward_spectral*): the row pass writes the spectrum
// row of x right after transforming it.
static Status save_spectrum_prepare(const Problem &p, int64_t batch, Shape *sh, Ptrs *P, Sched *sc) {
  Status s = validate_forward(p);
  if (!s.ok()) return s;
  if (!is_complex(p.dt)) return fail(HK_ERR_NOT_SUPPORTED, "stored spectra for the adjoint need a complex dtype");
  Layout lay;
  s = spectral_setup(p, &lay, sc, batch);
  if (!s.ok()) return s;
  s = build_shape(p, lay, *sc, sh, P, nullptr);
  if (!s.ok()) return s;
  int nx = 0;
  for (int o = 0; o < sh->nops; ++o)
    if (sh->ops[o].role == ROLE_X) {
      sh->ops[o].flags |= OPF_STORE_SPEC;
      ++nx;
    }
  if (nx != 1 || sh->ops[0].role != ROLE_H) return fail(HK_ERR_NOT_SUPPORTED, "unexpected operand layout");
  return Status();
}

hk_status_t hankel_tvp_save_spectrum_workspace_size(hk_dtype_t dt, int m, int64_t n, int64_t batch, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  if (batch < 0) return finish(fail(HK_ERR_INVALID_VALUE, "batch must be >= 0"));
  Problem p = tvp_problem(dt, (const void *)256, m, n, (const void *)256, (void *)256, (void *)256);
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = save_spectrum_prepare(p, std::max<int64_t>(1, batch), &sh, &P, &sc);
  if (!s.ok()) return finish(s);
  *bytes = instance_ws_bytes(sh, dt) * (size_t)batch;
  return finish(Status());
}

hk_status_t hankel_tvp_save_spectrum(hk_dtype_t dt, const void *h, int64_t h_stride, int m, int64_t n, const void *x,
                                     int64_t x_stride, void *y, int64_t y_stride, void *alpha, void *x_spec,
                                     int64_t spec_stride, int64_t batch, void *ws, size_t ws_bytes,
                                     hipStream_t stream) {
  if (batch < 0) return finish(fail(HK_ERR_INVALID_VALUE, "batch must be >= 0"));
  if (!x_spec) return finish(fail(HK_ERR_NULL_POINTER, "x_spec is NULL"));
  if (!aligned(x_spec, cplx_bytes(dt))) return finish(fail(HK_ERR_MISALIGNED, "x_spec not aligned to its element size"));
  Problem p = tvp_problem(dt, h, m, n, x, y, alpha);
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = save_spectrum_prepare(p, std::max<int64_t>(1, batch), &sh, &P, &sc);
  if (!s.ok()) return finish(s);
  const int64_t N = (int64_t)1 << (sh.logR + sh.logC);
  if (batch > 1 && spec_stride < N) return finish(fail(HK_ERR_INVALID_VALUE, "spec_stride is below the spectrum length"));
  if (batch == 0) return finish(Status());
  const size_t per = instance_ws_bytes(sh, dt);
  s = check_ws(per * (size_t)batch, ws, ws_bytes);
  if (!s.ok()) return finish(s);
  s = ensure_device();
  if (!s.ok()) return finish(s);
  const int64_t eb = (int64_t)elem_bytes(dt);
  Strides str;
  memset(&str, 0, sizeof(str));
  str.op[0] = h_stride * eb;  // operands: H, X
  str.op[1] = x_stride * eb;
  str.y = y_stride * eb;
  str.alpha = eb;
  str.out1 = spec_stride * (int64_t)cplx_bytes(dt);
  str.ws = (int64_t)per;
  P.out1 = x_spec;
  P.ws = ws;
  return finish(launch_shape(dt, sh, sc, P, str, batch, stream));
}

hk_status_t hankel_tvp_backward_spectral_strided_batched_workspace_size(hk_dtype_t dt, int m, int64_t n, int64_t batch,
                                                                        size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  if (batch < 0) return finish(fail(HK_ERR_INVALID_VALUE, "batch must be >= 0"));
  Problem p = bwd_problem(dt, (const void *)256, m, n, (const void *)256, (const void *)256, (const void *)256,
                          (void *)256, (void *)256);
  p.spec_mask = 2u;
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = backward_spectral_prepare(p, &sh, &P, &sc, std::max<int64_t>(1, batch));
  if (!s.ok()) return finish(s);
  *bytes = instance_ws_bytes(sh, dt) * (size_t)batch;
  return finish(Status());
}

hk_status_t hankel_tvp_backward_spectral_strided_batched(hk_dtype_t dt, const void *h, int64_t h_stride, int m,
                                                         int64_t n, const void *x_spec, int64_t spec_stride,
                                                         const void *grad_y, int64_t gy_stride, const void *grad_alpha,
                                                         void *grad_x, int64_t gx_stride, void *grad_h,
                                                         int64_t gh_stride, int64_t batch, void *ws, size_t ws_bytes,
                                                         hipStream_t stream) {
  if (batch < 0) return finish(fail(HK_ERR_INVALID_VALUE, "batch must be >= 0"));
  Problem p = bwd_problem(dt, h, m, n, x_spec, grad_y, grad_alpha, grad_x, grad_h);
  p.spec_mask = 2u;
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = backward_spectral_prepare(p, &sh, &P, &sc, std::max<int64_t>(1, batch));
  if (!s.ok()) return finish(s);
  if (!(sh.ops[0].flags & OPF_SPEC)) return finish(fail(HK_ERR_NOT_SUPPORTED, "unexpected operand layout"));
  const int64_t N = (int64_t)1 << (sh.logR + sh.logC);
  if (batch > 1 && spec_stride < N) return finish(fail(HK_ERR_INVALID_VALUE, "spec_stride is below the spectrum length"));
  if (batch == 0) return finish(Status());
  const size_t per = instance_ws_bytes(sh, dt);
  s = check_ws(per * (size_t)batch, ws, ws_bytes);
  if (!s.ok()) return finish(s);
  s = ensure_device();
  if (!s.ok()) return finish(s);
  const int64_t eb = (int64_t)elem_bytes(dt);
  // operand order of the adjoint shape: X (stored spectrum), [V], [H]
  Strides str;
  memset(&str, 0, sizeof(str));
  int o = 0;
  str.op[o++] = spec_stride * (int64_t)cplx_bytes(dt);
  if (grad_y) str.op[o++] = gy_stride * eb;
  if (grad_x) str.op[o++] = h_stride * eb;
  str.y = gh_stride * eb;
  str.out1 = gx_stride * eb;
  str.phi = eb;
  str.ws = (int64_t)per;
  P.ws = ws;
  return finish(launch_shape(dt, sh, sc, P, str, batch, stream));
}

// ---------------------------------------------------------------------------
// Adjoint of the products with distinct vectors, 1D and BHHB (complex
// autograd's J^H applied to the cotangents v of y and phi of alpha).  Every
// gradient is linear in the cotangent of mode 1, c = conj(v) + conj(phi) x_1:
//   grad_h     = conj(c * x_2 * ... * x_m)            (convolution program)
//   grad_{x_p} = conj(H x_1 c x_q (q != 1, p))         (mode p free, p >= 2)
//   grad_{x_1} = phi conj(H x_2 ... x_m) = conj(H x_2 (conj(phi) x_2) x_3 ... x_m)
// Each is one product of the forward kernels on power-of-two complex
// layouts (conjugated output, or the generating-vector-free convolution),
// run in turn on the stream; they share one workspace after the two
// cotangent vectors.
// ---------------------------------------------------------------------------
static Status adjoint_distinct(hk_dtype_t dt, bool is_block, const void *h, int m, const int64_t *dims,
                               const int64_t *bdims, const void *const *vectors, const void *grad_y,
                               const void *grad_alpha, void *const *grad_vectors, void *grad_h, void *ws,
                               size_t ws_bytes, size_t *ws_need, hipStream_t st) {
  if (!dims || !vectors || !grad_vectors || (is_block && !bdims))
    return fail(HK_ERR_NULL_POINTER, "dims, block_dims, vectors or grad_vectors is NULL");
  if (m < 2 || m > HK_MAX_ORDER) return fail(HK_ERR_INVALID_VALUE, "order m must be in [2, 8]");
  if (!is_complex(dt)) return fail(HK_ERR_NOT_SUPPORTED, "the adjoint is implemented for complex dtypes");
  const bool sizing = ws_need != nullptr;
  bool any = grad_h != nullptr;
  for (int q = 0; q < m; ++q) any = any || grad_vectors[q] != nullptr;
  if (!any) return fail(HK_ERR_NULL_POINTER, "no gradient requested");
  if (grad_alpha && !vectors[0]) return fail(HK_ERR_NULL_POINTER, "grad_alpha given but vector 1 is NULL");
  const size_t eb = elem_bytes(dt);
  int64_t len[HK_MAX_ORDER];
  for (int q = 0; q < m; ++q) {
    if (dims[q] < 1 || (is_block && bdims[q] < 1)) return fail(HK_ERR_INVALID_VALUE, "every dimension must be >= 1");
    len[q] = dims[q] * (is_block ? bdims[q] : 1);
  }
  const void *ptrs[] = {h, grad_y, grad_alpha, grad_h};
  for (const void *q : ptrs)
    if (q && !aligned(q, eb)) return fail(HK_ERR_MISALIGNED, "pointer not aligned to the element size");
  for (int q = 0; q < m; ++q)
    if ((vectors[q] && !aligned(vectors[q], eb)) || (grad_vectors[q] && !aligned(grad_vectors[q], eb)))
      return fail(HK_ERR_MISALIGNED, "vector not aligned to the element size");
  // workspace: c (len[0]), d = conj(phi) x_2 (len[1]), then the products' workspace
  const size_t off_d = align256(len[0] * cplx_bytes(dt));
  const size_t off_p = off_d + align256(len[1] * cplx_bytes(dt));
  char *base = (char *)ws;
  // sizing: distinct placeholder addresses, so that no operands merge (an
  // upper bound on the workspace of any call whose vectors may coincide)
  auto dummy_of = [](int q) { return (const void *)(uintptr_t)(256 * (q + 3)); };
  const void *c = sizing ? (const void *)256 : (const void *)base;
  const void *d = sizing ? (const void *)512 : (const void *)(base + off_d);
  void *pws = sizing ? nullptr : (void *)(base + off_p);
  const size_t pws_bytes = ws_bytes > off_p ? ws_bytes - off_p : 0;
  // the sub-products
  std::vector<Problem> subs;
  auto sub = [&](const int64_t *order, const void *const *vecs, void *y, bool conv) {
    Problem q;
    q.dt = dt;
    q.prog = PROG_FWD;
    q.is_block = is_block;
    q.m = m;
    for (int t = 0; t < m; ++t) {
      q.dims[t] = dims[order[t]];
      q.bdims[t] = is_block ? bdims[order[t]] : 0;
      q.vec[t] = vecs[t];
    }
    q.h = conv ? nullptr : h;
    q.y = y;
    q.conv = conv;
    q.conj_y = !conv;
    subs.push_back(q);
  };
  int64_t order[HK_MAX_ORDER];
  const void *vecs[HK_MAX_ORDER];
  if (grad_h) {
    for (int t = 0; t < m; ++t) {
      order[t] = t;
      vecs[t] = t == 0 ? c : (sizing ? dummy_of(t) : vectors[t]);
    }
    sub(order, vecs, sizing ? (void *)256 : grad_h, true);
  }
  for (int p = 1; p < m; ++p) {
    if (!grad_vectors[p]) continue;
    // mode p free, c in the next mode, the other vectors after it
    int k = 0;
    order[k] = p;
    vecs[k++] = nullptr;
    order[k] = 0;
    vecs[k++] = c;
    for (int q = 1; q < m; ++q)
      if (q != p) {
        order[k] = q;
        vecs[k++] = sizing ? dummy_of(q) : vectors[q];
      }
    sub(order, vecs, sizing ? (void *)256 : grad_vectors[p], false);
  }
  const bool x1_product = grad_vectors[0] && grad_alpha;
  if (x1_product) {
    for (int t = 0; t < m; ++t) {
      order[t] = t;
      vecs[t] = t == 0 ? nullptr : (t == 1 ? d : (sizing ? dummy_of(t) : vectors[t]));
    }
    sub(order, vecs, sizing ? (void *)256 : grad_vectors[0], false);
  }
  for (Problem &q : subs) {
    if (!sizing && !q.conv && !q.h) return fail(HK_ERR_NULL_POINTER, "generating vector/matrix is NULL");
    if (sizing && !q.conv) q.h = (const void *)256;
    Status s = validate_forward(q);
    if (!s.ok()) return s;
  }
  size_t need_p = 0;
  for (const Problem &q : subs) {
    Shape sh;
    Ptrs P;
    Sched sc;
    Status s = prepare(q, 1, &sh, &P, &sc);
    if (!s.ok()) return s;
    need_p = std::max(need_p, instance_ws_bytes(sh, dt));
  }
  const size_t need = off_p + need_p;
  if (sizing) {
    *ws_need = need;
    return Status();
  }
  Status s = check_ws(need, ws, ws_bytes);
  if (!s.ok()) return s;
  s = ensure_device();
  if (!s.ok()) return s;
  const bool dbl = dt == HK_C128;
  hipError_t e = hipSuccess;
  const bool need_c = grad_h || [&] {
    for (int p = 1; p < m; ++p)
      if (grad_vectors[p]) return true;
    return false;
  }();
  if (need_c) {
    count_launch();
    e = launch_mode1_cotangent(dbl, (void *)c, grad_y, grad_alpha, vectors[0], len[0], st);
  }
  if (e == hipSuccess && x1_product) {
    count_launch();
    e = launch_mode1_cotangent(dbl, (void *)d, nullptr, grad_alpha, vectors[1], len[1], st);
  }
  if (e == hipSuccess && grad_vectors[0] && !grad_alpha) {
    // x_1 enters alpha only: with no cotangent for alpha its gradient is zero
    count_launch();
    e = launch_mode1_cotangent(dbl, grad_vectors[0], nullptr, nullptr, nullptr, len[0], st);
  }
  if (e != hipSuccess) return fail(HK_ERR_HIP, std::string("cotangent kernel launch: ") + hipGetErrorString(e));
  for (const Problem &q : subs) {
    s = run_one(q, pws, pws_bytes, st);
    if (!s.ok()) return s;
  }
  return Status();
}

hk_status_t hankel_mode_products_backward_workspace_size(hk_dtype_t dt, int m, const int64_t *dims,
                                                         int grad_vectors_mask, int want_grad_h, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  void *gv[HK_MAX_ORDER] = {nullptr};
  const void *vv[HK_MAX_ORDER];
  for (int q = 0; q < HK_MAX_ORDER; ++q) {
    gv[q] = ((grad_vectors_mask >> q) & 1) ? (void *)256 : nullptr;
    vv[q] = (const void *)256;
  }
  return finish(adjoint_distinct(dt, false, (const void *)256, m, dims, nullptr, vv, (const void *)256,
                                 (const void *)256, gv, want_grad_h ? (void *)256 : nullptr, nullptr, 0, bytes,
                                 nullptr));
}

hk_status_t hankel_mode_products_backward(hk_dtype_t dt, const void *h, int m, const int64_t *dims,
                                          const void *const *vectors, const void *grad_y, const void *grad_alpha,
                                          void *const *grad_vectors, void *grad_h, void *ws, size_t ws_bytes,
                                          hipStream_t stream) {
  return finish(adjoint_distinct(dt, false, h, m, dims, nullptr, vectors, grad_y, grad_alpha, grad_vectors, grad_h,
                                 ws, ws_bytes, nullptr, stream));
}

hk_status_t block_hankel_tvp_backward_workspace_size(hk_dtype_t dt, int m, const int64_t *inner_dims,
                                                     const int64_t *block_dims, int grad_vectors_mask,
                                                     int want_grad_h, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  void *gv[HK_MAX_ORDER] = {nullptr};
  const void *vv[HK_MAX_ORDER];
  for (int q = 0; q < HK_MAX_ORDER; ++q) {
    gv[q] = ((grad_vectors_mask >> q) & 1) ? (void *)256 : nullptr;
    vv[q] = (const void *)256;
  }
  return finish(adjoint_distinct(dt, true, (const void *)256, m, inner_dims, block_dims, vv, (const void *)256,
                                 (const void *)256, gv, want_grad_h ? (void *)256 : nullptr, nullptr, 0, bytes,
                                 nullptr));
}

hk_status_t block_hankel_tvp_backward(hk_dtype_t dt, const void *H, int m, const int64_t *inner_dims,
                                      const int64_t *block_dims, const void *const *vectors, const void *grad_y,
                                      const void *grad_alpha, void *const *grad_vectors, void *grad_H, void *ws,
                                      size_t ws_bytes, hipStream_t stream) {
  return finish(adjoint_distinct(dt, true, H, m, inner_dims, block_dims, vectors, grad_y, grad_alpha, grad_vectors,
                                 grad_H, ws, ws_bytes, nullptr, stream));
}

hk_status_t block_hankel_tvp_layout(hk_dtype_t dt, int m, const int64_t *inner_dims, const int64_t *block_dims,
                                    int64_t batch, int64_t *grid_rows, int64_t *grid_cols) {
  if (!grid_rows || !grid_cols) return finish(fail(HK_ERR_NULL_POINTER, "grid_rows or grid_cols is NULL"));
  const void *vecs[HK_MAX_ORDER];
  for (int q = 0; q < HK_MAX_ORDER; ++q) vecs[q] = (const void *)256;
  Problem p;
  Status s = block_problem(dt, (const void *)256, m, inner_dims, block_dims, vecs, (void *)256, nullptr, &p);
  if (!s.ok()) return finish(s);
  Layout lay;
  s = layout_for(p, 0, &lay, true, std::max<int64_t>(1, batch));
  if (!s.ok()) return finish(s);
  *grid_rows = (int64_t)lay.odd << lay.logR;
  *grid_cols = (int64_t)lay.odd_c << lay.logC;
  return finish(Status());
}

hk_status_t block_hankel_tvp_workspace_size(hk_dtype_t dt, int m, const int64_t *inner_dims, const int64_t *block_dims,
                                            const void *const *vectors, int want_y, int want_alpha, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  Problem p;
  Status s = block_problem(dt, (const void *)16, m, inner_dims, block_dims, vectors, want_y ? (void *)16 : nullptr,
                           want_alpha ? (void *)16 : nullptr, &p);
  if (!s.ok()) return finish(s);
  s = validate_forward(p);
  if (!s.ok()) return finish(s);
  return finish(ws_size(p, 1, bytes));
}

hk_status_t block_hankel_tvp(hk_dtype_t dt, const void *H, int m, const int64_t *inner_dims, const int64_t *block_dims,
                             const void *const *vectors, void *y, void *alpha, void *ws, size_t ws_bytes,
                             hipStream_t stream) {
  Problem p;
  Status s = block_problem(dt, H, m, inner_dims, block_dims, vectors, y, alpha, &p);
  if (!s.ok()) return finish(s);
  s = validate_forward(p);
  if (!s.ok()) return finish(s);
  return finish(run_one(p, ws, ws_bytes, stream));
}

hk_status_t block_hankel_tvp_levels_workspace_size(hk_dtype_t dt, int m, int k, const int64_t *dims,
                                                   const void *const *vectors, int want_y, int want_alpha,
                                                   size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  LevelsRun r;
  Status s = levels_setup(dt, nullptr, m, k, dims, vectors, want_y != 0, want_alpha != 0, &r);
  if (!s.ok()) return finish(s);
  *bytes = r.total;
  return finish(Status());
}

hk_status_t block_hankel_tvp_levels(hk_dtype_t dt, const void *G, int m, int k, const int64_t *dims,
                                    const void *const *vectors, void *y, void *alpha, void *ws, size_t ws_bytes,
                                    hipStream_t stream) {
  if (!G) return finish(fail(HK_ERR_NULL_POINTER, "generating tensor is NULL"));
  LevelsRun r;
  Status s = levels_setup(dt, G, m, k, dims, vectors, y != nullptr, alpha != nullptr, &r);
  if (!s.ok()) return finish(s);
  const size_t es = elem_bytes(dt);
  if (!aligned(G, es) || (y && !aligned(y, es)) || (alpha && !aligned(alpha, es)))
    return finish(fail(HK_ERR_MISALIGNED, "pointer not aligned to the element size"));
  for (int p = 0; p < m; ++p)
    if (r.need[p] && !aligned(vectors[p], es))
      return finish(fail(HK_ERR_MISALIGNED, "vector not aligned to the element size"));
  s = check_ws(r.total, ws, ws_bytes);
  if (!s.ok()) return finish(s);
  s = ensure_device();
  if (!s.ok()) return finish(s);
  char *w = (char *)ws;
  Problem q = r.p1;
  q.h = G;
  q.alpha = alpha;
  // embed the distinct vectors (k = 1: the vectors themselves)
  for (int p = 0; p < m; ++p) {
    if (!r.need[p]) continue;
    if (k == 1) {
      q.vec[p] = vectors[p];
      continue;
    }
    if (r.src[p] == p) {
      Levels lv;
      memset(&lv, 0, sizeof(lv));
      lv.k = k;
      int64_t cnt = 1;
      for (int t = 0; t < k; ++t) {
        lv.ext[t] = dims[t * m + p];
        lv.stride[t] = r.S[t];
        cnt *= lv.ext[t];
      }
      count_launch();
      hipError_t e = launch_levels_fill(w + r.off_vec[p], r.L[p], (int)es, stream);
      if (e == hipSuccess) {
        count_launch();
        e = launch_levels_copy(const_cast<void *>(vectors[p]), w + r.off_vec[p], lv, cnt, 0, (int)es, stream);
      }
      if (e != hipSuccess) return finish(fail(HK_ERR_HIP, std::string("level embedding: ") + hipGetErrorString(e)));
    }
    q.vec[p] = w + r.off_vec[r.src[p]];
  }
  q.y = y ? (k == 1 ? y : (void *)(w + r.off_y)) : nullptr;
  Shape sh;
  Ptrs P;
  Sched sc;
  s = prepare(q, 1, &sh, &P, &sc);
  if (!s.ok()) return finish(s);
  P.ws = ws;
  Strides str;
  memset(&str, 0, sizeof(str));
  s = launch_shape(dt, sh, sc, P, str, 1, stream);
  if (!s.ok()) return finish(s);
  if (y && k > 1) {
    Levels lv;
    memset(&lv, 0, sizeof(lv));
    lv.k = k;
    int64_t cnt = 1;
    for (int t = 0; t < k; ++t) {
      lv.ext[t] = dims[t * m];
      lv.stride[t] = r.S[t];
      cnt *= lv.ext[t];
    }
    count_launch();
    hipError_t e = launch_levels_copy(y, w + r.off_y, lv, cnt, 1, (int)es, stream);
    if (e != hipSuccess) return finish(fail(HK_ERR_HIP, std::string("level extraction: ") + hipGetErrorString(e)));
  }
  return finish(Status());
}

hk_status_t hankel_tvp_backward_workspace_size(hk_dtype_t dt, int m, int64_t n, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  // The size with every optional operand present is an upper bound.
  Problem p = bwd_problem(dt, (const void *)16, m, n, (const void *)16, (const void *)16, (const void *)16,
                          (void *)16, (void *)16);
  Status s = validate_backward(p);
  if (!s.ok()) return finish(s);
  return finish(ws_size(p, 1, bytes));
}

hk_status_t hankel_tvp_backward(hk_dtype_t dt, const void *h, int m, int64_t n, const void *x, const void *grad_y,
                                const void *grad_alpha, void *grad_x, void *grad_h, void *ws, size_t ws_bytes,
                                hipStream_t stream) {
  Problem p = bwd_problem(dt, h, m, n, x, grad_y, grad_alpha, grad_x, grad_h);
  Status s = validate_backward(p);
  if (!s.ok()) return finish(s);
  return finish(run_one(p, ws, ws_bytes, stream));
}

// ---------------------------------------------------------------------------
// Strided batches of one shape.
// ---------------------------------------------------------------------------
static Status run_strided(const Problem &p, const Strides &str_elems, int64_t batch, void *ws, size_t ws_bytes,
                          hipStream_t st) {
  if (batch < 0) return fail(HK_ERR_INVALID_VALUE, "batch must be >= 0");
  if (batch == 0) return Status();
  Shape sh;
  Ptrs P;
  Sched sc;
  Status s = prepare(p, batch, &sh, &P, &sc);
  if (!s.ok()) return s;
  const size_t per = instance_ws_bytes(sh, p.dt);
  s = check_ws(per * (size_t)batch, ws, ws_bytes);
  if (!s.ok()) return s;
  s = ensure_device();
  if (!s.ok()) return s;
  P.ws = ws;
  // Map the caller's element strides onto the shape's operand slots.
  Strides str;
  memset(&str, 0, sizeof(str));
  for (int o = 0; o < sh.nops; ++o) str.op[o] = str_elems.op[o];
  str.y = str_elems.y;
  str.alpha = str_elems.alpha;
  str.out1 = str_elems.out1;
  str.phi = str_elems.phi;
  str.ws = (int64_t)per;
  return launch_shape(p.dt, sh, sc, P, str, batch, st);
}

hk_status_t hankel_tvp_strided_batched_workspace_size(hk_dtype_t dt, int m, int64_t n, int64_t batch, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  if (batch < 0) return finish(fail(HK_ERR_INVALID_VALUE, "batch must be >= 0"));
  Problem p = tvp_problem(dt, (const void *)16, m, n, (const void *)16, (void *)16, nullptr);
  Status s = validate_forward(p);
  if (!s.ok()) return finish(s);
  return finish(ws_size(p, batch, bytes));
}

hk_status_t hankel_tvp_strided_batched(hk_dtype_t dt, const void *h, int64_t h_stride, int m, int64_t n, const void *x,
                                       int64_t x_stride, void *y, int64_t y_stride, void *alpha, int64_t batch,
                                       void *ws, size_t ws_bytes, hipStream_t stream) {
  Problem p = tvp_problem(dt, h, m, n, x, y, alpha);
  Status s = validate_forward(p);
  if (!s.ok()) return finish(s);
  const int64_t eb = (int64_t)elem_bytes(dt);
  // Operand order of the equal-vector shape: H, X.
  Strides str;
  memset(&str, 0, sizeof(str));
  str.op[0] = h_stride * eb;
  str.op[1] = x_stride * eb;
  str.y = y_stride * eb;
  str.alpha = eb;
  return finish(run_strided(p, str, batch, ws, ws_bytes, stream));
}

hk_status_t hankel_tvp_backward_strided_batched_workspace_size(hk_dtype_t dt, int m, int64_t n, int64_t batch,
                                                               size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  if (batch < 0) return finish(fail(HK_ERR_INVALID_VALUE, "batch must be >= 0"));
  Problem p = bwd_problem(dt, (const void *)16, m, n, (const void *)16, (const void *)16, (const void *)16,
                          (void *)16, (void *)16);
  Status s = validate_backward(p);
  if (!s.ok()) return finish(s);
  return finish(ws_size(p, batch, bytes));
}

hk_status_t hankel_tvp_backward_strided_batched(hk_dtype_t dt, const void *h, int64_t h_stride, int m, int64_t n,
                                                const void *x, int64_t x_stride, const void *grad_y,
                                                int64_t gy_stride, const void *grad_alpha, void *grad_x,
                                                int64_t gx_stride, void *grad_h, int64_t gh_stride, int64_t batch,
                                                void *ws, size_t ws_bytes, hipStream_t stream) {
  Problem p = bwd_problem(dt, h, m, n, x, grad_y, grad_alpha, grad_x, grad_h);
  Status s = validate_backward(p);
  if (!s.ok()) return finish(s);
  const int64_t eb = (int64_t)elem_bytes(dt);
  // Operand order of the adjoint shape: X, [V], [H].
  Strides str;
  memset(&str, 0, sizeof(str));
  int o = 0;
  str.op[o++] = x_stride * eb;
  if (grad_y) str.op[o++] = gy_stride * eb;
  if (grad_x) str.op[o++] = h_stride * eb;
  str.y = gh_stride * eb;
  str.out1 = gx_stride * eb;
  str.phi = eb;
  return finish(run_strided(p, str, batch, ws, ws_bytes, stream));
}

hk_status_t block_hankel_tvp_strided_batched_workspace_size(hk_dtype_t dt, int m, const int64_t *inner_dims,
                                                            const int64_t *block_dims, int64_t batch, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  if (batch < 0) return finish(fail(HK_ERR_INVALID_VALUE, "batch must be >= 0"));
  const void *vecs[HK_MAX_ORDER];
  for (int q = 0; q < HK_MAX_ORDER; ++q) vecs[q] = (const void *)16;
  Problem p;
  Status s = block_problem(dt, (const void *)16, m, inner_dims, block_dims, vecs, (void *)16, nullptr, &p);
  if (!s.ok()) return finish(s);
  s = validate_forward(p);
  if (!s.ok()) return finish(s);
  return finish(ws_size(p, batch, bytes));
}

hk_status_t block_hankel_tvp_strided_batched(hk_dtype_t dt, const void *H, int64_t H_stride, int m,
                                             const int64_t *inner_dims, const int64_t *block_dims, const void *x,
                                             int64_t x_stride, void *y, int64_t y_stride, void *alpha, int64_t batch,
                                             void *ws, size_t ws_bytes, hipStream_t stream) {
  const void *vecs[HK_MAX_ORDER];
  for (int q = 0; q < HK_MAX_ORDER; ++q) vecs[q] = x;
  Problem p;
  Status s = block_problem(dt, H, m, inner_dims, block_dims, vecs, y, alpha, &p);
  if (!s.ok()) return finish(s);
  if (!alpha) p.vec[0] = x;
  s = validate_forward(p);
  if (!s.ok()) return finish(s);
  if (inner_dims && block_dims)
    for (int q = 1; q < m; ++q)
      if (inner_dims[q] != inner_dims[0] || block_dims[q] != block_dims[0])
        return finish(fail(HK_ERR_INVALID_VALUE, "the strided block batch shares one vector: all modes need equal sizes"));
  const int64_t eb = (int64_t)elem_bytes(dt);
  Strides str;
  memset(&str, 0, sizeof(str));
  str.op[0] = H_stride * eb;
  str.op[1] = x_stride * eb;
  str.y = y_stride * eb;
  str.alpha = eb;
  return finish(run_strided(p, str, batch, ws, ws_bytes, stream));
}

// ---------------------------------------------------------------------------
// Heterogeneous batches and plans.
// ---------------------------------------------------------------------------
hk_status_t hk_plan_create(hk_plan_t *plan, hk_dtype_t dt, const hk_problem_t *probs, int64_t count, unsigned flags) {
  Status s = plan_create(plan, dt, probs, count, flags);
  return finish(s);
}

hk_status_t hk_plan_workspace_size(hk_plan_t plan, size_t *bytes) { return finish(plan_ws_size(plan, bytes)); }

hk_status_t hk_plan_execute(hk_plan_t plan, void *ws, size_t ws_bytes, hipStream_t stream) {
  return finish(plan_execute(plan, ws, ws_bytes, stream));
}

hk_status_t hk_plan_status(hk_plan_t plan) { return finish(plan_status(plan)); }

hk_status_t hk_plan_destroy(hk_plan_t plan) { return finish(plan_destroy(plan)); }

hk_status_t hk_plan_set_wait_bound(hk_plan_t plan, uint32_t spins) { return finish(plan_set_wait_bound(plan, spins)); }

hk_status_t hk_plan_pass_bytes(hk_plan_t plan, int64_t *bytes) { return finish(plan_pass_bytes(plan, bytes)); }

hk_status_t hk_plan_tune_times(hk_plan_t plan, double *ms_default, double *ms_tuned, uint32_t *pow2_buckets) {
  return finish(plan_tune_times(plan, ms_default, ms_tuned, pow2_buckets));
}

hk_status_t hankel_tvp_batched_workspace_size(hk_dtype_t dt, const hk_problem_t *probs, int64_t count, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  hk_plan_t plan = nullptr;
  Status s = plan_create(&plan, dt, probs, count, 0);
  if (!s.ok()) return finish(s);
  s = plan_ws_size(plan, bytes);
  plan_destroy(plan);
  return finish(s);
}

hk_status_t hankel_tvp_batched(hk_dtype_t dt, const hk_problem_t *probs, int64_t count, void *ws, size_t ws_bytes,
                               hipStream_t stream) {
  hk_plan_t plan = nullptr;
  Status s = plan_create(&plan, dt, probs, count, 0);
  if (!s.ok()) return finish(s);
  plan_set_oneshot(plan);
  s = plan_execute(plan, ws, ws_bytes, stream);
  if (s.ok())
    s = plan_release_after(plan, stream);
  else
    plan_destroy(plan);
  return finish(s);
}

// Batches of one product kind: the heterogeneous batch after a check that
// every problem is of that kind (1D general Hankel tensors or BHHB tensors).
static Status check_kind(const hk_problem_t *probs, int64_t count, int is_block) {
  if (count > 0 && !probs) return fail(HK_ERR_NULL_POINTER, "probs is NULL");
  for (int64_t i = 0; i < count; ++i)
    if ((probs[i].is_block != 0) != (is_block != 0))
      return fail(HK_ERR_INVALID_VALUE, is_block ? "problem " + std::to_string(i) + " is not a BHHB product"
                                                 : "problem " + std::to_string(i) + " is a BHHB product");
  return Status();
}

hk_status_t hankel_mode_products_batched_workspace_size(hk_dtype_t dt, const hk_problem_t *probs, int64_t count,
                                                        size_t *bytes) {
  Status s = check_kind(probs, count, 0);
  if (!s.ok()) return finish(s);
  return hankel_tvp_batched_workspace_size(dt, probs, count, bytes);
}

hk_status_t hankel_mode_products_batched(hk_dtype_t dt, const hk_problem_t *probs, int64_t count, void *ws,
                                         size_t ws_bytes, hipStream_t stream) {
  Status s = check_kind(probs, count, 0);
  if (!s.ok()) return finish(s);
  return hankel_tvp_batched(dt, probs, count, ws, ws_bytes, stream);
}

hk_status_t block_hankel_tvp_batched_workspace_size(hk_dtype_t dt, const hk_problem_t *probs, int64_t count,
                                                    size_t *bytes) {
  Status s = check_kind(probs, count, 1);
  if (!s.ok()) return finish(s);
  return hankel_tvp_batched_workspace_size(dt, probs, count, bytes);
}

hk_status_t block_hankel_tvp_batched(hk_dtype_t dt, const hk_problem_t *probs, int64_t count, void *ws,
                                     size_t ws_bytes, hipStream_t stream) {
  Status s = check_kind(probs, count, 1);
  if (!s.ok()) return finish(s);
  return hankel_tvp_batched(dt, probs, count, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// Hankel tensor-matrix product T = H x_2 U ... x_m U (square H, the same U in
// modes 2..m).  Column (j_2, ..., j_m) of T is the mode product with the
// columns U[:, j_2], ..., U[:, j_m]; it is symmetric in the j's, so only the
// nondecreasing tuples are computed (one grouped batch of mode products) and
// the other columns are copies.
// ---------------------------------------------------------------------------
struct TmLayout {
  std::vector<hk_problem_t> probs;      // one per nondecreasing tuple
  std::vector<int32_t> pairs;           // (dst column, src column) for the others
};

static Status tm_layout(hk_dtype_t dt, const void *h, int m, int64_t n, int64_t R, const void *U, void *out,
                        TmLayout *L) {
  if (m < 2 || m > HK_MAX_ORDER) return fail(HK_ERR_INVALID_VALUE, "order m must be in [2, 8]");
  if (n < 1 || R < 1) return fail(HK_ERR_INVALID_VALUE, "n and R must be >= 1");
  int64_t ncols = 1;
  for (int p = 1; p < m; ++p) {
    ncols *= R;
    if (ncols > (1 << 20)) return fail(HK_ERR_SIZE_LIMIT, "R^(m-1) exceeds 2^20 columns");
  }
  if (!h || !U || !out) return fail(HK_ERR_NULL_POINTER, "h, U or out is NULL");
  if (dt < HK_C64 || dt > HK_F64) return fail(HK_ERR_INVALID_VALUE, "unknown dtype");
  const size_t eb = elem_bytes(dt);
  std::vector<int64_t> canon_of(ncols, -1);
  std::vector<int> j(m - 1);
  for (int64_t c = 0; c < ncols; ++c) {
    int64_t r = c;
    for (int p = 0; p < m - 1; ++p) {
      j[p] = (int)(r % R);
      r /= R;
    }
    std::vector<int> s = j;
    std::sort(s.begin(), s.end());
    int64_t cc = 0;
    for (int p = m - 2; p >= 0; --p) cc = cc * R + s[p];
    canon_of[c] = cc;
    if (cc == c) {
      hk_problem_t q;
      memset(&q, 0, sizeof(q));
      q.m = m;
      for (int p = 0; p < m; ++p) q.dims[p] = n;
      q.h = h;
      for (int p = 1; p < m; ++p) q.vectors[p] = (const char *)U + (size_t)j[p - 1] * n * eb;
      q.y = (char *)out + (size_t)c * n * eb;
      L->probs.push_back(q);
    }
  }
  for (int64_t c = 0; c < ncols; ++c)
    if (canon_of[c] != c) {
      L->pairs.push_back((int32_t)c);
      L->pairs.push_back((int32_t)canon_of[c]);
    }
  return Status();
}

// Tensor-matrix product from spectra (complex dtypes, three-pass layouts):
// h^ once, the R columns of U once, then for every nondecreasing tuple the
// product of its spectra and one output transform (the grouped batch of mode
// products transforms h and the tuple's columns again for every column of T).
// All tuples run in one strided launch per pass: operand t of tuple k is the
// spectrum of U[:, s_{t-1}(k)], looked up in a per-operand pointer table, and
// the outputs go to a staging area from which one gather fills every column
// of T (the symmetric ones included).
// Workspace: [h^ | U^ (R spectra) | B instances | staging (K columns) |
//             pointer tables ((m-1) K) | gather pairs (2 R^(m-1))].
struct TmSpectral {
  Layout lay;
  Sched sc;
  int64_t N = 0, K = 0, ncols = 0;
  int64_t batch = 0;    // instances per launch
  size_t inst_ws = 0;   // bytes per instance
  size_t off_u = 0, off_inst = 0, off_stage = 0, off_tab = 0, off_pairs = 0, bytes = 0;
  std::vector<int32_t> digits;  // K x (m-1) nondecreasing digits, tuple-major
  std::vector<int32_t> pairs;   // (column of T, tuple) for every column
};

static bool tm_spectral_plan(hk_dtype_t dt, int m, int64_t n, int64_t R, TmSpectral *T) {
  if (R < 1 || m < 2 || m > HK_MAX_ORDER) return false;
  int64_t dims[HK_MAX_ORDER];
  for (int q = 0; q < m; ++q) dims[q] = n;
  Shape sh;
  Ptrs P;
  Sched sc;
  if (!spectrum_prepare(dt, m, dims, -1, nullptr, nullptr, &sh, &P, &sc).ok()) return false;
  Problem p;
  if (!spectral_problem(dt, m, dims, &p).ok() || !spectral_setup(p, &T->lay, &T->sc).ok()) return false;
  T->N = (int64_t)1 << (T->lay.logR + T->lay.logC);
  // the product program (all operands spectra) needs one buffer, as the
  // spectrum program does
  T->inst_ws = instance_ws_bytes(sh, dt);
  int64_t ncols = 1;
  for (int q = 1; q < m; ++q) ncols *= R;
  if (ncols > (1 << 20)) return false;
  T->ncols = ncols;
  // tuples: the columns whose digits (least significant first) are nondecreasing
  const int d = m - 1;
  std::vector<int32_t> tuple_of(ncols, -1), j(d);
  T->digits.clear();
  for (int64_t c = 0; c < ncols; ++c) {
    int64_t r = c;
    bool sorted = true;
    for (int q = 0; q < d; ++q) {
      j[q] = (int32_t)(r % R);
      r /= R;
      if (q > 0 && j[q] < j[q - 1]) sorted = false;
    }
    if (sorted) {
      tuple_of[c] = (int32_t)(T->digits.size() / d);
      T->digits.insert(T->digits.end(), j.begin(), j.end());
    }
  }
  T->K = (int64_t)(T->digits.size() / d);
  // Below about 2^21 spectral elements of products the launches, not the
  // transforms, set the time, and the grouped batch (fewer launches) is
  // as fast or faster.
  if (T->K * T->N < ((int64_t)1 << 21)) return false;
  T->pairs.resize(2 * ncols);
  for (int64_t c = 0; c < ncols; ++c) {
    int64_t r = c;
    for (int q = 0; q < d; ++q) {
      j[q] = (int32_t)(r % R);
      r /= R;
    }
    std::sort(j.begin(), j.end());
    int64_t cc = 0;
    for (int q = d - 1; q >= 0; --q) cc = cc * R + j[q];
    T->pairs[2 * c] = (int32_t)c;
    T->pairs[2 * c + 1] = tuple_of[cc];
  }
  const size_t eb = elem_bytes(dt), cb = cplx_bytes(dt);
  T->batch = std::max<int64_t>(1, std::min<int64_t>({T->K, (int64_t)(((size_t)256 << 20) / T->inst_ws), 65535}));
  T->off_u = align256((size_t)T->N * cb);
  T->off_inst = T->off_u + align256((size_t)R * (size_t)T->N * cb);
  T->off_stage = T->off_inst + (size_t)T->batch * T->inst_ws;
  T->off_tab = T->off_stage + align256((size_t)T->K * (size_t)n * eb);
  T->off_pairs = T->off_tab + align256((size_t)d * (size_t)T->K * sizeof(void *));
  T->bytes = T->off_pairs + align256((size_t)T->pairs.size() * sizeof(int32_t));
  return T->bytes <= ((size_t)8 << 30);
}

static Status tm_spectral_run(const TmSpectral &T, hk_dtype_t dt, const void *h, int m, int64_t n, int64_t R,
                              const void *U, void *out, char *ws, hipStream_t st) {
  const size_t eb = elem_bytes(dt), cb = cplx_bytes(dt);  // vectors and outputs / spectra
  const int64_t N = T.N, K = T.K;
  const int d = m - 1;
  char *hspec = ws, *uspec = ws + T.off_u, *inst = ws + T.off_inst, *stage = ws + T.off_stage;
  const void **tab = (const void **)(ws + T.off_tab);
  int32_t *dpairs = (int32_t *)(ws + T.off_pairs);
  int64_t dims[HK_MAX_ORDER];
  for (int q = 0; q < m; ++q) dims[q] = n;
  // tables: operand t of tuple k -> spectrum of U[:, digit t-1 of k]
  std::vector<const void *> htab((size_t)d * K);
  for (int t = 0; t < d; ++t)
    for (int64_t k = 0; k < K; ++k) htab[(size_t)t * K + k] = uspec + (size_t)T.digits[(size_t)k * d + t] * N * cb;
  hipError_t e = hipMemcpyAsync(tab, htab.data(), htab.size() * sizeof(void *), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dpairs, T.pairs.data(), T.pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(HK_ERR_HIP, std::string("tensor-matrix tables: ") + hipGetErrorString(e));
  Shape sh;
  Ptrs P;
  Sched sc;
  Strides str;
  // h^
  Status s = spectrum_prepare(dt, m, dims, -1, h, hspec, &sh, &P, &sc);
  if (s.ok()) {
    P.ws = inst;
    memset(&str, 0, sizeof(str));
    s = launch_shape(dt, sh, sc, P, str, 1, st);
  }
  // the spectra of the columns of U
  if (s.ok()) s = spectrum_prepare(dt, m, dims, 1, U, uspec, &sh, &P, &sc);
  if (s.ok()) {
    str.op[0] = n * (int64_t)eb;
    str.out1 = N * (int64_t)cb;
    str.ws = (int64_t)T.inst_ws;
    for (int64_t c0 = 0; c0 < R && s.ok(); c0 += T.batch) {
      Ptrs Pc = P;
      Pc.op[0] = (const char *)U + (size_t)c0 * n * eb;
      Pc.out1 = uspec + (size_t)c0 * N * cb;
      Pc.ws = inst;
      s = launch_shape(dt, sh, sc, Pc, str, std::min(T.batch, R - c0), st);
    }
  }
  // every tuple: h^ times the m - 1 spectra of its digits (not merged, so
  // that all tuples share one shape), the output transform, to the staging
  if (s.ok()) {
    Problem q;
    q.dt = dt;
    q.prog = PROG_FWD;
    q.m = m;
    for (int t = 0; t < m; ++t) q.dims[t] = n;
    q.h = hspec;
    q.h_spec = true;
    for (int t = 1; t < m; ++t) {
      q.vec[t] = (const void *)(uintptr_t)(256 * t);  // distinct placeholders: one operand per mode
      q.spec_mask |= 1u << t;
    }
    q.y = stage;
    int op_src[MAXOPS];
    s = build_shape(q, T.lay, T.sc, &sh, &P, op_src);
    if (s.ok() && sh.nops != m) s = fail(HK_ERR_NOT_SUPPORTED, "tensor-matrix operand layout");
    for (int64_t k0 = 0; k0 < K && s.ok(); k0 += T.batch) {
      Ptrs Pk = P;
      memset(&str, 0, sizeof(str));
      for (int o = 1; o < sh.nops; ++o) {
        Pk.op[o] = tab + (size_t)(op_src[o] - 1) * K + k0;
        str.op[o] = OP_TABLE;
      }
      Pk.y = stage + (size_t)k0 * n * eb;
      str.y = n * (int64_t)eb;
      Pk.ws = inst;
      str.ws = (int64_t)T.inst_ws;
      s = launch_shape(dt, sh, T.sc, Pk, str, std::min(T.batch, K - k0), st);
    }
  }
  if (s.ok()) {
    count_launch();
    const bool dbl = dt == HK_C128 || dt == HK_F64;
    e = dbl ? launch_copy_cols_f64(out, stage, dpairs, T.ncols, n, is_complex(dt), st)
            : launch_copy_cols_f32(out, stage, dpairs, T.ncols, n, is_complex(dt), st);
    if (e != hipSuccess) s = fail(HK_ERR_HIP, std::string("tensor-matrix gather: ") + hipGetErrorString(e));
  }
  // the host copies of the tables must outlive the transfers enqueued above
  e = hipStreamSynchronize(st);
  if (s.ok() && e != hipSuccess) s = fail(HK_ERR_HIP, std::string("stream synchronize: ") + hipGetErrorString(e));
  return s;
}

// The columns of T that are not nondecreasing tuples: copies of their
// canonical column (the pair table goes to the workspace first).
static Status tm_copy_pairs(hk_dtype_t dt, const TmLayout &L, int64_t n, void *out, char *dst, hipStream_t stream) {
  int32_t *dpairs = (int32_t *)dst;
  hipError_t e =
      hipMemcpyAsync(dpairs, L.pairs.data(), L.pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
  const bool cplx = is_complex(dt);
  const bool dbl = dt == HK_C128 || dt == HK_F64;
  if (e == hipSuccess) {
    count_launch();
    e = dbl ? launch_copy_cols_f64(out, out, dpairs, (int64_t)(L.pairs.size() / 2), n, cplx, stream)
            : launch_copy_cols_f32(out, out, dpairs, (int64_t)(L.pairs.size() / 2), n, cplx, stream);
  }
  if (e != hipSuccess) return fail(HK_ERR_HIP, std::string("symmetric completion: ") + hipGetErrorString(e));
  return Status();
}

hk_status_t hankel_tensor_matrix_workspace_size(hk_dtype_t dt, int m, int64_t n, int64_t R, size_t *bytes) {
  if (!bytes) return finish(fail(HK_ERR_NULL_POINTER, "bytes is NULL"));
  TmLayout L;
  const void *dummy = (const void *)256;
  Status s = tm_layout(dt, dummy, m, n, R, dummy, (void *)256, &L);
  if (!s.ok()) return finish(s);
  TmSpectral T;
  if (tm_spectral_plan(dt, m, n, R, &T)) {
    *bytes = T.bytes;
    return finish(Status());
  }
  hk_plan_t plan = nullptr;
  s = plan_create(&plan, dt, L.probs.data(), (int64_t)L.probs.size(), 0);
  if (!s.ok()) return finish(s);
  size_t pb = 0;
  s = plan_ws_size(plan, &pb);
  plan_destroy(plan);
  if (!s.ok()) return finish(s);
  *bytes = ((pb + 255) & ~(size_t)255) + L.pairs.size() * sizeof(int32_t) + 256;
  return finish(Status());
}

hk_status_t hankel_tensor_matrix(hk_dtype_t dt, const void *h, int m, int64_t n, int64_t R, const void *U,
                                 void *out, void *ws, size_t ws_bytes, hipStream_t stream) {
  TmLayout L;
  Status s = tm_layout(dt, h, m, n, R, U, out, &L);
  if (!s.ok()) return finish(s);
  TmSpectral T;
  if (tm_spectral_plan(dt, m, n, R, &T)) {
    const size_t need = T.bytes;
    if (!ws || ws_bytes < need)
      return finish(fail(HK_ERR_WORKSPACE, "workspace smaller than hankel_tensor_matrix_workspace_size"));
    if (((uintptr_t)ws) % 256 != 0) return finish(fail(HK_ERR_MISALIGNED, "workspace must be 256-byte aligned"));
    const size_t a = elem_bytes(dt);
    if (!aligned(h, a) || !aligned(U, a) || !aligned(out, a))
      return finish(fail(HK_ERR_MISALIGNED, "pointer not aligned to the element size"));
    s = ensure_device();
    if (!s.ok()) return finish(s);
    return finish(tm_spectral_run(T, dt, h, m, n, R, U, out, (char *)ws, stream));
  }
  hk_plan_t plan = nullptr;
  s = plan_create(&plan, dt, L.probs.data(), (int64_t)L.probs.size(), 0);
  if (!s.ok()) return finish(s);
  size_t pb = 0;
  plan_ws_size(plan, &pb);
  const size_t pairs_off = (pb + 255) & ~(size_t)255;
  const size_t need = pairs_off + L.pairs.size() * sizeof(int32_t) + 256;
  if (!ws || ws_bytes < need) {
    plan_destroy(plan);
    return finish(fail(HK_ERR_WORKSPACE, "workspace smaller than hankel_tensor_matrix_workspace_size"));
  }
  plan_set_oneshot(plan);
  s = plan_execute(plan, ws, ws_bytes, stream);
  if (s.ok() && !L.pairs.empty()) s = tm_copy_pairs(dt, L, n, out, (char *)ws + pairs_off, stream);
  // the host tables (plan and pairs) must outlive the copies enqueued above
  if (s.ok())
    s = plan_release_after(plan, stream);
  else {
    (void)hipStreamSynchronize(stream);
    plan_destroy(plan);
  }
  return finish(s);
}

hk_status_t hk_profile_start(void) { return finish(prof_start()); }

hk_status_t hk_profile_stop(double *ms_by_kind, int64_t *launches_by_kind) {
  if (!ms_by_kind || !launches_by_kind) return finish(fail(HK_ERR_NULL_POINTER, "output array is NULL"));
  return finish(prof_stop(ms_by_kind, launches_by_kind));
}

hk_status_t hk_autotune_tvp(hk_dtype_t dt, int m, int64_t n, int verbose) {
  return finish(autotune_tvp(dt, m, n, verbose != 0));
}

hk_status_t hk_tune_save(const char *path) { return finish(sched_save(path)); }

hk_status_t hk_tune_load(const char *path, int *n_loaded) { return finish(sched_load(path, n_loaded)); }

hk_status_t hk_autotune(hk_dtype_t dt, int kind, int m, int64_t n, const int64_t *inner_dims,
                        const int64_t *block_dims, int64_t batch, int verbose) {
  if (kind == 2 && (!inner_dims || !block_dims)) return finish(fail(HK_ERR_NULL_POINTER, "block dims are NULL"));
  return finish(autotune_shape(dt, kind, m, n, inner_dims, block_dims, batch, verbose != 0));
}

}  // extern "C"
