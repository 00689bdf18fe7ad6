/*
 * Test oracle for the fast Hankel tensor-vector product (TEST INFRASTRUCTURE).
 *
 * This file is the plain, slow CPU definition that the GPU library is checked
 * against.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline load it; the product library never links, calls or falls back to
 * it, and it shares no code with the GPU path (no FFT anywhere in here).
 *
 * What it computes (paper, Section 1 definition of a Hankel tensor and
 * Section 2.1 definition of the mode-p product, Section 3 statement of the two
 * product types):
 *
 *   H_{i_1..i_m} = h_{i_1+...+i_m},  0 <= i_p < n_p,  len(h) = d_H = sum n_p - m + 1
 *   y   = H x_2 ... x_m   (mode 1 free):  y_i = sum_{i_2..i_m} h_{i+i_2+..+i_m} prod_p x_{p,i_p}
 *   alpha = H x_1 x_2 ... x_m
 *
 * Grouping the sum by s = i_2+...+i_m turns the inner product over index
 * tuples into the linear convolution w = x_2 * x_3 * ... * x_m followed by the
 * correlation y_i = sum_k h_{i+k} w_k (k < len(w) = d_H - n_1 + 1).  The scalar
 * is alpha = sum_s h_s u_s with u = x_1 * w.  Both are the definition with
 * the terms of each output gathered by the value of the index sum; nothing is
 * transformed.  The 2-level block (BHHB) case (Section 2.2 generating matrix,
 * Section 3 BHHB procedure) is the same with 2D convolutions: the entry of the
 * block tensor at in-block indices (i_p) and block indices (j_p) is
 * H[sum i_p, sum j_p], and mode-p vectors are un-vectorized column-major into
 * n_p x N_p matrices.
 *
 * Gradients (the paper does not treat differentiation): for the equal-vector
 * products g = H x^{m-1} and f = H x^m with cotangents v (for g) and phi
 * (for f), the functions below return the conjugate-transposed Jacobian
 * applied to the cotangents, J^H [v; phi], the convention of complex autograd
 * for holomorphic maps:
 *   grad_h[s] = sum_i conj(w_{s-i}) v_i + phi conj(u_s)        (w = x^{*(m-1)}, u = x^{*m})
 *   grad_x[l] = (m-1) conj( sum_k h_{l+k} c_k ) + m phi conj(g_l)   (c = conj(v) * x^{*(m-2)})
 *
 * Compensated mode (hko_tvp_comp): the same sums with every product split
 * exactly by an FMA (TwoProduct) and added by Neumaier's TwoSum, i.e. the
 * Dot2 algorithm of Ogita, Rump and Oishi: each convolution and correlation
 * as if computed in twice the working precision.  It measures the rounding
 * error of the blocked sums on small and medium sizes.
 *
 * Spectra: the fast procedures of Section 3 multiply h^ = ifft(pad_N h) and
 * x^ = fft(pad_N x).  hko_dft_sampled evaluates these two transforms at listed
 * bins as plain DFT sums (a sum over the samples per bin, with the phase
 * index j s reduced mod N exactly in integers); it is not an FFT.
 *
 * Arithmetic: FP64 (complex as interleaved re/im pairs).  Long sums are
 * accumulated in consecutive blocks of 256 terms whose partial sums are then
 * added in order, which keeps the rounding error of sums of ~10^6 terms well
 * under 1e-12 relative.  A complex int64 variant of the 1D and BHHB products
 * gives bit-exact results for small integer inputs.
 *
 * OpenMP is used only to split independent outputs across threads; each output
 * is always summed in the same order, so results do not depend on the thread
 * count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } hkc;
typedef struct { int64_t re, im; } hki;

#define BLOCK 256

static inline hkc cmul(hkc a, hkc b) {
    hkc r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}
static inline hkc cadd(hkc a, hkc b) { hkc r = { a.re + b.re, a.im + b.im }; return r; }
static inline hkc cconj(hkc a) { hkc r = { a.re, -a.im }; return r; }
static inline hkc cscale(hkc a, double s) { hkc r = { a.re * s, a.im * s }; return r; }

static inline hki imul(hki a, hki b) {
    hki r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}

static int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }
static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

int hko_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (n >= 1); returns the previous count. */
int hko_set_threads(int n) {
    const int prev = hko_max_threads();
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#endif
    return prev;
}

/* ------------------------------------------------------------------------ */
/* 1D linear convolution: out_k = sum_j a_j b_{k-j}, for k in [k0, k1).      */
/* ------------------------------------------------------------------------ */
int hko_conv_range(const hkc *a, int64_t na, const hkc *b, int64_t nb,
                   int64_t k0, int64_t k1, hkc *out) {
    if (na < 1 || nb < 1 || k0 < 0 || k1 > na + nb - 1 || k0 > k1) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = k0; k < k1; ++k) {
        int64_t jlo = max64(0, k - (nb - 1));
        int64_t jhi = min64(k, na - 1);
        hkc total = { 0.0, 0.0 }, part = { 0.0, 0.0 };
        int cnt = 0;
        for (int64_t j = jlo; j <= jhi; ++j) {
            part = cadd(part, cmul(a[j], b[k - j]));
            if (++cnt == BLOCK) { total = cadd(total, part); part.re = part.im = 0.0; cnt = 0; }
        }
        out[k - k0] = cadd(total, part);
    }
    return 0;
}

int hko_conv(const hkc *a, int64_t na, const hkc *b, int64_t nb, hkc *out) {
    return hko_conv_range(a, na, b, nb, 0, na + nb - 1, out);
}

/* Correlation with the generating vector: y_i = sum_{k<lw} h_{i+k} w_k, for the
 * listed output indices (requires i + lw - 1 < dh). */
static int corr_indices(const hkc *h, int64_t dh, const hkc *w, int64_t lw,
                        const int64_t *idx, int64_t nidx, hkc *y) {
    for (int64_t t = 0; t < nidx; ++t)
        if (idx[t] < 0 || idx[t] + lw - 1 >= dh) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nidx; ++t) {
        const hkc *hp = h + idx[t];
        hkc total = { 0.0, 0.0 }, part = { 0.0, 0.0 };
        int cnt = 0;
        for (int64_t k = 0; k < lw; ++k) {
            part = cadd(part, cmul(hp[k], w[k]));
            if (++cnt == BLOCK) { total = cadd(total, part); part.re = part.im = 0.0; cnt = 0; }
        }
        y[t] = cadd(total, part);
    }
    return 0;
}

int hko_corr(const hkc *h, int64_t dh, const hkc *w, int64_t lw, int64_t ny, hkc *y) {
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)max64(ny, 1));
    if (!idx) return -2;
    for (int64_t i = 0; i < ny; ++i) idx[i] = i;
    int rc = corr_indices(h, dh, w, lw, idx, ny, y);
    free(idx);
    return rc;
}

/* Plain sum of a[s] * b[s] (blocked), s < n. */
static hkc dot_plain(const hkc *a, const hkc *b, int64_t n) {
    hkc total = { 0.0, 0.0 }, part = { 0.0, 0.0 };
    int cnt = 0;
    for (int64_t s = 0; s < n; ++s) {
        part = cadd(part, cmul(a[s], b[s]));
        if (++cnt == BLOCK) { total = cadd(total, part); part.re = part.im = 0.0; cnt = 0; }
    }
    return cadd(total, part);
}

/* w = x_{first} * x_{first+1} * ... * x_{m-1}  (vectors[p] has length dims[p]).
 * Returns a malloc'd array and its length; a product of zero vectors is the
 * unit impulse [1]. */
static hkc *conv_chain(int first, int m, const int64_t *dims, const hkc *const *vectors, int64_t *len_out) {
    int64_t len = 1;
    hkc *w = (hkc *)malloc(sizeof(hkc));
    if (!w) return NULL;
    w[0].re = 1.0; w[0].im = 0.0;
    for (int p = first; p < m; ++p) {
        int64_t nl = len + dims[p] - 1;
        hkc *nw = (hkc *)malloc(sizeof(hkc) * (size_t)nl);
        if (!nw) { free(w); return NULL; }
        if (p == first) {
            memcpy(nw, vectors[p], sizeof(hkc) * (size_t)dims[p]);
        } else {
            hko_conv(w, len, vectors[p], dims[p], nw);
        }
        free(w);
        w = nw;
        len = nl;
    }
    *len_out = len;
    return w;
}

static int check_dims(int m, const int64_t *dims) {
    if (m < 2 || m > 16) return -1;
    for (int p = 0; p < m; ++p) if (dims[p] < 1) return -1;
    return 0;
}

/* y = H x_2 ... x_m at output indices idx (nullable when nidx == 0) and/or
 * alpha = H x_1 ... x_m (alpha nullable; needs vectors[0]). */
int hko_tvp_sampled(int m, const int64_t *dims, const hkc *h, const hkc *const *vectors,
                    const int64_t *idx, int64_t nidx, hkc *y, hkc *alpha) {
    if (check_dims(m, dims)) return -1;
    int64_t dh = 1 - m;
    for (int p = 0; p < m; ++p) dh += dims[p];
    int64_t lw = 0;
    hkc *w = conv_chain(1, m, dims, vectors, &lw);
    if (!w) return -2;
    int rc = 0;
    if (nidx > 0) {
        for (int64_t t = 0; t < nidx; ++t) if (idx[t] >= dims[0]) { free(w); return -1; }
        rc = corr_indices(h, dh, w, lw, idx, nidx, y);
    }
    if (rc == 0 && alpha) {
        /* u = x_1 * w has length d_H; alpha = sum_s h_s u_s */
        hkc *u = (hkc *)malloc(sizeof(hkc) * (size_t)dh);
        if (!u) { free(w); return -2; }
        hko_conv(vectors[0], dims[0], w, lw, u);
        *alpha = dot_plain(h, u, dh);
        free(u);
    }
    free(w);
    return rc;
}

int hko_tvp(int m, const int64_t *dims, const hkc *h, const hkc *const *vectors, hkc *y, hkc *alpha) {
    if (check_dims(m, dims)) return -1;
    int64_t n1 = y ? dims[0] : 0;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)max64(n1, 1));
    if (!idx) return -2;
    for (int64_t i = 0; i < n1; ++i) idx[i] = i;
    int rc = hko_tvp_sampled(m, dims, h, vectors, idx, n1, y, alpha);
    free(idx);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Exact complex-int64 1D product (small integer inputs).                   */
/* ------------------------------------------------------------------------ */
static hki *iconv(const hki *a, int64_t na, const hki *b, int64_t nb) {
    hki *out = (hki *)calloc((size_t)(na + nb - 1), sizeof(hki));
    if (!out) return NULL;
    for (int64_t i = 0; i < na; ++i)
        for (int64_t j = 0; j < nb; ++j) {
            hki t = imul(a[i], b[j]);
            out[i + j].re += t.re;
            out[i + j].im += t.im;
        }
    return out;
}

int hko_tvp_i64(int m, const int64_t *dims, const hki *h, const hki *const *vectors, hki *y, hki *alpha) {
    if (check_dims(m, dims)) return -1;
    int64_t dh = 1 - m;
    for (int p = 0; p < m; ++p) dh += dims[p];
    hki *w = (hki *)calloc(1, sizeof(hki));
    if (!w) return -2;
    w[0].re = 1;
    int64_t lw = 1;
    for (int p = 1; p < m; ++p) {
        hki *nw = iconv(w, lw, vectors[p], dims[p]);
        free(w);
        if (!nw) return -2;
        w = nw;
        lw += dims[p] - 1;
    }
    if (y) {
        for (int64_t i = 0; i < dims[0]; ++i) {
            hki acc = { 0, 0 };
            for (int64_t k = 0; k < lw; ++k) {
                hki t = imul(h[i + k], w[k]);
                acc.re += t.re; acc.im += t.im;
            }
            y[i] = acc;
        }
    }
    if (alpha) {
        hki *u = iconv(vectors[0], dims[0], w, lw);
        if (!u) { free(w); return -2; }
        hki acc = { 0, 0 };
        for (int64_t s = 0; s < dh; ++s) {
            hki t = imul(h[s], u[s]);
            acc.re += t.re; acc.im += t.im;
        }
        *alpha = acc;
        free(u);
    }
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 2-level block Hankel (BHHB).  Matrices are column-major: A[r + rows*c].   */
/* ------------------------------------------------------------------------ */
static hkc *conv2(const hkc *a, int64_t ar, int64_t ac, const hkc *b, int64_t br, int64_t bc) {
    int64_t orr = ar + br - 1, oc = ac + bc - 1;
    hkc *out = (hkc *)malloc(sizeof(hkc) * (size_t)(orr * oc));
    if (!out) return NULL;
#pragma omp parallel for collapse(2) schedule(dynamic, 64)
    for (int64_t c = 0; c < oc; ++c)
        for (int64_t r = 0; r < orr; ++r) {
            hkc total = { 0.0, 0.0 }, part = { 0.0, 0.0 };
            int cnt = 0;
            for (int64_t jc = max64(0, c - (bc - 1)); jc <= min64(c, ac - 1); ++jc)
                for (int64_t jr = max64(0, r - (br - 1)); jr <= min64(r, ar - 1); ++jr) {
                    part = cadd(part, cmul(a[jr + ar * jc], b[(r - jr) + br * (c - jc)]));
                    if (++cnt == BLOCK) { total = cadd(total, part); part.re = part.im = 0.0; cnt = 0; }
                }
            out[r + orr * c] = cadd(total, part);
        }
    return out;
}

int hko_block_tvp(int m, const int64_t *n, const int64_t *nblk, const hkc *H,
                  const hkc *const *vectors, hkc *y, hkc *alpha) {
    if (check_dims(m, n) || check_dims(m, nblk)) return -1;
    int64_t hr = 1 - m, hcols = 1 - m;
    for (int p = 0; p < m; ++p) { hr += n[p]; hcols += nblk[p]; }
    /* W = X_2 (*) ... (*) X_m, 2D linear convolution */
    int64_t wr = 1, wc = 1;
    hkc *w = (hkc *)malloc(sizeof(hkc));
    if (!w) return -2;
    w[0].re = 1.0; w[0].im = 0.0;
    for (int p = 1; p < m; ++p) {
        hkc *nw = conv2(w, wr, wc, vectors[p], n[p], nblk[p]);
        free(w);
        if (!nw) return -2;
        w = nw;
        wr += n[p] - 1;
        wc += nblk[p] - 1;
    }
    if (y) {
        /* Y[i, j] = sum_{k,l} H[i+k, j+l] W[k, l];  y = vec(Y), Y is n_1 x N_1 */
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
        for (int64_t j = 0; j < nblk[0]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                hkc total = { 0.0, 0.0 }, part = { 0.0, 0.0 };
                int cnt = 0;
                for (int64_t l = 0; l < wc; ++l)
                    for (int64_t k = 0; k < wr; ++k) {
                        part = cadd(part, cmul(H[(i + k) + hr * (j + l)], w[k + wr * l]));
                        if (++cnt == BLOCK) { total = cadd(total, part); part.re = part.im = 0.0; cnt = 0; }
                    }
                y[i + n[0] * j] = cadd(total, part);
            }
    }
    if (alpha) {
        hkc *u = conv2(vectors[0], n[0], nblk[0], w, wr, wc); /* hr x hcols */
        if (!u) { free(w); return -2; }
        *alpha = dot_plain(H, u, hr * hcols);
        free(u);
    }
    free(w);
    return 0;
}

/* BHHB product at the listed output indices only (flat column-major indices
 * into the n_1 x N_1 result), and/or the scalar.  Same sums as
 * hko_block_tvp. */
int hko_block_tvp_sampled(int m, const int64_t *n, const int64_t *nblk, const hkc *H,
                          const hkc *const *vectors, const int64_t *idx, int64_t nidx,
                          hkc *y, hkc *alpha) {
    if (check_dims(m, n) || check_dims(m, nblk)) return -1;
    for (int64_t t = 0; t < nidx; ++t)
        if (idx[t] < 0 || idx[t] >= n[0] * nblk[0]) return -1;
    int64_t hr = 1 - m, hcols = 1 - m;
    for (int p = 0; p < m; ++p) { hr += n[p]; hcols += nblk[p]; }
    int64_t wr = 1, wc = 1;
    hkc *w = (hkc *)malloc(sizeof(hkc));
    if (!w) return -2;
    w[0].re = 1.0; w[0].im = 0.0;
    for (int p = 1; p < m; ++p) {
        hkc *nw = conv2(w, wr, wc, vectors[p], n[p], nblk[p]);
        free(w);
        if (!nw) return -2;
        w = nw;
        wr += n[p] - 1;
        wc += nblk[p] - 1;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nidx; ++t) {
        const int64_t i = idx[t] % n[0], j = idx[t] / n[0];
        hkc total = { 0.0, 0.0 }, part = { 0.0, 0.0 };
        int cnt = 0;
        for (int64_t l = 0; l < wc; ++l)
            for (int64_t k = 0; k < wr; ++k) {
                part = cadd(part, cmul(H[(i + k) + hr * (j + l)], w[k + wr * l]));
                if (++cnt == BLOCK) { total = cadd(total, part); part.re = part.im = 0.0; cnt = 0; }
            }
        y[t] = cadd(total, part);
    }
    if (alpha) {
        hkc *u = conv2(vectors[0], n[0], nblk[0], w, wr, wc);
        if (!u) { free(w); return -2; }
        *alpha = dot_plain(H, u, hr * hcols);
        free(u);
    }
    free(w);
    return 0;
}

static hki *iconv2(const hki *a, int64_t ar, int64_t ac, const hki *b, int64_t br, int64_t bc) {
    int64_t orr = ar + br - 1, oc = ac + bc - 1;
    hki *out = (hki *)calloc((size_t)(orr * oc), sizeof(hki));
    if (!out) return NULL;
    for (int64_t ac_ = 0; ac_ < ac; ++ac_)
        for (int64_t ar_ = 0; ar_ < ar; ++ar_)
            for (int64_t bc_ = 0; bc_ < bc; ++bc_)
                for (int64_t br_ = 0; br_ < br; ++br_) {
                    hki t = imul(a[ar_ + ar * ac_], b[br_ + br * bc_]);
                    int64_t o = (ar_ + br_) + orr * (ac_ + bc_);
                    out[o].re += t.re; out[o].im += t.im;
                }
    return out;
}

int hko_block_tvp_i64(int m, const int64_t *n, const int64_t *nblk, const hki *H,
                      const hki *const *vectors, hki *y, hki *alpha) {
    if (check_dims(m, n) || check_dims(m, nblk)) return -1;
    int64_t hr = 1 - m, hcols = 1 - m;
    for (int p = 0; p < m; ++p) { hr += n[p]; hcols += nblk[p]; }
    int64_t wr = 1, wc = 1;
    hki *w = (hki *)calloc(1, sizeof(hki));
    if (!w) return -2;
    w[0].re = 1;
    for (int p = 1; p < m; ++p) {
        hki *nw = iconv2(w, wr, wc, vectors[p], n[p], nblk[p]);
        free(w);
        if (!nw) return -2;
        w = nw;
        wr += n[p] - 1;
        wc += nblk[p] - 1;
    }
    if (y) {
        for (int64_t j = 0; j < nblk[0]; ++j)
            for (int64_t i = 0; i < n[0]; ++i) {
                hki acc = { 0, 0 };
                for (int64_t l = 0; l < wc; ++l)
                    for (int64_t k = 0; k < wr; ++k) {
                        hki t = imul(H[(i + k) + hr * (j + l)], w[k + wr * l]);
                        acc.re += t.re; acc.im += t.im;
                    }
                y[i + n[0] * j] = acc;
            }
    }
    if (alpha) {
        hki *u = iconv2(vectors[0], n[0], nblk[0], w, wr, wc);
        if (!u) { free(w); return -2; }
        hki acc = { 0, 0 };
        for (int64_t s = 0; s < hr * hcols; ++s) {
            hki t = imul(H[s], u[s]);
            acc.re += t.re; acc.im += t.im;
        }
        *alpha = acc;
        free(u);
    }
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gradients of g = H x^{m-1} (cotangent v) and f = H x^m (cotangent phi).   */
/* v or phi may be NULL (zero cotangent); grad_x / grad_h may be NULL.       */
/* ------------------------------------------------------------------------ */
int hko_tvp_backward(int m, int64_t n, const hkc *h, const hkc *x, const hkc *v, const hkc *phi,
                     hkc *grad_x, hkc *grad_h) {
    if (m < 2 || m > 16 || n < 1) return -1;
    int64_t dh = m * (n - 1) + 1;
    int64_t *dims = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    const hkc **vecs = (const hkc **)malloc(sizeof(hkc *) * (size_t)m);
    if (!dims || !vecs) { free(dims); free(vecs); return -2; }
    for (int p = 0; p < m; ++p) { dims[p] = n; vecs[p] = x; }
    int64_t lw = 0, lw2 = 0;
    hkc *w = conv_chain(1, m, dims, vecs, &lw);      /* x^{*(m-1)}, length d_H - n + 1 */
    hkc *w2 = conv_chain(2, m, dims, vecs, &lw2);    /* x^{*(m-2)} ([1] when m = 2)   */
    int rc = (w && w2) ? 0 : -2;
    hkc ph = { 0.0, 0.0 };
    if (phi) ph = *phi;
    if (rc == 0 && grad_h) {
        hkc *u = NULL;
        if (phi) {
            u = (hkc *)malloc(sizeof(hkc) * (size_t)dh);
            if (!u) rc = -2; else hko_conv(x, n, w, lw, u);
        }
        if (rc == 0) {
#pragma omp parallel for schedule(dynamic, 64)
            for (int64_t s = 0; s < dh; ++s) {
                hkc total = { 0.0, 0.0 }, part = { 0.0, 0.0 };
                int cnt = 0;
                if (v) {
                    int64_t ilo = max64(0, s - (lw - 1));
                    int64_t ihi = min64(s, n - 1);
                    for (int64_t i = ilo; i <= ihi; ++i) {
                        part = cadd(part, cmul(cconj(w[s - i]), v[i]));
                        if (++cnt == BLOCK) { total = cadd(total, part); part.re = part.im = 0.0; cnt = 0; }
                    }
                }
                hkc g = cadd(total, part);
                if (u) g = cadd(g, cmul(ph, cconj(u[s])));
                grad_h[s] = g;
            }
        }
        free(u);
    }
    if (rc == 0 && grad_x) {
        hkc *corr = NULL, *gfwd = NULL;
        if (v) {
            /* c = conj(v) * x^{*(m-2)}, then corr_l = sum_k h_{l+k} c_k */
            hkc *cv = (hkc *)malloc(sizeof(hkc) * (size_t)n);
            hkc *c = (hkc *)malloc(sizeof(hkc) * (size_t)(n + lw2 - 1));
            corr = (hkc *)malloc(sizeof(hkc) * (size_t)n);
            if (!cv || !c || !corr) rc = -2;
            else {
                for (int64_t i = 0; i < n; ++i) cv[i] = cconj(v[i]);
                hko_conv(cv, n, w2, lw2, c);
                rc = hko_corr(h, dh, c, n + lw2 - 1, n, corr);
            }
            free(cv); free(c);
        }
        if (rc == 0 && phi) {
            gfwd = (hkc *)malloc(sizeof(hkc) * (size_t)n);
            if (!gfwd) rc = -2; else rc = hko_corr(h, dh, w, lw, n, gfwd);
        }
        if (rc == 0) {
            for (int64_t l = 0; l < n; ++l) {
                hkc g = { 0.0, 0.0 };
                if (corr) g = cscale(cconj(corr[l]), (double)(m - 1));
                if (gfwd) g = cadd(g, cscale(cmul(ph, cconj(gfwd[l])), (double)m));
                grad_x[l] = g;
            }
        }
        free(corr); free(gfwd);
    }
    free(w); free(w2); free(dims); free(vecs);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Gradients of the general products with distinct vectors (the paper does   */
/* not differentiate; complex autograd's convention, J^H applied to the      */
/* cotangents of these holomorphic maps):                                    */
/*   y = H x_2 ... x_m (cotangent v, dims[0] values),                        */
/*   alpha = H x_1 x_2 ... x_m (cotangent phi).                              */
/* y is linear in each x_p; its coefficient of x_p[l] multiplied by conj(v)  */
/* and summed over the free index is the mode-p-free product with conj(v)    */
/* in mode 1, and alpha's is the same with x_1 in mode 1.  With             */
/* c = conj(v) + conj(phi) x_1 (both linear in mode 1):                      */
/*   grad_{x_p}[l] = conj( sum_k h_{l+k} (c * x_q, q != 1, p)_k ),  p >= 2   */
/*   grad_{x_1}[l] = phi conj( sum_k h_{l+k} (x_2 * ... * x_m)_k )          */
/*   grad_h[s]     = conj( (c * x_2 * ... * x_m)_s ),   s < d_H              */
/* (* = linear convolution).  v or phi may be NULL (zero cotangent); x_1 is  */
/* read only with phi; grad_vectors[p] or grad_h may be NULL.                */
/* ------------------------------------------------------------------------ */
static hkc *cotangent_mode1(int64_t n1, const hkc *v, const hkc *phi, const hkc *x1) {
    hkc *c = (hkc *)malloc(sizeof(hkc) * (size_t)n1);
    if (!c) return NULL;
    for (int64_t i = 0; i < n1; ++i) {
        hkc t = { 0.0, 0.0 };
        if (v) t = cconj(v[i]);
        if (phi) t = cadd(t, cmul(cconj(*phi), x1[i]));
        c[i] = t;
    }
    return c;
}

int hko_mode_backward(int m, const int64_t *dims, const hkc *h, const hkc *const *vectors, const hkc *v,
                      const hkc *phi, hkc *const *grad_vectors, hkc *grad_h) {
    if (check_dims(m, dims)) return -1;
    if (phi && !vectors[0]) return -1;
    int64_t dh = 1 - m;
    for (int p = 0; p < m; ++p) dh += dims[p];
    hkc *c = cotangent_mode1(dims[0], v, phi, vectors[0]);
    const hkc **vecs = (const hkc **)malloc(sizeof(hkc *) * (size_t)m);
    int64_t *d2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    if (!c || !vecs || !d2) { free(c); free(vecs); free(d2); return -2; }
    int rc = 0;
    if (grad_h) {
        /* c * x_2 * ... * x_m, length d_H */
        vecs[0] = c;
        d2[0] = dims[0];
        for (int q = 1; q < m; ++q) { vecs[q] = vectors[q]; d2[q] = dims[q]; }
        int64_t lu = 0;
        hkc *u = conv_chain(0, m, d2, vecs, &lu);
        if (!u) rc = -2;
        else {
            for (int64_t s = 0; s < dh; ++s) grad_h[s] = cconj(u[s]);
            free(u);
        }
    }
    for (int p = 1; p < m && rc == 0; ++p) {
        if (!grad_vectors[p]) continue;
        /* c and the vectors of the modes other than 1 and p */
        int k = 0;
        vecs[k] = c;
        d2[k++] = dims[0];
        for (int q = 1; q < m; ++q)
            if (q != p) { vecs[k] = vectors[q]; d2[k++] = dims[q]; }
        int64_t lw = 0;
        hkc *w = conv_chain(0, k, d2, vecs, &lw); /* length d_H - n_p + 1 */
        if (!w) { rc = -2; break; }
        rc = hko_corr(h, dh, w, lw, dims[p], grad_vectors[p]);
        for (int64_t l = 0; l < dims[p] && rc == 0; ++l) grad_vectors[p][l] = cconj(grad_vectors[p][l]);
        free(w);
    }
    if (rc == 0 && grad_vectors[0]) {
        if (!phi) {
            for (int64_t l = 0; l < dims[0]; ++l) { grad_vectors[0][l].re = 0.0; grad_vectors[0][l].im = 0.0; }
        } else {
            int64_t lw = 0;
            hkc *w = conv_chain(1, m, dims, vectors, &lw); /* x_2 * ... * x_m */
            if (!w) rc = -2;
            else {
                rc = hko_corr(h, dh, w, lw, dims[0], grad_vectors[0]);
                for (int64_t l = 0; l < dims[0] && rc == 0; ++l)
                    grad_vectors[0][l] = cmul(*phi, cconj(grad_vectors[0][l]));
                free(w);
            }
        }
    }
    free(c); free(vecs); free(d2);
    return rc;
}

/* The same for the BHHB product (Section 3's 2-level form; matrices        */
/* column-major, X_p is n_p x N_p, H is (sum n - m + 1) x (sum N - m + 1)):  */
/* 2D linear convolutions and Y-style 2D correlations with H in place of    */
/* the 1D ones:                                                              */
/*   grad_{X_p}[i,j] = conj( sum_{k,l} H[i+k, j+l] (C (*) X_q, q != 1, p)[k,l] ), */
/*   grad_{X_1}[i,j] = phi conj( Y[i,j] ),  grad_H = conj( C (*) X_2 (*) ... (*) X_m ), */
/* C = conj(V) + conj(phi) X_1.                                              */
static hkc *conv2_chain(int k, const hkc *const *mats, const int64_t *rows, const int64_t *cols,
                        int64_t *r_out, int64_t *c_out) {
    int64_t wr = 1, wc = 1;
    hkc *w = (hkc *)malloc(sizeof(hkc));
    if (!w) return NULL;
    w[0].re = 1.0; w[0].im = 0.0;
    for (int p = 0; p < k; ++p) {
        hkc *nw = conv2(w, wr, wc, mats[p], rows[p], cols[p]);
        free(w);
        if (!nw) return NULL;
        w = nw;
        wr += rows[p] - 1;
        wc += cols[p] - 1;
    }
    *r_out = wr;
    *c_out = wc;
    return w;
}

/* out[i + outr*j] = conj( sum_{k,l} H[(i+k) + hr (j+l)] W[k + wr l] ) for i < outr, j < outc. */
static void corr2_conj(const hkc *H, int64_t hr, const hkc *W, int64_t wr, int64_t wc, int64_t outr,
                       int64_t outc, hkc *out) {
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t j = 0; j < outc; ++j)
        for (int64_t i = 0; i < outr; ++i) {
            hkc total = { 0.0, 0.0 }, part = { 0.0, 0.0 };
            int cnt = 0;
            for (int64_t l = 0; l < wc; ++l)
                for (int64_t k = 0; k < wr; ++k) {
                    part = cadd(part, cmul(H[(i + k) + hr * (j + l)], W[k + wr * l]));
                    if (++cnt == BLOCK) { total = cadd(total, part); part.re = part.im = 0.0; cnt = 0; }
                }
            out[i + outr * j] = cconj(cadd(total, part));
        }
}

int hko_block_backward(int m, const int64_t *n, const int64_t *nblk, const hkc *H, const hkc *const *vectors,
                       const hkc *v, const hkc *phi, hkc *const *grad_vectors, hkc *grad_H) {
    if (check_dims(m, n) || check_dims(m, nblk)) return -1;
    if (phi && !vectors[0]) return -1;
    int64_t hr = 1 - m, hc = 1 - m;
    for (int p = 0; p < m; ++p) { hr += n[p]; hc += nblk[p]; }
    hkc *c = cotangent_mode1(n[0] * nblk[0], v, phi, vectors[0]);
    const hkc **mats = (const hkc **)malloc(sizeof(hkc *) * (size_t)m);
    int64_t *rr = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *cc = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    if (!c || !mats || !rr || !cc) { free(c); free(mats); free(rr); free(cc); return -2; }
    int rc = 0;
    if (grad_H) {
        mats[0] = c; rr[0] = n[0]; cc[0] = nblk[0];
        for (int q = 1; q < m; ++q) { mats[q] = vectors[q]; rr[q] = n[q]; cc[q] = nblk[q]; }
        int64_t ur = 0, uc = 0;
        hkc *u = conv2_chain(m, mats, rr, cc, &ur, &uc); /* hr x hc */
        if (!u) rc = -2;
        else {
            for (int64_t s = 0; s < hr * hc; ++s) grad_H[s] = cconj(u[s]);
            free(u);
        }
    }
    for (int p = 1; p < m && rc == 0; ++p) {
        if (!grad_vectors[p]) continue;
        int k = 0;
        mats[k] = c; rr[k] = n[0]; cc[k++] = nblk[0];
        for (int q = 1; q < m; ++q)
            if (q != p) { mats[k] = vectors[q]; rr[k] = n[q]; cc[k++] = nblk[q]; }
        int64_t wr = 0, wc = 0;
        hkc *w = conv2_chain(k, mats, rr, cc, &wr, &wc);
        if (!w) { rc = -2; break; }
        corr2_conj(H, hr, w, wr, wc, n[p], nblk[p], grad_vectors[p]);
        free(w);
    }
    if (rc == 0 && grad_vectors[0]) {
        const int64_t len = n[0] * nblk[0];
        if (!phi) {
            for (int64_t s = 0; s < len; ++s) { grad_vectors[0][s].re = 0.0; grad_vectors[0][s].im = 0.0; }
        } else {
            int k = 0;
            for (int q = 1; q < m; ++q) { mats[k] = vectors[q]; rr[k] = n[q]; cc[k++] = nblk[q]; }
            int64_t wr = 0, wc = 0;
            hkc *w = conv2_chain(k, mats, rr, cc, &wr, &wc);
            if (!w) rc = -2;
            else {
                corr2_conj(H, hr, w, wr, wc, n[0], nblk[0], grad_vectors[0]);
                for (int64_t s = 0; s < len; ++s) grad_vectors[0][s] = cmul(*phi, grad_vectors[0][s]);
                free(w);
            }
        }
    }
    free(c); free(mats); free(rr); free(cc);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Spectra of the Section 3 procedures, as DFT sums at the bins idx[]:       */
/*   sign = -1:  out_i = sum_{s<len} a_s e^{-2 pi i j s / N}          (fft)   */
/*   sign = +1:  out_i = (1/N) sum_{s<len} a_s e^{+2 pi i j s / N}    (ifft)  */
/* with j = idx[i] mod N; a is zero-padded from len to N samples.            */
/* ------------------------------------------------------------------------ */
int hko_dft_sampled(int sign, const hkc *a, int64_t len, int64_t N, const int64_t *idx, int64_t nidx, hkc *out) {
    if (N < 1 || len < 0 || len > N || (sign != 1 && sign != -1) || nidx < 0) return -1;
    hkc *w = (hkc *)malloc(sizeof(hkc) * (size_t)N);
    if (!w) return -2;
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int64_t k = 0; k < N; ++k) {
        const long double t = two_pi * ((long double)k / (long double)N);
        w[k].re = (double)cosl(t);
        w[k].im = (double)(sign * sinl(t));
    }
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nidx; ++i) {
        const int64_t j = ((idx[i] % N) + N) % N;
        hkc total = { 0.0, 0.0 }, part = { 0.0, 0.0 };
        int cnt = 0;
        int64_t k = 0;  /* j s mod N */
        for (int64_t s = 0; s < len; ++s) {
            part = cadd(part, cmul(a[s], w[k]));
            if (++cnt == BLOCK) { total = cadd(total, part); part.re = part.im = 0.0; cnt = 0; }
            k += j;
            if (k >= N) k -= N;
        }
        total = cadd(total, part);
        out[i] = sign > 0 ? cscale(total, 1.0 / (double)N) : total;
    }
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Compensated mode (Dot2): TwoProduct by FMA, TwoSum (Neumaier).            */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } acc2;

static inline void acc_add(acc2 *a, double x) {
    const double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static inline void acc_prod(acc2 *a, double x, double y) {
    const double p = x * y;
    const double e = fma(x, y, -p);   /* exact: x y = p + e */
    acc_add(a, p);
    a->c += e;
}

/* sum_j a_j b_j over the given index pattern: a[ja + j], b[jb - j] (conv) or
 * b[jb + j] (corr), j < len */
static hkc dot2(const hkc *a, const hkc *b, int64_t len, int reverse_b) {
    acc2 re = { 0.0, 0.0 }, im = { 0.0, 0.0 };
    for (int64_t j = 0; j < len; ++j) {
        const hkc x = a[j];
        const hkc y = reverse_b ? b[-j] : b[j];
        acc_prod(&re, x.re, y.re);
        acc_prod(&re, -x.im, y.im);
        acc_prod(&im, x.re, y.im);
        acc_prod(&im, x.im, y.re);
    }
    hkc r = { re.s + re.c, im.s + im.c };
    return r;
}

static int conv_comp(const hkc *a, int64_t na, const hkc *b, int64_t nb, hkc *out) {
    if (na < 1 || nb < 1) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < na + nb - 1; ++k) {
        const int64_t jlo = max64(0, k - (nb - 1));
        const int64_t jhi = min64(k, na - 1);
        out[k] = dot2(a + jlo, b + (k - jlo), jhi - jlo + 1, 1);
    }
    return 0;
}

/* hko_tvp with compensated sums everywhere (y: dims[0] outputs, nullable;
 * alpha nullable, needs vectors[0]). */
int hko_tvp_comp(int m, const int64_t *dims, const hkc *h, const hkc *const *vectors, hkc *y, hkc *alpha) {
    if (check_dims(m, dims)) return -1;
    int64_t dh = 1 - m;
    for (int p = 0; p < m; ++p) dh += dims[p];
    /* w = x_2 * ... * x_m */
    int64_t lw = dims[1];
    hkc *w = (hkc *)malloc(sizeof(hkc) * (size_t)lw);
    if (!w) return -2;
    memcpy(w, vectors[1], sizeof(hkc) * (size_t)lw);
    for (int p = 2; p < m; ++p) {
        const int64_t nl = lw + dims[p] - 1;
        hkc *nw = (hkc *)malloc(sizeof(hkc) * (size_t)nl);
        if (!nw) { free(w); return -2; }
        conv_comp(w, lw, vectors[p], dims[p], nw);
        free(w);
        w = nw;
        lw = nl;
    }
    if (y) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < dims[0]; ++i) y[i] = dot2(h + i, w, lw, 0);
    }
    if (alpha) {
        hkc *u = (hkc *)malloc(sizeof(hkc) * (size_t)dh);
        if (!u) { free(w); return -2; }
        conv_comp(vectors[0], dims[0], w, lw, u);
        *alpha = dot2(h, u, dh, 0);
        free(u);
    }
    free(w);
    return 0;
}
