/*
 * hankel.h -- C ABI of the MI355X (gfx950) fast Hankel tensor-vector product.
 *
 * Method (Ding, Qi, Wei, "Fast Hankel tensor-vector products and application
 * to exponential data fitting"): an order-m Hankel tensor H of size
 * n_1 x ... x n_m is fixed by its generating vector h of length
 * d_H = n_1 + ... + n_m - m + 1 (Section 1).  It sits in the corner of the
 * anti-circulant tensor with compressed generating vector h, which the Fourier
 * matrix diagonalizes (Theorem 2.1), so each product becomes zero padding,
 * FFTs, one pointwise spectral product, an FFT and a slice (Section 3):
 *
 *   y     = H x_2 x_3 ... x_m  = fft( ifft(h~) .* fft(x~_2) .* ... .* fft(x~_m) )[0 : n_1)
 *   alpha = H x_1 x_2 ... x_m  = ifft(h~)^T ( fft(x~_1) .* ... .* fft(x~_m) )
 *
 * with fft(v)_k = sum_j v_j e^{-2 pi i jk/N}, ifft = (1/N) * conjugate kernel,
 * "~" = zero padding to length N >= d_H, and products taken without complex
 * conjugation (Section 2.1 mode-p product).  Any N >= d_H gives the same
 * result (the paper takes N = d_H, Section 3).  The library takes the smallest
 * N >= d_H of the form 2^k, 3 * 2^k or 5 * 2^k (N <= 2^24) for which it has
 * kernels: a length 3 * 2^k or 5 * 2^k transform is computed as a 2D
 * transform of 3 or 5 sequences of length 2^k through the Chinese-remainder
 * index map (no twiddles between the factors), which keeps the padding below
 * 25% of d_H for most lengths instead of up to 100%.  The 2-level block
 * (BHHB) form uses 2D FFTs on a grid of at least (sum n_p - m + 1) x
 * (sum N_p - m + 1) (Section 3, BHHB procedure), each axis 2^k, 3 * 2^k or
 * 5 * 2^k (block_hankel_tvp_layout).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Data pointers are DEVICE pointers owned by the caller.  Arrays are
 *    contiguous (stride 1).  Complex dtypes are interleaved (re, im) pairs;
 *    real dtypes (HK_F32, HK_F64) mean real inputs and real outputs.  Real
 *    forward products (1D) transform each real vector of padded length N as
 *    N/2 complex pairs and split the result by conjugate symmetry, so they
 *    move and transform half the data of a complex product (power-of-two N;
 *    the adjoint of real data, persistent plans and HK_PLAN_POW2 plans take
 *    the complex path and drop the imaginary part, rounding noise for real
 *    data).  Each pointer must be aligned to its element size.
 *  - Arrays of vector pointers ("vectors") are HOST arrays of device pointers.
 *  - Calls are asynchronous and stream-ordered on `stream` (NULL = default
 *    stream).  Outputs are fully overwritten; outputs must not alias inputs.
 *  - Workspace: `ws`/`ws_bytes` is caller-owned device scratch of at least the
 *    size the matching *_workspace_size call reports (it may be NULL when that
 *    size is 0).  The library allocates no device memory in these calls apart
 *    from a one-time, per-device twiddle-table setup on first use.
 *  - Errors are return codes; nothing is thrown or aborted across the ABI.
 *    Arguments are validated on the host before anything is enqueued.
 *    hk_last_error() gives a thread-local description of the last failure.
 */
#ifndef HANKEL_H_
#define HANKEL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

struct ihipStream_t;
typedef struct ihipStream_t *hipStream_t;

typedef enum {
    HK_C64 = 0,  /* complex float  (8-byte elements)  */
    HK_C128 = 1, /* complex double (16-byte elements) */
    HK_F32 = 2,  /* real float                        */
    HK_F64 = 3   /* real double                       */
} hk_dtype_t;

typedef int hk_status_t;
#define HK_SUCCESS 0
#define HK_ERR_INVALID_VALUE 1 /* m outside [2, HK_MAX_ORDER], a dim < 1, bad dtype/flags  */
#define HK_ERR_NULL_POINTER 2  /* a required pointer is NULL, or no output requested       */
#define HK_ERR_MISALIGNED 3    /* a data pointer is not aligned to its element size         */
#define HK_ERR_WORKSPACE 4     /* ws_bytes smaller than the reported workspace size         */
#define HK_ERR_SIZE_LIMIT 5    /* padded length (per axis) above HK_MAX_FFT_LOG2 or overflow */
#define HK_ERR_DEVICE 6        /* current device is not gfx950                              */
#define HK_ERR_HIP 7           /* a HIP runtime call or kernel launch failed                */
#define HK_ERR_DEVICE_FAULT 8  /* a batched plan's kernel reported an error (see status)    */
#define HK_ERR_NOT_SUPPORTED 9 /* valid request outside what the library implements         */

#define HK_MAX_ORDER 8
#define HK_MAX_FFT_LOG2 24 /* 1D: N <= 2^24; BHHB: each grid axis <= 2^12 */

/* -------------------------------------------------------------------------
 * Square Hankel tensor, all vectors equal (Section 3 procedures with
 * x_1 = ... = x_m = x; Qi's notation H x^{m-1}, H x^m, Section 2.1).
 *   h     : d_H = m(n-1)+1 elements
 *   x     : n elements
 *   y     : if non-NULL, receives H x^{m-1} (n elements)
 *   alpha : if non-NULL, receives H x^m (1 element, on the device)
 * At least one of y, alpha must be non-NULL.  Both come from one set of FFTs.
 * ------------------------------------------------------------------------- */
hk_status_t hankel_tvp_workspace_size(hk_dtype_t dt, int m, int64_t n, size_t *bytes);
hk_status_t hankel_tvp(hk_dtype_t dt, const void *h, int m, int64_t n, const void *x,
                       void *y, void *alpha, void *ws, size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * hankel_tvp without a workspace argument and without device allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and kernels as hankel_tvp; the workspace is a static device array
 * of HK_NOALLOC_SCRATCH_BYTES per device, held by every device the library
 * runs on until the process ends.
 *  - Products whose workspace (hankel_tvp_workspace_size) exceeds
 *    HK_NOALLOC_SCRATCH_BYTES are rejected with HK_ERR_WORKSPACE before
 *    anything is enqueued.  40 MiB covers, e.g., m = 4, n = 2^18 (N = 2^20)
 *    in HK_C64 and HK_C128.
 *  - The first call on a device looks up that device's copy of the array and
 *    uploads the twiddle tables (host-synchronous, once); make it outside
 *    graph capture.  Later calls enqueue kernels only.
 *  - All calls on one device share its array: calls that overlap in time on
 *    one device (different streams or threads without ordering) race and give
 *    unspecified results.  Calls on one stream are ordered and safe.
 * ------------------------------------------------------------------------- */
#define HK_NOALLOC_SCRATCH_BYTES ((size_t)40 << 20)
hk_status_t hankel_tvp_noalloc(hk_dtype_t dt, const void *h, int m, int64_t n, const void *x,
                               void *y, void *alpha, hipStream_t stream);

/* -------------------------------------------------------------------------
 * General Hankel tensor n_1 x ... x n_m, distinct vectors (Section 3, the two
 * product types y = H x_2 ... x_m and alpha = H x_1 ... x_m).
 *   dims    : host array of m sizes n_p >= 1
 *   h       : sum(dims) - m + 1 elements
 *   vectors : host array of m device pointers; vectors[p] has dims[p]
 *             elements.  vectors[0] is read only when alpha is requested.
 *             Identical pointers with identical lengths are transformed once.
 *   y       : if non-NULL, receives H x_2 ... x_m (dims[0] elements)
 *   alpha   : if non-NULL, receives H x_1 ... x_m (1 element)
 * ------------------------------------------------------------------------- */
hk_status_t hankel_mode_products_workspace_size(hk_dtype_t dt, int m, const int64_t *dims,
                                                const void *const *vectors, int want_y,
                                                int want_alpha, size_t *bytes);
hk_status_t hankel_mode_products(hk_dtype_t dt, const void *h, int m, const int64_t *dims,
                                 const void *const *vectors, void *y, void *alpha, void *ws,
                                 size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * Spectral form (Section 3: the products are pointwise products of the
 * spectra h^ = ifft(pad_N h) and x^_p = fft(pad_N x_p) on one transform length
 * N >= d_H, followed by one transform).  A spectrum computed once serves every
 * product that shares its operand: a fixed h met by many vectors (power
 * iterations, HOOI), a vector met by many h.  d_H = sum(dims) - m + 1 must
 * be above 4096 (smaller shapes return HK_ERR_NOT_SUPPORTED).  Every dtype:
 * a spectrum is N complex values of the dtype's precision (complex64 for
 * HK_F32, complex128 for HK_F64 and HK_C128); real inputs are transformed as
 * complex data with zero imaginary parts and real outputs keep the real part.
 *
 * Layout: N is the power of two >= d_H; R = 2^(ceil(log2(N) / 2) + 1) for
 * N >= 2^16 (at most 2^12), else R = 2^ceil(log2(N) / 2); C = N / R.
 * Element r R + c (r < C, c < R) of a spectrum holds bin r + C c.  The
 * layout depends only on d_H (not on hk_set_fft_lengths), so spectra of
 * separate calls combine whenever their shapes have the same d_H.  spec
 * pointers are aligned to the complex element (8 or 16 bytes).
 *
 * hankel_spectrum_layout: *n_fft = N, *row_len = R for the shape (m, dims).
 * hankel_spectrum: which = -1: src = h (d_H elements), spec receives h^
 *   (including the 1/N of the inverse transform); which = p in [0, m):
 *   src = x_p (dims[p] elements), spec receives x^_p.  spec must not overlap
 *   src or ws.  Workspace: hankel_spectrum_workspace_size.
 * hankel_mode_products_spectral: h_spec = h^ (from hankel_spectrum with
 *   which = -1 on the same shape).  Mode p's operand is specs[p] (a spectrum)
 *   when specs is non-NULL and specs[p] is non-NULL, else vectors[p] (the
 *   vector itself); vectors and specs may each be NULL.  Mode 0 is read only
 *   when alpha is requested.  y and alpha as in hankel_mode_products; equal
 *   operands (same pointer, length and kind) are used once, as a power.
 *   Workspace: hankel_mode_products_spectral_workspace_size, with the same
 *   vectors/specs pointers (they decide which operands are merged).
 * Errors as for hankel_mode_products.
 * ------------------------------------------------------------------------- */
hk_status_t hankel_spectrum_layout(hk_dtype_t dt, int m, const int64_t *dims, int64_t *n_fft,
                                   int64_t *row_len);
hk_status_t hankel_spectrum_workspace_size(hk_dtype_t dt, int m, const int64_t *dims, int which,
                                           size_t *bytes);
hk_status_t hankel_spectrum(hk_dtype_t dt, int m, const int64_t *dims, int which, const void *src,
                            void *spec, void *ws, size_t ws_bytes, hipStream_t stream);
hk_status_t hankel_mode_products_spectral_workspace_size(hk_dtype_t dt, int m, const int64_t *dims,
                                                         const void *const *vectors,
                                                         const void *const *specs, int want_y,
                                                         int want_alpha, size_t *bytes);
hk_status_t hankel_mode_products_spectral(hk_dtype_t dt, const void *h_spec, int m,
                                          const int64_t *dims, const void *const *vectors,
                                          const void *const *specs, void *y, void *alpha,
                                          void *ws, size_t ws_bytes, hipStream_t stream);
/* Strided batch of equal-vector products (square shape (m, n)) that share one
 * stored h^ (hankel_spectrum with which = -1 on dims = {n, ..., n}): instance b
 * uses x + b*x_stride and writes y + b*y_stride (H x^{m-1}) and alpha + b
 * (H x^m); y or alpha may be NULL.  One launch per pass covers the batch; the
 * h^ it reads is shared by all instances.  Rules as for the spectral form. */
hk_status_t hankel_tvp_spectral_strided_batched_workspace_size(hk_dtype_t dt, int m, int64_t n,
                                                               int64_t batch, size_t *bytes);
hk_status_t hankel_tvp_spectral_strided_batched(hk_dtype_t dt, const void *h_spec, int m,
                                                int64_t n, const void *x, int64_t x_stride,
                                                void *y, int64_t y_stride, void *alpha,
                                                int64_t batch, void *ws, size_t ws_bytes,
                                                hipStream_t stream);

/* -------------------------------------------------------------------------
 * 2-level block Hankel tensor with Hankel blocks (BHHB; Section 2.2
 * generating matrix, Section 3 BHHB procedure).  Mode p has N_p blocks of
 * size n_p; the tensor entry at in-block indices (i_p) and block indices
 * (j_p) is H[i_1+...+i_m, j_1+...+j_m].
 *   inner_dims : n_p (host array, m entries)
 *   block_dims : N_p (host array, m entries)
 *   H          : generating matrix, column-major,
 *                (sum n_p - m + 1) rows x (sum N_p - m + 1) columns
 *   vectors[p] : vec(X_p), n_p * N_p elements, X_p[i, j] = vectors[p][i + n_p j]
 *   y          : if non-NULL, receives vec(Y), Y = (H x_2 ... x_m) as an
 *                n_1 x N_1 column-major matrix
 *   alpha      : if non-NULL, receives H x_1 ... x_m (needs vectors[0])
 * ------------------------------------------------------------------------- */
/* The transform grid of a BHHB shape (rows along the in-block index, columns
 * along the block index) for a call of `batch` instances under the current
 * length policy: each axis is the smallest of 2^k, 3 * 2^k, 5 * 2^k (complex
 * dtypes; the axes' factors combine freely) >= its extent
 * (sum n_p - m + 1, sum N_p - m + 1) that has kernels, or the power of two.
 * An axis of length odd * 2^k is transformed as `odd` sequences of 2^k
 * through the Chinese-remainder index map.  Host-only. */
hk_status_t block_hankel_tvp_layout(hk_dtype_t dt, int m, const int64_t *inner_dims, const int64_t *block_dims,
                                    int64_t batch, int64_t *grid_rows, int64_t *grid_cols);
hk_status_t block_hankel_tvp_workspace_size(hk_dtype_t dt, int m, const int64_t *inner_dims,
                                            const int64_t *block_dims, const void *const *vectors,
                                            int want_y, int want_alpha, size_t *bytes);
hk_status_t block_hankel_tvp(hk_dtype_t dt, const void *H, int m, const int64_t *inner_dims,
                             const int64_t *block_dims, const void *const *vectors, void *y,
                             void *alpha, void *ws, size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * Batched products: heterogeneous problems (any mix of orders, sizes, 1D and
 * BHHB, equal or distinct vectors) executed together.  The paper motivates
 * this with the Hankel tensor-matrix products of HOOI (Section 4.2), which
 * are batches of tensor-vector products.
 *
 * One hk_problem_t per product.  For 1D problems block_dims is ignored; for
 * BHHB problems (is_block = 1) dims are the n_p and block_dims the N_p.
 * vectors[0] is read only when alpha != NULL.  y / alpha as above (at least
 * one non-NULL).  Problems must not write to overlapping outputs.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t m;
    int32_t is_block;
    int32_t reserved0;
    int32_t reserved1;
    int64_t dims[HK_MAX_ORDER];
    int64_t block_dims[HK_MAX_ORDER];
    const void *h;
    const void *vectors[HK_MAX_ORDER];
    void *y;
    void *alpha;
} hk_problem_t;

typedef struct hk_plan_s *hk_plan_t;

#define HK_PLAN_PERSISTENT 0x1u /* one persistent launch: task queues and grid-wide barriers   */
#define HK_PLAN_MULTIKERNEL 0x2u /* grouped launches: per phase, one kernel specialised for each
                                   (task kind, transform length) group; no in-kernel waits      */
#define HK_PLAN_GRAPH 0x4u      /* capture the plan's launches in a hipGraph on first execute */
#define HK_PLAN_AUTOTUNE 0x8u   /* grouped eager plans: at the first execute, choose per
                                   length bucket (log2 of the power-of-two length >= d_H)
                                   between the odd-factor lengths, the odd lengths without
                                   the factor 5 and the power-of-two lengths by timing the
                                   whole plan (coordinate descent, longest bucket first);
                                   the workspace size covers every candidate.  No effect
                                   together with HK_PLAN_GRAPH                               */
#define HK_PLAN_POW2 0x10u      /* power-of-two complex transforms only (no 3 * 2^k, 5 * 2^k,
                                   no half-length real transforms); implied by PERSISTENT      */

/* Creates a plan for `count` problems.  The plan copies the descriptors
 * (pointers included); on first execute it uploads them to a device table
 * that it owns until hk_plan_destroy.  With HK_PLAN_GRAPH it also owns a
 * captured graph.  flags without PERSISTENT pick the grouped launches (the
 * faster schedule on MI355X); PERSISTENT runs the whole batch in one launch
 * whose resident workgroups pull each phase's tasks from a queue and meet in
 * a grid-wide barrier (bounded wait) between phases.  That launch is a
 * cooperative one (hipLaunchCooperativeKernel: the runtime refuses a grid that
 * cannot be resident at once, and hk_plan_execute then fails with
 * HK_ERR_HIP), except inside a stream capture (HK_PLAN_GRAPH) and while
 * hk_profile_start timing is on, which launch the same occupancy-sized grid
 * plainly.  Grouped launches spread
 * a phase's groups over the caller's stream and three streams of the plan;
 * the process's streams share its few hardware queues, so the eager plan's
 * time varies with the streams the process created before it (by up to ~15 %
 * on one mixed batch), while a graph plan (HK_PLAN_GRAPH, on a non-default
 * stream) replays with the same time whatever they are. */
hk_status_t hk_plan_create(hk_plan_t *plan, hk_dtype_t dt, const hk_problem_t *probs,
                           int64_t count, unsigned flags);
hk_status_t hk_plan_workspace_size(hk_plan_t plan, size_t *bytes);
/* Enqueues the plan.  The workspace must stay untouched until the plan's work
 * on `stream` has finished. */
hk_status_t hk_plan_execute(hk_plan_t plan, void *ws, size_t ws_bytes, hipStream_t stream);
/* Synchronizes the last execute's stream and returns HK_SUCCESS or
 * HK_ERR_DEVICE_FAULT if the persistent kernel flagged an error (a barrier
 * wait that exceeded its bound: in a plain launch, the device could not hold
 * the whole grid at once, for example while other work occupied it; results
 * are then unspecified). */
hk_status_t hk_plan_status(hk_plan_t plan);
/* Diagnostics: the number of polling iterations (each a short sleep) a
 * persistent-plan workgroup waits at a grid barrier before it sets the error
 * word and continues (default 2^22, a fraction of a second).  A tiny bound
 * exercises the error path of hk_plan_status without any fault.  Not allowed
 * once the plan is captured in a graph. */
hk_status_t hk_plan_set_wait_bound(hk_plan_t plan, uint32_t spins);
/* Diagnostics (measurement): the bytes one hk_plan_execute reads and writes
 * in HBM under the pass model of its kernels, summed over the instances.
 * Resident instances (one workgroup per product) count their inputs and
 * outputs once; three-pass instances count pass A (each operand read, the
 * storage columns that can be nonzero written), pass B (those columns read,
 * the output columns the last pass reads written) and pass D (those read
 * back, the output slice written).  Host-only; *bytes receives the total. */
hk_status_t hk_plan_pass_bytes(hk_plan_t plan, int64_t *bytes);
/* Diagnostics: the times (ms per execute) the HK_PLAN_AUTOTUNE tuner measured
 * for the default plan and for the plan it kept, and the mask of length
 * buckets it moved to powers of two (bit b: power-of-two length 2^b); zeros
 * before the first execute or without the flag.  Any pointer may be NULL. */
hk_status_t hk_plan_tune_times(hk_plan_t plan, double *ms_default, double *ms_tuned, uint32_t *pow2_buckets);
hk_status_t hk_plan_destroy(hk_plan_t plan);

/* One-shot convenience: plan (grouped launches), execute with the descriptor
 * tables kept in the workspace, then wait for `stream` and free the plan
 * (this call blocks until the batch has finished). */
hk_status_t hankel_tvp_batched_workspace_size(hk_dtype_t dt, const hk_problem_t *probs,
                                              int64_t count, size_t *bytes);
hk_status_t hankel_tvp_batched(hk_dtype_t dt, const hk_problem_t *probs, int64_t count,
                               void *ws, size_t ws_bytes, hipStream_t stream);

/* The same one-shot batch restricted to one product kind: every problem a
 * general (1D) Hankel tensor with dims and distinct or equal vectors
 * (hankel_mode_products_batched, is_block = 0), or every problem a BHHB
 * tensor (block_hankel_tvp_batched, is_block = 1).  A problem of the other
 * kind is rejected with HK_ERR_INVALID_VALUE before anything is enqueued;
 * otherwise arguments, workspace and blocking behaviour are those of
 * hankel_tvp_batched. */
hk_status_t hankel_mode_products_batched_workspace_size(hk_dtype_t dt, const hk_problem_t *probs,
                                                        int64_t count, size_t *bytes);
hk_status_t hankel_mode_products_batched(hk_dtype_t dt, const hk_problem_t *probs, int64_t count,
                                         void *ws, size_t ws_bytes, hipStream_t stream);
hk_status_t block_hankel_tvp_batched_workspace_size(hk_dtype_t dt, const hk_problem_t *probs,
                                                    int64_t count, size_t *bytes);
hk_status_t block_hankel_tvp_batched(hk_dtype_t dt, const hk_problem_t *probs, int64_t count,
                                     void *ws, size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * Level-k block Hankel tensor, 1 <= k <= 4 (Section 2.2: a block Hankel tensor
 * whose blocks are level-(k-1) block Hankel tensors; k = 2 is the BHHB tensor
 * of block_hankel_tvp, k = 1 the Hankel tensor of hankel_mode_products).  The
 * tensor is fixed by its generating tensor G of order k (Section 2.2) and the
 * sizes of its modes at every level:
 *   dims    : HOST array of k*m sizes, dims[t*m + p] = size of mode p at level
 *             t (t = 0 the innermost level, the entries of the Hankel blocks);
 *   G       : d_0 x ... x d_{k-1}, d_t = dims[t*m] + ... + dims[t*m+m-1] - m + 1,
 *             column-major (entry (i_0, ..., i_{k-1}) at i_0 + d_0 (i_1 + d_1 (...)));
 *             prod_t d_t <= 2^24;
 *   vectors : HOST array of m device pointers, vectors[p] = vec(X_p), X_p of size
 *             dims[p] x dims[m+p] x ..., column-major like G (vectors[0] only
 *             for alpha);
 *   y       : if non-NULL, vec(Y) of size dims[0] x dims[m] x ... x dims[(k-1)m]:
 *             Y = H x_2 vec(X_2) ... x_m vec(X_m) (mode 1 free);
 *   alpha   : if non-NULL, H x_1 vec(X_1) ... x_m vec(X_m).
 * The paper computes these with k-dimensional FFTs on the padded grid.  This
 * call embeds each X_p at the strides of G's column-major layout, where the
 * index sums of a product never carry from one level into the next, so the
 * product equals a 1D Hankel product with generating vector G and the embedded
 * vectors, read back at the same strides (same result, one 1D transform of
 * length >= prod d_t).  Workspace: block_hankel_tvp_levels_workspace_size with
 * the same sizes, vectors and requested outputs (the vector pointers only
 * decide which modes share one embedding). */
hk_status_t block_hankel_tvp_levels_workspace_size(hk_dtype_t dt, int m, int k, const int64_t *dims,
                                                   const void *const *vectors, int want_y, int want_alpha,
                                                   size_t *bytes);
hk_status_t block_hankel_tvp_levels(hk_dtype_t dt, const void *G, int m, int k, const int64_t *dims,
                                    const void *const *vectors, void *y, void *alpha, void *ws,
                                    size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * Hankel tensor-matrix product (Section 4.2): for the square order-m Hankel
 * tensor H (generating vector h, m(n-1)+1 elements) and an n x R matrix U
 * (column-major, device), T = H x_2 U x_3 U ... x_m U with the Section 2.1
 * mode product, i.e. column (j_2, ..., j_m) of T is the tensor-vector product
 * H x_2 U[:, j_2] ... x_m U[:, j_m].  out is n x R^(m-1), column-major, column
 * index j_2 + R j_3 + ... + R^(m-2) j_m.  The columns are symmetric in the j's:
 * the library computes the nondecreasing tuples and copies the rest.  With
 * d_H > 4096 and (tuples x N) >= 2^21 it transforms h and
 * each column of U once (the spectral form above) and forms every tuple as a
 * product of those spectra followed by one transform; otherwise each tuple is
 * a mode product of a grouped batch.  R^(m-1) <= 2^20.  The call enqueues its
 * work on `stream` and waits for it (its descriptor tables live on the host
 * until then).  Used by HOOI (Algorithm 4.2) for the Hankel tensor-matrix
 * products that dominate it.
 * ------------------------------------------------------------------------- */
hk_status_t hankel_tensor_matrix_workspace_size(hk_dtype_t dt, int m, int64_t n, int64_t R, size_t *bytes);
hk_status_t hankel_tensor_matrix(hk_dtype_t dt, const void *h, int m, int64_t n, int64_t R, const void *U,
                                 void *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * Adjoint of the equal-vector products g = H x^{m-1} (n values) and
 * f = H x^m (a scalar).  The paper does not differentiate; this follows
 * complex autograd's convention for holomorphic maps: the returned gradients
 * are J^H applied to the cotangents,
 *   grad_h = conj( ifft( x^^{m-1} .* (V^ + conj(phi) x^) ) )[0 : d_H)
 *   grad_x = conj( fft( h^ .* x^^{m-2} .* ((m-1) V^ + m conj(phi) x^) ) )[0 : n)
 * with h^ = ifft(h~), x^ = fft(x~), V^ = fft(conj(v)~): spectral
 * correlations on the same padded grid as the forward product.
 *   grad_y     : cotangent v of g (n elements) or NULL (zero)
 *   grad_alpha : cotangent phi of f (1 element, device) or NULL (zero)
 *   grad_x     : n elements or NULL (not requested)
 *   grad_h     : d_H elements or NULL (not requested)
 * Complex dtypes only.
 * ------------------------------------------------------------------------- */
hk_status_t hankel_tvp_backward_workspace_size(hk_dtype_t dt, int m, int64_t n, size_t *bytes);
/* The same adjoint with x given by its stored spectrum x_spec (hankel_spectrum
 * on the shape (m, {n, ..., n}), any mode): the forward's x^ kept for the
 * backward, so x is not transformed again.  Complex dtypes and the rules of
 * the spectral form (d_H > 4096). */
hk_status_t hankel_tvp_backward_spectral_workspace_size(hk_dtype_t dt, int m, int64_t n, size_t *bytes);
hk_status_t hankel_tvp_backward_spectral(hk_dtype_t dt, const void *h, int m, int64_t n,
                                         const void *x_spec, const void *grad_y,
                                         const void *grad_alpha, void *grad_x, void *grad_h,
                                         void *ws, size_t ws_bytes, hipStream_t stream);
hk_status_t hankel_tvp_backward(hk_dtype_t dt, const void *h, int m, int64_t n, const void *x,
                                const void *grad_y, const void *grad_alpha, void *grad_x,
                                void *grad_h, void *ws, size_t ws_bytes, hipStream_t stream);

/* Forward products that keep x^ for the adjoint: the strided batch of
 * hankel_tvp_strided_batched (instance b: h + b*h_stride, x + b*x_stride,
 * y + b*y_stride, alpha + b; y or alpha may be NULL) that also writes each
 * instance's x^ = fft(pad_N x), in the row order of hankel_spectrum, to
 * x_spec + b*spec_stride (complex elements of x's precision; spec_stride >= N,
 * N from hankel_spectrum_layout).  The row pass stores x^ right after
 * transforming x, so the saved spectrum costs N element writes and no extra
 * transform.  Complex dtypes, d_H > 4096 (the spectral layout, power-of-two N). */
hk_status_t hankel_tvp_save_spectrum_workspace_size(hk_dtype_t dt, int m, int64_t n, int64_t batch,
                                                    size_t *bytes);
hk_status_t hankel_tvp_save_spectrum(hk_dtype_t dt, const void *h, int64_t h_stride, int m, int64_t n,
                                     const void *x, int64_t x_stride, void *y, int64_t y_stride,
                                     void *alpha, void *x_spec, int64_t spec_stride, int64_t batch,
                                     void *ws, size_t ws_bytes, hipStream_t stream);
/* Strided batch of hankel_tvp_backward_spectral: instance b reads h + b*h_stride,
 * x_spec + b*spec_stride (as stored by hankel_tvp_save_spectrum),
 * grad_y + b*gy_stride, grad_alpha + b, and writes grad_x + b*gx_stride,
 * grad_h + b*gh_stride (NULL pointers as in hankel_tvp_backward). */
hk_status_t hankel_tvp_backward_spectral_strided_batched_workspace_size(hk_dtype_t dt, int m, int64_t n,
                                                                        int64_t batch, size_t *bytes);
hk_status_t hankel_tvp_backward_spectral_strided_batched(
    hk_dtype_t dt, const void *h, int64_t h_stride, int m, int64_t n, const void *x_spec,
    int64_t spec_stride, const void *grad_y, int64_t gy_stride, const void *grad_alpha,
    void *grad_x, int64_t gx_stride, void *grad_h, int64_t gh_stride, int64_t batch, void *ws,
    size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * Adjoint of the products with distinct vectors: the general Hankel tensor
 * (hankel_mode_products: y = H x_2 ... x_m, alpha = H x_1 ... x_m) and the
 * BHHB tensor (block_hankel_tvp, vectors vec(X_p), y = vec(Y)).  The paper
 * does not differentiate; as for hankel_tvp_backward the gradients are J^H
 * applied to the cotangents v (of y) and phi (of alpha).  With
 * c = conj(v) + conj(phi) x_1:
 *   grad_h     = conj( c * x_2 * ... * x_m )            (d_H values; BHHB: 2D, the H grid)
 *   grad_{x_p} = conj( H x_1 c x_q (q != 1, p) )         (mode p free, dims[p] values), p >= 2
 *   grad_{x_1} = phi conj( H x_2 ... x_m )               (zero when grad_alpha is NULL)
 * (* = linear convolution; 2D for BHHB; Section 2.1 mode products).  Each
 * is computed by the forward kernels on the forward product's transform grid
 * (N or each BHHB axis 2^k, 3 * 2^k or 5 * 2^k under the length policy:
 * spectral correlations / convolutions), one after the other on `stream`.
 *   vectors      : host array of m device pointers; vectors[0] (x_1) is read
 *                  only when grad_alpha is given
 *   grad_y       : cotangent of y (dims[0] values; BHHB n_1 N_1) or NULL
 *   grad_alpha   : cotangent of alpha (1 value, device) or NULL
 *   grad_vectors : host array of m device pointers, grad_vectors[p] receives
 *                  grad_{x_p} (NULL = not requested)
 *   grad_h       : receives grad_h (NULL = not requested)
 * Workspace: *_workspace_size with the mask of requested grad_vectors (bit p)
 * and want_grad_h.  Complex dtypes only.
 * ------------------------------------------------------------------------- */
hk_status_t hankel_mode_products_backward_workspace_size(hk_dtype_t dt, int m, const int64_t *dims,
                                                         int grad_vectors_mask, int want_grad_h,
                                                         size_t *bytes);
hk_status_t hankel_mode_products_backward(hk_dtype_t dt, const void *h, int m, const int64_t *dims,
                                          const void *const *vectors, const void *grad_y,
                                          const void *grad_alpha, void *const *grad_vectors,
                                          void *grad_h, void *ws, size_t ws_bytes,
                                          hipStream_t stream);
hk_status_t block_hankel_tvp_backward_workspace_size(hk_dtype_t dt, int m, const int64_t *inner_dims,
                                                     const int64_t *block_dims, int grad_vectors_mask,
                                                     int want_grad_h, size_t *bytes);
hk_status_t block_hankel_tvp_backward(hk_dtype_t dt, const void *H, int m, const int64_t *inner_dims,
                                      const int64_t *block_dims, const void *const *vectors,
                                      const void *grad_y, const void *grad_alpha,
                                      void *const *grad_vectors, void *grad_H, void *ws,
                                      size_t ws_bytes, hipStream_t stream);

/* Strided batch of equal-vector products of one shape (m, n): instance b uses
 * h + b*h_stride, x + b*x_stride, y + b*y_stride, alpha + b (elements).
 * y or alpha may be NULL.  One launch per pass covers the whole batch. */
hk_status_t hankel_tvp_strided_batched_workspace_size(hk_dtype_t dt, int m, int64_t n,
                                                      int64_t batch, size_t *bytes);
hk_status_t hankel_tvp_strided_batched(hk_dtype_t dt, const void *h, int64_t h_stride, int m,
                                       int64_t n, const void *x, int64_t x_stride, void *y,
                                       int64_t y_stride, void *alpha, int64_t batch, void *ws,
                                       size_t ws_bytes, hipStream_t stream);
hk_status_t hankel_tvp_backward_strided_batched_workspace_size(hk_dtype_t dt, int m, int64_t n,
                                                               int64_t batch, size_t *bytes);
hk_status_t hankel_tvp_backward_strided_batched(
    hk_dtype_t dt, const void *h, int64_t h_stride, int m, int64_t n, const void *x,
    int64_t x_stride, const void *grad_y, int64_t gy_stride, const void *grad_alpha,
    void *grad_x, int64_t gx_stride, void *grad_h, int64_t gh_stride, int64_t batch, void *ws,
    size_t ws_bytes, hipStream_t stream);

/* Strided batch of BHHB products of one shape: instance b uses
 * H + b*H_stride, x + b*x_stride (all m vectors equal), y + b*y_stride,
 * alpha + b. */
hk_status_t block_hankel_tvp_strided_batched_workspace_size(hk_dtype_t dt, int m,
                                                            const int64_t *inner_dims,
                                                            const int64_t *block_dims,
                                                            int64_t batch, size_t *bytes);
hk_status_t block_hankel_tvp_strided_batched(hk_dtype_t dt, const void *H, int64_t H_stride,
                                             int m, const int64_t *inner_dims,
                                             const int64_t *block_dims, const void *x,
                                             int64_t x_stride, void *y, int64_t y_stride,
                                             void *alpha, int64_t batch, void *ws,
                                             size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------------------------
 * Schedule control and diagnostics.
 * ------------------------------------------------------------------------- */
/* Process-wide choice of transform lengths for the calls and plans created
 * afterwards.  HK_LENGTHS_SMALLEST takes the smallest length with kernels
 * (2^k, 3 * 2^k, 5 * 2^k); HK_LENGTHS_AUTO (default) does so when the call's
 * work is large enough to fill the device (instances * the power-of-two
 * length >= 2^18: a plan's instances, a strided batch's count) and takes the
 * power of two otherwise, where the odd lengths' longer per-lane sequences
 * would cost latency; under AUTO the factor 5 is taken for resident
 * transforms (5 * 2^k with 2^k <= 2048), for three-pass ones only where
 * instances * N >= 2^22 (strided batches and single calls; not in plans), and
 * for BHHB row axes where instances * grid >= 2^22: with less work its
 * three-pass row kernels are slower than the next length (3 * 2^k or 2^k);
 * HK_LENGTHS_POW2 takes power-of-two complex transforms
 * only.  Real forward products use their half-length transform under AUTO
 * and SMALLEST.  Workspace sizes depend on the policy: query them under the
 * policy the call runs with.  Not synchronized with calls running on other
 * host threads. */
#define HK_LENGTHS_AUTO 0
#define HK_LENGTHS_POW2 1
#define HK_LENGTHS_SMALLEST 2
hk_status_t hk_set_fft_lengths(int policy);
int hk_get_fft_lengths(void);
/* Padded FFT length N (1D) chosen for a single product with a given d_H
 * (complex64 data, current length policy, default schedule) and the row x
 * column split of each of its power-of-two sequences:
 * N = odd * n_row * n_col with odd = N / (n_row * n_col) in {1, 3, 5};
 * n_col = 1 means one workgroup holds the whole transform. */
hk_status_t hk_fft_layout(int64_t d_h, int64_t *n_fft, int64_t *n_row, int64_t *n_col);
/* Runs the in-house autotuner for the plain 1D path of one (dtype, m, n)
 * shape on the current device and stores the winner in the process-wide
 * schedule cache that later calls of that shape consult.  Allocates and
 * frees its own temporary device buffers and synchronizes the device. */
hk_status_t hk_autotune_tvp(hk_dtype_t dt, int m, int64_t n, int verbose);
/* General form: kind 0 = hankel_tvp / hankel_tvp_strided_batched shape
 * (m, n); kind 1 = the adjoint of that shape; kind 2 = equal-vector BHHB
 * shape (m, inner_dims, block_dims; n ignored).  batch = instances per call
 * (1 for single products); the cache is kept per batch class (1, < 16,
 * >= 16). */
#define HK_TUNE_FORWARD 0
#define HK_TUNE_ADJOINT 1
#define HK_TUNE_BLOCK 2
hk_status_t hk_autotune(hk_dtype_t dt, int kind, int m, int64_t n, const int64_t *inner_dims,
                        const int64_t *block_dims, int64_t batch, int verbose);

/* Schedule database.  hk_tune_save writes every cached schedule (autotuned or
 * loaded) to a text file, one line per shape key; hk_tune_load merges such a
 * file into the cache (*n_loaded = entries read, may be NULL) so that a
 * process can reuse schedules tuned earlier on the same kind of device
 * without running the autotuner.  Values: E_row 4, 8 or 16; 1-64 rows per
 * workgroup; E_col 8 or 16; a column-tile width that is a power of two from 1
 * to 64; split -4..4; XCD numbering 0 or 1; 1, 2 or 4 rows in turn.  A
 * malformed or out-of-range line rejects
 * the whole file with HK_ERR_INVALID_VALUE and leaves the cache unchanged;
 * loaded entries that the kernels cannot run are ignored at use time.  Host
 * only: no device work. */
hk_status_t hk_tune_save(const char *path);
hk_status_t hk_tune_load(const char *path, int *n_loaded);
/* Number of the library's kernel launches enqueued by the last call made on
 * this thread (diagnostics). */
int hk_last_launch_count(void);
/* Kernel timing (diagnostics).  Between start and stop, every kernel the
 * library enqueues is launched with a start/stop HIP event pair that the
 * runtime timestamps at that dispatch's own begin and end (the kernel's
 * execution time, as a kernel trace reports it).  Not for use during graph
 * capture.  hk_profile_stop synchronizes on those events and returns, per kernel kind,
 * the summed duration in milliseconds and the number of launches (arrays of
 * HK_PROF_KINDS entries): 0 resident single-workgroup transforms, 1 pass A
 * (column FFTs of the inputs), 2 pass B (row FFTs + spectral product),
 * 3 pass D (column FFTs of the output + slice), 4 batched task kernels (persistent or grouped). */
#define HK_PROF_KINDS 5
hk_status_t hk_profile_start(void);
hk_status_t hk_profile_stop(double *ms_by_kind, int64_t *launches_by_kind);

const char *hk_status_string(hk_status_t s);
const char *hk_last_error(void);
int hk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HANKEL_H_ */
