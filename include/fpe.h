/*
 * fpe.h — C ABI of the MI355X (gfx950) Fast Polynomial Evaluator library.
 *
 * The library implements the evaluation phase of the Fast Polynomial Evaluator
 * (FPE) of Anton, Mihalache and Vigneron, "Fast evaluation of real and complex
 * polynomials" (arXiv 2211.06320): many points z against one preconditioned
 * complex polynomial P(z) = a_0 + a_1 z + ... + a_d z^d.
 *
 * Conventions shared by every entry point:
 *   - Complex numbers are interleaved (re, im) pairs of IEEE binary64, the
 *     memory layout of C99 double complex and of torch.complex128.
 *   - Coefficients are ordered a_0 first (the paper's CSV convention, Section 8.1).
 *   - Arguments named *_dev are device pointers on the current HIP device;
 *     arguments named *_host are host pointers.  The library never allocates
 *     device memory: the caller provides every device buffer, including the
 *     workspaces sized by the *_workspace_size queries.
 *   - Values are returned as P(z) = m 2^e with m a complex double whose larger
 *     component lies in [1/2, 1) (or m = 0, e = 0) and e a 64-bit integer: the
 *     paper's number model has unbounded exponents (Section 2.2), and at the
 *     sizes this library targets |P(z)| routinely exceeds the FP64 range.
 *   - Every call returns an fpe_status; FPE_OK is 0.  Nothing is printed and no
 *     exception crosses the ABI.  fpe_last_error() gives a thread-local detail
 *     string for the last failing call on the calling thread.
 *   - Work is enqueued on the given stream.  These calls wait for it before
 *     returning (they read counters back to the host to build a host handle or
 *     to time): fpe_precondition, fpe_precondition_batched, fpe_cover_build,
 *     fpe_plan_from_cover, fpe_batch_create, fpe_autotune,
 *     fpe_batch_autotune and fpe_profile_read; fpe_plan_export copies from the
 *     device synchronously.  Every other call (fpe_eval, fpe_eval_noalloc,
 *     fpe_eval_deriv, fpe_newton_step, fpe_eval_adjoint, fpe_cancelled_bits,
 *     fpe_eval_batched, fpe_horner_eval) only enqueues kernels and returns, so
 *     a HIP graph can capture it once a first call has set the library up on
 *     the device (occupancy queries).
 *   - Evaluations keep no state in the plan or batch: calls on different
 *     streams may overlap as long as each has a workspace of its own.  Calls
 *     that share a workspace (or fpe_eval_noalloc's static one) must not
 *     overlap.  The tuning setters (fpe_plan_set_*, fpe_batch_set_chunk,
 *     the autotuners) change the plan or batch for later calls and must not
 *     run concurrently with calls that use it.
 */
#ifndef FPE_H
#define FPE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fpe_status;

enum {
    FPE_OK = 0,
    FPE_ERR_INVALID_ARG = 1,   /* NULL pointer, negative size, bad flag         */
    FPE_ERR_NONFINITE = 2,     /* a coefficient is NaN or infinite               */
    FPE_ERR_PRECISION = 3,     /* p_bits outside 1..53                           */
    FPE_ERR_WORKSPACE = 4,     /* workspace smaller than the size query's answer */
    FPE_ERR_HIP = 5,           /* a HIP runtime call failed                      */
    FPE_ERR_UNSUPPORTED = 6    /* input outside the supported range (see below)  */
};

/* Opaque handle of a preconditioned polynomial.  The handle lives in host
   memory; its tables live in the caller's precondition workspace, which must
   stay allocated and unmodified for the handle's lifetime. */
typedef struct fpe_plan_s *fpe_plan_t;

/* Human-readable name of a status code (static storage). */
const char *fpe_status_string(fpe_status s);

/* Detail message of the last failing call on this thread (thread-local storage;
   "" when the last call succeeded). */
const char *fpe_last_error(void);

/* ABI version, incremented on incompatible changes. */
int32_t fpe_abi_version(void);

/* ------------------------------------------------------------------------- */
/* Preconditioning (Algorithm A_p, first block; Section 5.1).                */
/* ------------------------------------------------------------------------- */

/* Precondition flags. */
enum {
    /* fpe_eval of this plan sums the windows in FP32 (requires p_bits <= 24):
     * the coefficients a_k (k in G_p) are also stored as FP32 numbers scaled
     * per chunk of C coefficients, each tile's window part runs a plain FP32
     * Horner recurrence over blocks of 8 coefficients, and the block partials
     * are accumulated in FP64 (Horner in z^8), as are z^l and the sum over
     * chunks.  A tile falls back to FP64 arithmetic where FP32 cannot hold it:
     * a chunk whose good coefficients span more than 120 binary orders (or
     * whose cover drops by more than 99 within the chunk), a wavefront holding
     * a point with |z| outside [2^-12, 2^12], the ragged start of windows
     * inside a tile.  Error bound: the FP32 block Horner contributes at most
     * about 24 2^-24 sum |a_k||z|^k (8 steps, the rounding of z and of a_k).
     * fpe_eval_deriv and fpe_newton_step sum Q and Q' the same way (the block
     * derivatives accumulated as Q' <- Q' z^8 + 8 z^7 Q + block's); the reverse
     * mode (fpe_eval_adjoint) stays in FP64.  Which tiles run in FP32 depends
     * on the points sharing a wavefront, so the last bits of an FP32 plan's
     * values can vary from call to call (within the bound). */
    FPE_PRECONDITION_FP32 = 1u,
    /* With FPE_PRECONDITION_FP32: each FP32 block runs the compensated Horner
     * recurrence instead of the plain one: the products s z split exactly by
     * TwoProd (fused multiply-add), the additions by TwoSum, and the lost parts
     * (with the rounding error of z in FP32) carried in an FP32 correction
     * term; the block's sum is the sum of the two.  The recurrence's error
     * drops to a few units of 2^-48 per step; the rounding of the coefficients
     * to FP32 (at most 2^-24 of each term) then bounds the error: about
     * 2^-24 sum |a_k||z|^k.  About ten times the FP32 operations of the plain
     * form; values only (fpe_eval_deriv runs the plain form). */
    FPE_PRECONDITION_FP32_COMPENSATED = 2u
};

/* Bytes of device workspace fpe_precondition needs for a polynomial of degree
   d (d + 1 coefficients) at precision p_bits.  flags: 0 or
   FPE_PRECONDITION_FP32 (then p_bits <= 24). */
fpe_status fpe_precondition_workspace_size(int64_t d, int32_t p_bits, uint32_t flags,
                                           size_t *bytes);

/* Preconditions P for precision p_bits (Algorithm A_p, preconditioning):
 * computes the scales s(a_k) = 1 + floor(log2|a_k|) (Section 2.3), their concave
 * cover Ehat (the least concave majorant, Section 4.1), and the good set
 * G_p = { k : s(a_k) >= Ehat(k) - p - s(d) - 3 } (eq. threshold).
 *
 *   coef_dev        2 (d + 1) doubles, a_0 first; read only; may be freed once
 *                   the call has returned.
 *   d               degree as given, 0 <= d < 2^31 - 1.  Zero coefficients at
 *                   either end are trimmed (the paper assumes a_0 != 0 and
 *                   a_d != 0, Section 4.3), so s(d) uses the trimmed degree.
 *   p_bits          1..53: the precision p of the truncation rule (53 = FP64,
 *                   24 = FP32).
 *   flags           0, or FPE_PRECONDITION_FP32 (p_bits <= 24; FP32 window sums).
 *   workspace_dev   device buffer of at least the queried size, 256-byte aligned;
 *                   owned by the caller, borrowed by the plan.
 *   stream          HIP stream the work is enqueued on; the call waits for it.
 *   out_plan        receives the handle (free it with fpe_plan_destroy).
 *
 * Errors: FPE_ERR_INVALID_ARG (NULL pointer, d out of range, misaligned
 * workspace, unknown flag), FPE_ERR_PRECISION (p_bits outside 1..53, or above
 * 24 with FPE_PRECONDITION_FP32), FPE_ERR_WORKSPACE, FPE_ERR_NONFINITE (a NaN or
 * infinite coefficient), FPE_ERR_UNSUPPORTED (the scales of the good
 * coefficients span more binary orders of magnitude than an FP64 window sum can
 * hold: max s - min good s > 2 (958 - T)), FPE_ERR_HIP.  An all-zero polynomial
 * is accepted (P == 0). */
fpe_status fpe_precondition(const double *coef_dev, int64_t d, int32_t p_bits, uint32_t flags,
                            void *workspace_dev, size_t workspace_bytes,
                            hipStream_t stream, fpe_plan_t *out_plan);

/* The two parts of preconditioning apart (Remark partialpreproc, Section 5.1:
 * the concave cover does not depend on p, only G_p does): fpe_cover_build
 * computes the scales and their concave cover once; fpe_plan_from_cover then
 * finishes a plan for a precision p (G_p and the tables, in O(d)) as often as
 * needed, e.g. for p = 53 and p = 24.  A plan from a cover is bit for bit the
 * plan fpe_precondition builds from the same coefficients and p. */
typedef struct fpe_cover_s *fpe_cover_t;

/* Bytes of device workspace fpe_cover_build needs for degree d. */
fpe_status fpe_cover_workspace_size(int64_t d, size_t *bytes);

/* The scales s(a_k) and their concave cover (Algorithm A_p, lines 2-3), in
 * workspace_dev (caller-owned, 256-byte aligned, borrowed by the cover: keep
 * it until fpe_cover_destroy).  coef_dev as fpe_precondition (only read here).
 * The call waits for stream.  Errors: FPE_ERR_INVALID_ARG, FPE_ERR_WORKSPACE,
 * FPE_ERR_NONFINITE, FPE_ERR_HIP. */
fpe_status fpe_cover_build(const double *coef_dev, int64_t d, void *workspace_dev, size_t workspace_bytes,
                           hipStream_t stream, fpe_cover_t *out_cover);

/* Cover summary, written to info_host[0..4]: d, v (first nonzero index, -1 if
 * P == 0), d' (last nonzero index), number of cover vertices, max s(a_k). */
fpe_status fpe_cover_info(fpe_cover_t cover, int64_t *info_host);

/* Frees the host handle (the workspace stays the caller's). */
fpe_status fpe_cover_destroy(fpe_cover_t cover);

/* Bytes of device workspace fpe_plan_from_cover needs (p_bits and flags as
 * fpe_precondition). */
fpe_status fpe_plan_from_cover_workspace_size(fpe_cover_t cover, int32_t p_bits, uint32_t flags, size_t *bytes);

/* Finishes the preconditioning for precision p_bits (Algorithm A_p, line 4):
 * G_p and the tables of a plan, in workspace_dev (caller-owned, 256-byte
 * aligned, borrowed by the plan).  coef_dev must hold the coefficients the
 * cover was built from (read again here; not checked).  The plan copies the
 * cover's vertices: the cover may be destroyed afterwards.  The call waits for
 * stream.  Arguments otherwise and errors as fpe_precondition. */
fpe_status fpe_plan_from_cover(fpe_cover_t cover, const double *coef_dev, int32_t p_bits, uint32_t flags,
                               void *workspace_dev, size_t workspace_bytes, hipStream_t stream,
                               fpe_plan_t *out_plan);

/* Many polynomials preconditioned by one launch sequence and one wait:
 * polynomial i has the coefficients coef_dev[2 off[i] .. 2 off[i+1] - 1]
 * (complex, a_0 first; off = coef_offsets_host, n_poly + 1 host int64,
 * off[0] = 0, at least one coefficient each).  Polynomials of at most 2^17
 * coefficients are preconditioned by one workgroup each, all in one launch;
 * larger ones by the per-coefficient kernels of fpe_precondition, on the same
 * stream.  plans_out (host array of n_poly handles) receives ordinary plans,
 * bit for bit those of fpe_precondition, each borrowing its part of
 * workspace_dev (caller-owned, 256-byte aligned, at least the queried size);
 * destroy each with fpe_plan_destroy.  p_bits and flags apply to every
 * polynomial.  On an error no plan is returned, and the message names the
 * first failing polynomial.  Errors as fpe_precondition. */
fpe_status fpe_precondition_batched_workspace_size(int32_t n_poly, const int64_t *coef_offsets_host,
                                                   int32_t p_bits, uint32_t flags, size_t *bytes);
fpe_status fpe_precondition_batched(const double *coef_dev, const int64_t *coef_offsets_host, int32_t n_poly,
                                    int32_t p_bits, uint32_t flags, void *workspace_dev, size_t workspace_bytes,
                                    hipStream_t stream, fpe_plan_t *plans_out);

/* Plan summary, written to info_host[0..9]:
 *   0 d (as given)      1 v (first nonzero index, -1 if P == 0)
 *   2 d' (last nonzero) 3 number of cover vertices
 *   4 |G_p|             5 T = p + s(d' - v) + 3
 *   6 p_bits            7 chunk length C of the window kernel
 *   8 max s(a_k)        9 minimum s(a_k) over G_p                              */
#define FPE_PLAN_INFO_LEN 10
fpe_status fpe_plan_info(fpe_plan_t plan, int64_t *info_host);

/* Copies the cover vertices (k_i, s(a_{k_i})), increasing k, into
 * hull_k_host / hull_s_host (capacity hull_cap entries each; at least
 * info[3] are needed) and the good-set indicator into good_host (d + 1 bytes,
 * 1 = k in G_p).  Any of the three pointers may be NULL to skip that table. */
fpe_status fpe_plan_export(fpe_plan_t plan, int64_t *hull_k_host, int64_t *hull_s_host,
                           int64_t hull_cap, uint8_t *good_host);

/* Frees the host handle; the workspace stays the caller's. */
fpe_status fpe_plan_destroy(fpe_plan_t plan);

/* ------------------------------------------------------------------------- */
/* Evaluation (Algorithm A_p, second block; Section 5.2).                    */
/* ------------------------------------------------------------------------- */

/* Bytes of device workspace fpe_eval needs for n points with this plan. */
fpe_status fpe_eval_workspace_size(fpe_plan_t plan, int64_t n, size_t *bytes);

/* Evaluates Q_lambda(z_j) = sum over k in G_p within [l_j, r_j] of a_k z_j^k
 * (eq. reducedQlambda) at n points, where lambda = log2|z| (eq. defLambda),
 * N = max(Ehat + lambda Id) (eq. defN) and [l, r] is the largest integer
 * interval on which Ehat(k) + lambda k >= N - p - s(d) - 3 (eq. def:LRN).
 *
 *   z_dev          2n doubles; read only.
 *   n              number of points, 0 <= n < 2^31 (n == 0 is a no-op).
 *   m_dev, e_dev   outputs: 2n doubles and n int64, Q_lambda(z_j) = m_j 2^{e_j}.
 *   terms_dev      optional (NULL to skip): n int32, #(G_p within [l_j, r_j]),
 *                  the number of terms the method keeps.
 *   window_dev     optional (NULL to skip): 2n int64, (l_j, r_j) per point;
 *                  l_j > r_j marks an empty window.
 *   workspace_dev  at least fpe_eval_workspace_size bytes, 256-byte aligned.
 *
 * Special points: z = 0 gives a_0 (window [0, 0]); a NaN or infinite
 * coordinate gives m = NaN, e = 0, an empty window and 0 terms; P == 0 gives
 * m = 0, e = 0.  Concurrent calls on one plan are safe with distinct
 * workspaces.  Errors are reported synchronously for bad arguments
 * (FPE_ERR_INVALID_ARG, FPE_ERR_WORKSPACE) and as FPE_ERR_HIP for a failed
 * launch. */
fpe_status fpe_eval(fpe_plan_t plan, const double *z_dev, int64_t n,
                    double *m_dev, int64_t *e_dev, int32_t *terms_dev, int64_t *window_dev,
                    void *workspace_dev, size_t workspace_bytes, hipStream_t stream);

/* fpe_eval without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * results as fpe_eval, bit for bit, with the workspace in a static device array
 * of 96 MiB that the library holds on each device it runs on until the process
 * ends.  The call makes no hipMalloc, hipFree or other allocating call; the
 * first call on a device looks up the array's address there
 * (hipGetSymbolAddress).
 *
 *   plan, z_dev, n, m_dev, e_dev, terms_dev, window_dev, stream: as fpe_eval.
 *
 * Limit: the evaluation's workspace (fpe_eval's layout, sized for this call
 * alone) must fit in the 96 MiB array; 2^17 points always fit, and larger n
 * fails with FPE_ERR_WORKSPACE (use fpe_eval then).  Every call on one device
 * shares that device's array, which keeps the last call's contents: calls that
 * overlap on one device (two streams, two threads) race and must be
 * serialised by the caller.  Errors: those of fpe_eval, with
 * FPE_ERR_WORKSPACE meaning "n above the static scratch's limit". */
fpe_status fpe_eval_noalloc(fpe_plan_t plan, const double *z_dev, int64_t n,
                            double *m_dev, int64_t *e_dev, int32_t *terms_dev, int64_t *window_dev,
                            hipStream_t stream);

/* Q_lambda(z_j) as fpe_eval does, and in the same pass its derivative
 * Q'_lambda(z_j) = sum over k in G_p within [l_j, r_j] of k a_k z_j^(k-1): the
 * derivative of the terms the method keeps, through the same window (the
 * Newton iteration of Section 7.2 divides P by P' evaluated this way).
 *
 *   z_dev, n       as fpe_eval.
 *   m_dev, e_dev   outputs: Q = m 2^e, as fpe_eval.
 *   md_dev, ed_dev outputs: 2n doubles and n int64, Q' = md 2^ed (same
 *                  normalisation as m, e).
 *   workspace_dev  at least fpe_eval_workspace_size bytes (the same workspace
 *                  serves fpe_eval and fpe_eval_deriv).
 *
 * Special points as fpe_eval; where no term of degree >= 1 is kept (z = 0, or
 * |z| so small that a_0 dominates by more than T bits) Q' = 0, e = 0; a
 * non-finite z gives NaN.  Errors as fpe_eval. */
fpe_status fpe_eval_deriv(fpe_plan_t plan, const double *z_dev, int64_t n,
                          double *m_dev, int64_t *e_dev, double *md_dev, int64_t *ed_dev,
                          void *workspace_dev, size_t workspace_bytes, hipStream_t stream);

/* Upper bound of the cancelled bits c (Theorem equivAlgo, eq. (def_prec_loss):
 * c = 0 if |P(z)| >= M, else s(M) - s(P(z)), M = max_k |a_k z^k|) for values
 * v_j = m_j 2^{e_j} standing for P(z_j), e.g. fpe_eval's outputs:
 *   bits_j = max(0, floor(N_j) + 1 - s(v_j)),  N_j = max over the cover of
 *   Ehat(k) + lambda_j k (eq. defN), in FP64 as fpe_eval computes it.
 * By eq. (shear) every term has s(a_k z^k) <= N + 1, so s(M) <= floor(N) + 1:
 * bits_j >= c, and bits_j <= c + 2 when v_j = P(z_j).  With eq. (target) the
 * returned value has at least p - bits_j - 2 correct leading bits (the report
 * of correct bits the paper's library writes per point, Section 8).  s(v) is
 * decided exactly; floor(N) in FP64 (lambda is FP64, as in fpe_eval).
 *   z_dev          2n doubles: the points.
 *   m_dev, e_dev   2n doubles and n int64: the values, normalised or not.
 *   bits_dev       output: n int32.  0 where z_j = 0 (P(0) = a_0 exactly),
 *                  z_j is not finite, or P == 0; INT32_MAX where v_j = 0.
 * No workspace; enqueued on stream (no synchronisation).  Errors:
 * FPE_ERR_INVALID_ARG (NULL plan, a NULL pointer with n > 0, n < 0 or
 * n >= 2^31 - 1, z or m not 16-byte aligned), FPE_ERR_HIP. */
fpe_status fpe_cancelled_bits(fpe_plan_t plan, const double *z_dev, int64_t n, const double *m_dev,
                              const int64_t *e_dev, int32_t *bits_dev, hipStream_t stream);

/* One Newton step per point (Section 7.2, eq. newton): z_out = z - Q / Q' with
 * Q and Q' from fpe_eval_deriv (written to m, e, md, ed as there; the caller
 * keeps them).  The quotient is taken on the mantissas and scaled by
 * 2^(e - ed), so it is finite wherever it is representable.  Where Q' = 0 or z
 * is not finite, z_out is NaN.  z_out_dev: 2n doubles (may alias nothing else).
 * Errors as fpe_eval. */
fpe_status fpe_newton_step(fpe_plan_t plan, const double *z_dev, int64_t n,
                           double *m_dev, int64_t *e_dev, double *md_dev, int64_t *ed_dev,
                           double *z_out_dev, void *workspace_dev, size_t workspace_bytes,
                           hipStream_t stream);

/* Reverse mode of the map (a, z) -> Q_lambda(z) at n points, for upstream
 * gradients g_j (eq. reducedQlambda; the kept set G_p within [l_j, r_j] is
 * held fixed, as the map is piecewise polynomial in a and z).  The convention
 * is that of complex reverse-mode differentiation (PyTorch's): the gradient of
 * a holomorphic map is the upstream gradient times the conjugate of its
 * derivative, so
 *   grad_a[k] = sum over the points j whose kept terms include k of g_j conj(z_j)^k,
 *   grad_z[j] = g_j conj(Q'_lambda(z_j)).
 *
 *   z_dev, n         as fpe_eval.
 *   g_dev            2n doubles: the upstream gradients, input order.
 *   g_exp_dev        NULL, or n int64: the upstream gradients are then
 *                    g_j 2^(-g_exp[j]) (the exponent applied inside, so that a
 *                    gradient with respect to a normalised value m_j = Q_j 2^-e_j
 *                    passes with g_exp = e and nothing underflows).
 *   md_dev, ed_dev   Q' = md 2^ed from fpe_eval_deriv at the same points (only
 *                    read when grad_z_dev is not NULL).
 *   grad_a_dev       output, or NULL to skip: 2 (d + 1) doubles, overwritten
 *                    (zero outside G_p and where no window reaches k).
 *   grad_z_dev       output, or NULL to skip: 2n doubles.
 *   workspace_dev    at least fpe_eval_workspace_size bytes (the workspace of
 *                    fpe_eval serves).
 *
 * Both gradients are plain doubles: a term beyond the double range saturates
 * to an infinity (or NaN where an infinity meets a zero), and one below it
 * flushes to zero.  A point with a non-finite coordinate contributes nothing
 * to grad_a and gets a NaN grad_z; z = 0 contributes g_j to grad_a[0] when
 * a_0 != 0.
 *
 * Summation of grad_a (fpe_plan_set_adjoint_mode): by default
 * (FPE_ADJOINT_EXACT) every term goes to fixed point relative to a per-index
 * scale 2^E_k (E_k bounds every term at k, from a first pass over the tiles)
 * and the terms are summed exactly with integer atomics, so grad_a has the
 * same bits from call to call and for any order of the points; each term is
 * rounded to 2^(E_k - 2S), S = min(47, 62 - bitlen(n)), before the exact sum,
 * and the sum to double once.  A non-finite term makes its grad_a entry NaN.
 * With FPE_ADJOINT_ATOMIC the wavefronts' partial sums go to grad_a with FP64
 * atomic additions instead (one pass, about a third of the time at 2^20
 * points; the last bits then vary from call to call).  Errors as fpe_eval. */
fpe_status fpe_eval_adjoint(fpe_plan_t plan, const double *z_dev, int64_t n, const double *g_dev,
                            const int64_t *g_exp_dev, const double *md_dev, const int64_t *ed_dev,
                            double *grad_a_dev, double *grad_z_dev, void *workspace_dev, size_t workspace_bytes,
                            hipStream_t stream);

/* How fpe_eval_adjoint sums grad_a on this plan (see above):
 * FPE_ADJOINT_EXACT (the default) or FPE_ADJOINT_ATOMIC.  Errors:
 * FPE_ERR_INVALID_ARG (NULL plan, unknown mode). */
enum { FPE_ADJOINT_EXACT = 0, FPE_ADJOINT_ATOMIC = 1 };
fpe_status fpe_plan_set_adjoint_mode(fpe_plan_t plan, int32_t mode);

/* ------------------------------------------------------------------------- */
/* Many polynomials in one evaluation (Algorithm A_p, second block, applied  */
/* to each polynomial of a batch with its own points; Section 5.2).          */
/* ------------------------------------------------------------------------- */

/* Opaque handle: the device tables of a batch (a plan per polynomial and the
 * layout of its points), built once, then evaluated any number of times. */
typedef struct fpe_batch_s *fpe_batch_t;

/* Bytes of device workspace fpe_batch_create needs for n_poly polynomials whose
 * points are laid out by z_offsets_host (n_poly + 1 host int64: polynomial i
 * owns points z_offsets[i] .. z_offsets[i+1] - 1, z_offsets[0] == 0).
 * Errors: FPE_ERR_INVALID_ARG (NULL, n_poly < 1, offsets not starting at 0 or
 * decreasing, 2^31 points or more), FPE_ERR_UNSUPPORTED (a polynomial with
 * more than 4096 points: evaluate it with fpe_eval). */
fpe_status fpe_batch_workspace_size(int32_t n_poly, const int64_t *z_offsets_host, size_t *bytes);

/* Builds a batch from n_poly plans (host array of handles, all on one device;
 * a plan may appear more than once) and the point layout z_offsets_host.  The
 * batch copies the plans' device views (their workspaces must outlive it) into
 * workspace_dev (caller-owned, 256-byte aligned, at least the queried size),
 * on stream; the call waits for the copies.  Errors as
 * fpe_batch_workspace_size, plus FPE_ERR_WORKSPACE and FPE_ERR_HIP. */
fpe_status fpe_batch_create(const fpe_plan_t *plans_host, int32_t n_poly, const int64_t *z_offsets_host,
                            void *workspace_dev, size_t workspace_bytes, hipStream_t stream,
                            fpe_batch_t *out_batch);

/* Releases the host handle (the workspace stays the caller's). */
fpe_status fpe_batch_destroy(fpe_batch_t batch);

/* Bytes of device workspace one fpe_eval_batched call needs. */
fpe_status fpe_eval_batched_workspace_size(fpe_batch_t batch, size_t *bytes);

/* Q_lambda(z_j) of polynomial i at each of its points, for every polynomial of
 * the batch, as fpe_eval would give it: one launch sequence for the whole batch
 * (a workgroup per polynomial computes its points' windows and sorts them by
 * lambda; the (point group, chunk) tiles of all polynomials are then split
 * evenly over the resident wavefronts).  Enqueues kernels only (no host
 * synchronisation, no allocation), so a HIP graph can capture it.
 *
 *   z_dev          2 N doubles, N = z_offsets[n_poly], in the batch's layout.
 *   m_dev, e_dev   outputs, as fpe_eval (input order).
 *   terms_dev      optional n int32 kept-term counts (NULL to skip).
 *   workspace_dev  at least fpe_eval_batched_workspace_size bytes, 256-byte
 *                  aligned; one call at a time per workspace.
 *
 * With FP64 plans the results are bit for bit those of fpe_eval on each plan
 * alone.  Errors: FPE_ERR_INVALID_ARG, FPE_ERR_WORKSPACE, FPE_ERR_HIP. */
fpe_status fpe_eval_batched(fpe_batch_t batch, const double *z_dev, double *m_dev, int64_t *e_dev,
                            int32_t *terms_dev, void *workspace_dev, size_t workspace_bytes,
                            hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Tile schedule: the chunk length C of the (point group, chunk) tiles        */
/* (the paper's window sum, Section 5.2, is cut into pieces of C coefficients */
/* that are summed exactly; C changes the work split, not the method).        */
/* ------------------------------------------------------------------------- */

/* Sets the chunk length of later evaluations of this plan: a power of two in
 * [256, 2048], or 0 for the automatic choice (the length fpe_autotune found for
 * the same bucket of degree and point count earlier in this process, else 512).
 * FP32 plans accept only 0 and 512 (FPE_ERR_UNSUPPORTED otherwise).  Errors:
 * FPE_ERR_INVALID_ARG. */
fpe_status fpe_plan_set_chunk(fpe_plan_t plan, int32_t chunk);

/* The form of fpe_eval's window sums (Section 5.2 sums the kept terms a_k z^k,
 * k in G_p within [l, r]; both forms sum exactly those terms):
 *   FPE_WINDOW_DENSE   Horner's rule over every index of the window, the
 *                      coefficients outside G_p masked to 0 (work ~ r - l + 1);
 *   FPE_WINDOW_SPARSE  Horner's rule over the list of G_p inside the window,
 *                      each gap between two consecutive indices jumped by the
 *                      powers z^(2^j) of its binary digits (the precomputed
 *                      powers of the paper's implementation notes, Section 8.2;
 *                      work ~ #(G_p within [l, r]) times the digits per gap).
 * fpe_eval_deriv, fpe_newton_step, fpe_eval_adjoint and batches run the dense
 * form; FP32 plans run the dense form only. */
enum { FPE_WINDOW_AUTO = 0, FPE_WINDOW_DENSE = 1, FPE_WINDOW_SPARSE = 2 };

/* Sets the window-sum form of later fpe_eval calls on this plan: one of the
 * FPE_WINDOW_* values (AUTO: the form fpe_autotune found for the same bucket
 * of degree, point count and |G_p| earlier in this process, else DENSE).
 * Errors: FPE_ERR_INVALID_ARG (NULL plan, unknown mode), FPE_ERR_UNSUPPORTED
 * (SPARSE on an FP32 plan). */
fpe_status fpe_plan_set_window_mode(fpe_plan_t plan, int32_t mode);

/* The chunk length and the window-sum form (FPE_WINDOW_DENSE or
 * FPE_WINDOW_SPARSE) an fpe_eval of n points on this plan would use now.
 * Either output pointer (host) may be NULL.  Errors: FPE_ERR_INVALID_ARG. */
fpe_status fpe_plan_tile_choice(fpe_plan_t plan, int64_t n, int32_t *chunk_out, int32_t *mode_out);

/* Times fpe_eval of these n points (writing m, e as fpe_eval does) with each
 * candidate chunk length 256, 512, 1024, 2048 in each window-sum form (one
 * untimed and three timed calls each, HIP events on stream; the call waits),
 * keeps the fastest pair for this plan, records it for the plan's bucket (bit
 * lengths of d, n and |G_p|) in a process-wide cache that untuned plans
 * consult, and writes the chunk length to *chunk_out (may be NULL); the form is
 * readable with fpe_plan_tile_choice.  FP32 plans keep 512 and the dense form.
 * Arguments and errors as fpe_eval. */
fpe_status fpe_autotune(fpe_plan_t plan, const double *z_dev, int64_t n, double *m_dev, int64_t *e_dev,
                        void *workspace_dev, size_t workspace_bytes, hipStream_t stream, int32_t *chunk_out);

/* The same for a batch (fpe_eval_batched; the cache bucket is the mean degree
 * and the point count of the batch). */
fpe_status fpe_batch_set_chunk(fpe_batch_t batch, int32_t chunk);
fpe_status fpe_batch_autotune(fpe_batch_t batch, const double *z_dev, double *m_dev, int64_t *e_dev,
                              void *workspace_dev, size_t workspace_bytes, hipStream_t stream,
                              int32_t *chunk_out);

/* ------------------------------------------------------------------------- */
/* Same-GPU baseline: Horner's rule on the full polynomial (Section 1).      */
/* ------------------------------------------------------------------------- */

/* P(z_j) = sum_{k=0}^{d} a_k z_j^k by Horner's rule in FP64, one lane per point,
 * with exact power-of-two rescaling so that the result is returned as
 * m_j 2^{e_j} like fpe_eval.  coef_dev: 2 (d + 1) doubles, a_0 first; no
 * workspace.  Errors: FPE_ERR_INVALID_ARG, FPE_ERR_HIP. */
fpe_status fpe_horner_eval(const double *coef_dev, int64_t d, const double *z_dev, int64_t n,
                           double *m_dev, int64_t *e_dev, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Instrumentation (for measurement only).                                   */
/* ------------------------------------------------------------------------- */

/* on != 0: every later fpe_eval records a HIP event pair around its window
 * kernel (the dominant kernel of an evaluation) on the call's stream; on == 0
 * stops recording.  Events come from a library-owned pool (hipEventCreate, no
 * device memory); the pool is process-wide and not thread-safe. */
fpe_status fpe_profile_enable(int32_t on);

/* Waits for every recorded event pair, writes the summed elapsed time of the
 * window kernels in milliseconds and the number of launches, then forgets them.
 * Either pointer may be NULL. */
fpe_status fpe_profile_read(double *window_ms_host, int64_t *launches_host);

#ifdef __cplusplus
}
#endif

#endif /* FPE_H */
