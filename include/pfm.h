/*
 * pfm.h -- C ABI of libpfm: parallel fractional matrix functions on MI355X.
 *
 * Implements the method of S. Blanes, "Parallel computation of functions of
 * matrices and their action on vectors" (arXiv:2210.03714):
 *
 *   f(B) ~ r(B) = a0 I + sum_k w_k (I - c_k B)^{-1} B,   w_k = b_k c_k,
 *
 * i.e. the approximant sum_i b_i (I - c_i B)^{-1} of §2 (eqs. 2 and 4) in the
 * round-off-reducing form of §4.3, with the shifts c_k and weights b_k of the
 * paper's sets for each solve count m.  The m shifted solves are independent
 * (the paper's "processors") and run concurrently on the GPU.  Large norms are
 * handled as in §1: B = A / 2^s followed by s squarings for f(A), or B = A / N
 * followed by the recurrence v_j = r(B) v_{j-1} (N steps) for f(A) V.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: PFM_OK (0) on success; a negative PFM_ERR_* code means that
 *   nothing was enqueued and outputs are untouched (text via pfm_last_error).
 *   Per-instance outcomes (a singular shift, non-finite input, an instance
 *   not computed) are decided on the device, after the call has returned:
 *   the calls return PFM_OK and the caller reads pfm_info.status once the
 *   stream has synchronised.
 * - Matrices are row-major with a leading dimension counted in elements
 *   (ld >= n).  Complex data is interleaved (re, im) binary64, the layout of
 *   C99 double _Complex and torch.complex128.
 * - Device pointers are HIP device pointers on the context's device.  The
 *   caller owns every buffer it passes; the library never frees them and never
 *   writes to inputs.  The context owns all workspace.
 * - All device work is enqueued on the caller's stream and the calls return
 *   without waiting for it: the norm, the plan (s or N), the route of every
 *   instance and the number of squarings are decided by kernels, and no
 *   result is read back (the one exception: an action on an instance above
 *   512, complex above 256, whose steps are launched one by one, reads its
 *   step count back).  A call waits on the stream only to grow the
 *   workspace.  One context must not be used from two streams at the same
 *   time (its workspace is shared between calls).
 */
#ifndef PFM_H
#define PFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfm_ctx pfm_ctx;
typedef void *pfm_stream_t; /* a hipStream_t; NULL is the null stream */

/* functions (bit mask: EXP|PHI1 computes both from one set of solves, §2) */
#define PFM_EXP 1
#define PFM_PHI1 2
/* log(1 - A) (§2 worked example): on its own (f == PFM_LOG1M), m = 5 (the
 * shifts 1/2..1/6), real binary64 full matrices.  It has no scaling
 * identity, so r(A) is evaluated directly (s = 0); the bound of §3 holds for
 * ||A||_1 <= θ (PFM_OUT_OF_RANGE otherwise).  The result goes to F_exp. */
#define PFM_LOG1M 4
/* phi2(A) = sum_k A^k / (k + 2)! (§1's phi_k with k = 2, the Taylor
 * polynomial of degree k - 1 removed): weights solving eq. (4) with
 * a_k = 1/(k + 2)! on the exponential's shifts, and the doubling
 * phi2(2B) = (phi1(B)^2 + 2 phi2(B)) / 4 between the squarings (the phi1
 * chain is computed for it even when F_phi1 is not requested).  Combines
 * with PFM_EXP and PFM_PHI1; real full matrices up to n = 512 in binary64
 * with m = 4, 5 or 8 (PFM_ERR_UNSUPPORTED otherwise: action, complex,
 * mixed, the hybrid sets, larger n, the tridiagonal / banded paths and the
 * serving queue). */
#define PFM_PHI2 8

/* element types */
#define PFM_R64 0  /* real binary64 */
#define PFM_C128 1 /* complex, interleaved binary64 */

/* precision paths */
#define PFM_FP64 0  /* LU, solves, combination and squaring in binary64 */
#define PFM_MIXED 1 /* LU and solves in binary32 on MFMA with binary64
                       iterative-refinement residuals; combination and
                       squaring in binary64 */

/* routes of the full-matrix FP64 path (pfm_set_route) */
#define PFM_ROUTE_AUTO 0
#define PFM_ROUTE_LU 1

/* return codes */
#define PFM_OK 0
#define PFM_ERR_INVALID (-1)     /* null pointer, n < 1, ld < n, p < 0, tol not in (0,1), an array not 8-byte aligned, ... */
#define PFM_ERR_UNSUPPORTED (-2) /* (f, m, dtype, prec) combination not provided */
#define PFM_ERR_BUDGET (-3)      /* workspace would exceed the context's HBM budget */
#define PFM_ERR_HIP (-4)         /* HIP runtime error */
#define PFM_ERR_DEVICE (-5)      /* a bounded device-side wait of the squaring queue gave up (pfm_check) */

/* per-instance status bits (pfm_info.status) */
#define PFM_SINGULAR_SHIFT 1 /* an exact zero pivot in I - c_k B; bad_shift = k */
#define PFM_NONFINITE 2      /* ||A||_1 is not finite (NaN or Inf in A) */
#define PFM_IR_STALL 4       /* mixed path: refinement did not reach the target */
#define PFM_NOT_COMPUTED 8   /* the instance was not computed and its outputs
                                were not written: n > 512 (complex: > 256)
                                with A not finite or some shifted matrix
                                I - c_k B not diagonally dominant enough for
                                the large-instance route (|c_k| ||B||_1 <= 1/2;
                                the planner's B always is, a forced plan may
                                not); the hybrid set (m = 10) on an instance
                                that is not (only a forced plan or non-finite
                                input can do that); more than PFM_MAX_SQUARINGS
                                squarings; or more than PFM_MAX_STEPS steps */
#define PFM_OUT_OF_RANGE 16  /* PFM_LOG1M: ||A||_1 > θ, so the tolerance is not
                                guaranteed (the result is still computed) */

/* One problem instance.  p == 0: full matrix, F_exp / F_phi1 / F_phi2 are n x n with
 * leading dimension ldf.  p >= 1: action on the n x p block V (leading
 * dimension ldv), F_exp / F_phi1 are n x p with leading dimension ldf.
 * Outputs not requested by the function mask may be NULL.  Every array is
 * device memory at an address that is a multiple of 8 (PFM_ERR_INVALID
 * otherwise). */
typedef struct {
  int32_t n;
  int32_t p;
  int64_t lda;
  int64_t ldv;
  int64_t ldf;
  const void *A;
  const void *V;
  void *F_exp;
  void *F_phi1;
  void *F_phi2;  /* PFM_PHI2 output (full matrices), else ignored */
} pfm_problem;

/* Per-instance report, written to device memory by pfm_eval_batched. */
typedef struct {
  int32_t status;    /* PFM_SINGULAR_SHIFT | PFM_NONFINITE | PFM_IR_STALL | PFM_NOT_COMPUTED */
  int32_t plan;      /* s (full matrix: B = A / 2^s) or N (action: B = A / N) */
  int32_t order;     /* order of the rational approximation (eq. 3) */
  int32_t ir_iters;  /* mixed path: refinement sweeps performed */
  int32_t bad_shift; /* first shift index with a zero pivot, -1 if none */
  int32_t route;     /* 1: shifted inverses by Gauss-Jordan without interchanges
                        (every |c_k| ||B||_1 <= 1/2); 2: the same for a large
                        instance (n > 512, complex n > 256), spread over many
                        workgroups; 0: pivoting LU route; 3: tridiagonal
                        action (pfm_tri_action); 4: banded action
                        (pfm_band_action) */
  double norm1;      /* ||A||_1 */
  double theta;      /* admissible ||B||_1 for the requested tolerance (§3) */
  double resid;      /* mixed path: largest relative refinement residual */
} pfm_info;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the
 * workspace the context may allocate (0 = no cap).  Allocation happens lazily
 * on the first call that needs it. */
int pfm_create(pfm_ctx **ctx, int device, size_t hbm_budget_bytes);

/* Destroy a context and free its workspace.  The caller must have
 * synchronised every stream that used it. */
int pfm_destroy(pfm_ctx *ctx);

/* Text of the last error on this context (never NULL). */
const char *pfm_last_error(const pfm_ctx *ctx);

/* Host only.  Coefficients of the set used for function `f` (PFM_EXP,
 * PFM_PHI1, PFM_PHI2 or PFM_LOG1M, one of them) with m solves: the round-off form of §4.3,
 * r(x) = a0 + sum_k w_k x / (1 - c_k x), with w_k = b_k c_k and b_k the
 * solution of eq. (4) (§2).  m = 1: the 4th-order Padé pair of eq. (5) (exp)
 * or eq. (6) (phi1) written in this form, one conjugate pair (the conjugate
 * term is implied, *is_pair = 1).  m = 4: the set of §4.1 with alpha = 5;
 * m = 5: the set of §5.1; m = 8: the set of §4.2 with alpha = 5.  phi1 weights
 * solve eq. (4) with a_k = 1/(k+1)! on the same shifts, phi2 weights
 * (m = 4, 5, 8) with a_k = 1/(k+2)!.  m = 10 (exp only):
 * the hybrid 10th-order set of §4.3 with the smaller coefficients
 * (c = -+1/8, -+1/10, ..., -+1/16; b_9 = 2000, b_10 = -3500), whose
 * polynomial part pfm_poly returns (a0 = d0 + sum_k b_k); m = PFM_R10STAR
 * (exp only): the other one, R*10 (c_i = 1/(6 + i), b_9 = -5 10^4,
 * b_10 = 3.5 10^5).  Arrays must hold 16 entries.  Returns
 * PFM_ERR_UNSUPPORTED for an unknown (f, m). */
int pfm_coeffs(int f, int m, int *n_terms, double *c_re, double *c_im,
               double *w_re, double *w_im, double *a0, int *order,
               int *is_pair);

/* Host only.  The polynomial part d1 x + d2 x^2 of the approximant of (f, m)
 * (§4.3, hybrid sets): r(x) = a0 + d1 x + d2 x^2 + sum_k w_k x / (1 - c_k x).
 * Both are 0 for the partial-fraction sets.  PFM_ERR_UNSUPPORTED for an
 * unknown (f, m). */
int pfm_poly(int f, int m, double *d1, double *d2);

/* Host only.  θ(f, m, tol): the largest x with sum_k |a_k - alpha_k| x^k <=
 * tol (forward bound of §3; absolute, any consistent norm).  For a mask
 * with several functions the minimum; PFM_PHI2 brings in the exponential's
 * and phi1's bounds too (its doubling squares phi1, whose doubling applies
 * e^B). */
int pfm_theta(int f, int m, double tol, double *theta);

/* Largest squaring count s of the full-matrix path (above it the instance is
 * PFM_NOT_COMPUTED). */
#define PFM_MAX_SQUARINGS 1000

/* The solve count that selects the other hybrid 10th-order set of §4.3,
 * R*10 (eqs. Frac10ciNO-Frac10biNO: c_i = 1/(6 + i), i = 1..10, b_9 = -5 10^4,
 * b_10 = 3.5 10^5), the set the θ_10 of §5.1 (Table 2) is computed for.
 * Ten shifted solves, exp only, like m = 10; its weights are large
 * (sum |w_k| about 1.3e6), so its rounding floor (pfm_eval_batched) is about
 * 2e-10: tolerances below it are refused. */
#define PFM_R10STAR 110

/* Evaluate a batch of problems.
 *   f          PFM_EXP, PFM_PHI1, PFM_PHI2 (any combination), or PFM_LOG1M
 *   m          number of shifted solves: 1, 4, 5 or 8; or 10, the hybrid set
 *              of §4.3, for PFM_EXP of real matrices in binary64: full
 *              matrices on the Gauss-Jordan routes (every |c_k| ||B||_1 <=
 *              1/2, which planned steps meet; PFM_ERR_UNSUPPORTED otherwise),
 *              the action (p >= 1) on every route, each step adding
 *              d1 B u + d2 B^2 u; or PFM_R10STAR, the other hybrid set,
 *              likewise
 *   tol        target of the forward bound per scaled step, in (0, 1), and
 *              not below the set's rounding floor (sum_k |w_k| + |d1| + |d2|)
 *              θ(tol) 2^-53, which the round-off form cannot go under
 *              (PFM_ERR_UNSUPPORTED: only R*10 has a floor above 1e-12)
 *   prec       PFM_FP64 or PFM_MIXED
 *   dtype      PFM_R64 or PFM_C128 (for A, V and outputs)
 *   batch      number of problems, >= 1
 *   probs      host array of `batch` problems; sizes may differ
 *   info       device array of `batch` pfm_info records, or NULL
 *   force_plan -1: planner (s or N from ||A||_1 and θ).  >= 0: use this s
 *              (full matrix) or N >= 1 (action) for every instance (tests).
 *   stream     HIP stream to enqueue on
 * A problem with p == 0 and one with p >= 1 may not be mixed in one call.
 * The call may be recorded into the caller's own stream capture (a hipGraph)
 * when it repeats the previous call on the same context exactly (same
 * arguments, problems and pointers) and that call ran eagerly: then it
 * allocates nothing, copies nothing from the host and only launches
 * kernels; otherwise, inside a capture, it returns PFM_ERR_INVALID with
 * nothing recorded.  A captured call stays valid while no other call on the
 * context runs (they share the workspace). */
int pfm_eval_batched(pfm_ctx *ctx, int f, int m, double tol, int prec,
                     int dtype, int batch, const pfm_problem *probs,
                     pfm_info *info, int force_plan, pfm_stream_t stream);

/* pfm_eval_batched with one tolerance per instance (host array tols[batch],
 * each in (0,1)); the scalar tol is ignored when tols is not NULL.  Each
 * instance is planned with its own θ(f, m, tol_i) and reports it in
 * pfm_info.theta; everything else is shared, so instances of different
 * tolerances batch together.  (The mixed path refines to the smallest.) */
int pfm_eval_batched_tols(pfm_ctx *ctx, int f, int m, const double *tols, double tol, int prec, int dtype,
                          int batch, const pfm_problem *probs, pfm_info *info, int force_plan,
                          pfm_stream_t stream);

/* A caller-given partial-fraction decomposition (§2: a rational function
 * with simple poles, r(x) = d0 + sum_k b_k / (1 - c_k x), each pole 1/c_k real
 * or complex): r(A) (p == 0; F_exp receives it) or r(A) V (p >= 1; one step,
 * F_exp), evaluated in the round-off form of §4.3 as
 *     a0 I + sum_k w_k (I - c_k A)^{-1} A,   w_k = b_k c_k,  a0 = d0 + sum_k b_k,
 * with no scaling (s = 0, N = 1: choose the norm range of A beforehand) and
 * every shifted solve independent.  c_k = c_re[k] + i c_im[k] and
 * w_k = w_re[k] + i w_im[k] (c_im, w_im may be NULL: all real).  With
 * conj_pairs != 0 every term with c_im[k] != 0 stands for itself and its
 * conjugate (c_k*, w_k*), so that a real A gives a real r(A); complex shifts on
 * real A require it.  A real shift needs a real weight on real A.
 *   nterms     1..16 terms (16 solves at most, conjugates included, for
 *              complex A)
 *   dtype      PFM_R64 or PFM_C128 (A, V and F_exp); the problems as for
 *              pfm_eval_batched, F_phi1 ignored
 * Real shifts on real A take the real routes (Gauss-Jordan where every
 * |c_k| ||A||_1 <= 1/2, else pivoting LU), anything complex the embedded
 * route (complex: n <= 256).  binary64 only.  pfm_info.plan is 0 (full) or
 * 1 (action), order 0, theta +inf (no bound is known for the set).
 * PFM_ERR_INVALID for a bad term, PFM_ERR_UNSUPPORTED for complex shifts on
 * real A without conj_pairs. */
int pfm_eval_rational(pfm_ctx *ctx, int nterms, const double *c_re, const double *c_im, const double *w_re,
                      const double *w_im, double a0, int conj_pairs, int dtype, int batch,
                      const pfm_problem *probs, pfm_info *info, pfm_stream_t stream);

/* ------------------------------------------------------------------------
 * Tridiagonal A (§2.1, §5): the action f(A)V for real A given by its three
 * diagonals, by the N-step recurrence of the action path (N = max(1,
 * ceil(||A||_1 / θ)), B = A / N) with r(B) y = a0 y + sum_k w_k (I - c_k B)^{-1}
 * B y (round-off form, §4.3).  I - c_k B is tridiagonal: its LU is formed
 * once per shift and reused by all N steps and all columns (§5.1); each
 * solve is one forward and one backward sweep.
 *
 * Problem (all pointers device memory, owned by the caller):
 *   d       dimension, 1 <= d <= PFM_TRI_MAX_D
 *   p       columns of V, 1 <= p <= PFM_TRI_MAX_P
 *   dl      subdiagonal, dl[i] = A[i+1][i], d - 1 entries (may be NULL if d = 1)
 *   dd      diagonal, dd[i] = A[i][i], d entries
 *   du      superdiagonal, du[i] = A[i][i+1], d - 1 entries (NULL if d = 1)
 *   V       d x p row-major, leading dimension ldv >= p; never written
 *   F_exp, F_phi1   d x p row-major outputs, leading dimension ldf >= p; must
 *           not overlap the inputs; NULL when f excludes them
 * Every array's address is a multiple of 8 (PFM_ERR_INVALID otherwise).
 * ------------------------------------------------------------------------ */
#define PFM_TRI_MAX_D (1 << 24)
#define PFM_TRI_MAX_P (1 << 20)

typedef struct {
  int32_t d;
  int32_t p;
  int64_t ldv;
  int64_t ldf;
  const double *dl;
  const double *dd;
  const double *du;
  const double *V;
  double *F_exp;
  double *F_phi1;
} pfm_tri_problem;

/* Evaluate a batch of tridiagonal actions (binary64).
 *   f, tol, info, force_plan, stream   as for pfm_eval_batched (force_plan:
 *              N >= 1 for every instance; a forced N that leaves some
 *              |c_k| ||B||_1 >= 1 may meet a zero pivot, reported as
 *              PFM_SINGULAR_SHIFT, since the sweeps do not interchange rows)
 *   m          4, 5 or 8 (the real shift sets; PFM_ERR_UNSUPPORTED for m = 1),
 *              or 10 / PFM_R10STAR: the hybrid sets of §4.3 in the round-off
 *              form (R10' of §5), exp only (PFM_ERR_UNSUPPORTED with
 *              PFM_PHI1 or a tol below the set's rounding floor)
 * pfm_info.route is 3.  With pfm_profile on, phase 0 times the
 * factorisations and phase 1 the N steps.  The call only enqueues work on
 * `stream` (nothing is read back): an instance whose N would exceed
 * PFM_MAX_STEPS is flagged PFM_NOT_COMPUTED on the device and its outputs
 * are not written.  Workspace (grown with hipMalloc when a call needs more,
 * after synchronising `stream`): about (3 + 3 m) d + n_f (3 + m / 8) d p
 * doubles per instance (n_f functions). */
#define PFM_MAX_STEPS (1 << 20)
int pfm_tri_action(pfm_ctx *ctx, int f, int m, double tol, int batch, const pfm_tri_problem *probs,
                   pfm_info *info, int force_plan, pfm_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as pfm_tri_action, with the same arguments, results and
 * per-instance status, but every scratch byte (descriptors, plans, B and the
 * factors, step vectors, checkpoints) lives in one fixed device array of
 * PFM_NOALLOC_MAX_BYTES that the library holds on each device from the
 * first pfm_create on it until the process ends.  The call allocates
 * nothing (no hipMalloc, hipFree or pinned host memory; the descriptors are
 * copied from a static host array).  Returns PFM_ERR_BUDGET, with nothing
 * enqueued, when batch > PFM_NOALLOC_MAX_BATCH or the call needs more than
 * PFM_NOALLOC_MAX_BYTES (about 8 d (3 + 3 m + n_f (3 + m / 8) p) bytes per
 * instance plus 256 per instance for its descriptor and plan).  All calls on
 * one device share that array, and each call overwrites what the previous
 * one left there: calls that overlap on one device (two streams, or two
 * threads) race and must be serialised by the caller. */
#define PFM_NOALLOC_MAX_BYTES (64u << 20)
#define PFM_NOALLOC_MAX_BATCH 1024
int pfm_tri_action_noalloc(pfm_ctx *ctx, int f, int m, double tol, int batch, const pfm_tri_problem *probs,
                           pfm_info *info, int force_plan, pfm_stream_t stream);

/* ------------------------------------------------------------------------
 * Banded A (§2.1 and §5 name the pentadiagonal case beside the tridiagonal
 * one): the action f(A)V for real A with half-bandwidth b (b = 2:
 * pentadiagonal), by the same N-step recurrence and round-off form as
 * pfm_tri_action.  I - c_k B keeps the band of A: its LU (no interchanges)
 * is formed once per shift and reused by all N steps and all columns (§5.1);
 * each solve is one banded forward and one backward sweep.
 *
 * Problem (all pointers device memory, owned by the caller):
 *   d       dimension, 1 <= d <= PFM_TRI_MAX_D
 *   p       columns of V, 1 <= p <= PFM_TRI_MAX_P
 *   bands   (2b + 1) x d row-major: bands[(b + o) d + i] = A[i][i + o] for
 *           o = -b..b; the entries with i + o outside [0, d) are not part of
 *           A and are never read; never written
 *   V       d x p row-major, leading dimension ldv >= p; never written
 *   F_exp, F_phi1   d x p row-major outputs, leading dimension ldf >= p; must
 *           not overlap the inputs; NULL when f excludes them
 * Every array's address is a multiple of 8 (PFM_ERR_INVALID otherwise).
 * ------------------------------------------------------------------------ */
#define PFM_BAND_MAX_B 4

typedef struct {
  int32_t d;
  int32_t p;
  int64_t ldv;
  int64_t ldf;
  const double *bands;
  const double *V;
  double *F_exp;
  double *F_phi1;
} pfm_band_problem;

/* Evaluate a batch of banded actions (binary64), all with half-bandwidth b.
 *   b          1 <= b <= PFM_BAND_MAX_B (PFM_ERR_INVALID otherwise)
 *   f, m, tol, info, force_plan, stream   as for pfm_tri_action (m = 4, 5,
 *              8, or 10: the hybrid set of §4.3, exp only)
 * pfm_info.route is 4.  ||A||_1 adds column j's entries from the top row
 * down.  With pfm_profile on, phase 0 times the factorisations and phase 1
 * the N steps.  As for pfm_tri_action, the call only enqueues work, and an
 * instance whose N would exceed PFM_MAX_STEPS is flagged PFM_NOT_COMPUTED.
 * Workspace: about (m + 1) (2b + 1) d + n_f (3 + m b / 4) d p doubles per
 * instance (n_f functions; one checkpoint per 4 rows). */
int pfm_band_action(pfm_ctx *ctx, int f, int m, double tol, int b, int batch, const pfm_band_problem *probs,
                    pfm_info *info, int force_plan, pfm_stream_t stream);

/* Block until `stream` is idle and report device-side failures of previous
 * calls on this context: PFM_ERR_DEVICE if a bounded wait of the persistent
 * squaring queue gave up (its results are then not to be trusted); the flag
 * is cleared. */
int pfm_check(pfm_ctx *ctx, pfm_stream_t stream);

/* Phase timing.  enable != 0: every later pfm_eval_batched on this context
 * records hipEvents on its stream around four phases -- 0: shifted LU
 * factorisations, 1: shifted solves fused with the combination, 2: squaring
 * levels, 3: store of the results -- and accumulates their elapsed times.
 * Enabling or disabling resets the totals. */
int pfm_profile(pfm_ctx *ctx, int enable);

/* Route of the full-matrix FP64 path on real A.
 *   PFM_ROUTE_AUTO (default): an instance whose shifts all satisfy
 *     |c_k| ||B||_1 <= 1/2 has strictly column diagonally dominant
 *     I - c_k B, on which partial pivoting performs no interchange; its
 *     shifted inverses (I - c_k B)^{-1} (§2) are formed by Gauss-Jordan
 *     and R = a0 I + (sum_k w_k (I - c_k B)^{-1}) B (§4.3).  Every other
 *     instance takes the pivoting LU route.
 *   PFM_ROUTE_LU: every instance takes the pivoting LU route: M_k = P L U,
 *     Z_k = M_k^{-1} B by substitution, R = a0 I + sum_k w_k Z_k.
 * Both routes evaluate the same r(B) up to rounding; pfm_info.route reports
 * the one taken.  Returns PFM_ERR_INVALID for another value.  Takes effect
 * on the next pfm_eval_batched call. */
int pfm_set_route(pfm_ctx *ctx, int route);

/* Squaring schedule of the full-matrix path (§1: s squarings per instance,
 * s decided on the device).  The first direct_levels levels are one launch
 * each over every instance's product tiles (a tile of an instance with fewer
 * squarings returns at once); the levels beyond them, however many, run in
 * one persistent launch that takes (level, instance, tile) tasks from a
 * queue built on the device, each task waiting (bounded) until the tiles of
 * its instance's previous level are done.  Default 8; 0 runs every level
 * from the queue.  0 <= direct_levels <= PFM_MAX_SQUARINGS (PFM_ERR_INVALID
 * otherwise); takes effect on the next call, and a tuned schedule
 * (pfm_tune) no longer overrides it. */
int pfm_set_schedule(pfm_ctx *ctx, int direct_levels);

/* Totals since the last pfm_profile call: ms[4] milliseconds per phase,
 * launches[4] kernel launches per phase (may be NULL), *calls the number of
 * timed calls (may be NULL).  Waits for the last timed call to finish. */
int pfm_profile_read(pfm_ctx *ctx, double *ms, int *launches, int *calls);

/* Launch-sequence reuse.  After the plan read-back, the rest of a call is a
 * fixed sequence of kernel launches determined by the descriptors, plans and
 * task lists.  With graphs enabled (the default), a call whose sequence
 * repeats the previous call's exactly (same pointers, sizes, plans, routes,
 * function, tolerance and stream) has it captured as a hipGraph on the
 * second occurrence and replayed from the third on; a new sequence runs
 * eagerly.  Never on the null stream, and not while pfm_profile is on.
 * The graph holds no memset nodes.  Takes effect on the next call. */
int pfm_set_graphs(pfm_ctx *ctx, int enable);

/* Graph captures and replays since the context was created. */
int pfm_graph_stats(pfm_ctx *ctx, int *captures, int *replays);

/* Autotuner.  Runs the batch (same arguments as pfm_eval_batched, outputs
 * written) under each policy that can make a difference for it, timing
 * `reps` calls of each with hipEvents on `stream` after one warm-up call,
 * and keeps the fastest for the batch's key (mode, complex, precision, size
 * bucket of the largest instance, batch-size bucket).  A policy is
 * route + 4 (schedule + 2 (tile + 2 block)):
 *   route    real full matrices: 0 single-workgroup Gauss-Jordan inverses
 *            where dominant, 1 the pivoting LU route; action or complex: 0
 *            the multi-workgroup route for sizes above 128, 2 only above 512;
 *   schedule full matrices: 0 the first 8 squaring levels launched one by
 *            one, 1 every level from the persistent queue (pfm_set_schedule);
 *   tile     full matrices: 0 128 x 128 product tiles from npad 256 on, 1
 *            64 x 64 tiles for every size up to 512;
 *   block    Gauss-Jordan inverses of padded size 256: 0 128-wide pivot
 *            blocks (two passes over each matrix), 1 64-wide (four passes).
 * Later calls with the same key use it (an explicit PFM_ROUTE_LU or
 * pfm_set_schedule still wins).  Synchronises the stream.  *policy and *ms
 * (may be NULL) receive the choice (0..31) and its time per call. */
int pfm_tune(pfm_ctx *ctx, int f, int m, double tol, int prec, int dtype, int batch, const pfm_problem *probs,
             int reps, pfm_stream_t stream, int *policy, double *ms);

/* The tuned table as text, one "key policy" line per entry, into buf
 * (truncated to size, NUL-terminated; buf may be NULL).  Returns the bytes
 * needed including the NUL. */
int pfm_tune_export(const pfm_ctx *ctx, char *buf, size_t size);

/* Replace the tuned table with one produced by pfm_tune_export.  Returns
 * PFM_ERR_INVALID (table unchanged) for unreadable text. */
int pfm_tune_import(pfm_ctx *ctx, const char *text);

/* The pivoting LU factorisation of shift `shift` (0-based, in the order of
 * pfm_coeffs) of instance `instance` of the most recent pfm_eval_batched
 * call on ctx (§8(a3): M_k = I - c_k B = P L U, partial pivoting, pivot = the
 * first index of the largest |.| in the column), as the solve kernels store
 * it.  lu (host, column-major, npad x npad with leading dimension
 * ldlu >= npad) receives the padded matrix's factors (npad = n rounded up to
 * a multiple of 16, the padding being the identity): L unit lower below the
 * diagonal, U on and above it, except that every off-diagonal 16 x 16 block
 * is stored multiplied by the inverse of the diagonal block of its block
 * column, L_ij L_jj^{-1} (i > j) and U_ij U_jj^{-1} (i < j); binary32
 * factors (PFM_MIXED) are widened.  ipiv (host, npad entries) receives the
 * LAPACK-style pivot sequence, 0-based: at step r rows r and ipiv[r] were
 * interchanged.  *npad (may be NULL) receives npad; with lu and ipiv both
 * NULL only npad is returned.  Synchronises the device.  PFM_ERR_INVALID if
 * there is no such factorisation (the instance took another route, the
 * indices are out of range, or a later call reused the workspace). */
int pfm_lu_factors(pfm_ctx *ctx, int instance, int shift, double *lu, int64_t ldlu, int32_t *ipiv, int32_t *npad);

/* Upper bound of the workspace bytes pfm_eval_batched would allocate for
 * this batch (host only; probs may hold NULL data pointers).  Returns 0 for
 * an invalid or unsupported batch. */
size_t pfm_workspace_bytes(int f, int m, int prec, int dtype, int batch, const pfm_problem *probs);

/* ------------------------------------------------------------------------
 * Serving: a scheduler thread with continuous batching over the calls above.
 *
 * Requests are submitted one at a time with their own function, solve count,
 * tolerance, precision and element type.  The scheduler admits a pending
 * request when its resident bytes (copies of A and V, its outputs) fit in the
 * resident share of the HBM budget, copies A (and V) into library-owned
 * device buffers, and groups admitted requests that can share one
 * pfm_eval_batched_tols call (same f, m, prec, dtype, mode and size bucket:
 * real dimension <= 128, <= 512 or larger, counting 2n for complex) into batches
 * whose workspace fits one lane's share of the budget.  Each lane is a
 * stream with its own workspace; up to `lanes` batches run concurrently.
 * With two or more lanes, a third of them (at least one) are express lanes
 * that take only requests of real dimension <= 512 (2n for complex), so
 * small requests never queue behind batches of large ones.  Requests
 * arriving meanwhile are admitted and batched as lanes free up.
 * A request's results stay in library memory until fetched or released.
 *
 * Latency is measured by the library from pfm_srv_submit to the host seeing
 * the batch's completion event (host steady clock).  Each lane has a launch
 * thread (the calls wait on their own stream for the plan read-back), so a
 * lane waiting for the GPU never delays the dispatch to another.
 * ------------------------------------------------------------------------ */
typedef struct pfm_server pfm_server;

/* Start a server on `device`.  lanes in [1, 16]; hbm_budget_bytes > 0 is
 * split half for resident request data, half across the lanes' workspaces;
 * max_batch caps the requests per call. */
int pfm_srv_start(pfm_server **srv, int device, int lanes, size_t hbm_budget_bytes, int max_batch);

/* Finish every submitted request, stop the thread and free all memory
 * (unfetched results are lost). */
int pfm_srv_stop(pfm_server *srv);

/* Queue one request.  pr holds device pointers A (and V for p >= 1); they
 * must stay valid and unchanged until the request is done (the copy into
 * resident memory happens at dispatch).  pr->F_exp / F_phi1 / ldf are
 * ignored: results go to library memory.  Returns PFM_ERR_INVALID /
 * PFM_ERR_UNSUPPORTED for a request pfm_eval_batched would reject, and
 * PFM_ERR_BUDGET for one that can never fit the budget. */
int pfm_srv_submit(pfm_server *srv, const pfm_problem *pr, int f, int m, double tol, int prec, int dtype,
                   uint64_t *ticket);

/* State of a request: 0 done (info and latency filled, may be NULL),
 * 1 queued or running, PFM_ERR_INVALID for an unknown ticket, PFM_ERR_HIP if
 * its batch failed. */
int pfm_srv_poll(pfm_server *srv, uint64_t ticket, pfm_info *info, double *latency_s);

/* Up to max completed requests not reported before: tickets, latencies (s)
 * and per-instance status.  Returns the count. */
int pfm_srv_drain(pfm_server *srv, int max, uint64_t *tickets, double *latency_s, int32_t *status);

/* Where a completed (or failed) request's latency went, in seconds, into
 * parts[4]: [0] waiting for admission (its resident copies to fit the
 * budget), [1] admitted and waiting for a lane, [2] the host enqueueing its
 * batch (copies and pfm_eval_batched_tols on the lane stream), [3] from the
 * end of the enqueue to the scheduler seeing the batch's completion event
 * (device time, plus the earlier work on that stream).  The four add up to
 * the latency that pfm_srv_poll and pfm_srv_drain report.  Returns 1 if the
 * request is not finished, PFM_ERR_INVALID for an unknown (or released)
 * ticket.  The request keeps its record until pfm_srv_release. */
int pfm_srv_timing(pfm_server *srv, uint64_t ticket, double *parts);

/* Copy a done request's result for function `which` (PFM_EXP or PFM_PHI1)
 * to the device buffer dst (row-major, leading dimension ldd, the request's
 * element type), synchronously.  The result stays until released. */
int pfm_srv_fetch(pfm_server *srv, uint64_t ticket, int which, void *dst, int64_t ldd);

/* Free a done request's results and forget the ticket. */
int pfm_srv_release(pfm_server *srv, uint64_t ticket);

/* Counters: submitted, done, batches launched, bytes resident now, peak
 * resident bytes, host seconds spent launching batches (summed over the
 * lanes' launch threads).  Any pointer may be NULL. */
int pfm_srv_stats(pfm_server *srv, uint64_t *submitted, uint64_t *done, uint64_t *batches,
                  uint64_t *resident_bytes, uint64_t *peak_resident_bytes, double *launch_s);

/* Library version string (static storage). */
const char *pfm_version(void);

/* Test hook.  Runs one v_mfma_f64_16x16x4 on device `device` with operands
 * A[i][k] = 4 i + k + 1 and B[k][j] = 100 (k + 1) + j (i, j < 16, k < 4) and
 * copies the 64 lanes x 4 accumulator values, lane-major, to the host array
 * `out[0..255]`; then the same for v_mfma_f32_16x16x4 into `out[256..511]`
 * (512 doubles in all).  Lets the tests confirm the fragment layouts the
 * kernels assume.  Synchronous; allocates and frees its own 4 KiB. */
int pfm_selftest_mfma(int device, double *out);

#ifdef __cplusplus
}
#endif

#endif /* PFM_H */
