/*
 * jsvd.h -- C ABI of the MI355X (gfx950) implementation of the parallel
 * one-sided Jacobi SVD hot path of V. Novakovic, "Vectorization of a
 * thread-parallel Jacobi singular value decomposition method",
 * arXiv:2202.08361 (SIAM J. Sci. Comput., 2023).
 *
 * General conventions
 * -------------------
 * - Every matrix and vector argument is a DEVICE pointer owned by the caller
 *   (the library never frees it).  The library owns only the workspace it
 *   allocates in *_create and frees in *_destroy.
 * - Matrices are column-major with a leading dimension in elements.  Complex
 *   data is split: a complex m x n matrix is two real m x n matrices (real and
 *   imaginary parts), as in Sect. 2.4.1 of the paper.  A NULL imaginary
 *   pointer selects the real (symmetric / orthogonal) variant.
 * - Every floating-point quantity is IEEE-754 binary64; integer exponents
 *   and counters are int32 / int64.
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls that only
 *   launch work return as soon as it is enqueued; calls documented as
 *   "synchronises" wait for the stream.
 * - Return value: JSVD_OK (0) on success, > 0 a warning, < 0 an error.  No
 *   C++ exception crosses the ABI.  Arguments are validated before anything
 *   is enqueued; on an error nothing is enqueued and no output is touched.
 */
#ifndef JSVD_H
#define JSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JSVD_VERSION_MAJOR 0
#define JSVD_VERSION_MINOR 1

enum {
    JSVD_OK = 0,
    JSVD_NOT_CONVERGED = 1, /* sweep limit reached (Alg. zvjsvd returns C = S) */
    JSVD_EINVAL = -1,       /* invalid argument (sizes, strides, NULL pointers, flags) */
    JSVD_ENONFINITE = -2,   /* the input holds Inf or NaN (M~_0 = inf, Sect. 3.2) */
    JSVD_EZERO = -3,        /* the input is the zero matrix (M~_0 = 0, Sect. 3.2) */
    JSVD_ENOMEM = -4,       /* device or host allocation failed */
    JSVD_EDEVICE = -5,      /* a HIP runtime call failed */
    JSVD_EAGAIN = -6,       /* serving: the request cannot be admitted now */
    JSVD_ENOTFOUND = -7     /* serving: unknown ticket */
};

/* flags of jsvd_gesvj / jsvd_gesvj_batched / jsvd_state_set_flags / serving */
#define JSVD_NO_PERMUTE 1u  /* apply U, not U P, during the iteration: the default,
                               named for explicitness; the final sort orders the
                               output either way */
#define JSVD_COMPENSATED 2u /* scaled dot-products with compensated summation
                               (Sect. SM2.2, Alg. zdpsclcs / ddpsclcs) instead of
                               Alg. zdpscl */
#define JSVD_NO_GS 4u       /* always rotate: no Gram-Schmidt replacement for pairs
                               whose norms differ by more than 2^eta_hat upsilon
                               (eq. GScond; by default such a pair is orthogonalised
                               by eq. GS, Sect. 3.5.1) */
#define JSVD_PERMUTE 8u     /* apply U P: the EVD's permutation P keeps each pivot pair
                               sorted by norm, larger column first (Sect. 2, optional
                               there).  Off by default: with round-robin pairs a swapped
                               column takes over its partner's remaining pairings of the
                               sweep, so a sweep stops meeting every column pair and
                               the iteration needs about twice the sweeps, more as n
                               grows.  Invalid together with JSVD_NO_PERMUTE. */

/* flags of jsvd_evd2_batched */
#define JSVD_EVD_SCALED  1u /* return lambda' = 2^zeta lambda (not backscaled), Sect. 2.3 */
#define JSVD_EVD_SINFORM 2u /* return e^{i alpha} sin(phi) instead of e^{i alpha} tan(phi), eq. (jacsec) */

/* Library version as (major << 16) | minor. */
int jsvd_version(void);
/* Static text of a status code. */
const char *jsvd_strerror(int status);

/* ----------------------------------------------------------------------
 * Stand-alone batched EVD of Hermitian / real symmetric 2x2 matrices
 * (Sect. 2, Listing 1, Alg. zbjac2 and dbjac2).
 *
 * Input: r matrices [[a11, conj(a21)], [a21, a22]] in structure-of-arrays
 * form: a11[i], a22[i], a21_re[i] and (complex) a21_im[i], all finite.
 * a21_im == NULL selects the real symmetric variant; then ctan_im must be
 * NULL too.
 * Output (each r elements, any of lambda1, lambda2, zp may be NULL):
 *   cos_phi[i]              cos(phi)
 *   ctan_re[i], ctan_im[i]  e^{i alpha} tan(phi) (real: sign(a21) tan(phi)),
 *                           or e^{i alpha} sin(phi) with JSVD_EVD_SINFORM
 *   lambda1[i], lambda2[i]  eigenvalues 2^-zeta lambda'_1,2 (or lambda' with
 *                           JSVD_EVD_SCALED); U = [[c, -conj(e) s], [e s, c]]
 *                           with A = U diag(lambda1, lambda2) U^*
 *   zp[i]                   (zeta' << 1) | p, zeta' = -zeta the exponent of
 *                           the backscaling, p = [lambda'_1 < lambda'_2]
 * Results are bit-for-bit those of the serial algorithm of Listing 1 in
 * IEEE double arithmetic with round-to-nearest-even and gradual underflow.
 * Input and output arrays must not overlap.  Asynchronous on `stream`.
 * ---------------------------------------------------------------------- */
int jsvd_evd2_batched(size_t r, const double *a11, const double *a22,
                      const double *a21_re, const double *a21_im,
                      double *cos_phi, double *ctan_re, double *ctan_im,
                      double *lambda1, double *lambda2, int32_t *zp,
                      unsigned flags, void *stream);

/* Measurement aid: moves exactly the bytes jsvd_evd2_batched moves for a
 * batch of r (the same input streams read, the same output streams written,
 * the same launch shape and access hints as its kernel for batches of 2^22
 * and more) without its arithmetic: every output is a copy of an input.  Its
 * throughput is the memory-system ceiling of the batched EVD on the device.
 * All pointers as for jsvd_evd2_batched, but lambda1, lambda2 and zp are
 * required; the outputs carry no meaning.  Async on `stream`. */
int jsvd_evd2_stream_ceiling(size_t r, const double *a11, const double *a22,
                             const double *a21_re, const double *a21_im,
                             double *cos_phi, double *ctan_re, double *ctan_im,
                             double *lambda1, double *lambda2, int32_t *zp, void *stream);

/* Single precision variant (Sect. 2.4.1: nu = FLT_MAX, fl(sqrt nu) =
 * 1.844674297E+19, FLT_TRUE_MIN, eta = FLT_MAX_EXP - 4): the same interface
 * on float arrays.  Results are bit-for-bit those of the serial algorithm
 * carried out in IEEE single arithmetic (round-to-nearest-even, gradual
 * underflow).  zeta' fits the same int32 packing. */
int jsvd_evd2_batched_f32(size_t r, const float *a11, const float *a22,
                          const float *a21_re, const float *a21_im,
                          float *cos_phi, float *ctan_re, float *ctan_im,
                          float *lambda1, float *lambda2, int32_t *zp,
                          unsigned flags, void *stream);

/* ----------------------------------------------------------------------
 * Device-resident SVD state: the hot path one parallel step at a time
 * (Sect. 4, Alg. zvjsvd).
 *
 * The state owns a working copy of the iteration matrix G (m x n, m >= n >= 1),
 * the accumulated right transformations V (n x n), the column norms (e, f)
 * (sigma-like pairs 2^e f, f in [1, 2), Sect. 3.2), the scaling exponent s,
 * the max-norm estimate M~ and the step / sweep / transformation counters.
 * The pivot pairs of step k are the round-robin pairs of k mod K,
 * K = n - 1 (n even) or n (n odd).
 * ---------------------------------------------------------------------- */
typedef struct jsvd_state_s *jsvd_state;

typedef struct {
    int64_t steps;        /* steps taken since the last load */
    int64_t sweeps;       /* sweeps that transformed or swapped (C of Alg. zvjsvd) */
    int64_t T;            /* transformations in the current sweep so far */
    int64_t last_t;       /* transformations in the last step */
    int64_t swaps;        /* column swaps without transformation in the current sweep */
    int32_t s;            /* effective scaling exponent: G_k = 2^s (G_0 V_k) */
    int32_t rescaled;     /* step-start downscalings performed (Sect. 3.2) */
    double Mt;            /* M~_k, the max-norm estimate of G_k */
    int32_t converged;    /* a full sweep with neither transformation nor swap */
    int32_t status;       /* JSVD_OK or the load error */
    int64_t last_sweep_T;     /* transformations in the last completed sweep */
    int64_t last_sweep_swaps; /* swaps without transformation in the last completed sweep */
    int64_t gs;               /* Gram-Schmidt steps in the current sweep so far (counted in T) */
    int64_t last_sweep_gs;    /* Gram-Schmidt steps in the last completed sweep */
    int64_t loop_sweeps;      /* sweeps since the load that ran as one persistent launch */
    int64_t loop_redos;       /* persistent sweeps that gave up and were redone step by step */
    int64_t skipped_pairs;    /* pairs of large-column steps since the load that were not read:
                                 both columns unchanged since the pair last met, one sweep
                                 earlier, so its outcome is that meeting's (no change) */
    int64_t local_sweeps;     /* persistent sweeps of the state that ran in the L2-local mode
                                 (jsvd_state_set_loop_local) */
} jsvd_info;

/* Allocate a state for an m x n real (is_complex = 0) or complex problem,
 * m <= 2^24.  Columns of more than 16384 (real) / 8192 (complex) rows, which
 * no workgroup holds in registers, are streamed from memory by the step: the
 * pair is read three times (max, sums of squares, dot-product) and read and
 * written once, with the same sums in the same lane order, so the results
 * are the same bits as the oracle's.  Returns JSVD_EINVAL for m < n, n < 1,
 * m > 2^24, JSVD_ENOMEM when out of memory. */
int jsvd_state_create(int m, int n, int is_complex, jsvd_state *out);
void jsvd_state_destroy(jsvd_state st);

/* Load G (device, column-major, leading dimension ldg >= m) into the state,
 * then initialise as in Alg. zvjsvd: M~_0 = max|component| (NaN counted as
 * Inf), s_0 = s_[0] of eq. (skn), G_1 = 2^{s_0} G, V_1 = I.  Synchronises.
 * Returns JSVD_ENONFINITE / JSVD_EZERO for a non-finite / zero G. */
int jsvd_state_load(jsvd_state st, const double *G_re, const double *G_im, size_t ldg,
                    void *stream);

/* One parallel Jacobi step on the state (the hot path): for every pivot pair
 * of the step, the Frobenius norms of both columns, the scaled dot-product
 * (Alg. zdpscl), the convergence test (Alg. cvg) and scaled Gram matrix
 * (Alg. Gram), the 2x2 EVD (Listing 1), and the rotation or swap of the G
 * and V column pairs (Alg. zjrot), with the step-start rescaling check of
 * Sect. 3.2.  A pair to be transformed whose norms differ by more than
 * 2^eta_hat upsilon (eq. GScond) takes the Gram-Schmidt step of eq. (GS) on
 * G instead (the smaller column orthogonalised against the larger, which
 * stays or moves to the first place), while V still takes the pair's
 * rotation; JSVD_NO_GS turns this off.  Step index, M~ and the counters stay
 * on the device; launches only.  For columns of more than 256 rows (and no
 * forced workgroup size) the V rotations of up to 32 consecutive steps are
 * applied together (a row of V never mixes with another row, so the result
 * is the same bit for bit): V is brought up to date whenever it is read
 * (jsvd_state_save, jsvd_state_finalize, the end of jsvd_sweep and of
 * jsvd_gesvj) or the fused small-column kernel takes over. */
int jsvd_step(jsvd_state st, void *stream);

/* K steps followed by the end-of-sweep bookkeeping; launches only (one
 * graph, captured once per state and launch configuration).  For columns of
 * more than 256 rows the graph applies each 32 steps' V rotations on a second
 * stream of the library's, beside the steps that follow, and joins it back
 * before its end: to the caller the sweep is ordered on `stream` like any
 * other launch. */
int jsvd_sweep(jsvd_state st, void *stream);

/* Sweeps until the state stops (converged, or the sweep limit), one
 * graph-launched sweep at a time with a synchronisation after each (the
 * device decides convergence): the iteration of jsvd_gesvj on a loaded
 * state.  For columns of at most 1024 rows and at most 192 pair slots
 * (automatic launch shape) a sweep runs as one persistent launch whenever
 * the device has found that the rescaling check of Sect. 3.2 cannot fire in
 * it (max(M~, (1 + 32 eps K) ||G||_F) below the threshold): one workgroup
 * per pair slot, each pair of
 * step k + 1 starting as soon as its two columns are out of step k.  The
 * result is the same, bit for bit, as K steps.  Such a sweep needs its
 * workgroups resident together; one that waits too long for a column gives
 * up and is redone step by step from a copy taken before it.
 * jsvd_state_query reports both counts.  Synchronises. */
int jsvd_state_iterate(jsvd_state st, void *stream);
/* How long (wall clock, seconds) a workgroup of a persistent sweep of
 * jsvd_state_iterate / jsvd_gesvj waits for one column before the sweep
 * gives up and is redone step by step (default 0.25; at most 60).  0 turns
 * persistent sweeps off for the state.  JSVD_EINVAL outside [0, 60]. */
int jsvd_state_set_loop_wait(jsvd_state st, double seconds);
/* Whether persistent sweeps of the state may run in the L2-local mode
 * (allow = 1, the default) or always spread over the device (0).  In the
 * L2-local mode, used where every pair slot's workgroup fits on one XCC with
 * one wavefront per SIMD (n <= 256, columns of at most 1024 real / 512
 * complex rows, at most 4 x CUs/8 slots), the workgroups of one XCC take the
 * slots and exchange columns through its L2 without cache write-back or
 * invalidation; the results are
 * the same bits.  A sweep in that mode that gives up turns it off for the
 * state until the next call of this function.  JSVD_EINVAL for another
 * value of allow. */
int jsvd_state_set_loop_local(jsvd_state st, int allow);

/* Read the scalars of the state.  Synchronises. */
int jsvd_state_query(jsvd_state st, jsvd_info *out, void *stream);

/* Copy the working G (scaled iteration matrix), V and the column norms of
 * the last step out of the state (any pointer may be NULL).  Synchronises. */
int jsvd_state_save(jsvd_state st, double *G_re, double *G_im, size_t ldg,
                    double *V_re, double *V_im, size_t ldv,
                    double *e, double *f, int32_t *s, double *Mt, int64_t *step,
                    void *stream);
/* Overwrite the working G and V and the scalars (resume a saved state).
 * Synchronises. */
int jsvd_state_restore(jsvd_state st, const double *G_re, const double *G_im, size_t ldg,
                       const double *V_re, const double *V_im, size_t ldv,
                       int32_t s, double Mt, int64_t step, void *stream);

/* Finalisation (Sect. 4.2.1): u_j = (g_j 2^{-e_j}) / f_j, sigma_j =
 * (e_j - s, f_j), then a stable sort of (sigma, u, v) into descending order.
 * U (m x n) and V (n x n) are caller buffers; sv_e/sv_f receive the pairs and
 * sv (may be NULL) the values 2^e f as doubles.  Launches only. */
int jsvd_state_finalize(jsvd_state st, double *U_re, double *U_im, size_t ldu,
                        double *V_re, double *V_im, size_t ldv,
                        double *sv_e, double *sv_f, double *sv, void *stream);

/* Force the workgroup size (threads per pivot pair: 64, 128, 256, 512 or
 * 1024; 0 = automatic).  Results do not depend on it (bit-identical). */
int jsvd_state_set_launch(jsvd_state st, int threads_per_pair);

/* Set the iteration flags of a state (JSVD_PERMUTE or JSVD_NO_PERMUTE,
 * JSVD_COMPENSATED, JSVD_NO_GS; default none).  They apply from the next step
 * on.  Returns JSVD_EINVAL for unknown flags and for JSVD_PERMUTE together
 * with JSVD_NO_PERMUTE. */
int jsvd_state_set_flags(jsvd_state st, unsigned flags);

/* Single precision state (Sect. SM8: the method in the precision of the
 * datatype, with that precision's range constants): G, V and the norms are
 * float arrays and every operation of the step is an IEEE single operation;
 * nu = FLT_MAX, eps = 2^-24 (upsilon = fl(sqrt m) 2^-24), s_(k) = 126
 * (real) / 124 (complex) - floor(lg M~), s_[k] from eq. (skn) with nu =
 * FLT_MAX, the Gram scaling with FLT_MAX_EXP - 1 and the single precision EVD
 * (Sect. 2.4.1).  The compensated dot-products are not offered.
 * jsvd_step, jsvd_sweep, jsvd_state_query (M~ as a double holding the float
 * value), jsvd_state_set_launch, jsvd_state_set_flags (JSVD_PERMUTE,
 * JSVD_NO_PERMUTE and JSVD_NO_GS; eta_hat = FLT_MAX_EXP - 1 in eq. GScond)
 * and jsvd_state_destroy take either kind of state; the calls below take a
 * single precision state and the double calls above reject one
 * (JSVD_EINVAL), and the other way round.  Arguments as for the double
 * calls, with float arrays. */
int jsvd_state_create_f32(int m, int n, int is_complex, jsvd_state *out);
int jsvd_state_load_f32(jsvd_state st, const float *G_re, const float *G_im, size_t ldg,
                        void *stream);
int jsvd_state_save_f32(jsvd_state st, float *G_re, float *G_im, size_t ldg,
                        float *V_re, float *V_im, size_t ldv,
                        float *e, float *f, int32_t *s, double *Mt, int64_t *step,
                        void *stream);
/* Mt must be a finite non-negative float value. */
int jsvd_state_restore_f32(jsvd_state st, const float *G_re, const float *G_im, size_t ldg,
                           const float *V_re, const float *V_im, size_t ldv,
                           int32_t s, double Mt, int64_t step, void *stream);
int jsvd_state_finalize_f32(jsvd_state st, float *U_re, float *U_im, size_t ldu,
                            float *V_re, float *V_im, size_t ldv,
                            float *sv_e, float *sv_f, float *sv, void *stream);

/* ----------------------------------------------------------------------
 * Batched scaled dot-products (Sect. 3.3): for j < npairs,
 *   z_j = (q_j / 2^{eq_j})^* (p_j / 2^{ep_j}) / (fq_j fp_j)
 * of the columns q_j = Q[:, j] and p_j = P[:, j] (m rows, column-major,
 * leading dimension ld >= m; complex columns split, Q_im/P_im NULL for real
 * data), by Alg. zdpscl, or by Alg. zdpsclcs / ddpsclcs with
 * JSVD_COMPENSATED.  With (e, f) the column norms this is the a21' of a
 * pivot pair; with e = 0, f = 1 it is the dot-product itself.  The sums run
 * in the same lane order as in jsvd_step, so the results are those of the
 * step.  All arrays are device arrays of the caller; z_im may be NULL for
 * real data.  m <= 4096 (complex) / 8192 (real).  Launches only.
 * ---------------------------------------------------------------------- */
int jsvd_dot_scaled_batched(int npairs, int m, const double *Q_re, const double *Q_im,
                            const double *P_re, const double *P_im, size_t ld,
                            const double *eq, const double *fq, const double *ep, const double *fp,
                            double *z_re, double *z_im, unsigned flags, void *stream);

/* ----------------------------------------------------------------------
 * Batched non-overflowing Frobenius norms with a widened exponent range
 * (Sect. SM6, Alg. rnF): for each column j < ncols of X (m rows, column-major,
 * leading dimension ld >= m; complex columns split, X_im NULL for real data),
 *   ||x_j||^2 = 2^{e2[j]} f2[j] and ||x_j|| = 2^{e[j]} f[j], 1 <= f < 2,
 * with e2, e integral doubles (-inf for a zero column, then f = 1) that may
 * exceed the exponent range of double, so no finite input overflows or
 * underflows to zero.  Steps: lanes (a power of two, 1 ... 1024) partial
 * sums, lane L taking the elements L, L + lanes, ... in order (complex: real
 * part, then imaginary part), each updated as fma(|x|, |x|, r) in (e, f) form
 * (Sect. SM6.2); the partial sums sorted by (e, f) (eq. vsort) and added
 * pairwise (eqs. 1red, redj); the square root of Sect. SM6.1.  Results depend
 * on `lanes` only (1024: the lane vector of the step's own sums).  e2 and f2
 * may be NULL.  Elements must be finite.  Device arrays of the caller;
 * launches only.
 * ---------------------------------------------------------------------- */
int jsvd_nrmf_batched(int ncols, int m, const double *X_re, const double *X_im, size_t ld, int lanes,
                      double *e2, double *f2, double *e, double *f, void *stream);

/* ----------------------------------------------------------------------
 * The whole SVD (Alg. zvjsvd with round-robin pairs): G = U Sigma V^*.
 * G (m x n, ldg >= m) is overwritten by U; V (n x n, ldv >= n) receives V;
 * sv_e/sv_f (n) receive sigma_j = 2^{sv_e[j]} sv_f[j] in descending order;
 * sv (n, may be NULL) the same as doubles.  *sweeps receives the number of
 * sweeps that transformed something (C in Alg. zvjsvd).  max_sweeps <= 0
 * selects 128.  Synchronises.  On JSVD_NOT_CONVERGED G holds the scaled
 * iteration matrix and sv_e/sv_f its current (unsorted) column norms.
 * ---------------------------------------------------------------------- */
int jsvd_gesvj(int m, int n, double *G_re, double *G_im, size_t ldg,
               double *V_re, double *V_im, size_t ldv,
               double *sv_e, double *sv_f, double *sv, int max_sweeps, int *sweeps,
               unsigned flags, void *stream);

/* The whole SVD in single precision (Sect. SM8; the step of
 * jsvd_state_create_f32): the same interface on float arrays, sv_e holding
 * the exponents as floats.  flags: JSVD_PERMUTE or JSVD_NO_PERMUTE, JSVD_NO_GS. */
int jsvd_gesvj_f32(int m, int n, float *G_re, float *G_im, size_t ldg,
                   float *V_re, float *V_im, size_t ldv,
                   float *sv_e, float *sv_f, float *sv, int max_sweeps, int *sweeps,
                   unsigned flags, void *stream);

/* ----------------------------------------------------------------------
 * Many independent SVDs of uneven sizes in persistent launches, one per
 * class of matrices (real or complex; rows up to 64, 128, 256 or 512).
 * Arrays of `count` host pointers / sizes describe the problems; every
 * matrix pointer is a device pointer.  Matrix i follows jsvd_gesvj exactly
 * (same results, bit for bit, whatever the launch shape).  status[i] and
 * sweeps[i] (host arrays; sweeps may be NULL) receive the per-matrix
 * outcome; transformations[i] (host array, may be NULL) the number of pairs
 * transformed over the whole iteration, -1 for a matrix that took the plain
 * path.  Matrices of more than 512 rows or columns take the plain path one
 * by one.  Synchronises.
 * ---------------------------------------------------------------------- */
int jsvd_gesvj_batched(int count, const int *m, const int *n, const int *is_complex,
                       double *const *G_re, double *const *G_im, const size_t *ldg,
                       double *const *V_re, double *const *V_im, const size_t *ldv,
                       double *const *sv_e, double *const *sv_f,
                       int max_sweeps, int *sweeps, int *status, int64_t *transformations,
                       unsigned flags, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): jsvd_gesvj_batched without any
 * allocation.  The same arguments and the same per-matrix results, bit
 * for bit, with these limits:
 * - at most 8192 matrices per call (JSVD_EINVAL beyond);
 * - every matrix must be a batched shape (at most 512 rows and columns):
 *   JSVD_EINVAL otherwise, since the plain path allocates a state;
 * - launch shapes are the ones measured earlier in the process
 *   (jsvd_batched_tune, or a jsvd_gesvj_batched call), else the default; this
 *   call measures nothing;
 * - the classes run one after another on `stream`.
 * The launch records (930 KiB: per-matrix records, the processing
 * order and the classes' work-queue counters, rewritten on every call) sit
 * in a file-scope device array that each GPU the library runs on holds until
 * the process ends.  Calls in one process are serialised by a lock, so they
 * never overlap on the array.  Synchronises. */
int jsvd_gesvj_batched_noalloc(int count, const int *m, const int *n, const int *is_complex,
                               double *const *G_re, double *const *G_im, const size_t *ldg,
                               double *const *V_re, double *const *V_im, const size_t *ldv,
                               double *const *sv_e, double *const *sv_f,
                               int max_sweeps, int *sweeps, int *status, int64_t *transformations,
                               unsigned flags, void *stream);

/* Launch schedule of the batched SVD, per class (real or complex; rows per
 * lane 1, 2, 4 or 8, i.e. at most 64, 128, 256 or 512 rows):
 *   - threads per matrix (128, 256 or 512; one wavefront per pivot pair at a
 *     time, so that many pairs of a matrix in flight);
 *   - the register budget of the kernel instance: the compiler's own, or
 *     "dense", at most 128 VGPRs (four waves per SIMD, a few spills where
 *     the default instance needs more);
 *   - workgroups per CU of the persistent grid (0 = as many as fit; fewer
 *     keeps fewer matrices in flight, whose columns then stay in the caches).
 * Chosen by measurement once per process and device: one sweep of up to 1024
 * random matrices of the class's median shape per candidate schedule, the
 * fastest kept.  jsvd_gesvj_batched measures the classes of its matrices that
 * are not measured yet; jsvd_batched_tune does it ahead of time for a list
 * of shapes (host arrays; is_complex may be NULL; flags as for the batched
 * call, of which JSVD_COMPENSATED selects the compensated kernels).
 * Synchronises.  The results do not depend on the schedule. */
int jsvd_batched_tune(int count, const int *m, const int *n, const int *is_complex, unsigned flags,
                      void *stream);
/* Force the threads per matrix for every class (128, 256 or 512; 0 = the
 * measured choice, the default), with the default instance and grid.  A
 * process-wide setting.  JSVD_EINVAL for other values. */
int jsvd_batched_set_launch(int threads_per_matrix);
/* Force a whole schedule for every class: threads per matrix as above (0 =
 * the measured choice, the other two arguments then ignored), dense 0 or 1,
 * workgroups per CU 0..64 (0 = as many as fit; more than fit is clamped).
 * JSVD_EINVAL for other values. */
int jsvd_batched_set_schedule(int threads_per_matrix, int dense, int workgroups_per_cu);
/* The candidates the measurement tries besides the three thread counts with
 * the default instance and a full grid: JSVD_TUNE_DENSE adds the dense
 * instances (where the default one takes more than 128 registers),
 * JSVD_TUNE_WGS adds half, 2 and 1 workgroups per CU; both are the default.
 * Forgets every measured schedule of the process.  JSVD_EINVAL for other
 * bits. */
#define JSVD_TUNE_DENSE 1u
#define JSVD_TUNE_WGS 2u
int jsvd_batched_set_tuning(unsigned candidates);
/* The schedule a batched call would use now for an m x n matrix (forced,
 * else measured, else 256 threads with the default instance and grid);
 * threads 0 when the shape is not batched.  JSVD_EINVAL for n < 1, m < n or
 * a NULL output. */
int jsvd_batched_schedule_of(int m, int n, int is_complex, unsigned flags, int *threads_per_matrix, int *dense,
                             int *workgroups_per_cu);
/* The threads per matrix a batched call would use now for an m x n matrix:
 * the forced value, else the measured one, else 256 (not measured yet);
 * 0 when the shape is not batched (more than 512 rows or columns), JSVD_EINVAL
 * for n < 1 or m < n. */
int jsvd_batched_launch_of(int m, int n, int is_complex, unsigned flags);

/* ----------------------------------------------------------------------
 * Serving: continuous batching of SVD requests under an HBM budget.
 * Requests are admitted as slots and device memory free up; admitted
 * requests advance concurrently on the device, sweep by sweep, with their
 * iteration state device-resident.  Buffers stay caller-owned and must stay
 * valid until the ticket completes, and complete (the server's streams do
 * not order after the caller's) when submitted.  Large requests (beyond the
 * batched kernel's m, n <= 512) each advance on their own state, at most
 * max_large at once.  Small requests run in batched launches when at least
 * 32 of them wait, with the launch shapes measured in this process
 * (jsvd_batched_tune), else the default; with fewer waiting, each runs on
 * its own state like a large one, which finishes it sooner.  The server
 * itself measures nothing, so as not to stall the requests in flight.
 * ---------------------------------------------------------------------- */
typedef struct jsvd_server_s *jsvd_server;

typedef struct {
    size_t hbm_budget_bytes; /* device bytes the server may allocate for work state */
    int max_slots;           /* requests on the device at once */
    int max_sweeps;          /* per request (<= 0: 128) */
    int max_queue;           /* waiting requests before submit returns JSVD_EAGAIN (<= 0: unbounded) */
    unsigned flags;          /* jsvd_gesvj flags applied to every request (JSVD_PERMUTE or
                                JSVD_NO_PERMUTE, JSVD_COMPENSATED, JSVD_NO_GS) */
    int max_large;           /* large requests (beyond the batched kernel's m, n <= 512, each
                                advanced sweep by sweep on its own state) on the device at once
                                (<= 0: 2); while that many are active, queued small requests
                                are admitted past a large one at the head of the queue */
} jsvd_serve_config;

typedef struct {
    int m, n, is_complex;
    double *G_re, *G_im; size_t ldg;   /* in: A; out: U */
    double *V_re, *V_im; size_t ldv;   /* out: V */
    double *sv_e, *sv_f;               /* out: sigma (device, n each) */
    uint64_t tag;
} jsvd_request;

typedef struct {
    uint64_t submitted, completed, rejected;
    double p50_ns, p99_ns;       /* submit-to-completion latency */
    double p50_queue_ns, p99_queue_ns; /* submit-to-admission */
    double svds_per_s;           /* completions per second since creation */
    int queue_depth, active;
    size_t hbm_in_use;
    double p50_service_ns, p99_service_ns; /* admission-to-completion */
    uint64_t persistent_sweeps;  /* sweeps of requests on their own state that ran as one
                                    persistent launch (while alone on the device) */
    uint64_t persistent_redos;   /* of those, sweeps that gave up and were redone step by step */
} jsvd_serve_stats;

int jsvd_serve_create(const jsvd_serve_config *cfg, jsvd_server *out);
/* Non-blocking; *ticket identifies the request. */
int jsvd_serve_submit(jsvd_server sv, const jsvd_request *req, uint64_t *ticket);
/* *done = 1 once finished; *status is its jsvd_gesvj status, *sweeps its C. */
int jsvd_serve_poll(jsvd_server sv, uint64_t ticket, int *done, int *status, int *sweeps);
int jsvd_serve_wait(jsvd_server sv, uint64_t ticket, int *status, int *sweeps);
/* Counters, rates and latency percentiles since creation (the name differs
 * from the struct's, which C does not allow to share it).  Takes a copy of
 * every recorded latency: O(completed) per call. */
int jsvd_serve_stats_get(jsvd_server sv, jsvd_serve_stats *out);
/* The server's load now, without the percentiles: cheap enough to call
 * before every submission.  Each output pointer may be NULL. */
int jsvd_serve_load(jsvd_server sv, int *queue_depth, int *active, size_t *hbm_in_use);
/* Waits for every admitted request, then frees the server. */
int jsvd_serve_destroy(jsvd_server sv);

/* ----------------------------------------------------------------------
 * Layout helpers (Sect. SM5): interleaved complex (re, im pairs) <-> split.
 * ---------------------------------------------------------------------- */
int jsvd_split(int m, int n, const double *Z, size_t ldz, double *X_re, double *X_im, size_t ldx,
               void *stream);
int jsvd_merge(int m, int n, const double *X_re, const double *X_im, size_t ldx, double *Z, size_t ldz,
               void *stream);

#ifdef __cplusplus
}
#endif
#endif /* JSVD_H */
