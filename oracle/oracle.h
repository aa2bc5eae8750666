/*
 * oracle.h -- CPU reference ("oracle") of the parallel one-sided Jacobi SVD
 * hot path of Novakovic, "Vectorization of a thread-parallel Jacobi singular
 * value decomposition method" (arXiv:2202.08361).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code; only the test suite, the smoke check and the CPU baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP library.
 *
 * Every routine is plain, sequential (the batch EVD loop may use OpenMP
 * threads, which does not change any result) and follows the paper's
 * formulas in the paper's order.  Build with -ffp-contract=off so that every
 * a*b+c is rounded twice unless fma() is written out, exactly as the paper's
 * operation lists require.
 *
 * Storage: matrices are column-major with a leading dimension (in elements);
 * complex data is split into separate real and imaginary arrays (Sect. 2.4.1).
 */
#ifndef JSVD_ORACLE_H
#define JSVD_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of lanes of the "vector" over which every sum (sum of squares,
 * scaled dot-product) is accumulated: lane L takes rows i = L, L+S, L+2S, ...
 * in increasing order, and the lanes are then combined by a pairwise
 * halving tree (lane j += lane j+h for h = S/2, S/4, ..., 1).  This is the
 * paper's vector accumulation followed by reduce_add (Alg. zdpscl), with the
 * vector width s taken as 1024. */
#define ORA_LANES 1024

/* flags of the stand-alone EVD */
#define ORA_EVD_SCALED  1u  /* return lambda' (not backscaled) */
#define ORA_EVD_SINFORM 2u  /* return e^{i alpha} sin(phi) instead of e^{i alpha} tan(phi) */

/* ---- 2x2 Hermitian / symmetric EVD (Sect. 2.1-2.3, Listing 1, Alg. d8jac2) ---- */
int ora_evd2_cplx(double a11, double a22, double a21r, double a21i,
                  double *cs, double *ctr, double *cti, double *l1, double *l2,
                  unsigned flags);
int ora_evd2_real(double a11, double a22, double a21,
                  double *cs, double *tn, double *l1, double *l2, unsigned flags);
/* Batched form (Alg. zbjac2 / dbjac2): a21i == NULL selects real symmetric.
 * Any output pointer may be NULL.  nthreads <= 0 uses the OpenMP default. */
void ora_evd2_batch(size_t r, const double *a11, const double *a22,
                    const double *a21r, const double *a21i,
                    double *cs, double *ctr, double *cti,
                    double *l1, double *l2, int32_t *zp,
                    unsigned flags, int nthreads);
int ora_omp_max_threads(void);

/* ---- single precision variants (Sect. 2.4.1: nu = FLT_MAX, fl(sqrt nu) =
 * 1.844674297E+19, FLT_TRUE_MIN, eta = FLT_MAX_EXP - 4) ---- */
int ora_sevd2_cplx(float a11, float a22, float a21r, float a21i,
                   float *cs, float *ctr, float *cti, float *l1, float *l2, unsigned flags);
int ora_sevd2_real(float a11, float a22, float a21,
                   float *cs, float *tn, float *l1, float *l2, unsigned flags);
void ora_sevd2_batch(size_t r, const float *a11, const float *a22,
                     const float *a21r, const float *a21i,
                     float *cs, float *ctr, float *cti,
                     float *l1, float *l2, int32_t *zp,
                     unsigned flags, int nthreads);

/* ---- scalar helpers ---- */
double ora_hypot(double x, double y);            /* Alg. hypot */
int    ora_getexp(double x);                      /* floor(lg|x|), x finite non-zero */
/* floor(lg(nu/(varsigma*m))) for the real (varsigma=2) and complex
 * (varsigma=4*sqrt(2)) cases, eq. (skn); exact integer evaluation. */
int    ora_lg_bound_m(int m, int cplx);
int    ora_s_round(double Mt, int cplx);          /* s_(k), eq. (skr) */
int    ora_s_square(double Mt, int m, int cplx);  /* s_[k], eq. (skn) */

/* ---- round-robin parallel pivot order ----
 * N = n (even) or n+1 (odd, index n is a phantom); K = N-1 steps per sweep.
 * Step k' in [0,K): pair 0 is (N-1, k'); pair l = 1..N/2-1 is
 * ((k'+l) mod K, (k'-l+K) mod K).  Each pair is returned ordered p < q.
 * Returns 0 if the pair contains the phantom column (skipped), 1 otherwise. */
int ora_rr_pair(int n, long kk, int l, int *p, int *q);
int ora_rr_steps(int n);                          /* K */

/* ---- column kernels (Sect. 3) ---- */
/* Frobenius norm of a real (xi == NULL) or complex column as (e, f), f in [1,2);
 * zero column -> (-inf, 1). */
void ora_colnorm(int m, const double *xr, const double *xi, double *e, double *f);
/* Scaled dot-product a21' = g_q^* g_p / (||g_q|| ||g_p||) (Alg. zdpscl). */
void ora_dpscl(int m, const double *qr, const double *qi, const double *pr, const double *pi,
               double eq, double fq, double ep, double fp, double *zr, double *zi);
/* Sect. SM2.2: RD(a b) (product rounded toward -infinity), eq. (d2sum) 2Sum,
 * and Alg. zdpsclcs / ddpsclcs (compensated scaled dot-product). */
double ora_mul_rd(double a, double b);
void ora_2sum(double a, double b, double *s, double *t);
void ora_dpscl_cs(int m, const double *qr, const double *qi, const double *pr, const double *pi,
                  double eq, double fq, double ep, double fp, double *zr, double *zi);
/* Scaled Gram matrix A'' (Alg. Gram). */
void ora_gram(double zr, double zi, double e1, double f1, double e2, double f2,
              double *a11, double *a22, double *a21r, double *a21i);
/* Rotation of a column pair (Alg. zjrot, eq. transf); returns the max-norm
 * of the transformed columns.  xi == NULL for real data (then S is ignored). */
double ora_rot(int l, double *xpr, double *xpi, double *xqr, double *xqi,
               double c, double C, double S, int swap);
void ora_swap(int l, double *xpr, double *xpi, double *xqr, double *xqi);

/* ---- the SVD driver (Sect. 4, Alg. zvjsvd) ---- */
typedef struct {
    int m, n, cplx;
    double *Gr, *Gi; size_t ldg;   /* iteration matrix, overwritten by U */
    double *Vr, *Vi; size_t ldv;   /* right singular vectors */
    double *e, *f;                 /* column norms (e,f), n each */
    int s;                         /* effective scaling exponent of G */
    double Mt;                     /* M~_k */
    long k;                        /* global step counter */
    long T;                        /* transformations in the current sweep */
    long last_t;                   /* transformations of the last step */
    long SW;                       /* swaps without transformation in the current sweep */
    long last_sw;                  /* swaps without transformation in the last step */
    int  rescaled;                 /* number of step-start downscalings */
    int  nosort;                   /* apply U instead of U P (the default; ORA_PERMUTE clears it) */
    int  comp;                     /* scaled dot-products with compensated summation */
    int  nogs;                     /* always rotate (no Gram-Schmidt replacement, eq. GScond) */
    long GS;                       /* Gram-Schmidt transformations in the current sweep */
    long last_gs;                  /* Gram-Schmidt transformations of the last step */
} ora_svd;

/* The EVD's permutation P (Sect. 2: the pivot columns are multiplied by U P
 * instead of U when they are also to be kept sorted by norm) is optional in
 * the paper.  With round-robin pairs it is off by default: a column swapped
 * by P takes over the other column's remaining partners of the sweep, so a
 * sweep no longer meets every pair of columns.  ORA_PERMUTE applies it;
 * ORA_NO_PERMUTE names the default explicitly; both together are invalid. */
#define ORA_NO_PERMUTE 1u
#define ORA_PERMUTE 8u
#define ORA_COMPENSATED 2u      /* Alg. zdpsclcs / ddpsclcs instead of zdpscl */
#define ORA_NO_GS 4u            /* rotate even where eq. (GScond) calls for Gram-Schmidt */

/* eq. (GScond) on the norms (e1,f1) = ||g_p||, (e2,f2) = ||g_q|| of a pair
 * that is to be transformed: 1 if ||g_p|| > 2^eta_hat upsilon ||g_q||, 2 if
 * ||g_q|| > 2^eta_hat upsilon ||g_p||, 0 otherwise (rotate). */
int ora_gs_case(double e1, double f1, double e2, double f2, double ups);
/* Alg. zgsscl / dgsscl (eq. GS): y <- (y 2^-ey - psi x 2^-ex) 2^ey with
 * psi = (wr + i wi) (fy/fx); x is left unchanged.  Returns the max-norm of
 * the new y. */
double ora_gs(int l, const double *xr, const double *xi, double *yr, double *yi,
              double ex, double fx, double ey, double fy, double wr, double wi);

/* ---- single precision SVD (Sect. SM8; constants in ora_ssvd.c) ---- */
float ora_s_hypot(float x, float y);
int ora_s_lg_bound_m(int m, int cplx);
int ora_s_s_round(float Mt, int cplx);
int ora_s_s_square(float Mt, int m, int cplx);
void ora_s_colnorm(int m, const float *xr, const float *xi, float *e, float *f);
void ora_s_dpscl(int m, const float *qr, const float *qi, const float *pr, const float *pi,
                 float eq, float fq, float ep, float fp, float *zr, float *zi);
void ora_s_gram(float zr, float zi, float e1, float f1, float e2, float f2,
                float *a11, float *a22, float *a21r, float *a21i);
float ora_s_rot(int l, float *xpr, float *xpi, float *xqr, float *xqi, float c, float C, float S, int swap);
/* eq. (GScond) / eq. (GS) in single precision (eta_hat = FLT_MAX_EXP - 1) */
int ora_s_gs_case(float e1, float f1, float e2, float f2, float ups);
float ora_s_gs(int l, const float *xr, const float *xi, float *yr, float *yi,
               float ex, float fx, float ey, float fy, float wr, float wi);
int ora_sgesvj(int m, int n, float *Gr, float *Gi, size_t ldg, float *Vr, float *Vi, size_t ldv,
               float *sv_e, float *sv_f, int max_sweeps, int *sweeps, long *steps, unsigned flags);
int ora_s_init_ext(int m, int n, float *Gr, float *Gi, size_t ldg, float *Vr, float *Vi, size_t ldv,
                   float *e, float *f, int *s, float *Mt);
void ora_s_step_ext(int m, int n, float *Gr, float *Gi, size_t ldg, float *Vr, float *Vi, size_t ldv,
                    float *e, float *f, int *s, float *Mt, long k, long *t, long *sw, long *gs, int *rescaled,
                    unsigned flags);

#define ORA_OK 0
#define ORA_NOT_CONVERGED 1
#define ORA_EINVAL (-1)
#define ORA_ENONFINITE (-2)
#define ORA_EZERO (-3)

/* Validate, find M~_0, scale G by 2^{s_0}, set V = I (Alg. zvjsvd, first two lines). */
int  ora_init(ora_svd *st);
/* One parallel step with pairs RR(k mod K); updates G, V, e, f, Mt, s, T. */
void ora_step(ora_svd *st);
/* U = G diag(2^{-e}) / f, sigma = (e - s, f), then a stable descending sort of
 * (sigma, u, v).  Writes the sorted U into G and sorted V into V. */
void ora_finalize(ora_svd *st, double *sv_e, double *sv_f);
/* The whole method: returns ORA_OK / ORA_NOT_CONVERGED / error; *sweeps = C,
 * the number of sweeps before the one that found nothing to do.  A sweep
 * converges when it neither transformed nor swapped a pair: a swap moves
 * columns, so a sweep that swapped did not meet every column pair. */
/* threads of the loops over a step's pairs (default 1); results do not
 * depend on it */
void ora_set_step_threads(int nthreads);
/* The exact mode (ora_exact.c): column norms and scaled dot-products of the
 * iteration from binary128 sums rounded once to double (superseding the
 * compensated dot-product); 0 = the ordered 1024-lane mode, the default. */
void ora_set_exact(int on);
int ora_get_exact(void);
void ora_colnorm_exact(int m, const double *xr, const double *xi, double *e, double *f);
void ora_dpscl_exact(int m, const double *qr, const double *qi, const double *pr, const double *pi,
                     double eq, double fq, double ep, double fp, double *zr, double *zi);
int  ora_gesvj(int m, int n, double *Gr, double *Gi, size_t ldg,
               double *Vr, double *Vi, size_t ldv,
               double *sv_e, double *sv_f, int max_sweeps, int *sweeps, long *steps,
               unsigned flags);

/* flat-argument forms of ora_init / ora_step / ora_finalize */
int  ora_init_ext(int m, int n, double *Gr, double *Gi, size_t ldg,
                  double *Vr, double *Vi, size_t ldv, double *e, double *f,
                  int *s, double *Mt);
void ora_step_ext(int m, int n, double *Gr, double *Gi, size_t ldg,
                  double *Vr, double *Vi, size_t ldv, double *e, double *f,
                  int *s, double *Mt, long k, long *t, long *sw, long *gs, int *rescaled, unsigned flags);
void ora_finalize_ext(int m, int n, double *Gr, double *Gi, size_t ldg,
                      double *Vr, double *Vi, size_t ldv, double *e, double *f,
                      int s, double *sv_e, double *sv_f);

/* ---- non-overflowing Frobenius norm with a widened exponent (Sect. SM6, Alg. rnF) ---- */
/* The s lane partial sums (e, f) of ||x||^2 (s a power of two), unsorted. */
int ora_nrmf_lanes(int m, const double *xr, const double *xi, int s, double *le, double *lf);
/* ||x||^2 = 2^e2 f2 and ||x|| = 2^e f (e2, e integral doubles, -inf for x = 0). */
int ora_nrmf(int m, const double *xr, const double *xi, int s, double *e2, double *f2, double *e, double *f);


#ifdef __cplusplus
}
#endif

#endif
