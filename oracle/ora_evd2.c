/*
 * ora_evd2.c -- oracle for the branch-free, power-of-two-scaled EVD of a
 * Hermitian (complex) or symmetric (real) matrix of order two.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The complex routine follows the serial algorithm of Sect. 2.3.1 (Listing 1)
 * of arXiv:2202.08361 step by step: the scaling exponent of eq. (z) with
 * eta' = DBL_MAX_EXP - 3, the exact power-of-two scaling, the polar form of
 * eq. (zpolar) with the naive hypot of eq. (hypot), the clamped tan(2 phi) of
 * eq. (tan2), tan(phi) of eq. (jactan), the secant form of eq. (jacsec) and
 * the eigenvalues of eq. (lamsec).  The real routine is the specialisation
 * of Alg. d8jac2 (Sect. SM2.1): e^{i alpha} = sign(a21).
 *
 * Build with -ffp-contract=off: every operation below is one IEEE-754
 * double operation, rounded to nearest-even, fma() written out explicitly.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"

/* fl(sqrt(nu)), the clamp of tan(2 phi) in eq. (tan2) */
static const double ORA_SQRT_NU = 1.34078079299425956E+154;

/* zeta_c = eta' - (exponent of |c|, zero treated as the smallest subnormal),
 * with eta' = DBL_MAX_EXP - 3 = 1021 and frexp's exponent being
 * floor(lg|c|) + 1. */
static int zeta_of(double c)
{
    int ex;
    (void)frexp(fmax(fabs(c), DBL_TRUE_MIN), &ex);
    return (DBL_MAX_EXP - 3) - ex;
}

static double flip_sign_by(double x, double s)
{
    /* x with its sign bit XOR-ed with the sign bit of s */
    uint64_t ux, us;
    memcpy(&ux, &x, 8);
    memcpy(&us, &s, 8);
    ux ^= (us & 0x8000000000000000ull);
    memcpy(&x, &ux, 8);
    return x;
}

int ora_evd2_cplx(double a11, double a22, double a21r, double a21i,
                  double *cs, double *ctr, double *cti, double *l1, double *l2,
                  unsigned flags)
{
    /* scaling exponent: the minimum over the four components (eq. z) */
    const int z11 = zeta_of(a11), z22 = zeta_of(a22);
    const int zr = zeta_of(a21r), zi = zeta_of(a21i);
    const int zR = (z11 <= z22) ? z11 : z22;
    const int zC = (zr <= zi) ? zr : zi;
    const int zeta = (zR <= zC) ? zR : zC;
    const int zeta_b = -zeta;

    /* A' = 2^zeta A, exact unless a component is pushed below the normal range */
    const double br = scalbn(a21r, zeta), bi = scalbn(a21i, zeta);
    const double b11 = scalbn(a11, zeta), b22 = scalbn(a22, zeta);

    /* polar form |a21'| e^{i alpha} with the naive hypot */
    const double abr = fabs(br), abi = fabs(bi);
    const double am = fmin(abr, abi), aM = fmax(abr, abi);
    const double mM = fmax(am / aM, 0.0);
    const double ab = sqrt(fma(mM, mM, 1.0)) * aM;
    const double ca = copysign(fmin(abr / ab, 1.0), br);
    const double sa = bi / fmax(ab, DBL_TRUE_MIN);

    /* the Jacobi rotation */
    const double o = ab * 2.0;
    const double a = b11 - b22;
    const double t2 = copysign(fmin(fmax(o / fabs(a), 0.0), ORA_SQRT_NU), a);
    const double t = t2 / (1.0 + sqrt(fma(t2, t2, 1.0)));
    const double sec2 = fma(t, t, 1.0);
    const double sec = sqrt(sec2);
    const double c = 1.0 / sec;
    double C = ca * t;
    double S = sa * t;
    if (flags & ORA_EVD_SINFORM) {
        C = C / sec;
        S = S / sec;
    }

    /* eigenvalues of A' */
    const double lp1 = fma(t, fma(b22, t, o), b11) / sec2;
    const double lp2 = fma(t, fma(b11, t, -o), b22) / sec2;

    if (cs) *cs = c;
    if (ctr) *ctr = C;
    if (cti) *cti = S;
    if (flags & ORA_EVD_SCALED) {
        if (l1) *l1 = lp1;
        if (l2) *l2 = lp2;
    } else {
        if (l1) *l1 = scalbn(lp1, zeta_b);
        if (l2) *l2 = scalbn(lp2, zeta_b);
    }
    return (int)(((unsigned)zeta_b << 1) | (unsigned)(lp1 < lp2));
}

int ora_evd2_real(double a11, double a22, double a21,
                  double *cs, double *tn, double *l1, double *l2, unsigned flags)
{
    const int z11 = zeta_of(a11), z22 = zeta_of(a22), z21 = zeta_of(a21);
    const int zR = (z11 <= z22) ? z11 : z22;
    const int zeta = (zR <= z21) ? zR : z21;
    const int zeta_b = -zeta;

    const double b21 = scalbn(a21, zeta);
    const double b11 = scalbn(a11, zeta), b22 = scalbn(a22, zeta);

    const double ab = fabs(b21);
    const double o = ab * 2.0;
    const double a = b11 - b22;
    const double t2 = copysign(fmin(fmax(o / fabs(a), 0.0), ORA_SQRT_NU), a);
    const double t = t2 / (1.0 + sqrt(fma(t2, t2, 1.0)));
    const double sec2 = fma(t, t, 1.0);
    const double sec = sqrt(sec2);
    const double c = 1.0 / sec;
    /* e^{i alpha} tan(phi) = sign(a21) tan(phi): the sign bits multiply */
    double T = flip_sign_by(t, b21);
    if (flags & ORA_EVD_SINFORM)
        T = T / sec;

    const double lp1 = fma(t, fma(b22, t, o), b11) / sec2;
    const double lp2 = fma(t, fma(b11, t, -o), b22) / sec2;

    if (cs) *cs = c;
    if (tn) *tn = T;
    if (flags & ORA_EVD_SCALED) {
        if (l1) *l1 = lp1;
        if (l2) *l2 = lp2;
    } else {
        if (l1) *l1 = scalbn(lp1, zeta_b);
        if (l2) *l2 = scalbn(lp2, zeta_b);
    }
    return (int)(((unsigned)zeta_b << 1) | (unsigned)(lp1 < lp2));
}

void ora_evd2_batch(size_t r, const double *a11, const double *a22,
                    const double *a21r, const double *a21i,
                    double *cs, double *ctr, double *cti,
                    double *l1, double *l2, int32_t *zp,
                    unsigned flags, int nthreads)
{
    long long i, rr = (long long)r;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#else
    (void)nthreads;
#endif
    for (i = 0; i < rr; ++i) {
        double c, C, S = 0.0, L1, L2;
        int z;
        if (a21i)
            z = ora_evd2_cplx(a11[i], a22[i], a21r[i], a21i[i], &c, &C, &S, &L1, &L2, flags);
        else
            z = ora_evd2_real(a11[i], a22[i], a21r[i], &c, &C, &L1, &L2, flags);
        if (cs) cs[i] = c;
        if (ctr) ctr[i] = C;
        if (cti && a21i) cti[i] = S;
        if (l1) l1[i] = L1;
        if (l2) l2[i] = L2;
        if (zp) zp[i] = z;
    }
}

int ora_omp_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
