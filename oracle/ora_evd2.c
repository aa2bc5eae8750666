/*
 * ora_evd2.c -- oracle for the branch-free, power-of-two-scaled EVD of a
 * Hermitian (complex) or symmetric (real) matrix of order two.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Written from the equations of Sect. 2 of arXiv:2202.08361, each in a
 * routine of its own:
 *   eq. (z)                     the scaling exponent zeta = min_c (eta -
 *                               floor(lg|c|)), eta = floor(lg(nu/8)),
 *                               lg 0 read as lg of the smallest subnormal;
 *   eqs. (hypot), (zpolar)      |a21'| and e^{i alpha} = cos + i sin;
 *   eqs. (tan2), (jactan),      tan(2 phi) clamped by fl(sqrt(nu)), tan(phi),
 *   (jacsec)                    sec^2, sec and cos(phi);
 *   eq. (lamsec)                the eigenvalues of A' = 2^zeta A.
 * The real case takes e^{i alpha} = sign(a21) = +-1 (eq. alpha, with
 * sign(+-0) = +-1).
 *
 * Build with -ffp-contract=off: every operation below is one IEEE-754
 * double operation, rounded to nearest-even, fma() written out where an
 * equation has one.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"

/* fl(sqrt(nu)) for nu = DBL_MAX: the bound on |tan(2 phi)| of eq. (tan2) */
static const double ORA_SQRT_NU = 1.34078079299425956E+154;

/* eq. (z) for one component c: eta - floor(lg|c|) with eta = floor(lg(nu/8))
 * = DBL_MAX_EXP - 4; frexp returns floor(lg|c|) + 1 and nothing useful for
 * zero, so zero is replaced by the smallest subnormal */
static int ora_zeta_part(double c)
{
    int e;
    (void)frexp(fmax(fabs(c), DBL_TRUE_MIN), &e);
    return (DBL_MAX_EXP - 4) - (e - 1);
}

/* eq. (z): the minimum over the k components */
static int ora_zeta(const double *comp, int k)
{
    int z = ora_zeta_part(comp[0]);
    for (int i = 1; i < k; ++i) {
        const int zi = ora_zeta_part(comp[i]);
        if (zi < z) z = zi;
    }
    return z;
}

/* eqs. (hypot), (zpolar): x + iy = r (cos + i sin).  r is the naive hypot
 * M sqrt(q^2 + 1) with q = m/M (0/0 read as 0); the cosine is clamped to 1
 * and takes the sign of x; the sine divides by r, kept from zero by the
 * smallest subnormal. */
static void ora_polar(double x, double y, double *r, double *cosv, double *sinv)
{
    const double m = fmin(fabs(x), fabs(y));
    const double M = fmax(fabs(x), fabs(y));
    const double q = fmax(m / M, 0.0);
    *r = sqrt(fma(q, q, 1.0)) * M;
    *cosv = copysign(fmin(fabs(x) / *r, 1.0), x);
    *sinv = y / fmax(*r, DBL_TRUE_MIN);
}

/* eqs. (tan2), (jactan), (jacsec): the rotation from 2|a21'| and
 * a = a11' - a22' */
typedef struct {
    double tan_phi, sec2_phi, sec_phi, cos_phi;
} ora_jrot;

static ora_jrot ora_rotation(double two_abs21, double a)
{
    ora_jrot g;
    const double tan_2phi = copysign(fmin(fmax(two_abs21 / fabs(a), 0.0), ORA_SQRT_NU), a);
    g.tan_phi = tan_2phi / (1.0 + sqrt(fma(tan_2phi, tan_2phi, 1.0)));
    g.sec2_phi = fma(g.tan_phi, g.tan_phi, 1.0);
    g.sec_phi = sqrt(g.sec2_phi);
    g.cos_phi = 1.0 / g.sec_phi;
    return g;
}

/* eq. (lamsec): ((y tan + o) tan + x) / sec^2.  lambda_1 takes
 * (x, y, o) = (a11', a22', 2|a21'|) and lambda_2 (a22', a11', -2|a21'|). */
static double ora_lamsec(double x, double y, double o, const ora_jrot *g)
{
    return fma(g->tan_phi, fma(y, g->tan_phi, o), x) / g->sec2_phi;
}

/* the outputs common to both cases; returns (zeta' << 1) | p */
static int ora_finish(double a11s, double a22s, double two_abs21, const ora_jrot *g, int zeta,
                      double *l1, double *l2, unsigned flags)
{
    const double lam1 = ora_lamsec(a11s, a22s, two_abs21, g);
    const double lam2 = ora_lamsec(a22s, a11s, -two_abs21, g);
    const int zeta_back = -zeta;
    const int scaled = (flags & ORA_EVD_SCALED) != 0;
    if (l1) *l1 = scaled ? lam1 : scalbn(lam1, zeta_back);
    if (l2) *l2 = scaled ? lam2 : scalbn(lam2, zeta_back);
    return (int)(((unsigned)zeta_back << 1) | (unsigned)(lam1 < lam2));
}

int ora_evd2_cplx(double a11, double a22, double a21r, double a21i,
                  double *cs, double *ctr, double *cti, double *l1, double *l2,
                  unsigned flags)
{
    const double comp[4] = {a11, a22, a21r, a21i};
    const int zeta = ora_zeta(comp, 4);
    /* A' = 2^zeta A */
    const double a11s = scalbn(a11, zeta), a22s = scalbn(a22, zeta);
    double r, cos_alpha, sin_alpha;
    ora_polar(scalbn(a21r, zeta), scalbn(a21i, zeta), &r, &cos_alpha, &sin_alpha);
    const double two_abs21 = r * 2.0;
    const ora_jrot g = ora_rotation(two_abs21, a11s - a22s);
    /* e^{i alpha} tan(phi), or e^{i alpha} sin(phi) = e^{i alpha} tan(phi) / sec(phi) */
    double re = cos_alpha * g.tan_phi, im = sin_alpha * g.tan_phi;
    if (flags & ORA_EVD_SINFORM) {
        re = re / g.sec_phi;
        im = im / g.sec_phi;
    }
    if (cs) *cs = g.cos_phi;
    if (ctr) *ctr = re;
    if (cti) *cti = im;
    return ora_finish(a11s, a22s, two_abs21, &g, zeta, l1, l2, flags);
}

int ora_evd2_real(double a11, double a22, double a21,
                  double *cs, double *tn, double *l1, double *l2, unsigned flags)
{
    const double comp[3] = {a11, a22, a21};
    const int zeta = ora_zeta(comp, 3);
    const double a11s = scalbn(a11, zeta), a22s = scalbn(a22, zeta);
    const double a21s = scalbn(a21, zeta);
    const double two_abs21 = fabs(a21s) * 2.0;
    const ora_jrot g = ora_rotation(two_abs21, a11s - a22s);
    /* e^{i alpha} = sign(a21) = +-1: multiplying by it is exact */
    double v = g.tan_phi * copysign(1.0, a21s);
    if (flags & ORA_EVD_SINFORM)
        v = v / g.sec_phi;
    if (cs) *cs = g.cos_phi;
    if (tn) *tn = v;
    return ora_finish(a11s, a22s, two_abs21, &g, zeta, l1, l2, flags);
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
