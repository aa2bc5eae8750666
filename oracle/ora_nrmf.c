/*
 * ora_nrmf.c -- oracle for the non-overflowing Frobenius norm with a widened
 * exponent range (Sect. SM6, Alg. rnF) of arXiv:2202.08361.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * A value r > 0 is held as (e, f), r = 2^e f, 1 <= f < 2, with e an integral
 * double (so e may exceed the exponent range of the data); zero is e = -inf.
 * With s lanes (lane L takes the elements L, L + s, L + 2s, ... in order;
 * complex data: the real part, then the imaginary part of each element):
 *
 *   per lane and element x (Sect. SM6.2):
 *     r' = (e - b, f 2^b), b the lowest bit of e (0 for e = -inf): an even
 *          (or infinite) exponent;
 *     |x| = (E(x), F(x)), E = getexp, F = the fraction in [1, 2);
 *     e_max = max(2 E(x), e');
 *     d_x = max(2 E(x) - e_max, -inf), d_r = max(e' - e_max, -inf), the max
 *          turning the NaN of -inf - (-inf) into -inf;
 *     f'' = fma(F(x) 2^{d_x/2}, F(x) 2^{d_x/2}, f' 2^{d_r});
 *     r <- (e_max + E(f''), F(f''));
 *   the s partial sums sorted non-decreasingly by (e, f) (eq. vsort);
 *   the sorted sums reduced pairwise, lg s levels (eqs. 1red, redj):
 *     (e_a, f_a) + (e_b, f_b) = (e_b, fma(2^{max(e_a - e_b, -inf)}, f_a, f_b)),
 *     normalised;
 *   ||x|| from ||x||^2 = (e, f) (Sect. SM6.1): (e/2, fl(sqrt f)) for even or
 *     infinite e, ((e-1)/2, fl(sqrt(2f))) for odd e.
 *
 * E(0) = -inf and F(0) = 0; scalef(x, y) = x 2^y with 2^-inf = 0.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* getexp: floor(lg |x|), -inf for 0 */
static double E_of(double x) { return x == 0.0 ? -INFINITY : (double)ilogb(x); }

/* getmant to [1, 2) with the sign dropped; 0 for 0 */
static double F_of(double x) { return x == 0.0 ? 0.0 : scalbn(fabs(x), -ilogb(x)); }

/* scalef for an integral or -inf exponent (the exponents here never reach +inf) */
static double scalef(double x, double y)
{
    if (y == -INFINITY) return x * 0.0;
    if (y < -4000.0) y = -4000.0;
    if (y > 4000.0) y = 4000.0;
    return scalbn(x, (int)y);
}

/* the lowest bit of an integral exponent, 0 for -inf */
static double lsb(double e)
{
    if (isinf(e)) return 0.0;
    return (double)(((long long)e) & 1LL);
}

/* one update r <- fma(|x|, |x|, r) of a lane */
static void lane_update(double *e, double *f, double x)
{
    const double b = lsb(*e);
    const double e1 = *e - b;
    const double f1 = scalef(*f, b);
    const double ex = E_of(x), fx = F_of(x);
    const double eh = ex * 2.0;
    const double emax = fmax(eh, e1);
    const double dx = fmax(eh - emax, -INFINITY);
    const double dr = fmax(e1 - emax, -INFINITY);
    const double fh = scalef(fx, dx * 0.5);
    const double fr = scalef(f1, dr);
    const double fn = fma(fh, fh, fr);
    *f = F_of(fn);
    *e = emax + E_of(fn);
}

typedef struct { double e, f; } ef_t;

static int ef_cmp(const void *pa, const void *pb)
{
    const ef_t *a = (const ef_t *)pa, *b = (const ef_t *)pb;
    if (a->e < b->e) return -1;
    if (a->e > b->e) return 1;
    if (a->f < b->f) return -1;
    if (a->f > b->f) return 1;
    return 0;
}

int ora_nrmf_lanes(int m, const double *xr, const double *xi, int s, double *le, double *lf)
{
    if (m < 0 || s < 1 || (s & (s - 1))) return ORA_EINVAL;
    for (int L = 0; L < s; ++L) {
        le[L] = -INFINITY;
        lf[L] = 1.0;
    }
    for (int i = 0; i < m; ++i) {
        const int L = i % s;
        lane_update(&le[L], &lf[L], xr[i]);
        if (xi) lane_update(&le[L], &lf[L], xi[i]);
    }
    return ORA_OK;
}

int ora_nrmf(int m, const double *xr, const double *xi, int s, double *e2, double *f2, double *e, double *f)
{
    if (m < 0 || s < 1 || s > (1 << 20) || (s & (s - 1))) return ORA_EINVAL;
    ef_t *r = (ef_t *)malloc(sizeof(ef_t) * (size_t)s);
    double *le = (double *)malloc(sizeof(double) * (size_t)s);
    double *lf = (double *)malloc(sizeof(double) * (size_t)s);
    (void)ora_nrmf_lanes(m, xr, xi, s, le, lf);
    for (int L = 0; L < s; ++L) {
        r[L].e = le[L];
        r[L].f = lf[L];
    }
    qsort(r, (size_t)s, sizeof(ef_t), ef_cmp);
    for (int h = s / 2; h >= 1; h /= 2) {
        for (int i = 0; i < h; ++i) {
            const ef_t a = r[2 * i], b = r[2 * i + 1];
            const double fn = fma(scalef(1.0, fmax(a.e - b.e, -INFINITY)), a.f, b.f);
            r[i].f = F_of(fn);
            r[i].e = b.e + E_of(fn);
        }
    }
    double ee = r[0].e, ff = r[0].f;
    if (ee == -INFINITY) ff = 1.0;   /* the norm of a zero array is (-inf, 1) */
    *e2 = ee;
    *f2 = ff;
    if (!isinf(ee) && lsb(ee) != 0.0) {
        *e = (ee - 1.0) * 0.5;
        *f = sqrt(2.0 * ff);
    } else {
        *e = ee * 0.5;
        *f = sqrt(ff);
    }
    free(r);
    free(le);
    free(lf);
    return ORA_OK;
}
