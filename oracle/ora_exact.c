/*
 * ora_exact.c -- the oracle's "exact" mode of the column kernels of
 * arXiv:2202.08361: column norms (Sect. 3.2) and scaled dot-products
 * (Alg. zdpscl, without its final division) evaluated in binary128 and
 * rounded once to double.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The product of two doubles has at most 106 significant bits, so every
 * square and every product below is exact in binary128 (113 bits, exponent
 * range far beyond double's); only the running sums and the square root
 * round, each to 113 bits, and the result is rounded once more, to double.
 * That is the correctly rounded value except when the exact value lies
 * within about m 2^-113 (relative) of a rounding boundary of double.
 *
 * The ordered mode (ora_svd.c) fixes the summation order instead (1024
 * lanes, a halving tree), which is what the GPU path reproduces bit for
 * bit; this mode is the reference that the ordered sums are measured
 * against, and an alternative iteration whose results agree with the
 * ordered one to rounding.
 */
#include <math.h>
#include <quadmath.h>
#include <stddef.h>
#include "oracle.h"

/* x 2^e rounded once to double, as (e', f') with f' in [1, 2) */
static void split_ef(__float128 x, double *e, double *f)
{
    int ex = 0;
    __float128 fr = frexpq(x, &ex);            /* x = fr 2^ex, fr in [1/2, 1) */
    double fd = (double)(fr * 2);              /* the one rounding, to [1, 2] */
    int E = ex - 1;
    if (fd == 2.0) {                           /* rounded up to the next binade */
        fd = 1.0;
        E += 1;
    }
    *e = (double)E;
    *f = fd;
}

/* ||x||_2 of a real or complex column (xi may be NULL) in (e, f) form:
 * sqrt of the exact sum of squares, rounded once.  A zero column gives
 * e = -inf, f = 1, as in the ordered mode. */
void ora_colnorm_exact(int m, const double *xr, const double *xi, double *e, double *f)
{
    __float128 s = 0;
    int nonzero = 0;
    for (int i = 0; i < m; ++i) {
        const __float128 a = xr[i];
        s += a * a;
        nonzero |= xr[i] != 0.0;
        if (xi) {
            const __float128 b = xi[i];
            s += b * b;
            nonzero |= xi[i] != 0.0;
        }
    }
    if (!nonzero) {
        *e = -INFINITY;
        *f = 1.0;
        return;
    }
    split_ef(sqrtq(s), e, f);
}

/* The scaled dot-product a21' of Alg. zdpscl from the exact sum: with
 * g_j = x_j 2^-e_j, h = sum conj(g_q) g_p (real part: qr pr + qi pi,
 * imaginary part: qr pi - qi pr) rounded once to double, then divided by
 * fl(f_q f_p) as in the ordered mode. */
void ora_dpscl_exact(int m, const double *qr, const double *qi, const double *pr, const double *pi,
                     double eq, double fq, double ep, double fp, double *zr, double *zi)
{
    __float128 hr = 0, hi = 0;
    for (int i = 0; i < m; ++i) {
        const __float128 a = qr[i], b = pr[i];
        hr += a * b;
        if (qi) {
            const __float128 c = qi[i], d = pi[i];
            hr += c * d;
            hi += a * d;
            hi -= c * b;
        }
    }
    const int sh = -((int)eq + (int)ep);
    const double hrd = (double)scalbnq(hr, sh);
    const double hid = qi ? (double)scalbnq(hi, sh) : 0.0;
    const double dd = fq * fp;
    *zr = hrd / dd;
    *zi = qi ? hid / dd : 0.0;
}
