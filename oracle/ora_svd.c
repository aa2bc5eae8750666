/*
 * ora_svd.c -- oracle for the column kernels and the parallel one-sided
 * Jacobi SVD driver of arXiv:2202.08361 (Sects. 3 and 4, Alg. zvjsvd).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain sequential C, one IEEE-754 operation per expression, fma() written
 * out (build with -ffp-contract=off).  Readings where the paper leaves a
 * choice open are stated next to the code that takes them.
 */
#include <fenv.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* ------------------------------------------------------------------ */
/* scalar helpers                                                      */
/* ------------------------------------------------------------------ */

/* Alg. hypot (Sect. 2.2.1): M sqrt((m/M)^2 + 1), q = max(m/M, 0). */
double ora_hypot(double x, double y)
{
    const double ax = fabs(x), ay = fabs(y);
    const double mn = fmin(ax, ay), mx = fmax(ax, ay);
    const double q = fmax(mn / mx, 0.0);
    return sqrt(fma(q, q, 1.0)) * mx;
}

int ora_getexp(double x) { return ilogb(x); }

/* floor(lg(nu / (varsigma m))), eq. (skn).
 * Real, varsigma = 2: 2^k * 2m <= nu with nu = 2^1024 (1 - 2^-53) gives
 * k = 1023 - floor(lg 2m) = 1022 - floor(lg m) (exact also when m is a power
 * of two, since nu is below 2^1024).
 * Complex, varsigma = 4 sqrt 2: k = floor(1021.5 - lg m - tiny); with
 * a = floor(lg m) this is 1021 - a, minus one more when m > 2^a sqrt 2,
 * i.e. when m^2 > 2^(2a+1) (m^2 is never exactly 2^(2a+1)). */
int ora_lg_bound_m(int m, int cplx)
{
    int a = 0;
    while ((2LL << a) <= (long long)m) ++a;        /* a = floor(lg m) */
    if (!cplx)
        return 1022 - a;
    {
        const unsigned long long mm = (unsigned long long)m * (unsigned long long)m;
        const unsigned long long b = 1ULL << (2 * a + 1);
        return 1021 - a - (mm > b ? 1 : 0);
    }
}

/* s_(k), eq. (skr): real floor(lg(nu/2)) - floor(lg M~) = 1022 - floor(lg M~);
 * complex floor(lg(nu/(4 sqrt 2))) - floor(lg M~) - 1 = 1020 - floor(lg M~). */
int ora_s_round(double Mt, int cplx)
{
    return (cplx ? 1020 : 1022) - ilogb(Mt);
}

/* s_[k], eq. (skn), with the unconditional subtraction of one. */
int ora_s_square(double Mt, int m, int cplx)
{
    return ora_lg_bound_m(m, cplx) - ilogb(Mt) - 1;
}

/* ------------------------------------------------------------------ */
/* round-robin pivot order                                             */
/* ------------------------------------------------------------------ */

int ora_rr_steps(int n)
{
    const int N = n + (n & 1);
    return N - 1;
}

int ora_rr_pair(int n, long kk, int l, int *p, int *q)
{
    const int N = n + (n & 1), K = N - 1;
    const int k = (int)(kk % K);
    int a, b;
    if (l == 0) {
        a = N - 1;
        b = k;
    } else {
        a = (k + l) % K;
        b = (k - l + K) % K;
    }
    if (a > b) { const int t = a; a = b; b = t; }
    *p = a;
    *q = b;
    return b < n;   /* b == n only for the phantom column of an odd n */
}

/* ------------------------------------------------------------------ */
/* lane accumulation                                                   */
/* ------------------------------------------------------------------ */

/* reduce_add of the ORA_LANES partial sums by the halving tree.
 * Only the first P lanes are touched, P the smallest power of two >= m
 * (capped at ORA_LANES): the others hold +0, and a partial sum that starts
 * at +0 and is only ever updated by fma or + never becomes -0, so the levels
 * h >= P only add +0 to the first P lanes and leave them unchanged. */
static int lanes_used(int m)
{
    int P = 1;
    while (P < m && P < ORA_LANES) P *= 2;
    return P;
}

static double lanes_reduce(double *a, int P)
{
    for (int h = P / 2; h >= 1; h /= 2)
        for (int j = 0; j < h; ++j)
            a[j] = a[j] + a[j + h];
    return a[0];
}

/* ------------------------------------------------------------------ */
/* column kernels                                                      */
/* ------------------------------------------------------------------ */

/* Frobenius norm of a column in the (e, f) form of Sect. 3.2 / SM6.1.
 * Reading of the norm routine (the paper leaves it to the implementation):
 * the column is prescaled by 2^-E, E = floor(lg max|x_i|) (exact), the
 * squares are accumulated with fma in the lane order, and for a complex
 * column the two real norms are combined by the naive hypot (Sect. 3.2,
 * last paragraph).  The prescaled sum lies in [1, 4m], so nothing
 * overflows and the goto-rescale of Alg. zvjsvd is never needed. */
void ora_colnorm(int m, const double *xr, const double *xi, double *e, double *f)
{
    double ar[ORA_LANES], ai[ORA_LANES];
    double mx = 0.0;
    for (int i = 0; i < m; ++i) {
        mx = fmax(mx, fabs(xr[i]));
        if (xi) mx = fmax(mx, fabs(xi[i]));
    }
    if (mx == 0.0) {
        *e = -INFINITY;
        *f = 1.0;
        return;
    }
    const int E = ilogb(mx);
    const int P = lanes_used(m);
    memset(ar, 0, sizeof(double) * (size_t)P);
    memset(ai, 0, sizeof(double) * (size_t)P);
    for (int i = 0; i < m; ++i) {
        const int L = i % ORA_LANES;
        const double yr = scalbn(xr[i], -E);
        ar[L] = fma(yr, yr, ar[L]);
        if (xi) {
            const double yi = scalbn(xi[i], -E);
            ai[L] = fma(yi, yi, ai[L]);
        }
    }
    const double sr = lanes_reduce(ar, P);
    double r;
    if (xi) {
        const double si = lanes_reduce(ai, P);
        r = ora_hypot(sqrt(sr), sqrt(si));
    } else {
        r = sqrt(sr);
    }
    const int er = ilogb(r);
    *e = (double)(E + er);
    *f = scalbn(r, -er);
}

/* Alg. zdpscl: the columns are prescaled by 2^-e_j, the products are
 * accumulated per lane (real part: qr*pr then qi*pi; imaginary part: qr*pi
 * then -qi*pr), the lanes are reduced, and the result is divided once by
 * fl(f_q f_p). */
void ora_dpscl(int m, const double *qr, const double *qi, const double *pr, const double *pi,
               double eq, double fq, double ep, double fp, double *zr, double *zi)
{
    double ar[ORA_LANES], ai[ORA_LANES];
    const int Eq = (int)eq, Ep = (int)ep;
    const int P = lanes_used(m);
    memset(ar, 0, sizeof(double) * (size_t)P);
    memset(ai, 0, sizeof(double) * (size_t)P);
    for (int i = 0; i < m; ++i) {
        const int L = i % ORA_LANES;
        const double gqr = scalbn(qr[i], -Eq), gpr = scalbn(pr[i], -Ep);
        if (qi) {
            const double gqi = scalbn(qi[i], -Eq), gpi = scalbn(pi[i], -Ep);
            ar[L] = fma(gqr, gpr, ar[L]);
            ai[L] = fma(gqr, gpi, ai[L]);
            ar[L] = fma(gqi, gpi, ar[L]);
            ai[L] = fma(-gqi, gpr, ai[L]);
        } else {
            ar[L] = fma(gqr, gpr, ar[L]);
        }
    }
    const double hr = lanes_reduce(ar, P);
    const double hi = qi ? lanes_reduce(ai, P) : 0.0;
    const double d = fq * fp;
    *zr = hr / d;
    *zi = qi ? hi / d : 0.0;
}

/* ------------------------------------------------------------------ */
/* compensated scaled dot-product (Sect. SM2.2, Alg. zdpsclcs/ddpsclcs) */
/* ------------------------------------------------------------------ */

/* RD(a b): the product rounded toward -infinity, computed by the host FPU
 * switched to that rounding mode (item G. of Sect. SM2.2).  The library is
 * built with -frounding-math, so the multiplication is not moved across
 * the mode switches or folded at compile time. */
double ora_mul_rd(double a, double b)
{
    const int old = fegetround();
    fesetround(FE_DOWNWARD);
    volatile double c = a * b;
    fesetround(old);
    return c;
}

/* eq. (d2sum), Moller's 2Sum: s = fl(a + b) and a + b = s + t exactly. */
void ora_2sum(double a, double b, double *s, double *t)
{
    const double s0 = a + b;
    double a1 = s0 - b;
    double b1 = s0 - a1;
    a1 = a - a1;
    b1 = b - b1;
    *s = s0;
    *t = a1 + b1;
}

/* One product term of the compensated sums: c = RD(x y) and c' = x y - c
 * (one fma), then Kahan's update of the value stream (s, t) with c and of
 * the error stream (s', t') with c', each by 2Sum (items G., M., K.). */
static void cs_term(double x, double y, double *s, double *t, double *s2, double *t2)
{
    const double c = ora_mul_rd(x, y);
    const double c2 = fma(x, y, -c);
    ora_2sum(*s, c + *t, s, t);
    ora_2sum(*s2, c2 + *t2, s2, t2);
}

/* Alg. zdpsclcs / ddpsclcs: the scaled dot-product g_q^* g_p / (|g_q| |g_p|)
 * with compensated summation.  Each lane of the 1024-lane vector keeps four
 * partial sums per real stream (s, t of the rounded-down products, s', t' of
 * their errors); the lanes are reduced one sum at a time by the halving
 * tree, and the four totals are added as ((s' + t') + t) + s (the real
 * algorithm writes s + (t + (s' + t')), the same value since floating-point
 * addition commutes).
 *
 * Reading: the paper states the result as g_q^* g_p for both routines, as
 * in Alg. zdpscl, but the imaginary-part updates printed in Alg. zdpsclcs
 * form Re(g_p) Im(g_q) - Im(g_p) Re(g_q), the imaginary part of g_p^* g_q.
 * The stated result is taken: the imaginary stream adds Re(g_q) Im(g_p),
 * then (-Im(g_q)) Re(g_p) (the sign flipped on the operand before the
 * rounded-down product, as the algorithm flips it). */
void ora_dpscl_cs(int m, const double *qr, const double *qi, const double *pr, const double *pi,
                  double eq, double fq, double ep, double fp, double *zr, double *zi)
{
    static _Thread_local double acc[8][ORA_LANES];
    const int Eq = (int)eq, Ep = (int)ep;
    const int P = lanes_used(m);
    for (int a = 0; a < 8; ++a) memset(acc[a], 0, sizeof(double) * (size_t)P);
    double *rs = acc[0], *rt = acc[1], *rs2 = acc[2], *rt2 = acc[3];
    double *is = acc[4], *it = acc[5], *is2 = acc[6], *it2 = acc[7];
    for (int i = 0; i < m; ++i) {
        const int L = i % ORA_LANES;
        const double gpr = scalbn(pr[i], -Ep), gqr = scalbn(qr[i], -Eq);
        cs_term(gpr, gqr, &rs[L], &rt[L], &rs2[L], &rt2[L]);
        if (qi) {
            const double gpi = scalbn(pi[i], -Ep), gqi = scalbn(qi[i], -Eq);
            cs_term(gpi, gqi, &rs[L], &rt[L], &rs2[L], &rt2[L]);
            cs_term(gqr, gpi, &is[L], &it[L], &is2[L], &it2[L]);
            cs_term(-gqi, gpr, &is[L], &it[L], &is2[L], &it2[L]);
        }
    }
    double hr = lanes_reduce(rs2, P) + lanes_reduce(rt2, P);
    hr = hr + lanes_reduce(rt, P);
    hr = hr + lanes_reduce(rs, P);
    double hi = 0.0;
    if (qi) {
        hi = lanes_reduce(is2, P) + lanes_reduce(it2, P);
        hi = hi + lanes_reduce(it, P);
        hi = hi + lanes_reduce(is, P);
    }
    const double d = fq * fp;
    *zr = hr / d;
    *zi = qi ? hi / d : 0.0;
}

/* Alg. Gram with eqs. (sGramEF), (efpq), (F): the diagonal entries are
 * ||g_p||/||g_q|| and ||g_q||/||g_p|| in normalised (e,f) form, and the
 * whole matrix is scaled by 2^{s_A}, s_A = min(DBL_MAX_EXP-1 - max(e12,e21), 0). */
void ora_gram(double zr, double zi, double e1, double f1, double e2, double f2,
              double *a11, double *a22, double *a21r, double *a21i)
{
    double f12 = f1 / f2;
    double f21 = f2 / f1;
    long e12 = (long)e1 - (long)e2;
    long e21 = (long)e2 - (long)e1;
    const int g12 = ilogb(f12), g21 = ilogb(f21);
    e12 += g12;
    f12 = scalbn(f12, -g12);
    e21 += g21;
    f21 = scalbn(f21, -g21);
    long sA = (DBL_MAX_EXP - 1) - (e12 > e21 ? e12 : e21);
    if (sA > 0) sA = 0;
    e12 += sA;
    e21 += sA;
    /* exponents below -2200 give zero either way; clamp keeps the int cast defined */
    if (e12 < -4000) e12 = -4000;
    if (e21 < -4000) e21 = -4000;
    if (sA < -4000) sA = -4000;
    *a11 = scalbn(f12, (int)e12);
    *a22 = scalbn(f21, (int)e21);
    *a21r = scalbn(zr, (int)sA);
    *a21i = scalbn(zi, (int)sA);
}

/* Alg. zjrot / eq. (transf) with the complex fma of eq. (zfma):
 *   x_p' = fma(x_q, e', x_p) c,  x_q' = fma(x_p, -conj(e'), x_q) c,  e' = C + iS,
 * stored swapped when P is the transposition.  Real data: e' = C = +-tan(phi). */
double ora_rot(int l, double *xpr, double *xpi, double *xqr, double *xqi,
               double c, double C, double S, int swap)
{
    double M = 0.0;
    for (int i = 0; i < l; ++i) {
        const double pr = xpr[i], qr = xqr[i];
        if (xpi) {
            const double pi = xpi[i], qi = xqi[i];
            const double npr = fma(qr, C, fma(-qi, S, pr)) * c;
            const double npi = fma(qr, S, fma(qi, C, pi)) * c;
            const double nqr = fma(pr, -C, fma(-pi, S, qr)) * c;
            const double nqi = fma(pr, S, fma(pi, -C, qi)) * c;
            if (swap) {
                xpr[i] = nqr; xpi[i] = nqi; xqr[i] = npr; xqi[i] = npi;
            } else {
                xpr[i] = npr; xpi[i] = npi; xqr[i] = nqr; xqi[i] = nqi;
            }
            M = fmax(M, fmax(fabs(npr), fabs(npi)));
            M = fmax(M, fmax(fabs(nqr), fabs(nqi)));
        } else {
            const double np = fma(qr, C, pr) * c;
            const double nq = fma(pr, -C, qr) * c;
            if (swap) {
                xpr[i] = nq; xqr[i] = np;
            } else {
                xpr[i] = np; xqr[i] = nq;
            }
            M = fmax(M, fmax(fabs(np), fabs(nq)));
        }
    }
    return M;
}

void ora_swap(int l, double *xpr, double *xpi, double *xqr, double *xqi)
{
    for (int i = 0; i < l; ++i) {
        double t = xpr[i]; xpr[i] = xqr[i]; xqr[i] = t;
        if (xpi) { t = xpi[i]; xpi[i] = xqi[i]; xqi[i] = t; }
    }
}

/* eq. (GScond), evaluated on the normalised quotient of the norms that
 * Alg. Gram forms (eq. efpq): ||g_p|| / ||g_q|| = 2^{e_{p/q}} f_{p/q} with
 * f_{p/q} = F(fl(f_p/f_q)), compared in (e, f) form with 2^eta_hat upsilon =
 * 2^{eta_hat + e_u} f_u, eta_hat = DBL_MAX_EXP - 1, upsilon = 2^{e_u} f_u. */
static int gs_exceeds(double ea, double fa, double eb, double fb, double ups, int eta_hat)
{
    double fab = fa / fb;
    const int g = ilogb(fab);
    const long eab = (long)ea - (long)eb + g;
    fab = scalbn(fab, -g);
    const int eu = ilogb(ups);
    const double fu = scalbn(ups, -eu);
    const long et = (long)eta_hat + eu;
    return eab > et || (eab == et && fab > fu);
}

int ora_gs_case(double e1, double f1, double e2, double f2, double ups)
{
    if (gs_exceeds(e1, f1, e2, f2, ups, DBL_MAX_EXP - 1)) return 1;
    if (gs_exceeds(e2, f2, e1, f1, ups, DBL_MAX_EXP - 1)) return 2;
    return 0;
}

/* eq. (GS) as Alg. zgsscl / dgsscl order it: x' = 2^-ex x and y' = 2^-ey y
 * exactly (barring underflow), then per component
 *   Re y'' = fma(-Re psi, Re x', fma(Im psi, Im x', Re y')),
 *   Im y'' = fma(-Re psi, Im x', fma(-Im psi, Re x', Im y')),
 * i.e. y' - psi x', and y <- 2^ey y''.  psi = w fl(fy/fx), one product per
 * part. */
double ora_gs(int l, const double *xr, const double *xi, double *yr, double *yi,
              double ex, double fx, double ey, double fy, double wr, double wi)
{
    const double fyx = fy / fx;
    const double psr = wr * fyx, psi = wi * fyx;
    const int Ex = (int)ex, Ey = (int)ey;
    double M = 0.0;
    for (int i = 0; i < l; ++i) {
        const double xpr = scalbn(xr[i], -Ex), ypr = scalbn(yr[i], -Ey);
        if (yi) {
            const double xpi = scalbn(xi[i], -Ex), ypi = scalbn(yi[i], -Ey);
            const double nr = scalbn(fma(-psr, xpr, fma(psi, xpi, ypr)), Ey);
            const double ni = scalbn(fma(-psr, xpi, fma(-psi, xpr, ypi)), Ey);
            yr[i] = nr;
            yi[i] = ni;
            M = fmax(M, fmax(fabs(nr), fabs(ni)));
        } else {
            const double nr = scalbn(fma(-psr, xpr, ypr), Ey);
            yr[i] = nr;
            M = fmax(M, fabs(nr));
        }
    }
    return M;
}

/* ------------------------------------------------------------------ */
/* the driver                                                          */
/* ------------------------------------------------------------------ */

#define COLR(st, j) ((st)->Gr + (size_t)(j) * (st)->ldg)
#define COLI(st, j) ((st)->cplx ? (st)->Gi + (size_t)(j) * (st)->ldg : NULL)
#define VCOLR(st, j) ((st)->Vr + (size_t)(j) * (st)->ldv)
#define VCOLI(st, j) ((st)->cplx ? (st)->Vi + (size_t)(j) * (st)->ldv : NULL)

int ora_init(ora_svd *st)
{
    const int m = st->m, n = st->n;
    if (n < 1 || m < n || st->ldg < (size_t)m || st->ldv < (size_t)n || !st->Gr || !st->Vr ||
        !st->e || !st->f || (st->cplx && (!st->Gi || !st->Vi)))
        return ORA_EINVAL;
    /* M~_0: max-norm with NaN turned into infinity (Sect. 3.2) */
    double M = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            M = fmax(M, fmin(fabs(COLR(st, j)[i]), INFINITY));
            if (st->cplx) M = fmax(M, fmin(fabs(COLI(st, j)[i]), INFINITY));
        }
    if (M == INFINITY) return ORA_ENONFINITE;
    if (M == 0.0) return ORA_EZERO;
    /* s_0 = s_[0] and G_1 = 2^{s_0} G_0, M~_1 = 2^{s_0} M~_0 */
    const int s0 = ora_s_square(M, m, st->cplx);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            COLR(st, j)[i] = scalbn(COLR(st, j)[i], s0);
            if (st->cplx) COLI(st, j)[i] = scalbn(COLI(st, j)[i], s0);
        }
    st->Mt = scalbn(M, s0);
    st->s = s0;
    /* V_1 = I */
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            VCOLR(st, j)[i] = (i == j) ? 1.0 : 0.0;
            if (st->cplx) VCOLI(st, j)[i] = 0.0;
        }
    for (int j = 0; j < n; ++j) {
        st->e[j] = -INFINITY;
        st->f[j] = 1.0;
    }
    st->k = 0;
    st->T = 0;
    st->last_t = 0;
    st->GS = 0;
    st->last_gs = 0;
    st->rescaled = 0;
    return ORA_OK;
}

/* Threads of ora_step's loops over the pairs of a step (1: sequential, the
 * default).  The pairs of a step are disjoint and the step's counts and its
 * max-norm are an integer sum and an exact max, so the result does not
 * depend on the thread count. */
static int g_step_threads = 1;

/* The oracle's exact mode (ora_exact.c): the iteration takes its column
 * norms and scaled dot-products from binary128 sums rounded once, instead
 * of the ordered 1024-lane sums (it supersedes the compensated
 * dot-product).  Off by default; the GPU path reproduces the ordered mode. */
static int g_exact = 0;
void ora_set_exact(int on) { g_exact = on != 0; }
int ora_get_exact(void) { return g_exact; }

static void norm_of(int m, const double *xr, const double *xi, double *e, double *f)
{
    if (g_exact)
        ora_colnorm_exact(m, xr, xi, e, f);
    else
        ora_colnorm(m, xr, xi, e, f);
}

void ora_set_step_threads(int nthreads) { g_step_threads = nthreads > 1 ? nthreads : 1; }

void ora_step(ora_svd *st)
{
    const int m = st->m, n = st->n, cplx = st->cplx;
    const int N = n + (n & 1), npairs = N / 2;
    const long kk = st->k;

    /* step-start rescaling check, Sect. 3.2 heuristic, second item */
    if (ora_s_round(st->Mt, cplx) < 0) {
        const int sp = ora_s_square(st->Mt, m, cplx);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                COLR(st, j)[i] = scalbn(COLR(st, j)[i], sp);
                if (cplx) COLI(st, j)[i] = scalbn(COLI(st, j)[i], sp);
            }
        st->Mt = scalbn(st->Mt, sp);
        st->s += sp;
        st->rescaled++;
    }

    /* column norms of every column taking part in this step */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(g_step_threads) if (g_step_threads > 1)
#endif
    for (int l = 0; l < npairs; ++l) {
        int p, q;
        if (!ora_rr_pair(n, kk, l, &p, &q)) continue;
        norm_of(m, COLR(st, p), COLI(st, p), &st->e[p], &st->f[p]);
        norm_of(m, COLR(st, q), COLI(st, q), &st->e[q], &st->f[q]);
    }

    /* tolerance upsilon = fl(eps sqrt m), eps = 2^-53 (eq. tol) */
    const double ups = scalbn(sqrt((double)m), -53);
    long t = 0, sw = 0, gs = 0;
    double M = 0.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(g_step_threads) if (g_step_threads > 1) \
    reduction(+ : t, sw, gs) reduction(max : M)
#endif
    for (int l = 0; l < npairs; ++l) {
        int p, q;
        if (!ora_rr_pair(n, kk, l, &p, &q)) continue;
        const double ep = st->e[p], fp = st->f[p], eq = st->e[q], fq = st->f[q];
        int transform = 0, pbit, gsc = 0;
        double c = 1.0, C = 0.0, S = 0.0, zr = 0.0, zi = 0.0;
        if (isinf(ep) || isinf(eq)) {
            /* a zero column: never rotated; the zero column goes last */
            pbit = isinf(ep) && !isinf(eq);
        } else {
            if (g_exact)
                ora_dpscl_exact(m, COLR(st, q), COLI(st, q), COLR(st, p), COLI(st, p), eq, fq, ep, fp, &zr, &zi);
            else if (st->comp)
                ora_dpscl_cs(m, COLR(st, q), COLI(st, q), COLR(st, p), COLI(st, p), eq, fq, ep, fp, &zr, &zi);
            else
                ora_dpscl(m, COLR(st, q), COLI(st, q), COLR(st, p), COLI(st, p), eq, fq, ep, fp, &zr, &zi);
            const double az = cplx ? ora_hypot(zr, zi) : fabs(zr);
            transform = (ups <= az);
            double a11, a22, a21r, a21i;
            ora_gram(zr, zi, ep, fp, eq, fq, &a11, &a22, &a21r, &a21i);
            double l1, l2;
            int zp;
            if (cplx)
                zp = ora_evd2_cplx(a11, a22, a21r, a21i, &c, &C, &S, &l1, &l2, ORA_EVD_SCALED);
            else
                zp = ora_evd2_real(a11, a22, a21r, &c, &C, &l1, &l2, ORA_EVD_SCALED);
            pbit = zp & 1;
            /* a pair to be transformed whose norms differ by more than
             * 2^eta_hat upsilon is orthogonalised by Gram-Schmidt instead
             * (Alg. zvjsvd, eq. GScond); the larger column stays in place
             * (first), so the permutation is the transposition exactly when
             * the larger one is g_q */
            if (transform && !st->nogs) {
                gsc = ora_gs_case(ep, fp, eq, fq, ups);
                if (gsc) pbit = (gsc == 2);
            }
        }
        if (st->nosort) pbit = 0;
        if (transform && gsc) {
            ++t;
            ++gs;
            double Mg;
            if (gsc == 1)   /* g_q <- g_q - conj(a21') (f_q/f_p) ... , eq. (GS) */
                Mg = ora_gs(m, COLR(st, p), COLI(st, p), COLR(st, q), COLI(st, q), ep, fp, eq, fq, zr, -zi);
            else            /* g_p <- g_p - a21' (f_p/f_q) ..., roles reversed */
                Mg = ora_gs(m, COLR(st, q), COLI(st, q), COLR(st, p), COLI(st, p), eq, fq, ep, fp, zr, zi);
            if (pbit) ora_swap(m, COLR(st, p), COLI(st, p), COLR(st, q), COLI(st, q));
            /* Gram-Schmidt replaces the rotation of G only: V still takes the
             * Jacobi rotation of the pair (Alg. zvjsvd applies zjrotf to V
             * either way), which agrees with the Gram-Schmidt update of V to
             * first order and keeps V unitary */
            (void)ora_rot(n, VCOLR(st, p), VCOLI(st, p), VCOLR(st, q), VCOLI(st, q), c, C, S, pbit);
            M = fmax(M, Mg);
        } else if (transform) {
            ++t;
            const double Mg = ora_rot(m, COLR(st, p), COLI(st, p), COLR(st, q), COLI(st, q), c, C, S, pbit);
            (void)ora_rot(n, VCOLR(st, p), VCOLI(st, p), VCOLR(st, q), VCOLI(st, q), c, C, S, pbit);
            M = fmax(M, Mg);
        } else if (pbit) {
            ++sw;
            ora_swap(m, COLR(st, p), COLI(st, p), COLR(st, q), COLI(st, q));
            ora_swap(n, VCOLR(st, p), VCOLI(st, p), VCOLR(st, q), VCOLI(st, q));
        }
        if (pbit) {
            double x = st->e[p]; st->e[p] = st->e[q]; st->e[q] = x;
            x = st->f[p]; st->f[p] = st->f[q]; st->f[q] = x;
        }
    }
    st->T += t;
    st->last_t = t;
    st->SW += sw;
    st->last_sw = sw;
    st->GS += gs;
    st->last_gs = gs;
    st->Mt = fmax(st->Mt, M);
    st->k++;
}

/* sigma_i before sigma_j in a descending order */
static int sv_greater(double ei, double fi, double ej, double fj)
{
    return ei > ej || (ei == ej && fi > fj);
}

void ora_finalize(ora_svd *st, double *sv_e, double *sv_f)
{
    const int m = st->m, n = st->n, cplx = st->cplx;
    double *e = (double *)malloc(sizeof(double) * (size_t)n);
    double *f = (double *)malloc(sizeof(double) * (size_t)n);
    int *pos = (int *)malloc(sizeof(int) * (size_t)n);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)m * (size_t)n * 2);
    double *tmpv = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n * 2);
    /* U = G diag(2^-e) / f, column by column (Sect. 4.2.1) */
    for (int j = 0; j < n; ++j) {
        norm_of(m, COLR(st, j), COLI(st, j), &e[j], &f[j]);
        const int zero = isinf(e[j]);
        const int E = zero ? 0 : (int)e[j];
        for (int i = 0; i < m; ++i) {
            COLR(st, j)[i] = zero ? 0.0 : scalbn(COLR(st, j)[i], -E) / f[j];
            if (cplx) COLI(st, j)[i] = zero ? 0.0 : scalbn(COLI(st, j)[i], -E) / f[j];
        }
        e[j] = e[j] - (double)st->s;
    }
    /* stable descending order: rank of column j */
    for (int j = 0; j < n; ++j) {
        int r = 0;
        for (int i = 0; i < n; ++i)
            if (sv_greater(e[i], f[i], e[j], f[j]) || (i < j && e[i] == e[j] && f[i] == f[j]))
                ++r;
        pos[j] = r;
    }
    for (int j = 0; j < n; ++j) {
        const int r = pos[j];
        memcpy(tmp + (size_t)r * m, COLR(st, j), sizeof(double) * (size_t)m);
        if (cplx) memcpy(tmp + ((size_t)n + r) * m, st->Gi + (size_t)j * st->ldg, sizeof(double) * (size_t)m);
        memcpy(tmpv + (size_t)r * n, VCOLR(st, j), sizeof(double) * (size_t)n);
        if (cplx) memcpy(tmpv + ((size_t)n + r) * n, st->Vi + (size_t)j * st->ldv, sizeof(double) * (size_t)n);
        sv_e[r] = e[j];
        sv_f[r] = f[j];
    }
    for (int j = 0; j < n; ++j) {
        memcpy(COLR(st, j), tmp + (size_t)j * m, sizeof(double) * (size_t)m);
        if (cplx) memcpy(st->Gi + (size_t)j * st->ldg, tmp + ((size_t)n + j) * m, sizeof(double) * (size_t)m);
        memcpy(VCOLR(st, j), tmpv + (size_t)j * n, sizeof(double) * (size_t)n);
        if (cplx) memcpy(st->Vi + (size_t)j * st->ldv, tmpv + ((size_t)n + j) * n, sizeof(double) * (size_t)n);
        st->e[j] = sv_e[j];
        st->f[j] = sv_f[j];
    }
    free(e); free(f); free(pos); free(tmp); free(tmpv);
}

int ora_gesvj(int m, int n, double *Gr, double *Gi, size_t ldg,
              double *Vr, double *Vi, size_t ldv,
              double *sv_e, double *sv_f, int max_sweeps, int *sweeps, long *steps,
              unsigned flags)
{
    ora_svd st;
    memset(&st, 0, sizeof(st));
    st.m = m; st.n = n; st.cplx = (Gi != NULL);
    st.Gr = Gr; st.Gi = Gi; st.ldg = ldg;
    st.Vr = Vr; st.Vi = Vi; st.ldv = ldv;
    st.nosort = (flags & ORA_PERMUTE) == 0;
    st.comp = (flags & ORA_COMPENSATED) != 0;
    st.nogs = (flags & ORA_NO_GS) != 0;
    if (n < 1 || m < n || !sv_e || !sv_f || max_sweeps < 1 ||
        (flags & ~(ORA_NO_PERMUTE | ORA_PERMUTE | ORA_COMPENSATED | ORA_NO_GS)) ||
        ((flags & ORA_PERMUTE) && (flags & ORA_NO_PERMUTE)))
        return ORA_EINVAL;
    st.e = (double *)malloc(sizeof(double) * (size_t)n);
    st.f = (double *)malloc(sizeof(double) * (size_t)n);
    int status = ora_init(&st);
    if (status != ORA_OK) {
        free(st.e); free(st.f);
        if (sweeps) *sweeps = 0;
        if (steps) *steps = 0;
        return status;
    }
    const int K = ora_rr_steps(n);
    int C;
    for (C = 0; C < max_sweeps; ++C) {
        st.T = 0;
        st.SW = 0;
        for (int kk = 0; kk < K; ++kk)
            ora_step(&st);
        if (st.T == 0 && st.SW == 0) break;
    }
    if (sweeps) *sweeps = C;
    if (steps) *steps = st.k;
    if (C < max_sweeps) {
        ora_finalize(&st, sv_e, sv_f);
        status = ORA_OK;
    } else {
        /* not converged: G stays the scaled iteration matrix; report its
         * current column norms, backscaled, in column order */
        for (int j = 0; j < n; ++j) {
            double e, f;
            norm_of(m, Gr + (size_t)j * ldg, Gi ? Gi + (size_t)j * ldg : NULL, &e, &f);
            sv_e[j] = e - (double)st.s;
            sv_f[j] = f;
        }
        status = ORA_NOT_CONVERGED;
    }
    free(st.e); free(st.f);
    return status;
}

/* ------------------------------------------------------------------ */
/* flat-argument entry points (for the test harness bindings)          */
/* ------------------------------------------------------------------ */

static void fill(ora_svd *st, int m, int n, double *Gr, double *Gi, size_t ldg,
                 double *Vr, double *Vi, size_t ldv, double *e, double *f)
{
    memset(st, 0, sizeof(*st));
    st->m = m; st->n = n; st->cplx = (Gi != NULL);
    st->Gr = Gr; st->Gi = Gi; st->ldg = ldg;
    st->Vr = Vr; st->Vi = Vi; st->ldv = ldv;
    st->e = e; st->f = f;
}

int ora_init_ext(int m, int n, double *Gr, double *Gi, size_t ldg,
                 double *Vr, double *Vi, size_t ldv, double *e, double *f,
                 int *s, double *Mt)
{
    ora_svd st;
    fill(&st, m, n, Gr, Gi, ldg, Vr, Vi, ldv, e, f);
    const int status = ora_init(&st);
    *s = st.s;
    *Mt = st.Mt;
    return status;
}

void ora_step_ext(int m, int n, double *Gr, double *Gi, size_t ldg,
                  double *Vr, double *Vi, size_t ldv, double *e, double *f,
                  int *s, double *Mt, long k, long *t, long *sw, long *gs, int *rescaled, unsigned flags)
{
    ora_svd st;
    fill(&st, m, n, Gr, Gi, ldg, Vr, Vi, ldv, e, f);
    st.s = *s;
    st.Mt = *Mt;
    st.k = k;
    st.nosort = (flags & ORA_PERMUTE) == 0;
    st.comp = (flags & ORA_COMPENSATED) != 0;
    st.nogs = (flags & ORA_NO_GS) != 0;
    ora_step(&st);
    *s = st.s;
    *Mt = st.Mt;
    *t = st.last_t;
    *sw = st.last_sw;
    *gs = st.last_gs;
    *rescaled = st.rescaled;
}

void ora_finalize_ext(int m, int n, double *Gr, double *Gi, size_t ldg,
                      double *Vr, double *Vi, size_t ldv, double *e, double *f,
                      int s, double *sv_e, double *sv_f)
{
    ora_svd st;
    fill(&st, m, n, Gr, Gi, ldg, Vr, Vi, ldv, e, f);
    st.s = s;
    ora_finalize(&st, sv_e, sv_f);
}
