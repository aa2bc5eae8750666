/*
 * ora_ssvd.c -- oracle for the single precision variant of the parallel
 * one-sided Jacobi SVD of arXiv:2202.08361 (Sect. SM8: the same method with
 * the datatype's range; Sect. 2.4.1 for the EVD constants).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The steps are those of ora_svd.c carried out in IEEE single arithmetic
 * (every constant a float constant, FLT_EVAL_METHOD = 0, -ffp-contract=off):
 *   nu = FLT_MAX, eps = 2^-24, upsilon = fl(sqrt(m)) 2^-24 (eq. tol);
 *   s_(k) = floor(lg(nu/2)) - floor(lg M~) = 126 - floor(lg M~) (real) and
 *           floor(lg(nu/(4 sqrt 2))) - floor(lg M~) - 1 = 124 - floor(lg M~)
 *           (complex), eq. (skr);
 *   s_[k] = floor(lg(nu/(varsigma m))) - floor(lg M~) - 1, eq. (skn), the
 *           first term evaluated exactly from its definition;
 *   the Gram scaling s_A = min(FLT_MAX_EXP - 1 - max(e12, e21), 0).
 * The scaled dot-products are those of Alg. zdpscl (the compensated variant
 * is offered in double precision only).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#if FLT_EVAL_METHOD != 0
#error "the single precision oracle needs float arithmetic evaluated in float"
#endif

float ora_s_hypot(float x, float y)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
    const float q = fmaxf(mn / mx, 0.0f);
    return sqrtf(fmaf(q, q, 1.0f)) * mx;
}

/* floor(lg(nu / (varsigma m))) of eq. (skn) for nu = FLT_MAX = 2^104 (2^24 - 1),
 * evaluated as its definition: the largest integer k with 2^k varsigma m <= nu,
 * compared in exact 128-bit integer arithmetic (real: 2^k 2 m <= nu; complex,
 * varsigma = 4 sqrt 2: (2^k 4 m)^2 2 <= nu^2).  (The closed form 126 -
 * floor(lg m) of the real case is exact only for m < 2^24: nu has 24
 * significant bits.) */
static int s_fits(int k, int m, int cplx)
{
    typedef unsigned __int128 u128;
    const u128 nu24 = (u128)((1u << 24) - 1);            /* nu = nu24 2^104 */
    if (!cplx) {
        /* 2m 2^k <= nu24 2^104 */
        const u128 lhs = (u128)(2ULL * (unsigned long long)m);
        if (k >= 104) return (lhs << (k - 104)) <= nu24;
        return lhs <= (nu24 << (104 - k));
    }
    /* 32 m^2 2^(2k) <= nu24^2 2^208 */
    const u128 lhs = (u128)32 * (u128)m * (u128)m;
    const int t = 2 * k - 208;
    if (t >= 0) return (lhs << t) <= nu24 * nu24;
    return lhs <= ((nu24 * nu24) << (-t));
}

int ora_s_lg_bound_m(int m, int cplx)
{
    int k = 128;
    while (!s_fits(k, m, cplx)) --k;
    return k;
}

int ora_s_s_round(float Mt, int cplx) { return (cplx ? 124 : 126) - ilogbf(Mt); }

int ora_s_s_square(float Mt, int m, int cplx) { return ora_s_lg_bound_m(m, cplx) - ilogbf(Mt) - 1; }

/* the 1024-lane accumulation of ora_svd.c, in float */
static int lanes_used_f(int m)
{
    int P = 1;
    while (P < m && P < ORA_LANES) P *= 2;
    return P;
}

static float lanes_reduce_f(float *a, int P)
{
    for (int h = P / 2; h >= 1; h /= 2)
        for (int j = 0; j < h; ++j)
            a[j] = a[j] + a[j + h];
    return a[0];
}

/* Frobenius norm in (e, f) form, as ora_colnorm: prescale by 2^-E,
 * E = floor(lg max|x_i|), fma sums of squares per lane, sqrt, naive hypot of
 * the real and imaginary norms for complex data. */
void ora_s_colnorm(int m, const float *xr, const float *xi, float *e, float *f)
{
    float ar[ORA_LANES], ai[ORA_LANES];
    float mx = 0.0f;
    for (int i = 0; i < m; ++i) {
        mx = fmaxf(mx, fabsf(xr[i]));
        if (xi) mx = fmaxf(mx, fabsf(xi[i]));
    }
    if (mx == 0.0f) {
        *e = -INFINITY;
        *f = 1.0f;
        return;
    }
    const int E = ilogbf(mx);
    const int P = lanes_used_f(m);
    memset(ar, 0, sizeof(float) * (size_t)P);
    memset(ai, 0, sizeof(float) * (size_t)P);
    for (int i = 0; i < m; ++i) {
        const int L = i % ORA_LANES;
        const float yr = scalbnf(xr[i], -E);
        ar[L] = fmaf(yr, yr, ar[L]);
        if (xi) {
            const float yi = scalbnf(xi[i], -E);
            ai[L] = fmaf(yi, yi, ai[L]);
        }
    }
    const float sr = lanes_reduce_f(ar, P);
    float r;
    if (xi) {
        const float si = lanes_reduce_f(ai, P);
        r = ora_s_hypot(sqrtf(sr), sqrtf(si));
    } else {
        r = sqrtf(sr);
    }
    const int er = ilogbf(r);
    *e = (float)(E + er);
    *f = scalbnf(r, -er);
}

/* Alg. zdpscl in float (the order of ora_dpscl). */
void ora_s_dpscl(int m, const float *qr, const float *qi, const float *pr, const float *pi,
                 float eq, float fq, float ep, float fp, float *zr, float *zi)
{
    float ar[ORA_LANES], ai[ORA_LANES];
    const int Eq = (int)eq, Ep = (int)ep;
    const int P = lanes_used_f(m);
    memset(ar, 0, sizeof(float) * (size_t)P);
    memset(ai, 0, sizeof(float) * (size_t)P);
    for (int i = 0; i < m; ++i) {
        const int L = i % ORA_LANES;
        const float gqr = scalbnf(qr[i], -Eq), gpr = scalbnf(pr[i], -Ep);
        if (qi) {
            const float gqi = scalbnf(qi[i], -Eq), gpi = scalbnf(pi[i], -Ep);
            ar[L] = fmaf(gqr, gpr, ar[L]);
            ai[L] = fmaf(gqr, gpi, ai[L]);
            ar[L] = fmaf(gqi, gpi, ar[L]);
            ai[L] = fmaf(-gqi, gpr, ai[L]);
        } else {
            ar[L] = fmaf(gqr, gpr, ar[L]);
        }
    }
    const float hr = lanes_reduce_f(ar, P);
    const float hi = qi ? lanes_reduce_f(ai, P) : 0.0f;
    const float d = fq * fp;
    *zr = hr / d;
    *zi = qi ? hi / d : 0.0f;
}

/* Alg. Gram in float: s_A = min(FLT_MAX_EXP - 1 - max(e12, e21), 0). */
void ora_s_gram(float zr, float zi, float e1, float f1, float e2, float f2,
                float *a11, float *a22, float *a21r, float *a21i)
{
    float f12 = f1 / f2;
    float f21 = f2 / f1;
    long e12 = (long)e1 - (long)e2;
    long e21 = (long)e2 - (long)e1;
    const int g12 = ilogbf(f12), g21 = ilogbf(f21);
    e12 += g12;
    f12 = scalbnf(f12, -g12);
    e21 += g21;
    f21 = scalbnf(f21, -g21);
    long sA = (FLT_MAX_EXP - 1) - (e12 > e21 ? e12 : e21);
    if (sA > 0) sA = 0;
    e12 += sA;
    e21 += sA;
    if (e12 < -1000) e12 = -1000;
    if (e21 < -1000) e21 = -1000;
    if (sA < -1000) sA = -1000;
    *a11 = scalbnf(f12, (int)e12);
    *a22 = scalbnf(f21, (int)e21);
    *a21r = scalbnf(zr, (int)sA);
    *a21i = scalbnf(zi, (int)sA);
}

/* Alg. zjrot / eq. (transf) with eq. (zfma), in float. */
float ora_s_rot(int l, float *xpr, float *xpi, float *xqr, float *xqi, float c, float C, float S, int swap)
{
    float M = 0.0f;
    for (int i = 0; i < l; ++i) {
        const float pr = xpr[i], qr = xqr[i];
        if (xpi) {
            const float pi = xpi[i], qi = xqi[i];
            const float npr = fmaf(qr, C, fmaf(-qi, S, pr)) * c;
            const float npi = fmaf(qr, S, fmaf(qi, C, pi)) * c;
            const float nqr = fmaf(pr, -C, fmaf(-pi, S, qr)) * c;
            const float nqi = fmaf(pr, S, fmaf(pi, -C, qi)) * c;
            if (swap) {
                xpr[i] = nqr; xpi[i] = nqi; xqr[i] = npr; xqi[i] = npi;
            } else {
                xpr[i] = npr; xpi[i] = npi; xqr[i] = nqr; xqi[i] = nqi;
            }
            M = fmaxf(M, fmaxf(fabsf(npr), fabsf(npi)));
            M = fmaxf(M, fmaxf(fabsf(nqr), fabsf(nqi)));
        } else {
            const float np = fmaf(qr, C, pr) * c;
            const float nq = fmaf(pr, -C, qr) * c;
            if (swap) {
                xpr[i] = nq; xqr[i] = np;
            } else {
                xpr[i] = np; xqr[i] = nq;
            }
            M = fmaxf(M, fmaxf(fabsf(np), fabsf(nq)));
        }
    }
    return M;
}

/* eq. (GScond) on the normalised quotient of the norms (eq. efpq), as
 * ora_gs_case, with eta_hat = FLT_MAX_EXP - 1 */
static int s_gs_exceeds(float ea, float fa, float eb, float fb, float ups)
{
    float fab = fa / fb;
    const int g = ilogbf(fab);
    const long eab = (long)ea - (long)eb + g;
    fab = scalbnf(fab, -g);
    const int eu = ilogbf(ups);
    const float fu = scalbnf(ups, -eu);
    const long et = (long)(FLT_MAX_EXP - 1) + eu;
    return eab > et || (eab == et && fab > fu);
}

int ora_s_gs_case(float e1, float f1, float e2, float f2, float ups)
{
    if (s_gs_exceeds(e1, f1, e2, f2, ups)) return 1;
    if (s_gs_exceeds(e2, f2, e1, f1, ups)) return 2;
    return 0;
}

/* eq. (GS) in float, in the order of ora_gs */
float ora_s_gs(int l, const float *xr, const float *xi, float *yr, float *yi,
               float ex, float fx, float ey, float fy, float wr, float wi)
{
    const float fyx = fy / fx;
    const float psr = wr * fyx, psi = wi * fyx;
    const int Ex = (int)ex, Ey = (int)ey;
    float M = 0.0f;
    for (int i = 0; i < l; ++i) {
        const float xpr = scalbnf(xr[i], -Ex), ypr = scalbnf(yr[i], -Ey);
        if (yi) {
            const float xpi = scalbnf(xi[i], -Ex), ypi = scalbnf(yi[i], -Ey);
            const float nr = scalbnf(fmaf(-psr, xpr, fmaf(psi, xpi, ypr)), Ey);
            const float ni = scalbnf(fmaf(-psr, xpi, fmaf(-psi, xpr, ypi)), Ey);
            yr[i] = nr;
            yi[i] = ni;
            M = fmaxf(M, fmaxf(fabsf(nr), fabsf(ni)));
        } else {
            const float nr = scalbnf(fmaf(-psr, xpr, ypr), Ey);
            yr[i] = nr;
            M = fmaxf(M, fabsf(nr));
        }
    }
    return M;
}

static void swap_f(int l, float *xpr, float *xpi, float *xqr, float *xqi)
{
    for (int i = 0; i < l; ++i) {
        float t = xpr[i]; xpr[i] = xqr[i]; xqr[i] = t;
        if (xpi) { t = xpi[i]; xpi[i] = xqi[i]; xqi[i] = t; }
    }
}

/* ------------------------------------------------------------------ */
/* the driver                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    int m, n, cplx;
    float *Gr, *Gi; size_t ldg;
    float *Vr, *Vi; size_t ldv;
    float *e, *f;
    int s;
    float Mt;
    long k, T, last_t, SW, last_sw, GS, last_gs;
    int rescaled, nosort, nogs;
} ora_ssvd;

#define SCOLR(st, j) ((st)->Gr + (size_t)(j) * (st)->ldg)
#define SCOLI(st, j) ((st)->cplx ? (st)->Gi + (size_t)(j) * (st)->ldg : NULL)
#define SVCOLR(st, j) ((st)->Vr + (size_t)(j) * (st)->ldv)
#define SVCOLI(st, j) ((st)->cplx ? (st)->Vi + (size_t)(j) * (st)->ldv : NULL)

static int s_init(ora_ssvd *st)
{
    const int m = st->m, n = st->n;
    if (n < 1 || m < n || st->ldg < (size_t)m || st->ldv < (size_t)n)
        return ORA_EINVAL;
    float M = 0.0f;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            M = fmaxf(M, fminf(fabsf(SCOLR(st, j)[i]), INFINITY));
            if (st->cplx) M = fmaxf(M, fminf(fabsf(SCOLI(st, j)[i]), INFINITY));
        }
    if (M == INFINITY) return ORA_ENONFINITE;
    if (M == 0.0f) return ORA_EZERO;
    const int s0 = ora_s_s_square(M, m, st->cplx);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            SCOLR(st, j)[i] = scalbnf(SCOLR(st, j)[i], s0);
            if (st->cplx) SCOLI(st, j)[i] = scalbnf(SCOLI(st, j)[i], s0);
        }
    st->Mt = scalbnf(M, s0);
    st->s = s0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            SVCOLR(st, j)[i] = (i == j) ? 1.0f : 0.0f;
            if (st->cplx) SVCOLI(st, j)[i] = 0.0f;
        }
    for (int j = 0; j < n; ++j) {
        st->e[j] = -INFINITY;
        st->f[j] = 1.0f;
    }
    st->k = 0;
    st->T = 0;
    st->last_t = 0;
    st->rescaled = 0;
    return ORA_OK;
}

static void s_step(ora_ssvd *st)
{
    const int m = st->m, n = st->n, cplx = st->cplx;
    const int N = n + (n & 1), npairs = N / 2;
    const long kk = st->k;

    if (ora_s_s_round(st->Mt, cplx) < 0) {
        const int sp = ora_s_s_square(st->Mt, m, cplx);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                SCOLR(st, j)[i] = scalbnf(SCOLR(st, j)[i], sp);
                if (cplx) SCOLI(st, j)[i] = scalbnf(SCOLI(st, j)[i], sp);
            }
        st->Mt = scalbnf(st->Mt, sp);
        st->s += sp;
        st->rescaled++;
    }
    for (int l = 0; l < npairs; ++l) {
        int p, q;
        if (!ora_rr_pair(n, kk, l, &p, &q)) continue;
        ora_s_colnorm(m, SCOLR(st, p), SCOLI(st, p), &st->e[p], &st->f[p]);
        ora_s_colnorm(m, SCOLR(st, q), SCOLI(st, q), &st->e[q], &st->f[q]);
    }
    /* upsilon = fl(eps sqrt m), eps = 2^-24 */
    const float ups = scalbnf(sqrtf((float)m), -24);
    long t = 0, sw = 0, gs = 0;
    float M = 0.0f;
    for (int l = 0; l < npairs; ++l) {
        int p, q;
        if (!ora_rr_pair(n, kk, l, &p, &q)) continue;
        const float ep = st->e[p], fp = st->f[p], eq = st->e[q], fq = st->f[q];
        int transform = 0, pbit, gsc = 0;
        float c = 1.0f, C = 0.0f, S = 0.0f, zr = 0.0f, zi = 0.0f;
        if (isinf(ep) || isinf(eq)) {
            pbit = isinf(ep) && !isinf(eq);
        } else {
            ora_s_dpscl(m, SCOLR(st, q), SCOLI(st, q), SCOLR(st, p), SCOLI(st, p), eq, fq, ep, fp, &zr, &zi);
            const float az = cplx ? ora_s_hypot(zr, zi) : fabsf(zr);
            transform = (ups <= az);
            float a11, a22, a21r, a21i, l1, l2;
            ora_s_gram(zr, zi, ep, fp, eq, fq, &a11, &a22, &a21r, &a21i);
            int zp;
            if (cplx)
                zp = ora_sevd2_cplx(a11, a22, a21r, a21i, &c, &C, &S, &l1, &l2, ORA_EVD_SCALED);
            else
                zp = ora_sevd2_real(a11, a22, a21r, &c, &C, &l1, &l2, ORA_EVD_SCALED);
            pbit = zp & 1;
            if (transform && !st->nogs) {
                gsc = ora_s_gs_case(ep, fp, eq, fq, ups);
                if (gsc) pbit = (gsc == 2);
            }
        }
        if (st->nosort) pbit = 0;
        if (transform && gsc) {
            ++t;
            ++gs;
            float Mg;
            if (gsc == 1)
                Mg = ora_s_gs(m, SCOLR(st, p), SCOLI(st, p), SCOLR(st, q), SCOLI(st, q), ep, fp, eq, fq, zr, -zi);
            else
                Mg = ora_s_gs(m, SCOLR(st, q), SCOLI(st, q), SCOLR(st, p), SCOLI(st, p), eq, fq, ep, fp, zr, zi);
            if (pbit) swap_f(m, SCOLR(st, p), SCOLI(st, p), SCOLR(st, q), SCOLI(st, q));
            (void)ora_s_rot(n, SVCOLR(st, p), SVCOLI(st, p), SVCOLR(st, q), SVCOLI(st, q), c, C, S, pbit);
            M = fmaxf(M, Mg);
        } else if (transform) {
            ++t;
            const float Mg = ora_s_rot(m, SCOLR(st, p), SCOLI(st, p), SCOLR(st, q), SCOLI(st, q), c, C, S, pbit);
            (void)ora_s_rot(n, SVCOLR(st, p), SVCOLI(st, p), SVCOLR(st, q), SVCOLI(st, q), c, C, S, pbit);
            M = fmaxf(M, Mg);
        } else if (pbit) {
            ++sw;
            swap_f(m, SCOLR(st, p), SCOLI(st, p), SCOLR(st, q), SCOLI(st, q));
            swap_f(n, SVCOLR(st, p), SVCOLI(st, p), SVCOLR(st, q), SVCOLI(st, q));
        }
        if (pbit) {
            float x = st->e[p]; st->e[p] = st->e[q]; st->e[q] = x;
            x = st->f[p]; st->f[p] = st->f[q]; st->f[q] = x;
        }
    }
    st->T += t;
    st->last_t = t;
    st->SW += sw;
    st->last_sw = sw;
    st->GS += gs;
    st->last_gs = gs;
    st->Mt = fmaxf(st->Mt, M);
    st->k++;
}

static int sv_greater_f(float ei, float fi, float ej, float fj)
{
    return ei > ej || (ei == ej && fi > fj);
}

static void s_finalize(ora_ssvd *st, float *sv_e, float *sv_f)
{
    const int m = st->m, n = st->n, cplx = st->cplx;
    float *e = (float *)malloc(sizeof(float) * (size_t)n);
    float *f = (float *)malloc(sizeof(float) * (size_t)n);
    int *pos = (int *)malloc(sizeof(int) * (size_t)n);
    float *tmp = (float *)malloc(sizeof(float) * (size_t)m * (size_t)n * 2);
    float *tmpv = (float *)malloc(sizeof(float) * (size_t)n * (size_t)n * 2);
    for (int j = 0; j < n; ++j) {
        ora_s_colnorm(m, SCOLR(st, j), SCOLI(st, j), &e[j], &f[j]);
        const int zero = isinf(e[j]);
        const int E = zero ? 0 : (int)e[j];
        for (int i = 0; i < m; ++i) {
            SCOLR(st, j)[i] = zero ? 0.0f : scalbnf(SCOLR(st, j)[i], -E) / f[j];
            if (cplx) SCOLI(st, j)[i] = zero ? 0.0f : scalbnf(SCOLI(st, j)[i], -E) / f[j];
        }
        e[j] = e[j] - (float)st->s;
    }
    for (int j = 0; j < n; ++j) {
        int r = 0;
        for (int i = 0; i < n; ++i)
            if (sv_greater_f(e[i], f[i], e[j], f[j]) || (i < j && e[i] == e[j] && f[i] == f[j]))
                ++r;
        pos[j] = r;
    }
    for (int j = 0; j < n; ++j) {
        const int r = pos[j];
        memcpy(tmp + (size_t)r * m, SCOLR(st, j), sizeof(float) * (size_t)m);
        if (cplx) memcpy(tmp + ((size_t)n + r) * m, st->Gi + (size_t)j * st->ldg, sizeof(float) * (size_t)m);
        memcpy(tmpv + (size_t)r * n, SVCOLR(st, j), sizeof(float) * (size_t)n);
        if (cplx) memcpy(tmpv + ((size_t)n + r) * n, st->Vi + (size_t)j * st->ldv, sizeof(float) * (size_t)n);
        sv_e[r] = e[j];
        sv_f[r] = f[j];
    }
    for (int j = 0; j < n; ++j) {
        memcpy(SCOLR(st, j), tmp + (size_t)j * m, sizeof(float) * (size_t)m);
        if (cplx) memcpy(st->Gi + (size_t)j * st->ldg, tmp + ((size_t)n + j) * m, sizeof(float) * (size_t)m);
        memcpy(SVCOLR(st, j), tmpv + (size_t)j * n, sizeof(float) * (size_t)n);
        if (cplx) memcpy(st->Vi + (size_t)j * st->ldv, tmpv + ((size_t)n + j) * n, sizeof(float) * (size_t)n);
        st->e[j] = sv_e[j];
        st->f[j] = sv_f[j];
    }
    free(e); free(f); free(pos); free(tmp); free(tmpv);
}

int ora_sgesvj(int m, int n, float *Gr, float *Gi, size_t ldg, float *Vr, float *Vi, size_t ldv,
               float *sv_e, float *sv_f, int max_sweeps, int *sweeps, long *steps, unsigned flags)
{
    ora_ssvd st;
    memset(&st, 0, sizeof(st));
    st.m = m; st.n = n; st.cplx = (Gi != NULL);
    st.Gr = Gr; st.Gi = Gi; st.ldg = ldg;
    st.Vr = Vr; st.Vi = Vi; st.ldv = ldv;
    st.nosort = (flags & ORA_PERMUTE) == 0;
    st.nogs = (flags & ORA_NO_GS) != 0;
    if (n < 1 || m < n || !sv_e || !sv_f || max_sweeps < 1 ||
        (flags & ~(ORA_NO_PERMUTE | ORA_PERMUTE | ORA_NO_GS)) ||
        ((flags & ORA_PERMUTE) && (flags & ORA_NO_PERMUTE)))
        return ORA_EINVAL;
    st.e = (float *)malloc(sizeof(float) * (size_t)n);
    st.f = (float *)malloc(sizeof(float) * (size_t)n);
    int status = s_init(&st);
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
            s_step(&st);
        if (st.T == 0 && st.SW == 0) break;
    }
    if (sweeps) *sweeps = C;
    if (steps) *steps = st.k;
    if (C < max_sweeps) {
        s_finalize(&st, sv_e, sv_f);
        status = ORA_OK;
    } else {
        for (int j = 0; j < n; ++j) {
            float e, f;
            ora_s_colnorm(m, Gr + (size_t)j * ldg, Gi ? Gi + (size_t)j * ldg : NULL, &e, &f);
            sv_e[j] = e - (float)st.s;
            sv_f[j] = f;
        }
        status = ORA_NOT_CONVERGED;
    }
    free(st.e); free(st.f);
    return status;
}

/* flat-argument entry points for the step-by-step test harness */
static void s_fill(ora_ssvd *st, int m, int n, float *Gr, float *Gi, size_t ldg, float *Vr, float *Vi, size_t ldv,
                   float *e, float *f)
{
    memset(st, 0, sizeof(*st));
    st->m = m; st->n = n; st->cplx = (Gi != NULL);
    st->Gr = Gr; st->Gi = Gi; st->ldg = ldg;
    st->Vr = Vr; st->Vi = Vi; st->ldv = ldv;
    st->e = e; st->f = f;
}

int ora_s_init_ext(int m, int n, float *Gr, float *Gi, size_t ldg, float *Vr, float *Vi, size_t ldv,
                   float *e, float *f, int *s, float *Mt)
{
    ora_ssvd st;
    s_fill(&st, m, n, Gr, Gi, ldg, Vr, Vi, ldv, e, f);
    const int status = s_init(&st);
    *s = st.s;
    *Mt = st.Mt;
    return status;
}

void ora_s_step_ext(int m, int n, float *Gr, float *Gi, size_t ldg, float *Vr, float *Vi, size_t ldv,
                    float *e, float *f, int *s, float *Mt, long k, long *t, long *sw, long *gs, int *rescaled,
                    unsigned flags)
{
    ora_ssvd st;
    s_fill(&st, m, n, Gr, Gi, ldg, Vr, Vi, ldv, e, f);
    st.s = *s;
    st.Mt = *Mt;
    st.k = k;
    st.nosort = (flags & ORA_PERMUTE) == 0;
    st.nogs = (flags & ORA_NO_GS) != 0;
    s_step(&st);
    *s = st.s;
    *Mt = st.Mt;
    *t = st.last_t;
    *sw = st.last_sw;
    *gs = st.last_gs;
    *rescaled = st.rescaled;
}
