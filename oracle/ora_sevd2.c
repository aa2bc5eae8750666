/*
 * ora_sevd2.c -- oracle for the single precision variant of the
 * branch-free, power-of-two-scaled EVD of a Hermitian (complex) or symmetric
 * (real) matrix of order two.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper converts its double precision routines to single precision by
 * redefining nu = FLT_MAX, fl(sqrt(nu)) = 1.844674297E+19, the smallest
 * subnormal FLT_TRUE_MIN and eta = FLT_MAX_EXP - 4 (Sect. 2.4.1).  The
 * equations are evaluated as in ora_evd2.c, every operation a single
 * precision IEEE-754 operation rounded to nearest-even (build with
 * -ffp-contract=off; on x86-64 float arithmetic is evaluated in float,
 * FLT_EVAL_METHOD = 0; every constant below is a float constant so nothing
 * is promoted).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"

#if FLT_EVAL_METHOD != 0
#error "the single precision oracle needs float arithmetic evaluated in float"
#endif

/* fl(sqrt(FLT_MAX)) = 0x1.fffffep+63, the bound on |tan(2 phi)| of eq. (tan2) */
static const float ORA_SQRT_NU_F = 1.844674297E+19f;

/* eq. (z) for one component: eta - floor(lg|c|), eta = floor(lg(FLT_MAX/8))
 * = FLT_MAX_EXP - 4, zero replaced by the smallest subnormal */
static int ora_s_zeta_part(float c)
{
    int e;
    (void)frexpf(fmaxf(fabsf(c), FLT_TRUE_MIN), &e);
    return (FLT_MAX_EXP - 4) - (e - 1);
}

/* eq. (z): the minimum over the k components */
static int ora_s_zeta(const float *comp, int k)
{
    int z = ora_s_zeta_part(comp[0]);
    for (int i = 1; i < k; ++i) {
        const int zi = ora_s_zeta_part(comp[i]);
        if (zi < z) z = zi;
    }
    return z;
}

/* eqs. (hypot), (zpolar) in single precision: x + iy = r (cos + i sin) */
static void ora_s_polar(float x, float y, float *r, float *cosv, float *sinv)
{
    const float m = fminf(fabsf(x), fabsf(y));
    const float M = fmaxf(fabsf(x), fabsf(y));
    const float q = fmaxf(m / M, 0.0f);
    *r = sqrtf(fmaf(q, q, 1.0f)) * M;
    *cosv = copysignf(fminf(fabsf(x) / *r, 1.0f), x);
    *sinv = y / fmaxf(*r, FLT_TRUE_MIN);
}

/* eqs. (tan2), (jactan), (jacsec) */
typedef struct {
    float tan_phi, sec2_phi, sec_phi, cos_phi;
} ora_s_jrot;

static ora_s_jrot ora_s_rotation(float two_abs21, float a)
{
    ora_s_jrot g;
    const float tan_2phi = copysignf(fminf(fmaxf(two_abs21 / fabsf(a), 0.0f), ORA_SQRT_NU_F), a);
    g.tan_phi = tan_2phi / (1.0f + sqrtf(fmaf(tan_2phi, tan_2phi, 1.0f)));
    g.sec2_phi = fmaf(g.tan_phi, g.tan_phi, 1.0f);
    g.sec_phi = sqrtf(g.sec2_phi);
    g.cos_phi = 1.0f / g.sec_phi;
    return g;
}

/* eq. (lamsec): ((y tan + o) tan + x) / sec^2 */
static float ora_s_lamsec(float x, float y, float o, const ora_s_jrot *g)
{
    return fmaf(g->tan_phi, fmaf(y, g->tan_phi, o), x) / g->sec2_phi;
}

static int ora_s_finish(float a11s, float a22s, float two_abs21, const ora_s_jrot *g, int zeta,
                        float *l1, float *l2, unsigned flags)
{
    const float lam1 = ora_s_lamsec(a11s, a22s, two_abs21, g);
    const float lam2 = ora_s_lamsec(a22s, a11s, -two_abs21, g);
    const int zeta_back = -zeta;
    const int scaled = (flags & ORA_EVD_SCALED) != 0;
    if (l1) *l1 = scaled ? lam1 : scalbnf(lam1, zeta_back);
    if (l2) *l2 = scaled ? lam2 : scalbnf(lam2, zeta_back);
    return (int)(((unsigned)zeta_back << 1) | (unsigned)(lam1 < lam2));
}

int ora_sevd2_cplx(float a11, float a22, float a21r, float a21i,
                   float *cs, float *ctr, float *cti, float *l1, float *l2, unsigned flags)
{
    const float comp[4] = {a11, a22, a21r, a21i};
    const int zeta = ora_s_zeta(comp, 4);
    const float a11s = scalbnf(a11, zeta), a22s = scalbnf(a22, zeta);
    float r, cos_alpha, sin_alpha;
    ora_s_polar(scalbnf(a21r, zeta), scalbnf(a21i, zeta), &r, &cos_alpha, &sin_alpha);
    const float two_abs21 = r * 2.0f;
    const ora_s_jrot g = ora_s_rotation(two_abs21, a11s - a22s);
    float re = cos_alpha * g.tan_phi, im = sin_alpha * g.tan_phi;
    if (flags & ORA_EVD_SINFORM) {
        re = re / g.sec_phi;
        im = im / g.sec_phi;
    }
    if (cs) *cs = g.cos_phi;
    if (ctr) *ctr = re;
    if (cti) *cti = im;
    return ora_s_finish(a11s, a22s, two_abs21, &g, zeta, l1, l2, flags);
}

int ora_sevd2_real(float a11, float a22, float a21,
                   float *cs, float *tn, float *l1, float *l2, unsigned flags)
{
    const float comp[3] = {a11, a22, a21};
    const int zeta = ora_s_zeta(comp, 3);
    const float a11s = scalbnf(a11, zeta), a22s = scalbnf(a22, zeta);
    const float a21s = scalbnf(a21, zeta);
    const float two_abs21 = fabsf(a21s) * 2.0f;
    const ora_s_jrot g = ora_s_rotation(two_abs21, a11s - a22s);
    /* e^{i alpha} = sign(a21) = +-1 (eq. alpha): an exact product */
    float v = g.tan_phi * copysignf(1.0f, a21s);
    if (flags & ORA_EVD_SINFORM)
        v = v / g.sec_phi;
    if (cs) *cs = g.cos_phi;
    if (tn) *tn = v;
    return ora_s_finish(a11s, a22s, two_abs21, &g, zeta, l1, l2, flags);
}

void ora_sevd2_batch(size_t r, const float *a11, const float *a22,
                     const float *a21r, const float *a21i,
                     float *cs, float *ctr, float *cti,
                     float *l1, float *l2, int32_t *zp,
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
        float c, C, S = 0.0f, L1, L2;
        int z;
        if (a21i)
            z = ora_sevd2_cplx(a11[i], a22[i], a21r[i], a21i[i], &c, &C, &S, &L1, &L2, flags);
        else
            z = ora_sevd2_real(a11[i], a22[i], a21r[i], &c, &C, &L1, &L2, flags);
        if (cs) cs[i] = c;
        if (ctr) ctr[i] = C;
        if (cti && a21i) cti[i] = S;
        if (l1) l1[i] = L1;
        if (l2) l2[i] = L2;
        if (zp) zp[i] = z;
    }
}
