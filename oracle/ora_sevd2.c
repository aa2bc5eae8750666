/*
 * ora_sevd2.c -- oracle for the single precision variant of the
 * branch-free, power-of-two-scaled EVD of a Hermitian (complex) or symmetric
 * (real) matrix of order two.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper converts its double precision routines to single precision by
 * redefining nu = FLT_MAX, fl(sqrt(nu)) = 1.844674297E+19, the smallest
 * subnormal FLT_TRUE_MIN and eta = FLT_MAX_EXP - 4 (Sect. 2.4.1), so
 * eta' = eta + 1 = FLT_MAX_EXP - 3 = 125 in the frexp form of Listing 1.
 * The steps are those of ora_evd2.c, every one of them a single precision
 * IEEE-754 operation rounded to nearest-even (build with -ffp-contract=off;
 * on x86-64 float arithmetic is evaluated in float, FLT_EVAL_METHOD = 0;
 * every constant below is a float constant so nothing is promoted).
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

/* fl(sqrt(FLT_MAX)) = 0x1.fffffep+63 */
static const float ORA_SQRT_NU_F = 1.844674297E+19f;

/* zeta_c = eta' - (frexp exponent of max(|c|, FLT_TRUE_MIN)), eta' = 125 */
static int zeta_of_f(float c)
{
    int ex;
    (void)frexpf(fmaxf(fabsf(c), FLT_TRUE_MIN), &ex);
    return (FLT_MAX_EXP - 3) - ex;
}

static float flip_sign_by_f(float x, float s)
{
    uint32_t ux, us;
    memcpy(&ux, &x, 4);
    memcpy(&us, &s, 4);
    ux ^= (us & 0x80000000u);
    memcpy(&x, &ux, 4);
    return x;
}

int ora_sevd2_cplx(float a11, float a22, float a21r, float a21i,
                   float *cs, float *ctr, float *cti, float *l1, float *l2, unsigned flags)
{
    const int z11 = zeta_of_f(a11), z22 = zeta_of_f(a22);
    const int zr = zeta_of_f(a21r), zi = zeta_of_f(a21i);
    const int zR = (z11 <= z22) ? z11 : z22;
    const int zC = (zr <= zi) ? zr : zi;
    const int zeta = (zR <= zC) ? zR : zC;
    const int zeta_b = -zeta;

    const float br = scalbnf(a21r, zeta), bi = scalbnf(a21i, zeta);
    const float b11 = scalbnf(a11, zeta), b22 = scalbnf(a22, zeta);

    const float abr = fabsf(br), abi = fabsf(bi);
    const float am = fminf(abr, abi), aM = fmaxf(abr, abi);
    const float mM = fmaxf(am / aM, 0.0f);
    const float ab = sqrtf(fmaf(mM, mM, 1.0f)) * aM;
    const float ca = copysignf(fminf(abr / ab, 1.0f), br);
    const float sa = bi / fmaxf(ab, FLT_TRUE_MIN);

    const float o = ab * 2.0f;
    const float a = b11 - b22;
    const float t2 = copysignf(fminf(fmaxf(o / fabsf(a), 0.0f), ORA_SQRT_NU_F), a);
    const float t = t2 / (1.0f + sqrtf(fmaf(t2, t2, 1.0f)));
    const float sec2 = fmaf(t, t, 1.0f);
    const float sec = sqrtf(sec2);
    const float c = 1.0f / sec;
    float C = ca * t;
    float S = sa * t;
    if (flags & ORA_EVD_SINFORM) {
        C = C / sec;
        S = S / sec;
    }
    const float lp1 = fmaf(t, fmaf(b22, t, o), b11) / sec2;
    const float lp2 = fmaf(t, fmaf(b11, t, -o), b22) / sec2;

    if (cs) *cs = c;
    if (ctr) *ctr = C;
    if (cti) *cti = S;
    if (flags & ORA_EVD_SCALED) {
        if (l1) *l1 = lp1;
        if (l2) *l2 = lp2;
    } else {
        if (l1) *l1 = scalbnf(lp1, zeta_b);
        if (l2) *l2 = scalbnf(lp2, zeta_b);
    }
    return (int)(((unsigned)zeta_b << 1) | (unsigned)(lp1 < lp2));
}

int ora_sevd2_real(float a11, float a22, float a21,
                   float *cs, float *tn, float *l1, float *l2, unsigned flags)
{
    const int z11 = zeta_of_f(a11), z22 = zeta_of_f(a22), z21 = zeta_of_f(a21);
    const int zR = (z11 <= z22) ? z11 : z22;
    const int zeta = (zR <= z21) ? zR : z21;
    const int zeta_b = -zeta;

    const float b21 = scalbnf(a21, zeta);
    const float b11 = scalbnf(a11, zeta), b22 = scalbnf(a22, zeta);

    const float ab = fabsf(b21);
    const float o = ab * 2.0f;
    const float a = b11 - b22;
    const float t2 = copysignf(fminf(fmaxf(o / fabsf(a), 0.0f), ORA_SQRT_NU_F), a);
    const float t = t2 / (1.0f + sqrtf(fmaf(t2, t2, 1.0f)));
    const float sec2 = fmaf(t, t, 1.0f);
    const float sec = sqrtf(sec2);
    const float c = 1.0f / sec;
    float T = flip_sign_by_f(t, b21);
    if (flags & ORA_EVD_SINFORM)
        T = T / sec;
    const float lp1 = fmaf(t, fmaf(b22, t, o), b11) / sec2;
    const float lp2 = fmaf(t, fmaf(b11, t, -o), b22) / sec2;

    if (cs) *cs = c;
    if (tn) *tn = T;
    if (flags & ORA_EVD_SCALED) {
        if (l1) *l1 = lp1;
        if (l2) *l2 = lp2;
    } else {
        if (l1) *l1 = scalbnf(lp1, zeta_b);
        if (l2) *l2 = scalbnf(lp2, zeta_b);
    }
    return (int)(((unsigned)zeta_b << 1) | (unsigned)(lp1 < lp2));
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
