// evd2_core.hpp -- device core of the branch-free, power-of-two-scaled EVD of
// a Hermitian / real symmetric 2x2 matrix (arXiv:2202.08361, Sect. 2:
// eqs. (z), (zpolar), (hypot), (tan2), (jactan), (jacsec), (lamsec);
// Listing 1 for the complex case, Alg. d8jac2 for the real case).
//
// One lane computes one matrix (the paper's SIMD lane becomes a wavefront
// lane).  Every expression is a single IEEE-754 binary64 operation rounded
// to nearest-even: the translation unit is compiled with -ffp-contract=off,
// fma() is written out where the paper writes fma, and '/' and sqrt() are
// the correctly rounded gfx950 expansions.  The results are therefore the
// same bits as the serial algorithm on any IEEE-754 machine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jsvd {

// fl(sqrt(nu)) = 0x1.fffffffffffffp+511, the clamp of tan(2 phi) in eq. (tan2)
__device__ constexpr double kSqrtNu = 1.34078079299425956e+154;
// smallest positive subnormal (the paper's mu-check)
__device__ constexpr double kTrueMin = 4.9406564584124654e-324;

// 1 + floor(lg x) for finite x > 0 (subnormals included): the exponent
// returned by frexp().
__device__ __forceinline__ int frexp_exp(double x) { return __builtin_amdgcn_frexp_exp(x); }

// zeta_c = eta' - frexp_exp(max(|c|, mu)), eta' = DBL_MAX_EXP - 3 = 1021
__device__ __forceinline__ int zeta_of(double c) { return 1021 - frexp_exp(fmax(fabs(c), kTrueMin)); }

// x * 2^e, correctly rounded (v_ldexp_f64)
__device__ __forceinline__ double scal2(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }

// x with its sign bit XOR-ed with that of s
__device__ __forceinline__ double xorsign(double x, double s)
{
    const uint64_t ux = __double_as_longlong(x);
    const uint64_t us = __double_as_longlong(s);
    return __longlong_as_double((long long)(ux ^ (us & 0x8000000000000000ull)));
}

struct Evd2Out {
    double c;      // cos(phi)
    double C, S;   // e^{i alpha} tan(phi) (or sin(phi) form)
    double l1, l2; // lambda'_1, lambda'_2 (scaled by 2^zeta)
    int zeta_b;    // zeta' = -zeta
    int p;         // [lambda'_1 < lambda'_2]
};

// Complex Hermitian matrix [[a11, conj a21], [a21, a22]] (Listing 1 order).
template <bool SINFORM>
__device__ __forceinline__ Evd2Out evd2_cplx(double a11, double a22, double a21r, double a21i)
{
    Evd2Out o;
    // scaling exponent of eq. (z): minimum over the four components
    const int z11 = zeta_of(a11), z22 = zeta_of(a22);
    const int zr = zeta_of(a21r), zi = zeta_of(a21i);
    const int zR = min(z11, z22), zC = min(zr, zi);
    const int zeta = min(zR, zC);
    o.zeta_b = -zeta;
    const double br = scal2(a21r, zeta), bi = scal2(a21i, zeta);
    const double b11 = scal2(a11, zeta), b22 = scal2(a22, zeta);
    // polar form with the naive hypot, eqs. (zpolar), (hypot)
    const double abr = fabs(br), abi = fabs(bi);
    const double am = fmin(abr, abi), aM = fmax(abr, abi);
    const double mM = fmax(am / aM, 0.0);
    const double ab = sqrt(fma(mM, mM, 1.0)) * aM;
    const double ca = copysign(fmin(abr / ab, 1.0), br);
    const double sa = bi / fmax(ab, kTrueMin);
    // the Jacobi rotation, eqs. (tan2), (jactan), (jacsec)
    const double ov = ab * 2.0;
    const double a = b11 - b22;
    const double t2 = copysign(fmin(fmax(ov / fabs(a), 0.0), kSqrtNu), a);
    const double t = t2 / (1.0 + sqrt(fma(t2, t2, 1.0)));
    const double sec2 = fma(t, t, 1.0);
    const double sec = sqrt(sec2);
    o.c = 1.0 / sec;
    o.C = ca * t;
    o.S = sa * t;
    if (SINFORM) {
        o.C = o.C / sec;
        o.S = o.S / sec;
    }
    // eigenvalues of the scaled matrix, eq. (lamsec)
    o.l1 = fma(t, fma(b22, t, ov), b11) / sec2;
    o.l2 = fma(t, fma(b11, t, -ov), b22) / sec2;
    o.p = (o.l1 < o.l2) ? 1 : 0;
    return o;
}

// Real symmetric matrix [[a11, a21], [a21, a22]] (Alg. d8jac2 order).
template <bool SINFORM>
__device__ __forceinline__ Evd2Out evd2_real(double a11, double a22, double a21)
{
    Evd2Out o;
    const int z11 = zeta_of(a11), z22 = zeta_of(a22), z21 = zeta_of(a21);
    const int zeta = min(min(z11, z22), z21);
    o.zeta_b = -zeta;
    const double b21 = scal2(a21, zeta);
    const double b11 = scal2(a11, zeta), b22 = scal2(a22, zeta);
    const double ab = fabs(b21);
    const double ov = ab * 2.0;
    const double a = b11 - b22;
    const double t2 = copysign(fmin(fmax(ov / fabs(a), 0.0), kSqrtNu), a);
    const double t = t2 / (1.0 + sqrt(fma(t2, t2, 1.0)));
    const double sec2 = fma(t, t, 1.0);
    const double sec = sqrt(sec2);
    o.c = 1.0 / sec;
    // e^{i alpha} tan(phi) = sign(a21) tan(phi): the sign bits multiply
    o.C = xorsign(t, b21);
    if (SINFORM) o.C = o.C / sec;
    o.S = 0.0;
    o.l1 = fma(t, fma(b22, t, ov), b11) / sec2;
    o.l2 = fma(t, fma(b11, t, -ov), b22) / sec2;
    o.p = (o.l1 < o.l2) ? 1 : 0;
    return o;
}

__device__ __forceinline__ int32_t pack_zp(int zeta_b, int p)
{
    return (int32_t)(((uint32_t)zeta_b << 1) | (uint32_t)p);
}

} // namespace jsvd
