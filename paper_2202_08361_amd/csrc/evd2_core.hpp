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

// Precision-dependent constants and primitives of the EVD (Sect. 2.4.1: the
// single precision routines redefine nu = FLT_MAX, fl(sqrt nu), the smallest
// subnormal and eta; eta' = eta + 1 in the frexp form of Listing 1).
template <typename T>
struct EvdFp;

template <>
struct EvdFp<double> {
    static constexpr int eta1 = 1021;   // DBL_MAX_EXP - 3
    __device__ static double sqrt_nu() { return 1.34078079299425956e+154; }
    __device__ static double true_min() { return 4.9406564584124654e-324; }
    __device__ static int frexp_exp(double x) { return __builtin_amdgcn_frexp_exp(x); }
    __device__ static double scal2(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
    __device__ static double xorsign(double x, double s)
    {
        const uint64_t ux = __double_as_longlong(x), us = __double_as_longlong(s);
        return __longlong_as_double((long long)(ux ^ (us & 0x8000000000000000ull)));
    }
};

template <>
struct EvdFp<float> {
    static constexpr int eta1 = 125;    // FLT_MAX_EXP - 3
    __device__ static float sqrt_nu() { return 1.844674297e+19f; }   // 0x1.fffffep+63
    __device__ static float true_min() { return 1.40129846e-45f; }   // 2^-149
    __device__ static int frexp_exp(float x) { return __builtin_amdgcn_frexp_expf(x); }
    __device__ static float scal2(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }
    __device__ static float xorsign(float x, float s)
    {
        const uint32_t ux = __float_as_uint(x), us = __float_as_uint(s);
        return __uint_as_float(ux ^ (us & 0x80000000u));
    }
};

template <typename T>
struct Evd2OutT {
    T c;           // cos(phi)
    T C, S;        // e^{i alpha} tan(phi) (or sin(phi) form)
    T l1, l2;      // lambda'_1, lambda'_2 (scaled by 2^zeta)
    int zeta_b;    // zeta' = -zeta
    int p;         // [lambda'_1 < lambda'_2]
};
using Evd2Out = Evd2OutT<double>;

// zeta_c = eta' - frexp_exp(max(|c|, mu)) of eq. (z) in the frexp form
template <typename T>
__device__ __forceinline__ int zeta_of_t(T c)
{
    using F = EvdFp<T>;
    return F::eta1 - F::frexp_exp(fmax(fabs(c), F::true_min()));
}

// Complex Hermitian matrix [[a11, conj a21], [a21, a22]] (Listing 1 order),
// in the precision of T.
template <bool SINFORM, typename T>
__device__ __forceinline__ Evd2OutT<T> evd2_cplx(T a11, T a22, T a21r, T a21i)
{
    using F = EvdFp<T>;
    Evd2OutT<T> o;
    // scaling exponent of eq. (z): minimum over the four components
    const int z11 = zeta_of_t(a11), z22 = zeta_of_t(a22);
    const int zr = zeta_of_t(a21r), zi = zeta_of_t(a21i);
    const int zR = min(z11, z22), zC = min(zr, zi);
    const int zeta = min(zR, zC);
    o.zeta_b = -zeta;
    const T br = F::scal2(a21r, zeta), bi = F::scal2(a21i, zeta);
    const T b11 = F::scal2(a11, zeta), b22 = F::scal2(a22, zeta);
    // polar form with the naive hypot, eqs. (zpolar), (hypot)
    const T abr = fabs(br), abi = fabs(bi);
    const T am = fmin(abr, abi), aM = fmax(abr, abi);
    const T mM = fmax(am / aM, T(0));
    const T ab = sqrt(fma(mM, mM, T(1))) * aM;
    const T ca = copysign(fmin(abr / ab, T(1)), br);
    const T sa = bi / fmax(ab, F::true_min());
    // the Jacobi rotation, eqs. (tan2), (jactan), (jacsec)
    const T ov = ab * T(2);
    const T a = b11 - b22;
    const T t2 = copysign(fmin(fmax(ov / fabs(a), T(0)), F::sqrt_nu()), a);
    const T t = t2 / (T(1) + sqrt(fma(t2, t2, T(1))));
    const T sec2 = fma(t, t, T(1));
    const T sec = sqrt(sec2);
    o.c = T(1) / sec;
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
template <bool SINFORM, typename T>
__device__ __forceinline__ Evd2OutT<T> evd2_real(T a11, T a22, T a21)
{
    using F = EvdFp<T>;
    Evd2OutT<T> o;
    const int z11 = zeta_of_t(a11), z22 = zeta_of_t(a22), z21 = zeta_of_t(a21);
    const int zeta = min(min(z11, z22), z21);
    o.zeta_b = -zeta;
    const T b21 = F::scal2(a21, zeta);
    const T b11 = F::scal2(a11, zeta), b22 = F::scal2(a22, zeta);
    const T ab = fabs(b21);
    const T ov = ab * T(2);
    const T a = b11 - b22;
    const T t2 = copysign(fmin(fmax(ov / fabs(a), T(0)), F::sqrt_nu()), a);
    const T t = t2 / (T(1) + sqrt(fma(t2, t2, T(1))));
    const T sec2 = fma(t, t, T(1));
    const T sec = sqrt(sec2);
    o.c = T(1) / sec;
    // e^{i alpha} tan(phi) = sign(a21) tan(phi): the sign bits multiply
    o.C = F::xorsign(t, b21);
    if (SINFORM) o.C = o.C / sec;
    o.S = T(0);
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
