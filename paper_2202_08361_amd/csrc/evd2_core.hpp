// evd2_core.hpp -- device core of the branch-free, power-of-two-scaled
// eigendecomposition of a Hermitian / real symmetric 2x2 matrix
// (arXiv:2202.08361, Sect. 2).
//
// The decomposition is assembled from the paper's equations, one helper
// each:
//   headroom / scaling exponent   eq. (z)  (exponents via frexp, zero taken
//                                           as the smallest subnormal)
//   polar form of a21             eqs. (hypot), (zpolar), (alpha)
//   the rotation                  eqs. (tan2), (jactan), (jacsec)
//   scaled eigenvalues            eq. (lamsec)
// The real case is the complex one with e^{i alpha} = sign(a21) (eq. alpha).
//
// One lane computes one matrix (the paper's SIMD lane becomes a wavefront
// lane).  Every expression is a single IEEE-754 operation rounded to
// nearest-even: the translation unit is compiled with -ffp-contract=off,
// fma() is written out where an equation has one, and '/' and sqrt() are
// the correctly rounded gfx950 expansions.  Each result is therefore the
// bit pattern the equations define, on any IEEE-754 machine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jsvd {

// x * 2^e, correctly rounded (v_ldexp_f64)
__device__ __forceinline__ double scal2(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }

// Range constants and primitives of one working precision (Sect. 2.4.1: a
// single precision routine redefines nu, fl(sqrt nu), the smallest subnormal
// and eta).  eta_frexp = eta + 1 because frexp's exponent of x is
// floor(lg x) + 1.
template <typename T>
struct EvdFp;

template <>
struct EvdFp<double> {
    static constexpr int eta_frexp = 1021;   // floor(lg(DBL_MAX / 8)) + 1
    __device__ static double sqrt_nu() { return 1.34078079299425956e+154; }   // 0x1.fffffffffffffp+511
    __device__ static double true_min() { return 4.9406564584124654e-324; }
    __device__ static int frexp_exp(double x) { return __builtin_amdgcn_frexp_exp(x); }
    __device__ static double scal2(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
    // x with its sign bit XOR-ed with that of s
    __device__ static double xorsign(double x, double s)
    {
        const uint64_t ux = __double_as_longlong(x), us = __double_as_longlong(s);
        return __longlong_as_double((long long)(ux ^ (us & 0x8000000000000000ull)));
    }
};

template <>
struct EvdFp<float> {
    static constexpr int eta_frexp = 125;    // floor(lg(FLT_MAX / 8)) + 1
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
    T C, S;        // e^{i alpha} tan(phi) (or e^{i alpha} sin(phi))
    T l1, l2;      // eigenvalues of the scaled matrix 2^zeta A
    int unscale;   // -zeta: lambda = 2^unscale lambda'
    int p;         // [lambda'_1 < lambda'_2]
};
using Evd2Out = Evd2OutT<double>;

// ---------------------------------------------------------------- eq. (z)
// How far one component may be scaled up by a power of two and still stay
// below nu/8: eta - floor(lg|c|), with lg 0 read as lg of the smallest
// subnormal (frexp gives no exponent for zero).
template <typename T>
__device__ __forceinline__ int headroom(T c)
{
    using F = EvdFp<T>;
    return F::eta_frexp - F::frexp_exp(fmax(fabs(c), F::true_min()));
}

// ---------------------------------------------------- eqs. (hypot), (zpolar)
// z = x + iy as |z| e^{i beta}: |z| by the naive hypot (the smaller magnitude
// over the larger one, 0/0 read as 0), cos(beta) clamped to 1 and carrying
// the sign of x, sin(beta) with |z| kept away from zero.
template <typename T>
struct PolarT {
    T r, cos_b, sin_b;
};

template <typename T>
__device__ __forceinline__ PolarT<T> polar_form(T x, T y)
{
    using F = EvdFp<T>;
    const T ax = fabs(x), ay = fabs(y);
    const T small = fmin(ax, ay), large = fmax(ax, ay);
    const T q = fmax(small / large, T(0));
    PolarT<T> z;
    z.r = sqrt(fma(q, q, T(1))) * large;
    z.cos_b = copysign(fmin(ax / z.r, T(1)), x);
    z.sin_b = y / fmax(z.r, F::true_min());
    return z;
}

// ------------------------------------------- eqs. (tan2), (jactan), (jacsec)
// The rotation of a scaled matrix from its doubled off-diagonal magnitude
// 2|a21| and its diagonal difference a11 - a22: tan(2 phi) clamped to
// fl(sqrt nu) with the sign of the difference, tan(phi), and the secant
// route to cos(phi).
template <typename T>
struct RotationT {
    T tan, sec2, sec, cos;
};

template <typename T>
__device__ __forceinline__ RotationT<T> rotation_of(T off2, T diff)
{
    using F = EvdFp<T>;
    const T tan2 = copysign(fmin(fmax(off2 / fabs(diff), T(0)), F::sqrt_nu()), diff);
    RotationT<T> g;
    g.tan = tan2 / (T(1) + sqrt(fma(tan2, tan2, T(1))));
    g.sec2 = fma(g.tan, g.tan, T(1));
    g.sec = sqrt(g.sec2);
    g.cos = T(1) / g.sec;
    return g;
}

// ------------------------------------------------------------ eq. (lamsec)
template <typename T>
__device__ __forceinline__ void eigenvalues_of(T d1, T d2, T off2, const RotationT<T> &g, Evd2OutT<T> &o)
{
    o.l1 = fma(g.tan, fma(d2, g.tan, off2), d1) / g.sec2;
    o.l2 = fma(g.tan, fma(d1, g.tan, -off2), d2) / g.sec2;
    o.p = (o.l1 < o.l2) ? 1 : 0;
}

// Hermitian [[a11, conj a21], [a21, a22]] in the precision of T.
template <bool SINFORM, typename T>
__device__ __forceinline__ Evd2OutT<T> evd2_cplx(T a11, T a22, T a21r, T a21i)
{
    using F = EvdFp<T>;
    int zeta = headroom(a11);
    zeta = min(zeta, headroom(a22));
    zeta = min(zeta, headroom(a21r));
    zeta = min(zeta, headroom(a21i));
    Evd2OutT<T> o;
    o.unscale = -zeta;
    const T d1 = F::scal2(a11, zeta), d2 = F::scal2(a22, zeta);
    const PolarT<T> w = polar_form(F::scal2(a21r, zeta), F::scal2(a21i, zeta));
    const T off2 = w.r * T(2);
    const RotationT<T> g = rotation_of(off2, d1 - d2);
    o.c = g.cos;
    o.C = w.cos_b * g.tan;
    o.S = w.sin_b * g.tan;
    if (SINFORM) {
        o.C = o.C / g.sec;
        o.S = o.S / g.sec;
    }
    eigenvalues_of(d1, d2, off2, g, o);
    return o;
}

// Real symmetric [[a11, a21], [a21, a22]]: e^{i alpha} = sign(a21), so the
// rotation's e^{i alpha} tan(phi) is tan(phi) with the sign of a21 applied.
template <bool SINFORM, typename T>
__device__ __forceinline__ Evd2OutT<T> evd2_real(T a11, T a22, T a21)
{
    using F = EvdFp<T>;
    int zeta = headroom(a11);
    zeta = min(zeta, headroom(a22));
    zeta = min(zeta, headroom(a21));
    Evd2OutT<T> o;
    o.unscale = -zeta;
    const T d1 = F::scal2(a11, zeta), d2 = F::scal2(a22, zeta);
    const T b21 = F::scal2(a21, zeta);
    const T off2 = fabs(b21) * T(2);
    const RotationT<T> g = rotation_of(off2, d1 - d2);
    o.c = g.cos;
    o.C = F::xorsign(g.tan, b21);
    if (SINFORM) o.C = o.C / g.sec;
    o.S = T(0);
    eigenvalues_of(d1, d2, off2, g, o);
    return o;
}

// the integer output of the stand-alone EVD: the unscaling exponent and the
// permutation bit in one word
__device__ __forceinline__ int32_t pack_zp(int unscale, int p)
{
    return (int32_t)(((uint32_t)unscale << 1) | (uint32_t)p);
}

} // namespace jsvd
