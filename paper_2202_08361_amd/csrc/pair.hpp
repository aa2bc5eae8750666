// pair.hpp -- device building blocks of one parallel one-sided Jacobi step
// for one pivot column pair (arXiv:2202.08361, Sects. 3-4).
//
// A group of W threads (W = 64 ... 1024, a power of two) owns one pivot pair
// (p, q).  Thread t keeps rows i = t + W j (j < R) of both columns in
// registers, so the pair is read from memory once and written once per step.
//
// Canonical summation order.  Every sum (sums of squares of the norms, the
// scaled dot-product) is the paper's vector accumulation (Alg. zdpscl) with a
// vector of S = 1024 lanes: lane L accumulates rows L, L+S, L+2S, ... in
// increasing order with fma, then the lanes are combined by the halving tree
// lane[L] += lane[L+h], h = S/2, ..., 1.  Row i = t + W j belongs to lane
// t + W (j mod S/W) at chain position j div (S/W), so every power-of-two W
// evaluates exactly the same expression tree: results are bit-identical for
// every launch shape and equal those of the sequential definition.  Lanes
// without rows hold +0, and a sum that starts at +0 and is only updated by
// fma or + never becomes -0, so adding them changes nothing and they are
// skipped.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "evd2_core.hpp"

namespace jsvd {

constexpr int kLanes = 1024;

__device__ __forceinline__ double bits2d(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long d2bits(double x) { return (unsigned long long)__double_as_longlong(x); }

// floor(lg |x|) for finite non-zero x (subnormals included)
__device__ __forceinline__ int getexp(double x) { return __builtin_amdgcn_frexp_exp(x) - 1; }
__device__ __forceinline__ int getexp(float x) { return __builtin_amdgcn_frexp_expf(x) - 1; }

// x * 2^e in single precision, correctly rounded (v_ldexp_f32)
__device__ __forceinline__ float scal2(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }

// Range constants of the SVD in the precision T (Sect. 3.2, eq. skr; Alg.
// Gram), from nu = DBL_MAX or FLT_MAX (the single precision routines redefine
// nu, Sect. 2.4.1):
//   round_real / round_cplx: floor(lg(nu/2)) and floor(lg(nu/(4 sqrt 2))) - 1,
//     so s_(k) = round - floor(lg M~);
//   gram_emax: the largest finite exponent, DBL_MAX_EXP - 1 or FLT_MAX_EXP - 1;
//   eps_exp: lg eps of the convergence tolerance upsilon = fl(sqrt m) eps.
template <typename T>
struct SvdFp;
template <>
struct SvdFp<double> {
    static constexpr int round_real = 1022, round_cplx = 1020, gram_emax = 1023, eps_exp = -53;
};
template <>
struct SvdFp<float> {
    static constexpr int round_real = 126, round_cplx = 124, gram_emax = 127, eps_exp = -24;
};

// Alg. hypot: M sqrt((m/M)^2 + 1), q = max(m/M, 0)
template <typename T>
__device__ __forceinline__ T hypot_naive(T x, T y)
{
    const T ax = fabs(x), ay = fabs(y);
    const T mn = fmin(ax, ay), mx = fmax(ax, ay);
    const T q = fmax(mn / mx, T(0));
    return sqrt(fma(q, q, T(1))) * mx;
}

// Round-robin pair l of step kk (circle method): N = n rounded up to even,
// K = N - 1; pair 0 is (N-1, kk), pair l > 0 is ((kk+l) mod K, (kk-l+K) mod K),
// ordered p < q.  Returns false when the pair holds the phantom column n of
// an odd n (then *p is the column sitting out).
__device__ __forceinline__ bool rr_pair(int n, long long kk, int l, int *p, int *q)
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
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
    *p = a;
    *q = b;
    return b < n;
}

// Workgroup barrier that orders LDS only: every wave first waits for its own
// LDS operations (lgkmcnt = 0), so LDS writes before the barrier are visible
// to LDS reads after it, while global loads and stores, including the
// asynchronous global->LDS prefetch, stay in flight.  (A fence-based barrier
// would also drain those, which stalls a pair on the prefetch of the next
// one.)  The empty asm statements keep the compiler from moving memory
// accesses across the barrier.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt not waited on
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// ---------------------------------------------------------------------------
// Cross-lane moves of the in-wave trees, on the VALU (no LDS round trip):
// lane i (i < h) receives lane i + h.  h = 32: v_permlane32_swap (the upper
// half of the wave into the lower one); h = 16: v_permlane16_swap (odd rows
// of 16 lanes into even ones); h <= 8: DPP row_shl within each row.  The
// other lanes receive values the trees do not use.
template <int H>
__device__ __forceinline__ unsigned lane_down_u32(unsigned v)
{
    if constexpr (H == 32) {
        return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
    } else if constexpr (H == 16) {
        return __builtin_amdgcn_permlane16_swap(v, v, false, false)[1];
    } else {
        static_assert(H >= 1 && H <= 8, "row shift");
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + H, 0xF, 0xF, false);
    }
}

template <int H, typename T>
__device__ __forceinline__ T lane_down(T x)
{
    if constexpr (sizeof(T) == 4) {
        return __uint_as_float(lane_down_u32<H>(__float_as_uint(x)));
    } else {
        const unsigned long long b = (unsigned long long)__double_as_longlong(x);
        const unsigned lo = lane_down_u32<H>((unsigned)b), hi = lane_down_u32<H>((unsigned)(b >> 32));
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
}

// lane 0's value in every lane (whatever the exec mask)
template <typename T>
__device__ __forceinline__ T lane0(T x)
{
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
    } else {
        const unsigned long long b = (unsigned long long)__double_as_longlong(x);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 0);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 0);
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
}

// In-wave halving tree: lane 0 ends with x_0 + x_1 + ... in the canonical
// order (lane i += lane i+h for h = 32, ..., 1); the total is broadcast to
// every lane.  VALU = false moves the lanes through the LDS crossbar
// (ds_bpermute) instead: the same sums, slower, but with fewer temporary
// registers, for kernels at the edge of their register budget.
template <bool VALU = true, typename T>
__device__ __forceinline__ T wave_tree_sum(T x)
{
    if constexpr (!VALU) {
#pragma unroll
        for (int h = 32; h >= 1; h >>= 1) x = x + __shfl_down(x, h, 64);
        return __shfl(x, 0, 64);
    }
    x = x + lane_down<32>(x);
    x = x + lane_down<16>(x);
    x = x + lane_down<8>(x);
    x = x + lane_down<4>(x);
    x = x + lane_down<2>(x);
    x = x + lane_down<1>(x);
    return lane0(x);
}

// The wave's maximum of non-negative values (exact, so any order), in every lane.
template <bool VALU = true, typename T>
__device__ __forceinline__ T wave_max(T x)
{
    if constexpr (!VALU) {
#pragma unroll
        for (int h = 32; h >= 1; h >>= 1) x = fmax(x, __shfl_xor(x, h, 64));
        return x;
    }
    x = fmax(x, lane_down<32>(x));
    x = fmax(x, lane_down<16>(x));
    x = fmax(x, lane_down<8>(x));
    x = fmax(x, lane_down<4>(x));
    x = fmax(x, lane_down<2>(x));
    x = fmax(x, lane_down<1>(x));
    return lane0(x);
}

// Group-wide canonical sum of NQ quantities (one value per thread each, the
// thread's in-thread tree already applied).  lds must hold NQ * W values and
// must not be reused by the caller until after the next workgroup barrier.
template <int W, int NQ, bool VALU = true, typename T>
__device__ __forceinline__ void group_tree_sum(T (&v)[NQ], T *lds)
{
    constexpr int NW = W / 64;
    if constexpr (NW == 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = wave_tree_sum<VALU>(v[q]);
    } else {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < NQ; ++q) lds[q * W + wv * 64 + lane] = v[q];
        lds_barrier();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            T x[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) x[w] = lds[q * W + w * 64 + lane];
            // thread index t = 64 w + lane: levels h >= 64 combine whole waves
#pragma unroll
            for (int h = NW / 2; h >= 1; h >>= 1)
#pragma unroll
                for (int w = 0; w < h; ++w) x[w] = x[w] + x[w + h];
            v[q] = wave_tree_sum<VALU>(x[0]);
        }
    }
}

// Group-wide max of NQ non-negative quantities (exact, order-free).
template <int W, int NQ, bool VALU = true, typename T>
__device__ __forceinline__ void group_max(T (&v)[NQ], T *lds)
{
    constexpr int NW = W / 64;
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = wave_max<VALU>(v[q]);
    if constexpr (NW > 1) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) lds[q * NW + wv] = v[q];
        }
        lds_barrier();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            T x = lds[q * NW];
#pragma unroll
            for (int w = 1; w < NW; ++w) x = fmax(x, lds[q * NW + w]);
            v[q] = x;
        }
    }
}

// The cross-lane method of the trees of a pair held at R rows per thread:
// the VALU moves where registers allow; from 16 rows per thread on (a
// column pair that fills most of the register file) the LDS permutes, whose
// fewer temporaries keep the kernel free of spills and at two workgroups
// per compute unit.
template <int R>
constexpr bool valu_trees() { return R < 16; }

// In-thread part of the canonical tree for a thread holding rows j < R:
// lane v = j mod V (V = S/W virtual lanes per thread), chain position
// j div V.  acc[v] for v < NL = min(R, V) is reduced by the halving tree over
// the V lanes; lanes >= NL are empty.
template <int W, int R>
struct LaneShape {
    static constexpr int V = kLanes / W;
    static constexpr int NL = (R < V) ? R : V;
    static constexpr int CH = (R + V - 1) / V;
};

template <int V, int NL, typename T>
__device__ __forceinline__ T thread_tree(T (&acc)[NL])
{
#pragma unroll
    for (int h = V / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int v = 0; v < h; ++v)
            if (v + h < NL) acc[v] = acc[v] + acc[v + h];
    return acc[0];
}

// ---------------------------------------------------------------------------
// Compensated summation (Sect. SM2.2): RD(a b), the product rounded toward
// -infinity (item G.), without touching the rounding mode of the wave.
// A product of magnitude >= 2^-960 has an exactly representable error
// a b - fl(a b), which one fma yields; then RD(a b) is fl(a b) when that
// error is >= 0 and the next double towards -infinity otherwise.  Smaller
// products, zeros and non-finite values take the exact slow path.
__device__ __noinline__ double mul_rd_slow(double a, double b, double p)
{
    if (p != p || a == 0.0 || b == 0.0 || __builtin_isinf(a) || __builtin_isinf(b)) return p;
    const bool neg = (a < 0.0) != (b < 0.0);
    if (__builtin_isinf(p)) return neg ? -INFINITY : 1.79769313486231570815e308;
    // |a b| < 2^-960: a b = (hi + lo) 2^E exactly, with a', b' in [1, 2)
    const int ea = getexp(a), eb = getexp(b);
    const double am = scal2(fabs(a), -ea), bm = scal2(fabs(b), -eb);
    const double hi = am * bm;
    const double lo = fma(am, bm, -hi);
    const int E = ea + eb;
    if (E + getexp(hi) >= -1022) {
        // normal result: fl(|a b|) = hi 2^E exactly; step down when the exact
        // value lies below the rounded one
        const double r = neg ? -scal2(hi, E) : scal2(hi, E);
        const bool down = neg ? (lo > 0.0) : (lo < 0.0);
        return down ? __longlong_as_double(__double_as_longlong(r) + (neg ? 1 : -1)) : r;
    }
    // subnormal result: the grid is 2^-1074, |a b| 2^1074 = (hi + lo) 2^S
    const int S = E + 1074;
    if (S < -2) return neg ? -4.9406564584124654e-324 : 0.0;   // 0 < |a b| < 2^-1074
    const double q = scal2(hi, S);    // exact, >= 1/4
    const double f = floor(q);
    const double fr = q - f;          // exact; when > 0 it exceeds |lo| 2^S
    if (!neg) return scal2((fr == 0.0 && lo < 0.0) ? f - 1.0 : f, -1074);
    return -scal2((fr > 0.0 || lo > 0.0) ? f + 1.0 : f, -1074);
}

// The next double below a normal p: p - |p| (2^-53 + 2^-105) rounded to
// nearest, one fma.  |p| times that factor lies strictly between half and
// one and a half of the spacing below p (also at powers of two, where that
// spacing halves), so the nearest double is the next one down.
__device__ __forceinline__ double next_down_normal(double p) { return fma(-fabs(p), 0x1p-53 + 0x1p-105, p); }

// RD(a b) by the fma test alone: exact when the product's magnitude is in
// [2^-960, max] or an operand is zero (the caller rules the rest out)
__device__ __forceinline__ double mul_rd_fast(double a, double b)
{
    const double p = a * b;
    const double e = fma(a, b, -p);
    return e < 0.0 ? next_down_normal(p) : p;
}

__device__ __forceinline__ double mul_rd(double a, double b)
{
    const double p = a * b;
    const double ap = fabs(p);
    if (ap >= 0x1p-960 && ap <= 1.79769313486231570815e308) {
        const double e = fma(a, b, -p);
        return e < 0.0 ? next_down_normal(p) : p;
    }
    return mul_rd_slow(a, b, p);
}

// a nonzero operand below 2^-480: only a product with such an operand can
// fall below 2^-960 (operands scaled by their columns' norm exponents stay
// below 4 in magnitude, so no product overflows)
__device__ __forceinline__ bool tiny_operand(double x) { return fabs(x) < 0x1p-480 && x != 0.0; }

// eq. (d2sum): s = fl(a + b), a + b = s + t exactly
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &t)
{
    const double s0 = a + b;
    double a1 = s0 - b;
    double b1 = s0 - a1;
    a1 = a - a1;
    b1 = b - b1;
    s = s0;
    t = a1 + b1;
}

// Kahan's summation with 2Sum of c = RD(x y) into (s, t) and of c' = x y - c
// into (s', t') (items G., M., K.)
__device__ __forceinline__ void cs_term(double x, double y, double &s, double &t, double &s2, double &t2)
{
    const double c = mul_rd(x, y);
    const double c2 = fma(x, y, -c);
    two_sum(s, c + t, s, t);
    two_sum(s2, c2 + t2, s2, t2);
}

__device__ __forceinline__ void cs_term_fast(double x, double y, double &s, double &t, double &s2, double &t2)
{
    const double c = mul_rd_fast(x, y);
    const double c2 = fma(x, y, -c);
    two_sum(s, c + t, s, t);
    two_sum(s2, c2 + t2, s2, t2);
}

// The compensated sums of one thread's NL lanes from its n rows in x
// (x[0..3][j]: Re g_p, Re g_q, Im g_p, Im g_q of the thread's row j, lane j
// mod V, in the row order of the lane), with the exact RD(x y): the rare
// pass for products outside the fma test's range.  Out of line and over
// memory, so that the register-resident first pass keeps its registers.
template <bool CPLX>
__device__ __noinline__ void cs_lanes_exact(const double *x, int n, int V, int NL, int ep, int eq, double *out)
{
    constexpr int NS = CPLX ? 2 : 1;
    for (int i = 0; i < NS * 4 * NL; ++i) out[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        const int v = j % V;
        double *a0 = out + v, *a1 = out + (NS - 1) * 4 * NL + v;
        const double gpr = scal2(x[j], -ep), gqr = scal2(x[n + j], -eq);
        cs_term(gpr, gqr, a0[0], a0[NL], a0[2 * NL], a0[3 * NL]);
        if (CPLX) {
            const double gpi = scal2(x[2 * n + j], -ep), gqi = scal2(x[3 * n + j], -eq);
            cs_term(gpi, gqi, a0[0], a0[NL], a0[2 * NL], a0[3 * NL]);
            cs_term(gqr, gpi, a1[0], a1[NL], a1[2 * NL], a1[3 * NL]);
            cs_term(-gqi, gpr, a1[0], a1[NL], a1[2 * NL], a1[3 * NL]);
        }
    }
}

// ---------------------------------------------------------------------------
// Column norm in (e, f) form (Sect. 3.2 and SM6.1): prescale by 2^-E with
// E = floor(lg max|x|), canonical sum of squares, sqrt, and for complex data
// the naive hypot of the real and imaginary norms.  Zero column: e = -inf.
template <typename T>
struct NormT {
    int zero;   // the column is zero
    int e;      // exponent (valid when !zero)
    T f;        // fraction in [1, 2)
};
using Norm = NormT<double>;

template <typename T>
__device__ __forceinline__ NormT<T> norm_from_sums(int E, T sr, T si, bool cplx)
{
    NormT<T> o;
    const T r = cplx ? hypot_naive(sqrt(sr), sqrt(si)) : sqrt(sr);
    const int er = getexp(r);
    o.zero = 0;
    o.e = E + er;
    o.f = scal2(r, -er);
    return o;
}

} // namespace jsvd

namespace jsvd {

// Alg. Gram (eqs. sGramEF, efpq, F): A'' = 2^{sA} [[|g_p|/|g_q|, .], [a21', |g_q|/|g_p|]],
// sA = min(DBL_MAX_EXP - 1 - max(e12, e21), 0) (FLT_MAX_EXP - 1 in single precision)
template <typename T>
__device__ __forceinline__ void gram_scaled(T zr, T zi, int e1, T f1, int e2, T f2, T *a11, T *a22, T *a21r,
                                            T *a21i)
{
    T f12 = f1 / f2;
    T f21 = f2 / f1;
    int e12 = e1 - e2, e21 = e2 - e1;
    const int g12 = getexp(f12), g21 = getexp(f21);
    e12 += g12;
    f12 = scal2(f12, -g12);
    e21 += g21;
    f21 = scal2(f21, -g21);
    const int sA = min(SvdFp<T>::gram_emax - max(e12, e21), 0);
    e12 += sA;
    e21 += sA;
    *a11 = scal2(f12, e12);
    *a22 = scal2(f21, e21);
    *a21r = scal2(zr, sA);
    *a21i = scal2(zi, sA);
}

// eq. (GScond) for norms ||g_a|| = 2^ea fa and ||g_b|| = 2^eb fb: is
// ||g_a|| > 2^eta_hat upsilon ||g_b||?  Decided on the normalised quotient of
// eq. (efpq), 2^{ea - eb + g} F(fl(fa/fb)) with g = getexp(fl(fa/fb)), against
// 2^{eta_hat} upsilon = 2^{eta_hat + eu} fu in (e, f) form (exact comparisons).
template <typename T>
__device__ __forceinline__ bool gs_exceeds(int ea, T fa, int eb, T fb, T ups)
{
    T q = fa / fb;
    const int g = getexp(q);
    const int eab = ea - eb + g;
    q = scal2(q, -g);
    const int eu = getexp(ups);
    const T fu = scal2(ups, -eu);
    const int et = SvdFp<T>::gram_emax + eu;
    return eab > et || (eab == et && q > fu);
}

// eq. (GS) on a register column pair (Alg. zgsscl / dgsscl order): column D
// <- (x_D 2^-eD - psi x_S 2^-eS) 2^eD with psi = (wr + i wi) fl(fD/fS),
// column S unchanged.  Per component, with x' = 2^-eS x_S, y' = 2^-eD x_D:
// Re = fma(-Re psi, Re x', fma(Im psi, Im x', Re y')), Im = fma(-Re psi,
// Im x', fma(-Im psi, Re x', Im y')).  Returns the thread's max-norm of the
// new column D.
template <bool CPLX, int R, int S, int D, typename T>
__device__ __forceinline__ T gs_regs(T (&xr)[2][R], T (&xi)[2][R], int eS, T fS, int eD, T fD, T wr, T wi)
{
    const T fds = fD / fS;
    const T pr = wr * fds, pi = wi * fds;
    T Mx = T(0);
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const T sr = scal2(xr[S][j], -eS), dr = scal2(xr[D][j], -eD);
        if (CPLX) {
            const T si = scal2(xi[S][j], -eS), di = scal2(xi[D][j], -eD);
            const T nr = scal2(fma(-pr, sr, fma(pi, si, dr)), eD);
            const T ni = scal2(fma(-pr, si, fma(-pi, sr, di)), eD);
            xr[D][j] = nr;
            xi[D][j] = ni;
            Mx = fmax(Mx, fmax(fabs(nr), fabs(ni)));
        } else {
            const T nr = scal2(fma(-pr, sr, dr), eD);
            xr[D][j] = nr;
            Mx = fmax(Mx, fabs(nr));
        }
    }
    return Mx;
}

// The scaled dot-product of the pair without its final division, \hat z =
// (g_q 2^-e_q)^* (g_p 2^-e_p), in the canonical lane order (h[0] = Re,
// h[1] = Im): Alg. zdpscl (fma per lane), or with COMP Alg. zdpsclcs /
// ddpsclcs (compensated per lane; the four sums of each real stream reduced
// one by one and added as ((s' + t') + t) + s).  The imaginary stream takes
// Re(g_q) Im(g_p), then (-Im(g_q)) Re(g_p), which is the stated result
// g_q^* g_p.  lds: (COMP ? 4 : 1) * (CPLX ? 2 : 1) * W values (W > 64).  The
// compensated variant is defined for double precision only.
template <bool CPLX, int W, int R, bool COMP, typename T>
__device__ __forceinline__ void pair_dot(const T (&xr)[2][R], const T (&xi)[2][R], int ep, int eq, T (&h)[2],
                                         T *lds)
{
    using LS = LaneShape<W, R>;
    constexpr int V = LS::V, NL = LS::NL, CH = LS::CH;
    static_assert(!COMP || sizeof(T) == sizeof(double), "compensated dot-products are double precision");
    if constexpr (!COMP) {
        T dr[NL], di[NL];
#pragma unroll
        for (int v = 0; v < NL; ++v) {
            dr[v] = T(0);
            di[v] = T(0);
        }
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
#pragma unroll
            for (int v = 0; v < NL; ++v) {
                const int j = ch * V + v;
                if (j < R) {
                    const T gqr = scal2(xr[1][j], -eq), gpr = scal2(xr[0][j], -ep);
                    if (CPLX) {
                        const T gqi = scal2(xi[1][j], -eq), gpi = scal2(xi[0][j], -ep);
                        dr[v] = fma(gqr, gpr, dr[v]);
                        di[v] = fma(gqr, gpi, di[v]);
                        dr[v] = fma(gqi, gpi, dr[v]);
                        di[v] = fma(-gqi, gpr, di[v]);
                    } else {
                        dr[v] = fma(gqr, gpr, dr[v]);
                    }
                }
            }
        constexpr int ND = CPLX ? 2 : 1;
        T g[ND];
        g[0] = thread_tree<V>(dr);
        if (CPLX) g[ND - 1] = thread_tree<V>(di);
        group_tree_sum<W, ND, valu_trees<R>()>(g, lds);
        h[0] = g[0];
        h[1] = CPLX ? g[ND - 1] : T(0);
    } else {
        // [stream][s, t, s', t'][lane]
        constexpr int NS = CPLX ? 2 : 1;
        double a[NS][4][NL];
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < NL; ++v) a[st][u][v] = 0.0;
        bool odd = false;
#pragma unroll
        for (int ch = 0; ch < CH; ++ch)
#pragma unroll
            for (int v = 0; v < NL; ++v) {
                const int j = ch * V + v;
                if (j < R) {
                    const double gpr = scal2(xr[0][j], -ep), gqr = scal2(xr[1][j], -eq);
                    odd |= tiny_operand(gpr) || tiny_operand(gqr);
                    cs_term_fast(gpr, gqr, a[0][0][v], a[0][1][v], a[0][2][v], a[0][3][v]);
                    if (CPLX) {
                        const double gpi = scal2(xi[0][j], -ep), gqi = scal2(xi[1][j], -eq);
                        odd |= tiny_operand(gpi) || tiny_operand(gqi);
                        cs_term_fast(gpi, gqi, a[0][0][v], a[0][1][v], a[0][2][v], a[0][3][v]);
                        cs_term_fast(gqr, gpi, a[NS - 1][0][v], a[NS - 1][1][v], a[NS - 1][2][v], a[NS - 1][3][v]);
                        cs_term_fast(-gqi, gpr, a[NS - 1][0][v], a[NS - 1][1][v], a[NS - 1][2][v], a[NS - 1][3][v]);
                    }
                }
            }
        if (odd) {
            // a product that may lie outside the fma test's range: this
            // thread's lanes again with the exact RD(x y), out of line
            double x[4 * R], out[NS * 4 * NL];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                x[j] = xr[0][j];
                x[R + j] = xr[1][j];
                x[2 * R + j] = CPLX ? xi[0][j] : 0.0;
                x[3 * R + j] = CPLX ? xi[1][j] : 0.0;
            }
            cs_lanes_exact<CPLX>(x, R, V, NL, ep, eq, out);
#pragma unroll
            for (int st = 0; st < NS; ++st)
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < NL; ++v) a[st][u][v] = out[(st * 4 + u) * NL + v];
        }
        double g[4 * NS];
#pragma unroll
        for (int st = 0; st < NS; ++st)
#pragma unroll
            for (int u = 0; u < 4; ++u) g[4 * st + u] = thread_tree<V>(a[st][u]);
        group_tree_sum<W, 4 * NS, valu_trees<R>()>(g, lds);
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            double z = g[4 * st + 2] + g[4 * st + 3];
            z = z + g[4 * st + 1];
            h[st] = z + g[4 * st + 0];
        }
        if (!CPLX) h[1] = 0.0;
    }
}

// Decision for one pivot pair held in registers by a group of W threads.
template <typename T>
struct PairDecisionT {
    NormT<T> np, nq;   // the column norms (e, f) before the transformation
    bool transform;
    int pbit;          // the permutation of the EVD (0 when ignored)
    int gs;            // 0: rotate; 1: Gram-Schmidt of g_q against g_p; 2: of g_p against g_q
    T c, C, S;
    T zr, zi;          // a21'
};
using PairDecision = PairDecisionT<double>;

// The decision for a pair from its norms (zero flags set) and, when neither
// column is zero, the scaled dot-product without its final division (h):
// a21' (Alg. zdpscl's division), the convergence test (Alg. cvg), the
// scaled Gram matrix (Alg. Gram), its EVD, and the Gram-Schmidt choice of
// eq. (GScond).  Every thread computes the same decision.
template <bool CPLX, typename T>
__device__ __forceinline__ PairDecisionT<T> pair_decide(const NormT<T> &np, const NormT<T> &nq, const T (&h)[2], T ups,
                                                       int nosort, int nogs)
{
    PairDecisionT<T> o;
    o.np = np;
    o.nq = nq;
    o.transform = false;
    o.gs = 0;
    o.c = T(1);
    o.C = T(0);
    o.S = T(0);
    o.zr = T(0);
    o.zi = T(0);
    if (np.zero || nq.zero) {
        // a zero column is never rotated; it goes after the other one
        o.pbit = (np.zero && !nq.zero) ? 1 : 0;
    } else {
        const T dd = o.nq.f * o.np.f;
        const T zr = h[0] / dd;
        const T zi = CPLX ? h[1] / dd : T(0);
        const T az = CPLX ? hypot_naive(zr, zi) : fabs(zr);
        o.transform = ups <= az;
        T a11, a22, a21r, a21i;
        gram_scaled(zr, zi, o.np.e, o.np.f, o.nq.e, o.nq.f, &a11, &a22, &a21r, &a21i);
        const Evd2OutT<T> e = CPLX ? evd2_cplx<false>(a11, a22, a21r, a21i) : evd2_real<false>(a11, a22, a21r);
        o.c = e.c;
        o.C = e.C;
        o.S = e.S;
        o.pbit = e.p;
        o.zr = zr;
        o.zi = zi;
        if (o.transform && !nogs) {
            if (gs_exceeds(o.np.e, o.np.f, o.nq.e, o.nq.f, ups))
                o.gs = 1;
            else if (gs_exceeds(o.nq.e, o.nq.f, o.np.e, o.np.f, ups))
                o.gs = 2;
            if (o.gs) o.pbit = (o.gs == 2) ? 1 : 0;
        }
    }
    if (nosort) o.pbit = 0;
    return o;
}

// Norms (Sect. 3.2), scaled dot-product (Alg. zdpscl, or zdpsclcs /
// ddpsclcs with COMP), convergence test (Alg. cvg), scaled Gram matrix
// (Alg. Gram) and 2x2 EVD (Listing 1) of the pair (xr/xi[0] = column p,
// [1] = column q; rows t + W j, zeros beyond m).  A pair to be transformed
// whose norms differ by more than 2^eta_hat upsilon is marked for the
// Gram-Schmidt replacement of eq. (GScond) unless nogs; its permutation is
// then the transposition exactly when g_q is the larger column.  Scratch:
// red_norm (4 W values), red_dot (2 W values, 8 W with COMP), mxs (2 W/64
// values); unused for W = 64.  Every thread returns the same decision.  All of
// it in the precision T, with that precision's constants.
template <bool CPLX, int W, int R, bool COMP = false, typename T>
__device__ __forceinline__ PairDecisionT<T> pair_core(const T (&xr)[2][R], const T (&xi)[2][R], T ups, int nosort,
                                                      int nogs, T *red_norm, T *red_dot, T *mxs)
{
    using LS = LaneShape<W, R>;
    constexpr int V = LS::V, NL = LS::NL, CH = LS::CH;
    T mx[2] = {T(0), T(0)};
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            mx[c] = fmax(mx[c], fabs(xr[c][j]));
            if (CPLX) mx[c] = fmax(mx[c], fabs(xi[c][j]));
        }
    group_max<W, 2, valu_trees<R>()>(mx, mxs);
    const bool zp_ = mx[0] == T(0), zq_ = mx[1] == T(0);
    const int Ep = zp_ ? 0 : getexp(mx[0]);
    const int Eq = zq_ ? 0 : getexp(mx[1]);
    constexpr int NQ = CPLX ? 4 : 2;
    T acc[NQ][NL];
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq)
#pragma unroll
        for (int v = 0; v < NL; ++v) acc[qq][v] = T(0);
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int v = 0; v < NL; ++v) {
            const int j = ch * V + v;
            if (j < R) {
                const T ypr = scal2(xr[0][j], -Ep), yqr = scal2(xr[1][j], -Eq);
                acc[0][v] = fma(ypr, ypr, acc[0][v]);
                acc[1][v] = fma(yqr, yqr, acc[1][v]);
                if (CPLX) {
                    const T ypi = scal2(xi[0][j], -Ep), yqi = scal2(xi[1][j], -Eq);
                    acc[2][v] = fma(ypi, ypi, acc[2][v]);
                    acc[3][v] = fma(yqi, yqi, acc[3][v]);
                }
            }
        }
    T s[NQ];
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) s[qq] = thread_tree<V>(acc[qq]);
    group_tree_sum<W, NQ, valu_trees<R>()>(s, red_norm);
    NormT<T> np = norm_from_sums(Ep, s[0], CPLX ? s[2] : T(0), CPLX);
    NormT<T> nq = norm_from_sums(Eq, s[1], CPLX ? s[3] : T(0), CPLX);
    np.zero = zp_;
    nq.zero = zq_;
    T h[2] = {T(0), T(0)};
    if (!zp_ && !zq_) pair_dot<CPLX, W, R, COMP>(xr, xi, np.e, nq.e, h, red_dot);
    return pair_decide<CPLX>(np, nq, h, ups, nosort, nogs);
}

// The transformation of a register pair that pair_core decided on: the
// rotation of Alg. zjrot or the Gram-Schmidt step of eq. (GS) (g_q against
// g_p with conj(a21'), or g_p against g_q with a21').  Returns the thread's
// max-norm of the changed column(s).
template <bool CPLX, int R, typename T>
__device__ __forceinline__ T transform_regs(T (&xr)[2][R], T (&xi)[2][R], const PairDecisionT<T> &dc);

// Rotation of a register pair (Alg. zjrot, eq. transf with the complex fma
// of eq. zfma): xr/xi[0] <- x_p', [1] <- x_q'; returns the thread's max-norm.
template <bool CPLX, int R, typename T>
__device__ __forceinline__ T rot_regs(T (&xr)[2][R], T (&xi)[2][R], T c, T C, T S)
{
    T Mx = T(0);
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const T pr = xr[0][j], qr = xr[1][j];
        if (CPLX) {
            const T pi = xi[0][j], qi = xi[1][j];
            xr[0][j] = fma(qr, C, fma(-qi, S, pr)) * c;
            xi[0][j] = fma(qr, S, fma(qi, C, pi)) * c;
            xr[1][j] = fma(pr, -C, fma(-pi, S, qr)) * c;
            xi[1][j] = fma(pr, S, fma(pi, -C, qi)) * c;
            Mx = fmax(Mx, fmax(fabs(xr[0][j]), fabs(xi[0][j])));
            Mx = fmax(Mx, fmax(fabs(xr[1][j]), fabs(xi[1][j])));
        } else {
            xr[0][j] = fma(qr, C, pr) * c;
            xr[1][j] = fma(pr, -C, qr) * c;
            Mx = fmax(Mx, fmax(fabs(xr[0][j]), fabs(xr[1][j])));
        }
    }
    return Mx;
}

template <bool CPLX, int R, typename T>
__device__ __forceinline__ T transform_regs(T (&xr)[2][R], T (&xi)[2][R], const PairDecisionT<T> &dc)
{
    if (dc.gs == 1)
        return gs_regs<CPLX, R, 0, 1>(xr, xi, dc.np.e, dc.np.f, dc.nq.e, dc.nq.f, dc.zr, -dc.zi);
    if (dc.gs == 2)
        return gs_regs<CPLX, R, 1, 0>(xr, xi, dc.nq.e, dc.nq.f, dc.np.e, dc.np.f, dc.zr, dc.zi);
    return rot_regs<CPLX, R>(xr, xi, dc.c, dc.C, dc.S);
}

} // namespace jsvd
