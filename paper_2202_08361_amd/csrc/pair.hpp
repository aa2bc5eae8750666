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

// Alg. hypot: M sqrt((m/M)^2 + 1), q = max(m/M, 0)
__device__ __forceinline__ double hypot_naive(double x, double y)
{
    const double ax = fabs(x), ay = fabs(y);
    const double mn = fmin(ax, ay), mx = fmax(ax, ay);
    const double q = fmax(mn / mx, 0.0);
    return sqrt(fma(q, q, 1.0)) * mx;
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

// ---------------------------------------------------------------------------
// In-wave halving tree: after the call lane 0 holds x_0 + x_1 + ... in the
// canonical order (lane i += lane i+h for h = 32, ..., 1); the total is
// broadcast to every lane.
__device__ __forceinline__ double wave_tree_sum(double x)
{
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) x = x + __shfl_down(x, h, 64);
    return __shfl(x, 0, 64);
}

__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) x = fmax(x, __shfl_xor(x, h, 64));
    return x;
}

// Group-wide canonical sum of NQ quantities (one value per thread each, the
// thread's in-thread tree already applied).  lds must hold NQ * W doubles and
// must not be reused by the caller until after the next __syncthreads().
template <int W, int NQ>
__device__ __forceinline__ void group_tree_sum(double (&v)[NQ], double *lds)
{
    constexpr int NW = W / 64;
    if constexpr (NW == 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = wave_tree_sum(v[q]);
    } else {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < NQ; ++q) lds[q * W + wv * 64 + lane] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double x[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) x[w] = lds[q * W + w * 64 + lane];
            // thread index t = 64 w + lane: levels h >= 64 combine whole waves
#pragma unroll
            for (int h = NW / 2; h >= 1; h >>= 1)
#pragma unroll
                for (int w = 0; w < h; ++w) x[w] = x[w] + x[w + h];
            v[q] = wave_tree_sum(x[0]);
        }
    }
}

// Group-wide max of NQ non-negative quantities (exact, order-free).
template <int W, int NQ>
__device__ __forceinline__ void group_max(double (&v)[NQ], double *lds)
{
    constexpr int NW = W / 64;
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = wave_max(v[q]);
    if constexpr (NW > 1) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) lds[q * NW + wv] = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double x = lds[q * NW];
#pragma unroll
            for (int w = 1; w < NW; ++w) x = fmax(x, lds[q * NW + w]);
            v[q] = x;
        }
    }
}

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

template <int V, int NL>
__device__ __forceinline__ double thread_tree(double (&acc)[NL])
{
#pragma unroll
    for (int h = V / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int v = 0; v < h; ++v)
            if (v + h < NL) acc[v] = acc[v] + acc[v + h];
    return acc[0];
}

// ---------------------------------------------------------------------------
// Column norm in (e, f) form (Sect. 3.2 and SM6.1): prescale by 2^-E with
// E = floor(lg max|x|), canonical sum of squares, sqrt, and for complex data
// the naive hypot of the real and imaginary norms.  Zero column: e = -inf.
struct Norm {
    int zero;   // the column is zero
    int e;      // exponent (valid when !zero)
    double f;   // fraction in [1, 2)
};

__device__ __forceinline__ Norm norm_from_sums(int E, double sr, double si, bool cplx)
{
    Norm o;
    const double r = cplx ? hypot_naive(sqrt(sr), sqrt(si)) : sqrt(sr);
    const int er = getexp(r);
    o.zero = 0;
    o.e = E + er;
    o.f = scal2(r, -er);
    return o;
}

} // namespace jsvd
