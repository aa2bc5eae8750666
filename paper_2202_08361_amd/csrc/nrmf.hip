// nrmf.hip -- batched non-overflowing Frobenius norms with a widened
// exponent range (arXiv:2202.08361, Sect. SM6, Alg. rnF) on gfx950.
//
// A value r > 0 is the pair (e, f), r = 2^e f, 1 <= f < 2, with e an integral
// double (so it may leave the exponent range of the data); zero is e = -inf.
// With s lanes (lane L takes the elements L, L + s, ... in order; complex data
// the real part, then the imaginary part of each element):
//   * per element, r <- fma(|x|, |x|, r) in (e, f) form (Sect. SM6.2): the
//     partial sum's exponent made even, the exponents of x^2 and r equalised
//     to their max, one fma of the scaled fractions, renormalisation;
//   * the s partial sums sorted by (e, f) (eq. vsort), then added pairwise,
//     lg s levels (eqs. 1red, redj);
//   * ||x|| = ((e - b)/2, fl(sqrt(2^b f))), b the lowest bit of e
//     (Sect. SM6.1).
// One workgroup of 256 threads per column.  Lane L belongs to thread L mod
// 256, so for s = 1024 every load of a wavefront covers 64 consecutive rows.
// The sort is a bitonic network over the positions p = t + 256 v: partners at
// distance j < 64 are in the same wavefront (shuffles), j = 64, 128 in
// another one (LDS), j >= 256 in the same thread (registers).  The sorted
// sequence is unique (equal keys are equal pairs), so it is that of any other
// sort.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>

#include "kernels.hpp"
#include "pair.hpp"

namespace jsvd {

namespace {

constexpr int kNT = 256;          // threads per column
constexpr int kMaxLanes = 1024;   // largest s

// getexp: floor(lg |x|), -inf for 0
__device__ __forceinline__ double E_of(double x) { return x == 0.0 ? -INFINITY : (double)getexp(x); }

// the fraction of |x| in [1, 2); 0 for 0
__device__ __forceinline__ double F_of(double x) { return x == 0.0 ? 0.0 : scal2(fabs(x), -getexp(x)); }

// x 2^y for an integral y or y = -inf (2^-inf = 0); exponents beyond +-4000
// give the same result as +-4000 for any double x
__device__ __forceinline__ double scalef(double x, double y)
{
    if (y == -INFINITY) return x * 0.0;
    const double yc = fmin(fmax(y, -4000.0), 4000.0);
    return scal2(x, (int)yc);
}

// the lowest bit of an integral exponent, 0 for -inf
__device__ __forceinline__ double low_bit(double e) { return isinf(e) ? 0.0 : (double)(((int)e) & 1); }

__device__ __forceinline__ void lane_update(double &e, double &f, double x)
{
    const double b = low_bit(e);
    const double e1 = e - b;
    const double f1 = scalef(f, b);
    const double ex = E_of(x), fx = F_of(x);
    const double eh = ex * 2.0;
    const double emax = fmax(eh, e1);
    const double dx = fmax(eh - emax, -INFINITY);   // -inf - (-inf) = NaN -> -inf
    const double dr = fmax(e1 - emax, -INFINITY);
    const double fh = scalef(fx, dx * 0.5);
    const double fr = scalef(f1, dr);
    const double fn = fma(fh, fh, fr);
    f = F_of(fn);
    e = emax + E_of(fn);
}

// (e, f) pairs during the sort: the integral exponent as an int (-inf as
// INT_MIN; exponents of double data stay within +-5000) and the fraction
struct Key {
    int e;
    double f;
};

__device__ __forceinline__ bool key_less(const Key &a, const Key &b) { return a.e < b.e || (a.e == b.e && a.f < b.f); }

__device__ __forceinline__ Key key_of(double e, double f)
{
    Key k;
    k.e = isinf(e) ? INT_MIN : (int)e;
    k.f = f;
    return k;
}

__device__ __forceinline__ double e_of(const Key &k) { return k.e == INT_MIN ? -INFINITY : (double)k.e; }

// the value a position of a bitonic stage keeps: of itself (a) and its
// partner (b), the smaller when (ascending block) == (lower position)
__device__ __forceinline__ Key bitonic_keep(const Key &a, const Key &b, bool asc, bool lower)
{
    const bool b_first = key_less(b, a);
    const bool take_min = asc == lower;
    const bool take_b = take_min == b_first;
    Key r;   // field by field, so the keys stay in registers
    r.e = take_b ? b.e : a.e;
    r.f = take_b ? b.f : a.f;
    return r;
}

__device__ __forceinline__ Key shfl_xor_key(const Key &k, int j)
{
    Key o;
    o.e = __shfl_xor(k.e, j, 64);
    o.f = __shfl_xor(k.f, j, 64);
    return o;
}

__device__ __forceinline__ Key shfl_down_key(const Key &k, int d)
{
    Key o;
    o.e = __shfl_down(k.e, d, 64);
    o.f = __shfl_down(k.f, d, 64);
    return o;
}

// (a, b) adjacent in sorted order, a <= b (eq. redj)
__device__ __forceinline__ Key red_add(const Key &a, const Key &b)
{
    const double ea = e_of(a), eb = e_of(b);
    const double fn = fma(scalef(1.0, fmax(ea - eb, -INFINITY)), a.f, b.f);
    return key_of(eb + E_of(fn), F_of(fn));
}

// bitonic stage with the partner in the same thread (position v ^ JV; used
// when s >= 512, so every thread holds nl = s / 256 > JV positions and
// positions >= nl, never read, may change freely)
template <int JV, int V>
__device__ __forceinline__ void bitonic_regs(Key (&key)[V], int t, int k, int j)
{
    Key nk[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int p = t + kNT * v;
        nk[v] = bitonic_keep(key[v], key[v ^ JV], (p & k) == 0, (p & j) == 0);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) key[v] = nk[v];
}

// reduction level with the partner in the same thread (position v + DV)
template <int DV, int V>
__device__ __forceinline__ void reduce_regs(Key (&key)[V], int nl)
{
#pragma unroll
    for (int v = 0; v + DV < V; ++v)
        if ((v % (2 * DV)) == 0 && v + DV < nl) key[v] = red_add(key[v], key[v + DV]);
}

// ---- the sort for s = 1024 with positions p = 4 t + v (thread t holds four
// consecutive positions): distances 1, 2 within the thread, 4, 8 to the
// neighbouring threads of a quad (DPP), 16 ... 64 within 32 lanes
// (ds_swizzle), 128 across the wavefront (bpermute), 256, 512 across
// wavefronts (LDS).
__device__ __forceinline__ int xlane(int x, int d)
{
    switch (d) {   // d = thread distance (xor), a constant after unrolling
    case 1: return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
    case 2: return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
    case 4: return __builtin_amdgcn_ds_swizzle(x, (4 << 10) | 0x1F);     // bit mode: lane xor 4
    case 8: return __builtin_amdgcn_ds_swizzle(x, (8 << 10) | 0x1F);
    case 16: return __builtin_amdgcn_ds_swizzle(x, (16 << 10) | 0x1F);
    default: return __shfl_xor(x, d, 64);
    }
}

__device__ __forceinline__ Key xlane_key(const Key &k, int d)
{
    Key o;
    o.e = xlane(k.e, d);
    const long long b = __double_as_longlong(k.f);
    const int lo = xlane((int)(unsigned)b, d);
    const int hi = xlane((int)(unsigned)(b >> 32), d);
    o.f = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    return o;
}

__device__ __forceinline__ void sort1024(Key (&key)[4], int t, int *se, double *sf)
{
#pragma unroll
    for (int k = 2; k <= 1024; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
            if (j < 4) {
                Key nk[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int p = 4 * t + v;
                    nk[v] = bitonic_keep(key[v], key[v ^ j], (p & k) == 0, (p & j) == 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) key[v] = nk[v];
            } else if (j < 256) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int p = 4 * t + v;
                    const Key b = xlane_key(key[v], j / 4);
                    key[v] = bitonic_keep(key[v], b, (p & k) == 0, (p & j) == 0);
                }
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    se[4 * t + v] = key[v].e;
                    sf[4 * t + v] = key[v].f;
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int p = 4 * t + v;
                    Key b;
                    b.e = se[p ^ j];
                    b.f = sf[p ^ j];
                    key[v] = bitonic_keep(key[v], b, (p & k) == 0, (p & j) == 0);
                }
                __syncthreads();
            }
        }
    }
}

// the reduction for s = 1024 on the positions p = 4 t + v
__device__ __forceinline__ void reduce1024(Key (&key)[4], int t, int *se, double *sf)
{
    key[0] = red_add(key[0], key[1]);
    key[2] = red_add(key[2], key[3]);
    key[0] = red_add(key[0], key[2]);
    // positions 4 t now hold the sums of their quads; threads t, t + dt
#pragma unroll
    for (int dt = 1; dt < 64; dt <<= 1) {
        const Key b = shfl_down_key(key[0], dt);
        if ((t % (2 * dt)) == 0) key[0] = red_add(key[0], b);
    }
    // the four wavefronts: thread 0 of wavefront w holds positions 256 w
    if ((t & 63) == 0) {
        se[t >> 6] = key[0].e;
        sf[t >> 6] = key[0].f;
    }
    __syncthreads();
    if (t == 0) {
        Key a[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            a[w].e = se[w];
            a[w].f = sf[w];
        }
        a[0] = red_add(a[0], a[1]);
        a[2] = red_add(a[2], a[3]);
        key[0] = red_add(a[0], a[2]);
    }
}

template <bool CPLX>
__global__ __launch_bounds__(kNT) void nrmf_kernel(int m, const double *Xr, const double *Xi, long long ld, int s,
                                                   double *e2o, double *f2o, double *eo, double *fo)
{
    __shared__ int se[kMaxLanes];
    __shared__ double sf[kMaxLanes];
    const int t = threadIdx.x;
    const int col = blockIdx.x;
    const double *xr = Xr + (size_t)col * ld;
    const double *xi = CPLX ? Xi + (size_t)col * ld : nullptr;
    constexpr int V = kMaxLanes / kNT;   // positions (lanes) per thread at most
    const int nl = s >= kNT ? s / kNT : (t < s ? 1 : 0);   // lanes of this thread
    double le[V], lf[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        le[v] = -INFINITY;
        lf[v] = 1.0;
    }
    // ---- lane partial sums; the next chain's elements are loaded while the
    // current ones are added
    const int chains = (m + s - 1) / s;
    double nr[V], ni[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int i = t + kNT * v;
        const bool in = v < nl && i < m;
        nr[v] = in ? xr[i] : 0.0;
        ni[v] = (CPLX && in) ? xi[i] : 0.0;
    }
    for (int c = 0; c < chains; ++c) {
        double cr[V], ci[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            cr[v] = nr[v];
            ci[v] = ni[v];
            const int i = (c + 1) * s + t + kNT * v;
            const bool in = v < nl && c + 1 < chains && i < m;
            nr[v] = in ? xr[i] : 0.0;
            ni[v] = (CPLX && in) ? xi[i] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (v < nl && c * s + t + kNT * v < m) {
                lane_update(le[v], lf[v], cr[v]);
                if (CPLX) lane_update(le[v], lf[v], ci[v]);
            }
        }
    }
    Key key[V];
#pragma unroll
    for (int v = 0; v < V; ++v) key[v] = key_of(le[v], lf[v]);
    if (s == kMaxLanes) {
        // the thread's four lane sums become the sort positions 4 t ... 4 t + 3
        sort1024(key, t, se, sf);
        reduce1024(key, t, se, sf);
    } else {
    // ---- bitonic sort of the s pairs, position p = t + 256 v
    for (int k = 2; k <= s; k <<= 1) {
        for (int j = k >> 1; j >= 1; j >>= 1) {
            if (j >= kNT) {
                // partner in this thread: v ^ (j / 256)
                if (j == kNT)
                    bitonic_regs<1>(key, t, k, j);
                else
                    bitonic_regs<2>(key, t, k, j);
            } else if (j >= 64) {
                // partner in another wavefront: through LDS
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (v < nl) {
                        se[t + kNT * v] = key[v].e;
                        sf[t + kNT * v] = key[v].f;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (v < nl) {
                        const int p = t + kNT * v;
                        Key b;
                        b.e = se[p ^ j];
                        b.f = sf[p ^ j];
                        key[v] = bitonic_keep(key[v], b, (p & k) == 0, (p & j) == 0);
                    }
                }
                __syncthreads();
            } else {
                // partner in this wavefront
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int p = t + kNT * v;
                    const Key b = shfl_xor_key(key[v], j);
                    if (v < nl) key[v] = bitonic_keep(key[v], b, (p & k) == 0, (p & j) == 0);
                }
            }
        }
    }
    // ---- pairwise reduction (eqs. 1red, redj) in strided form: at distance
    // d the position p (a multiple of 2d) takes p + d; the tree and the
    // operand order are those of the compacted levels
    for (int d = 1; d < s; d <<= 1) {
        if (d >= kNT) {
            // partner in this thread: v + d / 256 (positions p = 256 v, v a multiple of 2 d / 256)
            if (d == kNT)
                reduce_regs<1>(key, nl);
            else
                reduce_regs<2>(key, nl);
        } else if (d >= 64) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (v < nl) {
                    se[t + kNT * v] = key[v].e;
                    sf[t + kNT * v] = key[v].f;
                }
            }
            __syncthreads();
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int p = t + kNT * v;
                if (v < nl && (p % (2 * d)) == 0) {
                    Key b;
                    b.e = se[p + d];
                    b.f = sf[p + d];
                    key[v] = red_add(key[v], b);
                }
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int p = t + kNT * v;
                const Key b = shfl_down_key(key[v], d);
                if (v < nl && (p % (2 * d)) == 0) key[v] = red_add(key[v], b);
            }
        }
    }
    }
    if (t == 0) {
        const double e = e_of(key[0]);
        const double f = (e == -INFINITY) ? 1.0 : key[0].f;   // the norm of a zero array is (-inf, 1)
        if (e2o) e2o[col] = e;
        if (f2o) f2o[col] = f;
        if (!isinf(e) && low_bit(e) != 0.0) {
            eo[col] = (e - 1.0) * 0.5;
            fo[col] = sqrt(2.0 * f);
        } else {
            eo[col] = e * 0.5;
            fo[col] = sqrt(f);
        }
    }
}

} // namespace

hipError_t launch_nrmf(int ncols, int m, const double *Xr, const double *Xi, long long ld, int lanes, double *e2,
                       double *f2, double *e, double *f, hipStream_t s)
{
    if (ncols <= 0) return hipSuccess;
    if (lanes < 1 || lanes > kMaxLanes || (lanes & (lanes - 1))) return hipErrorInvalidValue;
    if (Xi)
        hipLaunchKernelGGL(nrmf_kernel<true>, dim3(ncols), dim3(kNT), 0, s, m, Xr, Xi, ld, lanes, e2, f2, e, f);
    else
        hipLaunchKernelGGL(nrmf_kernel<false>, dim3(ncols), dim3(kNT), 0, s, m, Xr, Xi, ld, lanes, e2, f2, e, f);
    return hipGetLastError();
}

} // namespace jsvd
