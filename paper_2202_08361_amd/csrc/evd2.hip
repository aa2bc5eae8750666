// evd2.hip -- batched EVD of Hermitian / real symmetric 2x2 matrices on
// gfx950 (arXiv:2202.08361, Sect. 2, Alg. zbjac2 / dbjac2; Sect. SM10 for the
// one-matrix-per-thread GPU mapping).
//
// Structure-of-arrays streams in, structure-of-arrays streams out: the
// kernel is bound by HBM bandwidth (60 B per real, 76 B per complex matrix).
// A batch larger than the caches runs one matrix per lane (8-byte accesses,
// the most lanes in flight: measured 9-10% faster than two per lane on
// MI355X); a smaller batch with 16-byte aligned streams runs two consecutive
// matrices per lane with 16-byte accesses (faster out of the caches).
// Streams are read and written once, with non-temporal hints so the batch
// does not evict other data from the caches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "evd2_core.hpp"
#include "kernels.hpp"

namespace jsvd {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef int i2v __attribute__((ext_vector_type(2)));

struct Evd2Args {
    size_t r;
    const double *a11, *a22, *ar, *ai;
    double *cs, *cr, *ci, *l1, *l2;
    int32_t *zp;
};

template <bool CPLX, bool SINFORM, bool SCALED>
__device__ __forceinline__ void evd2_one(const Evd2Args &A, size_t i)
{
    const double a11 = __builtin_nontemporal_load(A.a11 + i);
    const double a22 = __builtin_nontemporal_load(A.a22 + i);
    const double ar = __builtin_nontemporal_load(A.ar + i);
    Evd2Out o;
    if (CPLX) {
        const double ai = __builtin_nontemporal_load(A.ai + i);
        o = evd2_cplx<SINFORM>(a11, a22, ar, ai);
    } else {
        o = evd2_real<SINFORM>(a11, a22, ar);
    }
    __builtin_nontemporal_store(o.c, A.cs + i);
    __builtin_nontemporal_store(o.C, A.cr + i);
    if (CPLX) __builtin_nontemporal_store(o.S, A.ci + i);
    const double L1 = SCALED ? o.l1 : scal2(o.l1, o.unscale);
    const double L2 = SCALED ? o.l2 : scal2(o.l2, o.unscale);
    if (A.l1) __builtin_nontemporal_store(L1, A.l1 + i);
    if (A.l2) __builtin_nontemporal_store(L2, A.l2 + i);
    if (A.zp) __builtin_nontemporal_store(pack_zp(o.unscale, o.p), A.zp + i);
}

template <bool CPLX, bool SINFORM, bool SCALED>
__global__ __launch_bounds__(256) void evd2_kernel_v1(Evd2Args A)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < A.r) evd2_one<CPLX, SINFORM, SCALED>(A, i);
}

template <bool CPLX, bool SINFORM, bool SCALED>
__global__ __launch_bounds__(256) void evd2_kernel_v2(Evd2Args A)
{
    const size_t i = ((size_t)blockIdx.x * 256 + threadIdx.x) * 2;
    if (i >= A.r) return;
    if (i + 1 >= A.r) {
        evd2_one<CPLX, SINFORM, SCALED>(A, i);
        return;
    }
    const d2v a11 = __builtin_nontemporal_load((const d2v *)(A.a11 + i));
    const d2v a22 = __builtin_nontemporal_load((const d2v *)(A.a22 + i));
    const d2v ar = __builtin_nontemporal_load((const d2v *)(A.ar + i));
    d2v ai = {0.0, 0.0};
    if (CPLX) ai = __builtin_nontemporal_load((const d2v *)(A.ai + i));
    Evd2Out o0, o1;
    if (CPLX) {
        o0 = evd2_cplx<SINFORM>(a11.x, a22.x, ar.x, ai.x);
        o1 = evd2_cplx<SINFORM>(a11.y, a22.y, ar.y, ai.y);
    } else {
        o0 = evd2_real<SINFORM>(a11.x, a22.x, ar.x);
        o1 = evd2_real<SINFORM>(a11.y, a22.y, ar.y);
    }
    __builtin_nontemporal_store(d2v{o0.c, o1.c}, (d2v *)(A.cs + i));
    __builtin_nontemporal_store(d2v{o0.C, o1.C}, (d2v *)(A.cr + i));
    if (CPLX) __builtin_nontemporal_store(d2v{o0.S, o1.S}, (d2v *)(A.ci + i));
    if (A.l1) {
        const d2v L = SCALED ? d2v{o0.l1, o1.l1} : d2v{scal2(o0.l1, o0.unscale), scal2(o1.l1, o1.unscale)};
        __builtin_nontemporal_store(L, (d2v *)(A.l1 + i));
    }
    if (A.l2) {
        const d2v L = SCALED ? d2v{o0.l2, o1.l2} : d2v{scal2(o0.l2, o0.unscale), scal2(o1.l2, o1.unscale)};
        __builtin_nontemporal_store(L, (d2v *)(A.l2 + i));
    }
    if (A.zp)
        __builtin_nontemporal_store(i2v{pack_zp(o0.unscale, o0.p), pack_zp(o1.unscale, o1.p)},
                                    (i2v *)(A.zp + i));
}

// ---------------------------------------------------------------------------
// single precision (Sect. 2.4.1): V consecutive matrices per lane with
// V * 4-byte accesses; a tail shorter than V runs one matrix at a time.
struct SEvd2Args {
    size_t r;
    const float *a11, *a22, *ar, *ai;
    float *cs, *cr, *ci, *l1, *l2;
    int32_t *zp;
};

template <bool CPLX, bool SINFORM, bool SCALED>
__device__ __forceinline__ void sevd2_one(const SEvd2Args &A, size_t i)
{
    const float a11 = __builtin_nontemporal_load(A.a11 + i);
    const float a22 = __builtin_nontemporal_load(A.a22 + i);
    const float ar = __builtin_nontemporal_load(A.ar + i);
    Evd2OutT<float> o;
    if (CPLX)
        o = evd2_cplx<SINFORM>(a11, a22, ar, __builtin_nontemporal_load(A.ai + i));
    else
        o = evd2_real<SINFORM>(a11, a22, ar);
    __builtin_nontemporal_store(o.c, A.cs + i);
    __builtin_nontemporal_store(o.C, A.cr + i);
    if (CPLX) __builtin_nontemporal_store(o.S, A.ci + i);
    if (A.l1) __builtin_nontemporal_store(SCALED ? o.l1 : __builtin_amdgcn_ldexpf(o.l1, o.unscale), A.l1 + i);
    if (A.l2) __builtin_nontemporal_store(SCALED ? o.l2 : __builtin_amdgcn_ldexpf(o.l2, o.unscale), A.l2 + i);
    if (A.zp) __builtin_nontemporal_store(pack_zp(o.unscale, o.p), A.zp + i);
}

template <bool CPLX, bool SINFORM, bool SCALED, int V>
__global__ __launch_bounds__(256) void sevd2_kernel(SEvd2Args A)
{
    const size_t i = ((size_t)blockIdx.x * 256 + threadIdx.x) * V;
    if (i >= A.r) return;
    if constexpr (V == 1) {
        sevd2_one<CPLX, SINFORM, SCALED>(A, i);
    } else {
        if (i + V > A.r) {
            for (size_t k = i; k < A.r; ++k) sevd2_one<CPLX, SINFORM, SCALED>(A, k);
            return;
        }
        typedef float fv __attribute__((ext_vector_type(V)));
        typedef int iv __attribute__((ext_vector_type(V)));
        const fv a11 = __builtin_nontemporal_load((const fv *)(A.a11 + i));
        const fv a22 = __builtin_nontemporal_load((const fv *)(A.a22 + i));
        const fv ar = __builtin_nontemporal_load((const fv *)(A.ar + i));
        fv ai = {};
        if (CPLX) ai = __builtin_nontemporal_load((const fv *)(A.ai + i));
        fv c, C, S, L1, L2;
        iv z;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const Evd2OutT<float> o = CPLX ? evd2_cplx<SINFORM>(a11[u], a22[u], ar[u], ai[u])
                                           : evd2_real<SINFORM>(a11[u], a22[u], ar[u]);
            c[u] = o.c;
            C[u] = o.C;
            S[u] = o.S;
            L1[u] = SCALED ? o.l1 : __builtin_amdgcn_ldexpf(o.l1, o.unscale);
            L2[u] = SCALED ? o.l2 : __builtin_amdgcn_ldexpf(o.l2, o.unscale);
            z[u] = pack_zp(o.unscale, o.p);
        }
        __builtin_nontemporal_store(c, (fv *)(A.cs + i));
        __builtin_nontemporal_store(C, (fv *)(A.cr + i));
        if (CPLX) __builtin_nontemporal_store(S, (fv *)(A.ci + i));
        if (A.l1) __builtin_nontemporal_store(L1, (fv *)(A.l1 + i));
        if (A.l2) __builtin_nontemporal_store(L2, (fv *)(A.l2 + i));
        if (A.zp) __builtin_nontemporal_store(z, (iv *)(A.zp + i));
    }
}

template <bool CPLX, bool SINFORM, bool SCALED>
static hipError_t launch_s_t(const SEvd2Args &A, int V, hipStream_t s)
{
    const size_t threads = (A.r + V - 1) / V;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    switch (V) {
    case 4: hipLaunchKernelGGL((sevd2_kernel<CPLX, SINFORM, SCALED, 4>), dim3(blocks), dim3(256), 0, s, A); break;
    case 2: hipLaunchKernelGGL((sevd2_kernel<CPLX, SINFORM, SCALED, 2>), dim3(blocks), dim3(256), 0, s, A); break;
    default: hipLaunchKernelGGL((sevd2_kernel<CPLX, SINFORM, SCALED, 1>), dim3(blocks), dim3(256), 0, s, A); break;
    }
    return hipGetLastError();
}

static bool aligned_to(const void *p, unsigned a) { return p == nullptr || ((uintptr_t)p & (a - 1)) == 0; }

// matrices per lane of the single precision kernel: the widest access that
// every stream's alignment allows, up to the width measured fastest
int sevd2_lanes(size_t r, const void *const *ptrs, int nptr, int widest)
{
    (void)r;
    for (int V = widest; V > 1; V /= 2) {
        bool ok = true;
        for (int k = 0; k < nptr; ++k) ok = ok && aligned_to(ptrs[k], 4u * (unsigned)V);
        if (ok) return V;
    }
    return 1;
}

hipError_t launch_sevd2(size_t r, const float *a11, const float *a22, const float *ar, const float *ai, float *cs,
                        float *cr, float *ci, float *l1, float *l2, int32_t *zp, unsigned flags, int widest,
                        hipStream_t s)
{
    if (r == 0) return hipSuccess;
    SEvd2Args A{r, a11, a22, ar, ai, cs, cr, ci, l1, l2, zp};
    const void *ptrs[10] = {a11, a22, ar, ai, cs, cr, ci, l1, l2, zp};
    const int V = sevd2_lanes(r, ptrs, 10, widest);
    const bool cplx = ai != nullptr;
    const bool sinf = (flags & 2u) != 0, scaled = (flags & 1u) != 0;
    if (cplx) {
        if (sinf) return scaled ? launch_s_t<true, true, true>(A, V, s) : launch_s_t<true, true, false>(A, V, s);
        return scaled ? launch_s_t<true, false, true>(A, V, s) : launch_s_t<true, false, false>(A, V, s);
    }
    if (sinf) return scaled ? launch_s_t<false, true, true>(A, V, s) : launch_s_t<false, true, false>(A, V, s);
    return scaled ? launch_s_t<false, false, true>(A, V, s) : launch_s_t<false, false, false>(A, V, s);
}

static bool aligned16(const void *p) { return p == nullptr || ((uintptr_t)p & 15u) == 0; }

template <bool CPLX, bool SINFORM, bool SCALED>
static hipError_t launch_t(const Evd2Args &A, bool vec2, hipStream_t s)
{
    if (vec2) {
        const size_t threads = (A.r + 1) / 2;
        const unsigned blocks = (unsigned)((threads + 255) / 256);
        hipLaunchKernelGGL((evd2_kernel_v2<CPLX, SINFORM, SCALED>), dim3(blocks), dim3(256), 0, s, A);
    } else {
        const unsigned blocks = (unsigned)((A.r + 255) / 256);
        hipLaunchKernelGGL((evd2_kernel_v1<CPLX, SINFORM, SCALED>), dim3(blocks), dim3(256), 0, s, A);
    }
    return hipGetLastError();
}

// batches from this size on stream from HBM (beyond the 256 MB last-level cache)
constexpr size_t kLargeBatch = (size_t)1 << 22;

hipError_t launch_evd2(size_t r, const double *a11, const double *a22, const double *ar,
                       const double *ai, double *cs, double *cr, double *ci, double *l1,
                       double *l2, int32_t *zp, unsigned flags, hipStream_t s)
{
    if (r == 0) return hipSuccess;
    Evd2Args A{r, a11, a22, ar, ai, cs, cr, ci, l1, l2, zp};
    const bool vec2 = r < kLargeBatch && aligned16(a11) && aligned16(a22) && aligned16(ar) &&
                      aligned16(ai) && aligned16(cs) && aligned16(cr) && aligned16(ci) &&
                      aligned16(l1) && aligned16(l2) && ((uintptr_t)zp & 7u) == 0;
    const bool cplx = ai != nullptr;
    const bool sinf = (flags & 2u) != 0, scaled = (flags & 1u) != 0;
    if (cplx) {
        if (sinf)
            return scaled ? launch_t<true, true, true>(A, vec2, s) : launch_t<true, true, false>(A, vec2, s);
        return scaled ? launch_t<true, false, true>(A, vec2, s) : launch_t<true, false, false>(A, vec2, s);
    }
    if (sinf)
        return scaled ? launch_t<false, true, true>(A, vec2, s) : launch_t<false, true, false>(A, vec2, s);
    return scaled ? launch_t<false, false, true>(A, vec2, s) : launch_t<false, false, false>(A, vec2, s);
}

// ---------------------------------------------------------------------------
// The memory-system ceiling of the EVD kernels: the same streams read and
// written with the same launch shapes and access hints, every output a copy
// of an input (no arithmetic).  A measurement aid for the roofline of
// jsvd_evd2_batched.
template <bool CPLX>
__device__ __forceinline__ void stream_one(const Evd2Args &A, size_t i)
{
    const double a11 = __builtin_nontemporal_load(A.a11 + i);
    const double a22 = __builtin_nontemporal_load(A.a22 + i);
    const double ar = __builtin_nontemporal_load(A.ar + i);
    __builtin_nontemporal_store(a11, A.cs + i);
    __builtin_nontemporal_store(a22, A.cr + i);
    if (CPLX) __builtin_nontemporal_store(__builtin_nontemporal_load(A.ai + i), A.ci + i);
    __builtin_nontemporal_store(ar, A.l1 + i);
    __builtin_nontemporal_store(a11, A.l2 + i);
    __builtin_nontemporal_store((int32_t)(__double_as_longlong(a22) >> 32), A.zp + i);
}

template <bool CPLX>
__global__ __launch_bounds__(256) void evd2_stream_kernel_v1(Evd2Args A)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < A.r) stream_one<CPLX>(A, i);
}

hipError_t launch_evd2_stream(size_t r, const double *a11, const double *a22, const double *ar, const double *ai,
                              double *cs, double *cr, double *ci, double *l1, double *l2, int32_t *zp, hipStream_t s)
{
    if (r == 0) return hipSuccess;
    Evd2Args A{r, a11, a22, ar, ai, cs, cr, ci, l1, l2, zp};
    const unsigned blocks = (unsigned)((r + 255) / 256);
    if (ai)
        hipLaunchKernelGGL((evd2_stream_kernel_v1<true>), dim3(blocks), dim3(256), 0, s, A);
    else
        hipLaunchKernelGGL((evd2_stream_kernel_v1<false>), dim3(blocks), dim3(256), 0, s, A);
    return hipGetLastError();
}

} // namespace jsvd
