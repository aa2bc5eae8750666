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
    const double L1 = SCALED ? o.l1 : scal2(o.l1, o.zeta_b);
    const double L2 = SCALED ? o.l2 : scal2(o.l2, o.zeta_b);
    if (A.l1) __builtin_nontemporal_store(L1, A.l1 + i);
    if (A.l2) __builtin_nontemporal_store(L2, A.l2 + i);
    if (A.zp) __builtin_nontemporal_store(pack_zp(o.zeta_b, o.p), A.zp + i);
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
        const d2v L = SCALED ? d2v{o0.l1, o1.l1} : d2v{scal2(o0.l1, o0.zeta_b), scal2(o1.l1, o1.zeta_b)};
        __builtin_nontemporal_store(L, (d2v *)(A.l1 + i));
    }
    if (A.l2) {
        const d2v L = SCALED ? d2v{o0.l2, o1.l2} : d2v{scal2(o0.l2, o0.zeta_b), scal2(o1.l2, o1.zeta_b)};
        __builtin_nontemporal_store(L, (d2v *)(A.l2 + i));
    }
    if (A.zp)
        __builtin_nontemporal_store(i2v{pack_zp(o0.zeta_b, o0.p), pack_zp(o1.zeta_b, o1.p)},
                                    (i2v *)(A.zp + i));
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

} // namespace jsvd
