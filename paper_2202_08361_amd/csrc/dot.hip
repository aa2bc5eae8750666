// dot.hip -- batched scaled dot-products a21' = g_q^* g_p / (|g_q| |g_p|)
// (arXiv:2202.08361, Sect. 3.3: Alg. zdpscl, and Sect. SM2.2: Alg. zdpsclcs /
// ddpsclcs with the compensated summation).
//
// One workgroup of 256 threads per column pair, the pair in registers, the
// sums by pair_dot: the same code and the same canonical lane order as the
// Jacobi step, so a pair gives here exactly the a21' it gets in a step.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "evd2_core.hpp"
#include "kernels.hpp"
#include "pair.hpp"

namespace jsvd {

constexpr int kDW = 256;   // threads per column pair

struct DotArgs {
    int m;
    const double *Qr, *Qi, *Pr, *Pi;
    long long ld;
    const double *eq, *fq, *ep, *fp;
    double *zr, *zi;
};

template <bool CPLX, int R, bool COMP>
__global__ __launch_bounds__(kDW) void dot_kernel(DotArgs A)
{
    __shared__ double red[(COMP ? 8 : 2) * kDW];
    const int j = blockIdx.x;
    const int t = threadIdx.x;
    const double eqd = A.eq[j], epd = A.ep[j];
    if (!(fabs(eqd) <= 4096.0 && fabs(epd) <= 4096.0)) {
        // a norm exponent that is not that of a non-zero column
        if (t == 0) {
            A.zr[j] = NAN;
            if (CPLX) A.zi[j] = NAN;
        }
        return;
    }
    const double *q = A.Qr + (size_t)j * A.ld, *p = A.Pr + (size_t)j * A.ld;
    const double *qi = CPLX ? A.Qi + (size_t)j * A.ld : nullptr;
    const double *pi = CPLX ? A.Pi + (size_t)j * A.ld : nullptr;
    double xr[2][R], xi[2][R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = t + kDW * k;
        const bool in = i < A.m;
        xr[0][k] = in ? p[i] : 0.0;
        xr[1][k] = in ? q[i] : 0.0;
        xi[0][k] = (CPLX && in) ? pi[i] : 0.0;
        xi[1][k] = (CPLX && in) ? qi[i] : 0.0;
    }
    double h[2];
    pair_dot<CPLX, kDW, R, COMP>(xr, xi, (int)epd, (int)eqd, h, red);
    if (t == 0) {
        const double dd = A.fq[j] * A.fp[j];
        A.zr[j] = h[0] / dd;
        if (CPLX) A.zi[j] = h[1] / dd;
    }
}

int dot_rows(int m, int cplx)
{
    const int R = (m + kDW - 1) / kDW;
    if (R > (cplx ? 16 : 32)) return 0;
    int r = 1;
    while (r < R) r *= 2;
    return r;
}

template <bool CPLX, bool COMP>
static hipError_t launch_dot_t(int npairs, const DotArgs &A, int R, hipStream_t s)
{
    switch (R) {
#define JSVD_DT(r)                                                                               \
    case r:                                                                                      \
        if constexpr (r <= (CPLX ? 16 : 32)) {                                                   \
            hipLaunchKernelGGL((dot_kernel<CPLX, r, COMP>), dim3(npairs), dim3(kDW), 0, s, A);   \
            return hipGetLastError();                                                            \
        }                                                                                        \
        break;
        JSVD_DT(1) JSVD_DT(2) JSVD_DT(4) JSVD_DT(8) JSVD_DT(16) JSVD_DT(32)
#undef JSVD_DT
    }
    return hipErrorInvalidValue;
}

hipError_t launch_dot(int npairs, int m, const double *Qr, const double *Qi, const double *Pr, const double *Pi,
                      long long ld, const double *eq, const double *fq, const double *ep, const double *fp,
                      double *zr, double *zi, bool comp, hipStream_t s)
{
    const bool cplx = Qi != nullptr;
    const int R = dot_rows(m, cplx);
    if (R == 0 || npairs <= 0) return hipErrorInvalidValue;
    const DotArgs A{m, Qr, Qi, Pr, Pi, ld, eq, fq, ep, fp, zr, zi};
    if (cplx) return comp ? launch_dot_t<true, true>(npairs, A, R, s) : launch_dot_t<true, false>(npairs, A, R, s);
    return comp ? launch_dot_t<false, true>(npairs, A, R, s) : launch_dot_t<false, false>(npairs, A, R, s);
}

} // namespace jsvd
