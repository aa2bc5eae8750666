// gstep.hip -- the parallel Jacobi step for large columns (arXiv:2202.08361,
// Alg. zvjsvd phases; the same arithmetic, bit for bit, as step.hip).
//
// Two kernels per step:
//
// * gpair_kernel: one workgroup per pivot pair.  The G column pair is read
//   once into registers; norms, scaled dot-product (Alg. zdpscl),
//   convergence test (Alg. cvg), Gram matrix (Alg. Gram), 2x2 EVD
//   (Listing 1) and rotation (Alg. zjrot) run on it there, and it is written
//   once.  Two workgroups per compute unit overlap one pair's reductions and
//   EVD with the other's memory traffic.
// * vrot_kernel: a fully occupied streaming kernel that applies the step's
//   rotations and swaps to the V column pairs; its first workgroup also folds
//   the step into the device scalars (M~, counts, s, k) from the per-pair
//   outcomes, so no workgroup of either kernel needs an atomic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "evd2_core.hpp"
#include "kernels.hpp"
#include "pair.hpp"

namespace jsvd {

constexpr int kPW = 256;   // threads per pivot pair of the G kernel

// Workgroups of the G kernel resident per compute unit: two (at most 256
// VGPRs), one with the compensated dot-products (more registers), and four
// (at most 128 VGPRs) for real single precision pairs of up to 8192 rows,
// which fit there without spilling.  (Complex single precision pairs measured
// the same with two or four.)
template <typename T, bool CPLX, int R, bool COMP>
constexpr int gpair_wgs_per_cu()
{
    if (COMP) return 1;
    if (sizeof(T) == sizeof(float) && !CPLX && R <= 32) return 4;
    return 2;
}

// G part of the step: one workgroup of W = 256 threads per pivot pair, the
// pair held in registers from its load to its store.  Several workgroups
// share a compute unit, so one computes (reductions, EVD) while the others
// wait on their loads or stores.  The outcome of the pair (rotation,
// permutation, max-norm of the rotated columns) goes to prm.
template <bool CPLX, int W, int R, bool COMP, typename T>
__global__ __launch_bounds__(W, (gpair_wgs_per_cu<T, CPLX, R, COMP>() * W / 256)) void gpair_kernel(SvdDescT<T> d,
                                                                                                      PairParam *prm)
{
    __shared__ T red[(COMP ? 12 : 6) * W];
    __shared__ T mxs[4 * (W / 64)];
    DevScalars *sc = d.sc;
    if (*(volatile int *)&sc->stop) return;
    const long long k = *(volatile long long *)&sc->k;
    const T Mt = (T)bits2d(*(volatile unsigned long long *)&sc->Mt_bits);
    const int m = d.m, n = d.n;
    const int t = threadIdx.x;
    const int l = blockIdx.x;
    const int sr = (CPLX ? SvdFp<T>::round_cplx : SvdFp<T>::round_real) - getexp(Mt);
    const bool rescale = sr < 0;
    const int sp = rescale ? (d.lgbound - getexp(Mt) - 1) : 0;
    int p, q;
    const bool valid = rr_pair(n, k, l, &p, &q);
    T *const Gpr = d.Gr + (size_t)p * d.ldg;
    T *const Gqr = d.Gr + (size_t)q * d.ldg;
    T *const Gpi = CPLX ? d.Gi + (size_t)p * d.ldg : nullptr;
    T *const Gqi = CPLX ? d.Gi + (size_t)q * d.ldg : nullptr;
    PairParam pp;
    pp.p = p;
    pp.q = q;
    pp.flag = 0;
    pp.c = 1.0;
    pp.C = 0.0;
    pp.S = 0.0;
    pp.mx = 0.0;
    if (!valid) {
        // the column sitting out (odd n): only the rescaling applies
        if (rescale) {
            for (int i = t; i < m; i += W) {
                Gpr[i] = scal2(Gpr[i], sp);
                if (CPLX) Gpi[i] = scal2(Gpi[i], sp);
            }
        }
        if (t == 0) prm[l] = pp;
    } else {
        T xr[2][R], xi[2][R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = t + W * j;
            const bool in = i < m;
            xr[0][j] = in ? Gpr[i] : T(0);
            xr[1][j] = in ? Gqr[i] : T(0);
            if (CPLX) {
                xi[0][j] = in ? Gpi[i] : T(0);
                xi[1][j] = in ? Gqi[i] : T(0);
            }
        }
        if (rescale) {
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    xr[c][j] = scal2(xr[c][j], sp);
                    if (CPLX) xi[c][j] = scal2(xi[c][j], sp);
                }
        }
        const PairDecisionT<T> dc =
            pair_core<CPLX, W, R, COMP>(xr, xi, d.ups, d.nosort, d.nogs, red, red + 4 * W, mxs);
        const int pbit = dc.pbit;
        T *const Dp_r = pbit ? Gqr : Gpr;
        T *const Dq_r = pbit ? Gpr : Gqr;
        T *const Dp_i = pbit ? Gqi : Gpi;
        T *const Dq_i = pbit ? Gpi : Gqi;
        if (dc.transform) {
            T mm[1] = {transform_regs<CPLX, R>(xr, xi, dc)};
            group_max<W, 1>(mm, mxs + 2 * (W / 64));
            pp.mx = mm[0];
            pp.flag = 1 | (pbit ? 2 : 0) | (dc.gs ? 4 : 0);
            pp.c = dc.c;
            pp.C = dc.C;
            pp.S = dc.S;
        } else if (pbit) {
            pp.flag = 2;
        }
        if (dc.transform || pbit || rescale) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = t + W * j;
                if (i < m) {
                    Dp_r[i] = xr[0][j];
                    Dq_r[i] = xr[1][j];
                    if (CPLX) {
                        Dp_i[i] = xi[0][j];
                        Dq_i[i] = xi[1][j];
                    }
                }
            }
        }
        if (t == 0) {
            prm[l] = pp;
            const int dp = pbit ? q : p, dq = pbit ? p : q;
            d.e[dp] = dc.np.zero ? T(-INFINITY) : (T)dc.np.e;
            d.f[dp] = dc.np.zero ? T(1) : dc.np.f;
            d.e[dq] = dc.nq.zero ? T(-INFINITY) : (T)dc.nq.e;
            d.f[dq] = dc.nq.zero ? T(1) : dc.nq.f;
        }
    }
}


// rotation or swap of one V column pair, rows of row block blockIdx.y (the
// parameters, kept as doubles in prm, convert back to T exactly)
template <bool CPLX, typename T>
__device__ __forceinline__ void vrot_pair(const SvdDescT<T> &d, const PairParam &pp)
{
    const int n = d.n;
    const int i0 = blockIdx.y * 512 + threadIdx.x;
    T *const Vpr = d.Vr + (size_t)pp.p * d.ldv;
    T *const Vqr = d.Vr + (size_t)pp.q * d.ldv;
    T *const Vpi = CPLX ? d.Vi + (size_t)pp.p * d.ldv : nullptr;
    T *const Vqi = CPLX ? d.Vi + (size_t)pp.q * d.ldv : nullptr;
    const bool swap = (pp.flag & 2) != 0;
    T *const Ep_r = swap ? Vqr : Vpr;
    T *const Eq_r = swap ? Vpr : Vqr;
    T *const Ep_i = swap ? Vqi : Vpi;
    T *const Eq_i = swap ? Vpi : Vqi;
    const T c = (T)pp.c, C = (T)pp.C, S = (T)pp.S;
    T pr[2], qr[2], pi[2] = {T(0), T(0)}, qi[2] = {T(0), T(0)};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = i0 + 256 * u;
        const bool in = i < n;
        pr[u] = in ? Vpr[i] : T(0);
        qr[u] = in ? Vqr[i] : T(0);
        if (CPLX) {
            pi[u] = in ? Vpi[i] : T(0);
            qi[u] = in ? Vqi[i] : T(0);
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = i0 + 256 * u;
        if (i >= n) continue;
        if (pp.flag & 1) {
            if (CPLX) {
                Ep_r[i] = fma(qr[u], C, fma(-qi[u], S, pr[u])) * c;
                Ep_i[i] = fma(qr[u], S, fma(qi[u], C, pi[u])) * c;
                Eq_r[i] = fma(pr[u], -C, fma(-pi[u], S, qr[u])) * c;
                Eq_i[i] = fma(pr[u], S, fma(pi[u], -C, qi[u])) * c;
            } else {
                Ep_r[i] = fma(qr[u], C, pr[u]) * c;
                Eq_r[i] = fma(pr[u], -C, qr[u]) * c;
            }
        } else {
            Vpr[i] = qr[u];
            Vqr[i] = pr[u];
            if (CPLX) {
                Vpi[i] = qi[u];
                Vqi[i] = pi[u];
            }
        }
    }
}

// End of step (Alg. zvjsvd): from the outcomes of all pairs, M~_{k+1} =
// max(2^{s_[k]} M~_k, M) with M the max-norm of the rotated columns, the
// counts of rotations and of swaps, the scaling exponent and the step index.
// One workgroup of 256 threads; max and integer sums are exact, so the order
// does not matter.  The max-norms are values of the working precision T held
// as doubles, so the max and the rescaling below are those of T.
template <typename T>
__device__ void fold_step(const SvdDescT<T> &d, const PairParam *prm, int npairs)
{
    __shared__ double smx[4];
    __shared__ unsigned long long scnt[12];
    DevScalars *sc = d.sc;
    const int t = threadIdx.x;
    double mx = 0.0;
    unsigned long long tc = 0, swc = 0, gsc = 0;
    for (int l = t; l < npairs; l += 256) {
        const int fl = prm[l].flag;
        if (fl & 1) {
            mx = fmax(mx, prm[l].mx);
            ++tc;
            if (fl & 4) ++gsc;
        } else if (fl & 2) {
            ++swc;
        }
    }
    mx = wave_max(mx);
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) {
        tc += __shfl_xor(tc, h, 64);
        swc += __shfl_xor(swc, h, 64);
        gsc += __shfl_xor(gsc, h, 64);
    }
    if ((t & 63) == 0) {
        smx[t >> 6] = mx;
        scnt[t >> 6] = tc;
        scnt[4 + (t >> 6)] = swc;
        scnt[8 + (t >> 6)] = gsc;
    }
    __syncthreads();
    if (t == 0) {
        double M = smx[0];
        unsigned long long tt = scnt[0], sw = scnt[4], gg = scnt[8];
        for (int w = 1; w < 4; ++w) {
            M = fmax(M, smx[w]);
            tt += scnt[w];
            sw += scnt[4 + w];
            gg += scnt[8 + w];
        }
        const T Mt = (T)bits2d(sc->Mt_bits);
        const bool rescale = (d.cplx ? SvdFp<T>::round_cplx : SvdFp<T>::round_real) - getexp(Mt) < 0;
        const int sp = rescale ? (d.lgbound - getexp(Mt) - 1) : 0;
        const T Mt2 = rescale ? scal2(Mt, sp) : Mt;
        sc->Mt_bits = d2bits((double)fmax(Mt2, (T)M));
        sc->T += (long long)tt;
        sc->SW += (long long)sw;
        sc->GS += (long long)gg;
        sc->last_t = (long long)tt;
        if (rescale) {
            sc->s += sp;
            sc->rescaled += 1;
        }
        sc->k += 1;
    }
}

// V column pairs: rotate (flag & 1) and/or swap (flag & 2) with the step's
// parameters; 2 rows per thread, grid (pairs, row blocks).  Workgroup (0, 0)
// also folds the step into the device scalars (every G column of the step is
// final once this kernel runs).
template <bool CPLX, typename T>
__global__ __launch_bounds__(256) void vrot_kernel(SvdDescT<T> d, const PairParam *prm)
{
    if (*(volatile int *)&d.sc->stop) return;
    const PairParam pp = prm[blockIdx.x];
    if (pp.flag != 0) vrot_pair<CPLX>(d, pp);
    if (blockIdx.x == 0 && blockIdx.y == 0) fold_step(d, prm, (d.n + (d.n & 1)) / 2);
}

// rows per thread of the G kernel for m rows (0 = not supported): a column
// pair takes at most 128 registers per thread, so single precision allows
// twice the rows
int gpair_rows(int m, int cplx, bool fp32)
{
    const int R = (m + kPW - 1) / kPW;
    const int rmax = (cplx ? 16 : 32) * (fp32 ? 2 : 1);
    if (R > rmax) return 0;
    int r = 1;
    while (r < R) r *= 2;
    return r;
}

template <bool CPLX, typename T>
static hipError_t launch_gpair_t(const SvdDescT<T> &d, PairParam *prm, int R, hipStream_t s)
{
    constexpr bool F32 = sizeof(T) == sizeof(float);
    const int npairs = (d.n + (d.n & 1)) / 2;
    constexpr int RM = (CPLX ? 16 : 32) * (F32 ? 2 : 1);
    if (d.comp && F32) return hipErrorInvalidValue;
    switch (R) {
#define JSVD_GP(r)                                                                                              \
    case r:                                                                                                     \
        if constexpr (r <= RM) {                                                                                \
            if constexpr (!F32) {                                                                               \
                if (d.comp) {                                                                                   \
                    hipLaunchKernelGGL((gpair_kernel<CPLX, kPW, r, true, T>), dim3(npairs), dim3(kPW), 0, s, d, \
                                       prm);                                                                    \
                    return hipGetLastError();                                                                   \
                }                                                                                               \
            }                                                                                                   \
            hipLaunchKernelGGL((gpair_kernel<CPLX, kPW, r, false, T>), dim3(npairs), dim3(kPW), 0, s, d, prm);  \
            return hipGetLastError();                                                                           \
        }                                                                                                       \
        break;
        JSVD_GP(1) JSVD_GP(2) JSVD_GP(4) JSVD_GP(8) JSVD_GP(16) JSVD_GP(32) JSVD_GP(64)
#undef JSVD_GP
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_vrot(const SvdDescT<T> &d, const PairParam *prm, hipStream_t s)
{
    const int npairs = (d.n + (d.n & 1)) / 2;
    dim3 vgrid(npairs, (d.n + 511) / 512);
    if (d.cplx)
        hipLaunchKernelGGL((vrot_kernel<true, T>), vgrid, dim3(256), 0, s, d, prm);
    else
        hipLaunchKernelGGL((vrot_kernel<false, T>), vgrid, dim3(256), 0, s, d, prm);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gpair(const SvdDescT<T> &d, PairParam *prm, hipStream_t s)
{
    const int R = gpair_rows(d.m, d.cplx, sizeof(T) == sizeof(float));
    if (R == 0) return hipErrorInvalidValue;
    const hipError_t e = d.cplx ? launch_gpair_t<true>(d, prm, R, s) : launch_gpair_t<false>(d, prm, R, s);
    if (e != hipSuccess) return e;
    return launch_vrot(d, prm, s);
}

template hipError_t launch_vrot<double>(const SvdDescT<double> &, const PairParam *, hipStream_t);
template hipError_t launch_vrot<float>(const SvdDescT<float> &, const PairParam *, hipStream_t);
template hipError_t launch_gpair<double>(const SvdDescT<double> &, PairParam *, hipStream_t);
template hipError_t launch_gpair<float>(const SvdDescT<float> &, PairParam *, hipStream_t);

} // namespace jsvd
