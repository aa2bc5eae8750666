// sstep.hip -- one parallel Jacobi step for columns longer than the register
// tile of the fused step kernel (more than 16384 real / 8192 complex rows):
// the pivot pair is streamed from memory instead of held in registers.
//
// One workgroup of 1024 threads per pair; thread t is lane t of the 1024-lane
// vector of every sum and takes rows t, t + 1024, ... in order, as in the
// register kernels (Sect. 3: Alg. zdpscl's lane-wise accumulation, the
// norms' sums of squares), so the sums, and with them the whole step, are
// the same bits.  The passes over the pair:
//   1. max |component| of each column (the norms' prescaling exponent);
//   2. the sums of squares (column norms in (e, f) form);
//   3. the scaled dot-product (Alg. zdpscl, or zdpsclcs / ddpsclcs);
//   then the decision (Alg. cvg, Alg. Gram, the 2x2 EVD, eq. GScond) and
//   4. the rotation (Alg. zjrot) or Gram-Schmidt step (eq. GS) or swap of the
//      G pair, rows read and written once, then the same for the V pair.
// Passes 1-3 read the pair three times (the columns stay in the L2 / MALL
// between them); the rescaling check of Sect. 3.2, the outcome log and the
// fold of the previous step are those of the fused kernel.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "evd2_core.hpp"
#include "fold.hpp"
#include "kernels.hpp"
#include "pair.hpp"

namespace jsvd {

constexpr int kSW = 1024;   // threads per pair
constexpr int kSC = 4;      // rows per thread per chunk (loads in flight)

template <bool COMP, typename T>
struct StreamSmem {
    T red[(COMP ? 8 : 4) * kSW];
    T mx[2 * (kSW / 64)];
};

// rows i0 + t + kSW j (j < kSC) of column x, 2^sp-scaled, 0 beyond m
template <typename T>
__device__ __forceinline__ void stream_load(const T *x, int m, long long i0, int sp, bool rescale, T (&v)[kSC])
{
#pragma unroll
    for (int j = 0; j < kSC; ++j) {
        const long long i = i0 + threadIdx.x + (long long)kSW * j;
        const T a = i < m ? x[i] : T(0);
        v[j] = rescale ? scal2(a, sp) : a;
    }
}

template <bool CPLX, bool COMP, typename T>
__global__ __launch_bounds__(kSW) void stream_step_kernel(SvdDescT<T> d, StepSlot slot, StepSlot prev)
{
    __shared__ StreamSmem<COMP, T> sm;
    DevScalars *sc = d.sc;
    PairParam *const prm = slot.prm;
    const int t = threadIdx.x;
    const int l = blockIdx.x;
    if (*(volatile int *)&sc->stop) {
        if (t == 0) {
            PairParam z;
            z.c = 1.0;
            z.C = z.S = 0.0;
            z.pq = z.flag = 0;
            prm[l] = z;
            slot.mx[l] = 0.0;
        }
        return;
    }
    const int m = d.m, n = d.n;
    const int npairs = (n + 1) / 2;
    const long long k = prev.prm ? prev.hdr->k + 1 : *(volatile long long *)&sc->k;
    const unsigned long long pkey = prev.prm ? *prev.mxkey : 0ull;
    int p, q;
    const bool valid = rr_pair(n, k, l, &p, &q);
    T *const Gpr = d.Gr + (size_t)p * d.ldg;
    T *const Gqr = d.Gr + (size_t)q * d.ldg;
    T *const Gpi = CPLX ? d.Gi + (size_t)p * d.ldg : nullptr;
    T *const Gqi = CPLX ? d.Gi + (size_t)q * d.ldg : nullptr;
    T *const Vpr = d.Vr + (size_t)p * d.ldv;
    T *const Vqr = d.Vr + (size_t)q * d.ldv;
    T *const Vpi = CPLX ? d.Vi + (size_t)p * d.ldv : nullptr;
    T *const Vqi = CPLX ? d.Vi + (size_t)q * d.ldv : nullptr;

    // floor(lg M~) of this step, as in the fused kernel (and workgroup 0
    // folds the previous step when its fold is due)
    int eMt;
    if (prev.prm) {
        const T Mp = (T)bits2d(prev.hdr->Mt_bits);
        const bool rp = (CPLX ? SvdFp<T>::round_cplx : SvdFp<T>::round_real) - getexp(Mp) < 0;
        const T Mp2 = rp ? scal2(Mp, d.lgbound - getexp(Mp) - 1) : Mp;
        eMt = max(getexp(Mp2), step_max_exp(pkey, k - 1));
        if (l == 0) {
            const unsigned long long Mt_bits = fold_step<kSW, T>(d, prev.prm, prev.mx, npairs);
            if (t == 0) {
                slot.hdr->k = k;
                slot.hdr->Mt_bits = Mt_bits;
            }
        }
    } else {
        const unsigned long long Mt_bits = *(volatile unsigned long long *)&sc->Mt_bits;
        eMt = getexp((T)bits2d(Mt_bits));
        if (l == 0 && t == 0) {
            slot.hdr->k = k;
            slot.hdr->Mt_bits = Mt_bits;
        }
    }
    const int sr = (CPLX ? SvdFp<T>::round_cplx : SvdFp<T>::round_real) - eMt;
    const bool rescale = sr < 0;
    const int sp = rescale ? (d.lgbound - eMt - 1) : 0;

    PairParam pp;
    pp.pq = p | (q << 16);
    pp.flag = 0;
    pp.c = 1.0;
    pp.C = 0.0;
    pp.S = 0.0;
    if (!valid) {
        if (rescale) {
            for (int i = t; i < m; i += kSW) {
                Gpr[i] = scal2(Gpr[i], sp);
                if (CPLX) Gpi[i] = scal2(Gpi[i], sp);
            }
        }
        if (t == 0) {
            prm[l] = pp;
            slot.mx[l] = 0.0;
        }
        return;
    }

    // ---- pass 1: max |component| of each column
    T mx[2] = {T(0), T(0)};
    for (long long i0 = 0; i0 < m; i0 += (long long)kSW * kSC) {
        T a[kSC], b[kSC], ai[kSC], bi[kSC];
        stream_load(Gpr, m, i0, sp, rescale, a);
        stream_load(Gqr, m, i0, sp, rescale, b);
        if (CPLX) {
            stream_load(Gpi, m, i0, sp, rescale, ai);
            stream_load(Gqi, m, i0, sp, rescale, bi);
        }
#pragma unroll
        for (int j = 0; j < kSC; ++j) {
            mx[0] = fmax(mx[0], fabs(a[j]));
            mx[1] = fmax(mx[1], fabs(b[j]));
            if (CPLX) {
                mx[0] = fmax(mx[0], fabs(ai[j]));
                mx[1] = fmax(mx[1], fabs(bi[j]));
            }
        }
    }
    group_max<kSW, 2>(mx, sm.mx);
    const bool zp_ = mx[0] == T(0), zq_ = mx[1] == T(0);
    const int Ep = zp_ ? 0 : getexp(mx[0]);
    const int Eq = zq_ ? 0 : getexp(mx[1]);

    // ---- pass 2: sums of squares, lane t taking its rows in order
    constexpr int NQ = CPLX ? 4 : 2;
    T s[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) s[u] = T(0);
    for (long long i0 = 0; i0 < m; i0 += (long long)kSW * kSC) {
        T a[kSC], b[kSC], ai[kSC], bi[kSC];
        stream_load(Gpr, m, i0, sp, rescale, a);
        stream_load(Gqr, m, i0, sp, rescale, b);
        if (CPLX) {
            stream_load(Gpi, m, i0, sp, rescale, ai);
            stream_load(Gqi, m, i0, sp, rescale, bi);
        }
#pragma unroll
        for (int j = 0; j < kSC; ++j) {
            if (i0 + t + (long long)kSW * j >= m) break;
            const T ypr = scal2(a[j], -Ep), yqr = scal2(b[j], -Eq);
            s[0] = fma(ypr, ypr, s[0]);
            s[1] = fma(yqr, yqr, s[1]);
            if (CPLX) {
                const T ypi = scal2(ai[j], -Ep), yqi = scal2(bi[j], -Eq);
                s[2] = fma(ypi, ypi, s[2]);
                s[3] = fma(yqi, yqi, s[3]);
            }
        }
    }
    __syncthreads();
    group_tree_sum<kSW, NQ>(s, sm.red);
    NormT<T> np = norm_from_sums(Ep, s[0], CPLX ? s[2] : T(0), CPLX);
    NormT<T> nq = norm_from_sums(Eq, s[1], CPLX ? s[3] : T(0), CPLX);
    np.zero = zp_;
    nq.zero = zq_;

    // ---- pass 3: the scaled dot-product g_q^* g_p (without its division)
    T h[2] = {T(0), T(0)};
    if (!zp_ && !zq_) {
        const int ep = np.e, eq = nq.e;
        if constexpr (!COMP) {
            T dr = T(0), di = T(0);
            for (long long i0 = 0; i0 < m; i0 += (long long)kSW * kSC) {
                T a[kSC], b[kSC], ai[kSC], bi[kSC];
                stream_load(Gpr, m, i0, sp, rescale, a);
                stream_load(Gqr, m, i0, sp, rescale, b);
                if (CPLX) {
                    stream_load(Gpi, m, i0, sp, rescale, ai);
                    stream_load(Gqi, m, i0, sp, rescale, bi);
                }
#pragma unroll
                for (int j = 0; j < kSC; ++j) {
                    if (i0 + t + (long long)kSW * j >= m) break;
                    const T gqr = scal2(b[j], -eq), gpr = scal2(a[j], -ep);
                    if (CPLX) {
                        const T gqi = scal2(bi[j], -eq), gpi = scal2(ai[j], -ep);
                        dr = fma(gqr, gpr, dr);
                        di = fma(gqr, gpi, di);
                        dr = fma(gqi, gpi, dr);
                        di = fma(-gqi, gpr, di);
                    } else {
                        dr = fma(gqr, gpr, dr);
                    }
                }
            }
            constexpr int ND = CPLX ? 2 : 1;
            T g[ND];
            g[0] = dr;
            if (CPLX) g[ND - 1] = di;
            __syncthreads();
            group_tree_sum<kSW, ND>(g, sm.red);
            h[0] = g[0];
            h[1] = CPLX ? g[ND - 1] : T(0);
        } else {
            // [stream][s, t, s', t'] per lane (Alg. zdpsclcs / ddpsclcs)
            constexpr int NS = CPLX ? 2 : 1;
            double acc[NS][4];
#pragma unroll
            for (int st = 0; st < NS; ++st)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[st][u] = 0.0;
            for (long long i0 = 0; i0 < m; i0 += (long long)kSW * kSC) {
                T a[kSC], b[kSC], ai[kSC], bi[kSC];
                stream_load(Gpr, m, i0, sp, rescale, a);
                stream_load(Gqr, m, i0, sp, rescale, b);
                if (CPLX) {
                    stream_load(Gpi, m, i0, sp, rescale, ai);
                    stream_load(Gqi, m, i0, sp, rescale, bi);
                }
#pragma unroll
                for (int j = 0; j < kSC; ++j) {
                    if (i0 + t + (long long)kSW * j >= m) break;
                    const double gpr = scal2(a[j], -ep), gqr = scal2(b[j], -eq);
                    cs_term(gpr, gqr, acc[0][0], acc[0][1], acc[0][2], acc[0][3]);
                    if (CPLX) {
                        const double gpi = scal2(ai[j], -ep), gqi = scal2(bi[j], -eq);
                        cs_term(gpi, gqi, acc[0][0], acc[0][1], acc[0][2], acc[0][3]);
                        cs_term(gqr, gpi, acc[NS - 1][0], acc[NS - 1][1], acc[NS - 1][2], acc[NS - 1][3]);
                        cs_term(-gqi, gpr, acc[NS - 1][0], acc[NS - 1][1], acc[NS - 1][2], acc[NS - 1][3]);
                    }
                }
            }
            double g[4 * NS];
#pragma unroll
            for (int st = 0; st < NS; ++st)
#pragma unroll
                for (int u = 0; u < 4; ++u) g[4 * st + u] = acc[st][u];
            __syncthreads();
            group_tree_sum<kSW, 4 * NS>(g, (double *)sm.red);
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                double z = g[4 * st + 2] + g[4 * st + 3];
                z = z + g[4 * st + 1];
                h[st] = (T)(z + g[4 * st + 0]);
            }
            if (!CPLX) h[1] = T(0);
        }
    }
    const PairDecisionT<T> dc = pair_decide<CPLX>(np, nq, h, d.ups, d.nosort, d.nogs);
    const bool transform = dc.transform;
    const int pbit = dc.pbit;

    // ---- pass 4: transform or swap (or only rescale) the G pair, then V
    T *const Dp_r = pbit ? Gqr : Gpr;
    T *const Dq_r = pbit ? Gpr : Gqr;
    T *const Dp_i = pbit ? Gqi : Gpi;
    T *const Dq_i = pbit ? Gpi : Gqi;
    T *const Ep_r = pbit ? Vqr : Vpr;
    T *const Eq_r = pbit ? Vpr : Vqr;
    T *const Ep_i = pbit ? Vqi : Vpi;
    T *const Eq_i = pbit ? Vpi : Vqi;
    T Mx = T(0);
    if (transform || pbit || rescale) {
        for (long long i0 = 0; i0 < m; i0 += (long long)kSW * kSC) {
            T xr[2][kSC], xi[2][kSC];
            stream_load(Gpr, m, i0, sp, rescale, xr[0]);
            stream_load(Gqr, m, i0, sp, rescale, xr[1]);
            if (CPLX) {
                stream_load(Gpi, m, i0, sp, rescale, xi[0]);
                stream_load(Gqi, m, i0, sp, rescale, xi[1]);
            }
            // rows beyond m hold zeros: they change no max and are not stored
            if (transform) Mx = fmax(Mx, transform_regs<CPLX, kSC>(xr, xi, dc));
#pragma unroll
            for (int j = 0; j < kSC; ++j) {
                const long long i = i0 + t + (long long)kSW * j;
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
    }
    if (transform || pbit) {
        for (long long i0 = 0; i0 < n; i0 += (long long)kSW * kSC) {
            T vr[2][kSC], vi[2][kSC];
            stream_load(Vpr, n, i0, 0, false, vr[0]);
            stream_load(Vqr, n, i0, 0, false, vr[1]);
            if (CPLX) {
                stream_load(Vpi, n, i0, 0, false, vi[0]);
                stream_load(Vqi, n, i0, 0, false, vi[1]);
            }
            if (transform) (void)rot_regs<CPLX, kSC>(vr, vi, dc.c, dc.C, dc.S);
#pragma unroll
            for (int j = 0; j < kSC; ++j) {
                const long long i = i0 + t + (long long)kSW * j;
                if (i < n) {
                    Ep_r[i] = vr[0][j];
                    Eq_r[i] = vr[1][j];
                    if (CPLX) {
                        Ep_i[i] = vi[0][j];
                        Eq_i[i] = vi[1][j];
                    }
                }
            }
        }
    }
    T Mblk = T(0);
    if (transform) {
        T mm[1] = {Mx};
        __syncthreads();
        group_max<kSW, 1>(mm, sm.mx);
        Mblk = mm[0];
        pp.flag = 1 | (pbit ? 2 : 0) | (dc.gs ? 4 : 0);
        pp.c = dc.c;
        pp.C = dc.C;
        pp.S = dc.S;
    } else if (pbit) {
        pp.flag = 2;
    }
    // ---- the pair's outcome for the fold of this step, and its norms
    if (t == 0) {
        prm[l] = pp;
        slot.mx[l] = (double)Mblk;
        if (transform && Mblk > T(0)) step_max_add(slot.mxkey, k, getexp(Mblk));
        const T ep = np.zero ? T(-INFINITY) : (T)np.e;
        const T eq = nq.zero ? T(-INFINITY) : (T)nq.e;
        const int dp = pbit ? q : p, dq = pbit ? p : q;
        d.e[dp] = ep;
        d.f[dp] = np.zero ? T(1) : np.f;
        d.e[dq] = eq;
        d.f[dq] = nq.zero ? T(1) : nq.f;
    }
}

template <typename T>
hipError_t launch_stream_step(const SvdDescT<T> &d, StepSlot slot, StepSlot prev, hipStream_t s)
{
    const int N = d.n + (d.n & 1);
    const unsigned blocks = (unsigned)(N / 2);
    if (d.comp) {
        if constexpr (sizeof(T) == sizeof(double)) {
            if (d.cplx)
                hipLaunchKernelGGL((stream_step_kernel<true, true, T>), dim3(blocks), dim3(kSW), 0, s, d, slot, prev);
            else
                hipLaunchKernelGGL((stream_step_kernel<false, true, T>), dim3(blocks), dim3(kSW), 0, s, d, slot, prev);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        if (d.cplx)
            hipLaunchKernelGGL((stream_step_kernel<true, false, T>), dim3(blocks), dim3(kSW), 0, s, d, slot, prev);
        else
            hipLaunchKernelGGL((stream_step_kernel<false, false, T>), dim3(blocks), dim3(kSW), 0, s, d, slot, prev);
    }
    return hipGetLastError();
}

template hipError_t launch_stream_step<double>(const SvdDescT<double> &, StepSlot, StepSlot, hipStream_t);
template hipError_t launch_stream_step<float>(const SvdDescT<float> &, StepSlot, StepSlot, hipStream_t);

} // namespace jsvd
