// fold.hpp -- the end of a Jacobi step (Alg. zvjsvd) folded from the
// pairs' logged outcomes, shared by the step kernels (step.hip, gstep.hip).
//
// Each workgroup of a step writes its pair's outcome (rotation, swap,
// Gram-Schmidt, max-norm of the rotated columns) to the step's slot of the
// outcome log and, if it rotated, adds the exponent of that max-norm to the
// slot's key with one relaxed atomic max.  The next step's workgroups derive
// the step index and floor(lg M~) (all the rescaling check needs) from the
// slot, and its workgroup 0 folds the slot into the device scalars.  No
// workgroup waits on another.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "pair.hpp"

namespace jsvd {

// End of step (Alg. zvjsvd): from the outcomes of all pairs, M~_{k+1} =
// max(2^{s_[k]} M~_k, M) with M the max-norm of the rotated columns, the
// counts of rotations and of swaps, the scaling exponent and the step index.
// One workgroup of FW threads; max and integer sums are exact, so the order
// does not matter.  The max-norms are values of the working precision T held
// as doubles, so the max and the rescaling below are those of T.
constexpr int kFoldW = 1024;   // threads of the fold kernel

template <int FW, typename T>
__device__ unsigned long long fold_step(const SvdDescT<T> &d, const PairParam *prm, const double *pmx, int npairs)
{
    constexpr int NW = FW / 64;
    __shared__ double smx[NW];
    __shared__ unsigned long long scnt[4 * NW];
    DevScalars *sc = d.sc;
    const int t = threadIdx.x;
    // the scalars the fold updates, loaded (by thread 0) beside the outcomes
    unsigned long long Mt_bits = 0;
    long long T0 = 0, SW0 = 0, GS0 = 0, k0 = 0, SK0 = 0;
    int s0 = 0, resc0 = 0;
    if (t == 0) {
        Mt_bits = sc->Mt_bits;
        T0 = sc->T;
        SW0 = sc->SW;
        GS0 = sc->GS;
        SK0 = sc->skipped;
        k0 = sc->k;
        s0 = sc->s;
        resc0 = sc->rescaled;
    }
    double mx = 0.0;
    unsigned long long tc = 0, swc = 0, gsc = 0, skc = 0;
    // four outcomes per thread in flight at once (the log was written by
    // other compute units: each load goes past this one's L2)
    for (int l0 = 0; l0 < npairs; l0 += 4 * FW) {
        int fl[4];
        double m4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            // unconditional loads (an index past the end reads entry 0, masked)
            const int l = l0 + t + FW * u;
            const int lc = l < npairs ? l : 0;
            const int f = prm[lc].flag;
            const double mv = pmx[lc];
            fl[u] = l < npairs ? f : 0;
            m4[u] = mv;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (fl[u] & 1) {
                mx = fmax(mx, m4[u]);
                ++tc;
                if (fl[u] & 4) ++gsc;
            } else if (fl[u] & 2) {
                ++swc;
            }
            if (fl[u] & 8) ++skc;
        }
    }
    mx = wave_max(mx);
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) {
        tc += __shfl_xor(tc, h, 64);
        swc += __shfl_xor(swc, h, 64);
        gsc += __shfl_xor(gsc, h, 64);
        skc += __shfl_xor(skc, h, 64);
    }
    if ((t & 63) == 0) {
        smx[t >> 6] = mx;
        scnt[t >> 6] = tc;
        scnt[NW + (t >> 6)] = swc;
        scnt[2 * NW + (t >> 6)] = gsc;
        scnt[3 * NW + (t >> 6)] = skc;
    }
    __syncthreads();
    if (t == 0) {
        double M = smx[0];
        unsigned long long tt = scnt[0], sw = scnt[NW], gg = scnt[2 * NW], sk = scnt[3 * NW];
        for (int w = 1; w < NW; ++w) {
            M = fmax(M, smx[w]);
            tt += scnt[w];
            sw += scnt[NW + w];
            gg += scnt[2 * NW + w];
            sk += scnt[3 * NW + w];
        }
        const T Mt = (T)bits2d(Mt_bits);
        const bool rescale = (d.cplx ? SvdFp<T>::round_cplx : SvdFp<T>::round_real) - getexp(Mt) < 0;
        const int sp = rescale ? (d.lgbound - getexp(Mt) - 1) : 0;
        const T Mt2 = rescale ? scal2(Mt, sp) : Mt;
        Mt_bits = d2bits((double)fmax(Mt2, (T)M));
        sc->Mt_bits = Mt_bits;
        sc->T = T0 + (long long)tt;
        sc->SW = SW0 + (long long)sw;
        sc->GS = GS0 + (long long)gg;
        sc->skipped = SK0 + (long long)sk;
        sc->last_t = (long long)tt;
        if (rescale) {
            sc->s = s0 + sp;
            sc->rescaled = resc0 + 1;
        }
        sc->k = k0 + 1;
    }
    return Mt_bits;   // the new M~ in thread 0
}

// The max-norm of a step's rotated columns enters the next step's
// rescaling check only through its exponent.  Every workgroup that rotates
// adds the key (k << 12) | (floor(lg mx) + 1075) to its step's slot with an
// atomic max (exact and order-free); a key of an earlier step (smaller k, or
// the zero a load leaves) means that no pair was rotated in step k.
constexpr int kNoExp = -(1 << 20);

__device__ __forceinline__ void step_max_add(unsigned long long *key, long long k, int e)
{
    const unsigned long long v = ((unsigned long long)k << 12) | (unsigned long long)(e + 1075);
    (void)__hip_atomic_fetch_max(key, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int step_max_exp(unsigned long long key, long long k)
{
    return (key >> 12) == (unsigned long long)k ? (int)(key & 0xFFF) - 1075 : kNoExp;
}

} // namespace jsvd
