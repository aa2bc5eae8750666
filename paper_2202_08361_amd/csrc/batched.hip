// batched.hip -- many independent SVDs of uneven sizes in persistent
// launches (the batched form of Alg. zvjsvd, arXiv:2202.08361).
//
// One workgroup of NT threads owns one matrix at a time and runs its whole
// SVD: initial scaling, sweeps of round-robin steps, the convergence test and
// the finalisation.  Within a step each wavefront takes pivot pairs (one pair
// per wavefront at a time, the same canonical sums as every other launch
// shape, so each matrix's result is bit-for-bit the one jsvd_gesvj gives); a
// workgroup barrier separates the steps, so no step ever needs the host or a
// grid-wide synchronisation.  G and V are iterated in place in the caller's
// buffers; the final sort is an in-place cycle permutation through LDS.
//
// The matrices are grouped by class (real or complex, rows per lane R): each
// class runs as its own kernel instance, with registers and LDS sized for its
// largest matrix, so that small matrices run at high occupancy.  Per class a
// persistent grid (as many workgroups as fit on the GPU) pulls matrices from
// an atomic queue ordered by decreasing cost, which balances the uneven
// sizes.  The workgroup size of a class is chosen by measurement (batch_tune)
// and cached for the process.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/jsvd.h"
#include "evd2_core.hpp"
#include "batch.hpp"
#include "kernels.hpp"
#include "pair.hpp"
#include "state.hpp"

namespace jsvd {

constexpr int kBMaxN = 512;        // largest n of the batched kernel
constexpr int kBMaxRowsR = 512;    // largest m (real)
constexpr int kBMaxRowsC = 512;    // largest m (complex)

struct BatchCtl {
    unsigned int next;
    int count;
    int max_sweeps;
    int nosort;
    int nogs;
};

// LDS of a workgroup of NT threads on matrices of class R (n <= m <= 64 R)
template <int R, int NT>
struct BatchSmem {
    static constexpr int MM = 64 * R;
    static constexpr int NN = MM < kBMaxN ? MM : kBMaxN;
    static constexpr int NW = NT / 64;
    double e[NN], f[NN];
    int rank[NN], inv[NN];   // the final sort; rank holds each column's last-change step before it
    double tmp[2 * (MM + NN)];
    double wM[NW];
    unsigned long long wt[NW], wsw[NW];
    double red[NW];
    int item;
};

// block-wide max of a non-negative value (exact)
template <int NW>
__device__ __forceinline__ double block_max(double x, double *red)
{
    x = wave_max(x);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r = fmax(r, red[w]);
    __syncthreads();
    return r;
}

// canonical column norm by one wavefront (rows lane + 64 j)
template <bool CPLX, int R>
__device__ __forceinline__ Norm wave_colnorm(const double *xr, const double *xi, int m)
{
    using LS = LaneShape<64, R>;
    constexpr int V = LS::V, NL = LS::NL, CH = LS::CH;
    const int lane = threadIdx.x & 63;
    double vr[R], vi[R];
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = lane + 64 * j;
        vr[j] = i < m ? xr[i] : 0.0;
        vi[j] = (CPLX && i < m) ? xi[i] : 0.0;
        mx = fmax(mx, fabs(vr[j]));
        if (CPLX) mx = fmax(mx, fabs(vi[j]));
    }
    mx = wave_max(mx);
    Norm o;
    if (mx == 0.0) {
        o.zero = 1;
        o.e = 0;
        o.f = 1.0;
        return o;
    }
    const int E = getexp(mx);
    double ar[NL], ai[NL];
#pragma unroll
    for (int v = 0; v < NL; ++v) {
        ar[v] = 0.0;
        ai[v] = 0.0;
    }
#pragma unroll
    for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int v = 0; v < NL; ++v) {
            const int j = ch * V + v;
            if (j < R) {
                const double y = scal2(vr[j], -E);
                ar[v] = fma(y, y, ar[v]);
                if (CPLX) {
                    const double z = scal2(vi[j], -E);
                    ai[v] = fma(z, z, ai[v]);
                }
            }
        }
    const double sr = wave_tree_sum(thread_tree<V>(ar));
    const double si = CPLX ? wave_tree_sum(thread_tree<V>(ai)) : 0.0;
    o = norm_from_sums(E, sr, si, CPLX);
    return o;
}

template <bool CPLX, int R, bool COMP, int NT>
__device__ void svd_workgroup(BatchItem &it, int max_sweeps, int nosort, int nogs, BatchSmem<R, NT> &sm)
{
    constexpr int kBT = NT, kBWaves = NT / 64;
    const int m = it.m, n = it.n;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long long ldg = it.ldg, ldv = it.ldv;
    double *const Gr = it.Gr;
    double *const Gi = it.Gi;
    double *const Vr = it.Vr;
    double *const Vi = it.Vi;

    // ---- M~_0 (NaN counted as Inf), s_0 = s_[0], G_1 = 2^{s_0} G, V_1 = I
    double mx = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = tid; i < m; i += kBT) {
            mx = fmax(mx, fmin(fabs(Gr[(size_t)j * ldg + i]), INFINITY));
            if (CPLX) mx = fmax(mx, fmin(fabs(Gi[(size_t)j * ldg + i]), INFINITY));
        }
    const double M0 = block_max<kBWaves>(mx, sm.red);
    if (!(M0 <= 1.79769313486231570815e308) || M0 == 0.0) {
        if (tid == 0) {
            it.status = (M0 == 0.0) ? JSVD_EZERO : JSVD_ENONFINITE;
            it.sweeps = 0;
            it.transformations = 0;
        }
        return;
    }
    int s = it.lgbound - getexp(M0) - 1;
    for (int j = 0; j < n; ++j) {
        for (int i = tid; i < m; i += kBT) {
            Gr[(size_t)j * ldg + i] = scal2(Gr[(size_t)j * ldg + i], s);
            if (CPLX) Gi[(size_t)j * ldg + i] = scal2(Gi[(size_t)j * ldg + i], s);
        }
        for (int i = tid; i < n; i += kBT) {
            Vr[(size_t)j * ldv + i] = (i == j) ? 1.0 : 0.0;
            if (CPLX) Vi[(size_t)j * ldv + i] = 0.0;
        }
    }
    double Mt = scal2(M0, s);
    // per column, the step that last changed it (sm.rank, free until the
    // finalisation): the scaling above counts as a change at step 0
    for (int j = tid; j < n; j += kBT) sm.rank[j] = 0;
    __syncthreads();

    const int N = n + (n & 1), K = N - 1, npairs = N / 2;
    int C = 0;
    bool converged = false;
    long long k = 0, Tall = 0;
    for (;;) {
        long long T = 0, SW = 0;
        for (int kk = 0; kk < K; ++kk, ++k) {
            const int sr = (CPLX ? 1020 : 1022) - getexp(Mt);
            const bool rescale = sr < 0;
            const int sp = rescale ? (it.lgbound - getexp(Mt) - 1) : 0;
            double Mw = 0.0;
            unsigned long long tw = 0, sww = 0;
            for (int l = wv; l < npairs; l += kBWaves) {
                int p, q;
                const bool valid = rr_pair(n, k, l, &p, &q);
                double *const Gpr = Gr + (size_t)p * ldg;
                double *const Gpi = CPLX ? Gi + (size_t)p * ldg : nullptr;
                if (!valid) {
                    if (rescale) {
                        for (int i = lane; i < m; i += 64) {
                            Gpr[i] = scal2(Gpr[i], sp);
                            if (CPLX) Gpi[i] = scal2(Gpi[i], sp);
                        }
                        if (lane == 0) sm.rank[p] = (int)k;
                    }
                    continue;
                }
                // both columns unchanged since the pair last met, one sweep
                // ago: that meeting's outcome (no change) holds, nothing to read
                if (!rescale && sm.rank[p] < k - K && sm.rank[q] < k - K) continue;
                double *const Gqr = Gr + (size_t)q * ldg;
                double *const Gqi = CPLX ? Gi + (size_t)q * ldg : nullptr;
                double xr[2][R], xi[2][R];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int i = lane + 64 * j;
                    const bool in = i < m;
                    xr[0][j] = in ? Gpr[i] : 0.0;
                    xr[1][j] = in ? Gqr[i] : 0.0;
                    xi[0][j] = (CPLX && in) ? Gpi[i] : 0.0;
                    xi[1][j] = (CPLX && in) ? Gqi[i] : 0.0;
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
                const PairDecision dc = pair_core<CPLX, 64, R, COMP>(xr, xi, it.ups, nosort, nogs, (double *)nullptr,
                                                                     (double *)nullptr, (double *)nullptr);
                const int pbit = dc.pbit;
                double *const Dp_r = pbit ? Gqr : Gpr;
                double *const Dq_r = pbit ? Gpr : Gqr;
                double *const Dp_i = pbit ? Gqi : Gpi;
                double *const Dq_i = pbit ? Gpi : Gqi;
                if (dc.transform) {
                    Mw = fmax(Mw, transform_regs<CPLX, R>(xr, xi, dc));
                    ++tw;
                }
                if (dc.transform || pbit || rescale) {
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const int i = lane + 64 * j;
                        if (i < m) {
                            Dp_r[i] = xr[0][j];
                            Dq_r[i] = xr[1][j];
                            if (CPLX) {
                                Dp_i[i] = xi[0][j];
                                Dq_i[i] = xi[1][j];
                            }
                        }
                    }
                    if (lane == 0) {
                        sm.rank[p] = (int)k;
                        sm.rank[q] = (int)k;
                    }
                }
                if (dc.transform || pbit) {
                    double *const Vpr = Vr + (size_t)p * ldv;
                    double *const Vqr = Vr + (size_t)q * ldv;
                    double *const Vpi = CPLX ? Vi + (size_t)p * ldv : nullptr;
                    double *const Vqi = CPLX ? Vi + (size_t)q * ldv : nullptr;
                    double vr[2][R], vi[2][R];
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const int i = lane + 64 * j;
                        const bool in = i < n;
                        vr[0][j] = in ? Vpr[i] : 0.0;
                        vr[1][j] = in ? Vqr[i] : 0.0;
                        vi[0][j] = (CPLX && in) ? Vpi[i] : 0.0;
                        vi[1][j] = (CPLX && in) ? Vqi[i] : 0.0;
                    }
                    if (dc.transform) (void)rot_regs<CPLX, R>(vr, vi, dc.c, dc.C, dc.S);
                    else ++sww;
                    double *const Ep_r = pbit ? Vqr : Vpr;
                    double *const Eq_r = pbit ? Vpr : Vqr;
                    double *const Ep_i = pbit ? Vqi : Vpi;
                    double *const Eq_i = pbit ? Vpi : Vqi;
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const int i = lane + 64 * j;
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
            // step end: fold the wavefronts' counts and max (exact, order-free);
            // the max-norm first over the lanes of each wavefront
            Mw = wave_max(Mw);
            if (lane == 0) {
                sm.wM[wv] = Mw;
                sm.wt[wv] = tw;
                sm.wsw[wv] = sww;
            }
            __syncthreads();
            double Ms = 0.0;
            unsigned long long ts = 0, sws = 0;
#pragma unroll
            for (int w = 0; w < kBWaves; ++w) {
                Ms = fmax(Ms, sm.wM[w]);
                ts += sm.wt[w];
                sws += sm.wsw[w];
            }
            __syncthreads();
            if (rescale) {
                Mt = scal2(Mt, sp);
                s += sp;
            }
            Mt = fmax(Mt, Ms);
            T += (long long)ts;
            SW += (long long)sws;
        }
        Tall += T;
        if (T == 0 && SW == 0) {
            converged = true;
            break;
        }
        ++C;
        if (C >= max_sweeps) break;
    }

    // ---- finalisation: norms of all columns
    for (int j = wv; j < n; j += kBWaves) {
        const Norm nn = wave_colnorm<CPLX, R>(Gr + (size_t)j * ldg, CPLX ? Gi + (size_t)j * ldg : nullptr, m);
        if (lane == 0) {
            sm.e[j] = nn.zero ? -INFINITY : (double)nn.e;
            sm.f[j] = nn.zero ? 1.0 : nn.f;
        }
    }
    __syncthreads();
    if (!converged) {
        for (int j = tid; j < n; j += kBT) {
            const bool zero = isinf(sm.e[j]);
            it.sv_e[j] = zero ? -INFINITY : sm.e[j] - (double)s;
            it.sv_f[j] = sm.f[j];
        }
        if (tid == 0) {
            it.status = JSVD_NOT_CONVERGED;
            it.sweeps = C;
            it.transformations = Tall;
        }
        return;
    }
    // stable descending rank of sigma_j = (e_j, f_j); output column r = input inv[r]
    for (int j = tid; j < n; j += kBT) {
        const double ej = sm.e[j], fj = sm.f[j];
        int r = 0;
        for (int i = 0; i < n; ++i) {
            const double ei = sm.e[i], fi = sm.f[i];
            r += ((ei > ej || (ei == ej && fi > fj)) || ((ei == ej && fi == fj) && i < j)) ? 1 : 0;
        }
        sm.rank[j] = r;
        sm.inv[r] = j;
    }
    __syncthreads();
    for (int r = tid; r < n; r += kBT) {
        const int j = sm.inv[r];
        const bool zero = isinf(sm.e[j]);
        it.sv_e[r] = zero ? -INFINITY : sm.e[j] - (double)s;
        it.sv_f[r] = sm.f[j];
    }
    // in place: output column r <- normalised input column inv[r], following cycles
    for (int r0 = 0; r0 < n; ++r0) {
        // a cycle is handled from its smallest position
        int x = sm.inv[r0];
        bool smallest = true;
        while (x != r0) {
            if (x < r0) {
                smallest = false;
                break;
            }
            x = sm.inv[x];
        }
        if (!smallest) continue;
        if (sm.inv[r0] == r0) {
            // fixed point: normalise in place
            const int j = r0;
            const bool zero = isinf(sm.e[j]);
            const int E = zero ? 0 : (int)sm.e[j];
            const double f = sm.f[j];
            for (int i = tid; i < m; i += kBT) {
                Gr[(size_t)j * ldg + i] = zero ? 0.0 : scal2(Gr[(size_t)j * ldg + i], -E) / f;
                if (CPLX) Gi[(size_t)j * ldg + i] = zero ? 0.0 : scal2(Gi[(size_t)j * ldg + i], -E) / f;
            }
            continue;
        }
        // save input column r0 (goes to position rank[r0])
        for (int i = tid; i < m; i += kBT) {
            sm.tmp[i] = Gr[(size_t)r0 * ldg + i];
            if (CPLX) sm.tmp[m + i] = Gi[(size_t)r0 * ldg + i];
        }
        for (int i = tid; i < n; i += kBT) {
            sm.tmp[2 * m + i] = Vr[(size_t)r0 * ldv + i];
            if (CPLX) sm.tmp[2 * m + n + i] = Vi[(size_t)r0 * ldv + i];
        }
        __syncthreads();
        int pos = r0;
        for (;;) {
            const int src = sm.inv[pos];
            if (src == r0) break;
            const bool zero = isinf(sm.e[src]);
            const int E = zero ? 0 : (int)sm.e[src];
            const double f = sm.f[src];
            for (int i = tid; i < m; i += kBT) {
                Gr[(size_t)pos * ldg + i] = zero ? 0.0 : scal2(Gr[(size_t)src * ldg + i], -E) / f;
                if (CPLX) Gi[(size_t)pos * ldg + i] = zero ? 0.0 : scal2(Gi[(size_t)src * ldg + i], -E) / f;
            }
            for (int i = tid; i < n; i += kBT) {
                Vr[(size_t)pos * ldv + i] = Vr[(size_t)src * ldv + i];
                if (CPLX) Vi[(size_t)pos * ldv + i] = Vi[(size_t)src * ldv + i];
            }
            __syncthreads();
            pos = src;
        }
        {
            const bool zero = isinf(sm.e[r0]);
            const int E = zero ? 0 : (int)sm.e[r0];
            const double f = sm.f[r0];
            for (int i = tid; i < m; i += kBT) {
                Gr[(size_t)pos * ldg + i] = zero ? 0.0 : scal2(sm.tmp[i], -E) / f;
                if (CPLX) Gi[(size_t)pos * ldg + i] = zero ? 0.0 : scal2(sm.tmp[m + i], -E) / f;
            }
            for (int i = tid; i < n; i += kBT) {
                Vr[(size_t)pos * ldv + i] = sm.tmp[2 * m + i];
                if (CPLX) Vi[(size_t)pos * ldv + i] = sm.tmp[2 * m + n + i];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        it.status = JSVD_OK;
        it.sweeps = C;
        it.transformations = Tall;
    }
}

// the matrices of one class (CPLX, R), NT threads per matrix.  DENSE: the
// instance compiled for four waves per SIMD (at most 128 VGPRs, a few spills
// in the phases that need more), else the compiler's own register budget.
template <bool COMP, bool CPLX, int R, int NT, bool DENSE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(DENSE ? 4 : (NT >= 512 ? 2 : 1)))) void
batched_kernel(BatchItem *items, const int *order, BatchCtl *ctl)
{
    __shared__ BatchSmem<R, NT> sm;
    const int count = ctl->count;
    for (;;) {
        if (threadIdx.x == 0) sm.item = (int)atomicAdd(&ctl->next, 1u);
        __syncthreads();
        const int idx = sm.item;
        __syncthreads();
        if (idx >= count) return;
        BatchItem it = items[order[idx]];
        svd_workgroup<CPLX, R, COMP, NT>(it, ctl->max_sweeps, ctl->nosort, ctl->nogs, sm);
        if (threadIdx.x == 0) {
            items[order[idx]].status = it.status;
            items[order[idx]].sweeps = it.sweeps;
            items[order[idx]].transformations = it.transformations;
        }
        __syncthreads();
    }
}

// rows per lane class of the batched kernel (0: use the plain path)
int batch_rows(int m, int n, int cplx)
{
    if (n > kBMaxN || m > (cplx ? kBMaxRowsC : kBMaxRowsR)) return 0;
    const int R = (m + 63) / 64;
    int r = 1;
    while (r < R) r *= 2;
    return r;
}

int lg_bound_b(int m, int cplx)
{
    int a = 0;
    while ((2LL << a) <= (long long)m) ++a;
    if (!cplx) return 1022 - a;
    const unsigned long long mm = (unsigned long long)m * (unsigned long long)m;
    return 1021 - a - (mm > (1ULL << (2 * a + 1)) ? 1 : 0);
}

BatchItem make_batch_item(int m, int n, int cplx, double *Gr, double *Gi, size_t ldg, double *Vr, double *Vi,
                          size_t ldv, double *sv_e, double *sv_f)
{
    BatchItem it;
    memset(&it, 0, sizeof(it));
    it.m = m;
    it.n = n;
    it.cplx = cplx;
    it.R = batch_rows(m, n, cplx);
    it.Gr = Gr;
    it.Gi = cplx ? Gi : nullptr;
    it.ldg = (long long)ldg;
    it.Vr = Vr;
    it.Vi = cplx ? Vi : nullptr;
    it.ldv = (long long)ldv;
    it.sv_e = sv_e;
    it.sv_f = sv_f;
    it.lgbound = lg_bound_b(m, cplx);
    it.ups = ldexp(sqrt((double)m), -53);
    it.status = JSVD_EDEVICE;
    return it;
}

// ---------------------------------------------------------------------------
// classes, launch schedules and the autotuner
//
// A class's schedule: threads per matrix NT (one pivot pair per wavefront
// at a time, so NT/64 pairs of a matrix in flight), the register budget of
// the instance (dense: four waves per SIMD), and the workgroups per CU of the
// persistent grid (0: as many as fit; fewer keeps fewer matrices in flight,
// whose columns then stay in the caches).  Every schedule gives the same bits.

constexpr int kNumNT = 3;
constexpr int kNTs[kNumNT] = {128, 256, 512};   // threads per matrix tried

static int class_index(int cplx, int R)
{
    const int r = R <= 1 ? 0 : R <= 2 ? 1 : R <= 4 ? 2 : 3;
    return (cplx ? 4 : 0) + r;
}

// packed schedule: nt | dense << 10 | wpc << 11 (0: none)
static int sched_pack(const BatchSched &b) { return b.nt | (b.dense ? 1 << 10 : 0) | (b.wpc << 11); }
static BatchSched sched_unpack(int v) { return BatchSched{v & 1023, (v >> 10) & 1, v >> 11}; }

template <bool COMP, bool CPLX, int R>
static const void *class_kernel_r(int NT, bool dense)
{
    switch (NT) {
    case 128:
        return dense ? (const void *)batched_kernel<COMP, CPLX, R, 128, true>
                     : (const void *)batched_kernel<COMP, CPLX, R, 128, false>;
    case 256:
        return dense ? (const void *)batched_kernel<COMP, CPLX, R, 256, true>
                     : (const void *)batched_kernel<COMP, CPLX, R, 256, false>;
    case 512:
        return dense ? (const void *)batched_kernel<COMP, CPLX, R, 512, true>
                     : (const void *)batched_kernel<COMP, CPLX, R, 512, false>;
    default: return nullptr;
    }
}

template <bool COMP, bool CPLX>
static const void *class_kernel_c(int R, int NT, bool dense)
{
    switch (R) {
    case 1: return class_kernel_r<COMP, CPLX, 1>(NT, dense);
    case 2: return class_kernel_r<COMP, CPLX, 2>(NT, dense);
    case 4: return class_kernel_r<COMP, CPLX, 4>(NT, dense);
    case 8: return class_kernel_r<COMP, CPLX, 8>(NT, dense);
    default: return nullptr;
    }
}

// the kernel instance of a class and schedule (nullptr: no such instance)
static const void *class_kernel_of(bool comp, int cplx, int R, int NT, bool dense)
{
    if (comp) return cplx ? class_kernel_c<true, true>(R, NT, dense) : class_kernel_c<true, false>(R, NT, dense);
    return cplx ? class_kernel_c<false, true>(R, NT, dense) : class_kernel_c<false, false>(R, NT, dense);
}

// workgroups of an instance that fit on one CU (at least 1)
static int class_per_cu(const void *fn, int NT)
{
    int per_cu = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return per_cu;
}

// registers per lane of an instance (0 if unknown)
static int class_regs(const void *fn)
{
    hipFuncAttributes a;
    if (!fn || hipFuncGetAttributes(&a, fn) != hipSuccess) return 0;
    return a.numRegs;
}

// one persistent launch over the `count` matrices of class (cplx, R) listed
// (longest first) in order
static hipError_t launch_class(bool comp, int cplx, int R, const BatchSched &sc, BatchItem *items, const int *order,
                               BatchCtl *ctl, int count, int ncu, hipStream_t s)
{
    const void *fn = class_kernel_of(comp, cplx, R, sc.nt, sc.dense != 0);
    if (!fn) return hipErrorInvalidValue;
    const int per_cu = class_per_cu(fn, sc.nt);
    const int wpc = sc.wpc > 0 ? std::min(sc.wpc, per_cu) : per_cu;
    const int grid = std::min(count, wpc * ncu);
    void *args[] = {(void *)&items, (void *)&order, (void *)&ctl};
    return hipLaunchKernel(fn, dim3(grid), dim3(sc.nt), args, 0, s);
}

// the tuner's results per (device, compensated, class), packed; 0 = not
// measured yet.  A forced schedule (jsvd_batched_set_schedule) overrides.
constexpr int kMaxDev = 64;
static std::mutex g_tune_mu;
static int g_tuned[kMaxDev][2][8];
static int g_forced = 0;
static unsigned g_tuning = JSVD_TUNE_DENSE | JSVD_TUNE_WGS;

// fill a sample matrix with values in [-1, 1) from a counter hash
__global__ void batch_fill_kernel(double *x, size_t count, unsigned long long seed)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        x[i] = (double)(z >> 11) * 0x1p-52 - 1.0;
    }
}

// The candidate schedules of a class: every NT with the default instance and
// a full grid; with JSVD_TUNE_DENSE the dense instance where the default one
// takes more than 128 registers; with JSVD_TUNE_WGS also half, 2 and 1
// workgroups per CU (each below the most that fit).
static std::vector<BatchSched> class_candidates(bool comp, int cplx, int R, unsigned tuning)
{
    std::vector<BatchSched> cand;
    for (int ci = 0; ci < kNumNT; ++ci) {
        for (int dense = 0; dense < 2; ++dense) {
            if (dense && (!(tuning & JSVD_TUNE_DENSE) ||
                          class_regs(class_kernel_of(comp, cplx, R, kNTs[ci], false)) <= 128))
                continue;
            const int per_cu = class_per_cu(class_kernel_of(comp, cplx, R, kNTs[ci], dense != 0), kNTs[ci]);
            BatchSched sc{kNTs[ci], dense, 0};
            cand.push_back(sc);
            if (!(tuning & JSVD_TUNE_WGS)) continue;
            for (int w : {per_cu / 2, 2, 1}) {
                bool dup = w < 1 || w >= per_cu;
                for (const BatchSched &o : cand)
                    dup = dup || (o.nt == sc.nt && o.dense == sc.dense && o.wpc == w);
                if (dup) continue;
                sc.wpc = w;
                cand.push_back(sc);
            }
        }
    }
    return cand;
}

// Measure the threads per matrix of one class: one sweep of up to 1024
// sample matrices of the class's median shape (random entries), per
// candidate, after a warm-up; the fastest wins.  Returns 0 on failure.
static int measure_class(bool comp, int cplx, int R, int m, int n, int ncu, unsigned tuning, hipStream_t s)
{
    const int c = cplx ? 2 : 1;
    const size_t per = (size_t)c * ((size_t)m * n + (size_t)n * n) + 2 * (size_t)n;
    size_t S = std::min<size_t>(1024, std::max<size_t>(1, ((size_t)1 << 30) / (per * sizeof(double))));
    const size_t bytes = S * per * sizeof(double) + 4096 + S * (sizeof(BatchItem) + sizeof(int));
    char *mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return 0;
    double *base = (double *)mem;
    std::vector<BatchItem> items(S);
    std::vector<int> order(S);
    for (size_t i = 0; i < S; ++i) {
        double *G = base + i * per;
        double *V = G + (size_t)c * m * n;
        double *e = V + (size_t)c * n * n;
        items[i] = make_batch_item(m, n, cplx, G, cplx ? G + (size_t)m * n : nullptr, m, V,
                                   cplx ? V + (size_t)n * n : nullptr, n, e, e + n);
        order[i] = (int)i;
    }
    char *tail = mem + S * per * sizeof(double);
    BatchItem *ditems = (BatchItem *)tail;
    int *dorder = (int *)(tail + S * sizeof(BatchItem));
    BatchCtl *dctl = (BatchCtl *)(((uintptr_t)(dorder + S) + 255) & ~(uintptr_t)255);
    const std::vector<BatchSched> cand = class_candidates(comp, cplx, R, tuning);
    hipEvent_t a = nullptr, b = nullptr;
    int best = 0;
    float best_ms = 0.f;
    bool ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess &&
              hipMemcpyAsync(dorder, order.data(), sizeof(int) * S, hipMemcpyHostToDevice, s) == hipSuccess;
    for (size_t ci = 0; ok && ci < cand.size(); ++ci) {
        const BatchSched &sc = cand[ci];
        for (int rep = 0; ok && rep < 2; ++rep) {
            // fresh random G (the SVD works in place) and fresh queue
            hipLaunchKernelGGL(batch_fill_kernel, dim3(1024), dim3(256), 0, s, base, S * per, 1234567ull);
            BatchCtl ctl;
            ctl.next = 0;
            ctl.count = (int)S;
            ctl.max_sweeps = 1;
            ctl.nosort = 1;
            ctl.nogs = 0;
            ok = hipGetLastError() == hipSuccess &&
                 hipMemcpyAsync(ditems, items.data(), sizeof(BatchItem) * S, hipMemcpyHostToDevice, s) == hipSuccess &&
                 hipMemcpyAsync(dctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, s) == hipSuccess &&
                 hipEventRecord(a, s) == hipSuccess &&
                 launch_class(comp, cplx, R, sc, ditems, dorder, dctl, (int)S, ncu, s) == hipSuccess &&
                 hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
            float ms = 0.f;
            if (ok && rep == 1 && hipEventElapsedTime(&ms, a, b) == hipSuccess && (best == 0 || ms < best_ms)) {
                best = sched_pack(sc);
                best_ms = ms;
            }
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(s);
    (void)hipFree(mem);
    return ok ? best : 0;
}

static int current_device_ncu(int *dev)
{
    int ncu = 256;
    *dev = 0;
    (void)hipGetDevice(dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, *dev) != hipSuccess || ncu <= 0) ncu = 256;
    return ncu;
}

// Trial schedules of the joint refinement (batch_tune), per class, packed (0:
// none): seen by class_sched on the tuning thread only.
static thread_local int t_trial[8];
static thread_local bool t_trial_on = false;

// the schedule of a class: a trial of the joint refinement, forced, else
// measured (once per process and device), else 256 threads with the default
// instance and grid
static BatchSched class_sched(bool comp, int cplx, int R, int m, int n, hipStream_t s, bool measure)
{
    if (t_trial_on && t_trial[class_index(cplx, R)]) return sched_unpack(t_trial[class_index(cplx, R)]);
    int dev = 0;
    const int ncu = current_device_ncu(&dev);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_forced) return sched_unpack(g_forced);
    int v = 0;
    if (dev >= 0 && dev < kMaxDev) {
        int &t = g_tuned[dev][comp ? 1 : 0][class_index(cplx, R)];
        if (t == 0 && measure) t = measure_class(comp, cplx, R, m, n, ncu, g_tuning, s);
        v = t;
    }
    return sched_unpack(v ? v : 256);
}

// One sweep of the sample, every class side by side on its own stream as in
// a real launch, after refilling the sample's G with random entries; the
// span in milliseconds (negative on failure).
static float sample_span(const std::vector<BatchItem> &sample, unsigned flags, double *buf, size_t nbuf,
                         hipEvent_t a, hipEvent_t b, hipStream_t s)
{
    hipLaunchKernelGGL(batch_fill_kernel, dim3(1024), dim3(256), 0, s, buf, nbuf, 7654321ull);
    if (hipGetLastError() != hipSuccess || hipEventRecord(a, s) != hipSuccess) return -1.f;
    BatchLaunch *bl = batch_launch(sample.data(), (int)sample.size(), 1, flags, s, false);
    if (!bl) return -1.f;
    float ms = -1.f;
    if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess)
        ms = -1.f;
    (void)hipStreamSynchronize(s);
    batch_release(bl);
    return ms;
}

// Measure the schedules of the classes of these items that are not measured
// yet.  First each class alone, threads per matrix only (measure_class).
// Then, when the tuning allows more, a joint refinement: the classes of a
// batch run side by side and share the compute units, so a class's other
// candidates are timed on a sample of this batch's own shapes (every class,
// in the batch's proportions, one sweep), the largest class first, each
// change kept when it shortens the whole sample's span by more than 1 %.
void batch_tune(const BatchItem *items, int cnt, unsigned flags, hipStream_t s)
{
    const bool comp = (flags & JSVD_COMPENSATED) != 0;
    int dev = 0;
    const int ncu = current_device_ncu(&dev);
    if (dev < 0 || dev >= kMaxDev || cnt <= 0) return;
    std::vector<int> by[8];
    double cost[8] = {};
    for (int i = 0; i < cnt; ++i) {
        const int k = class_index(items[i].cplx, items[i].R);
        by[k].push_back(i);
        cost[k] += (items[i].cplx ? 2.0 : 1.0) * items[i].n * (double)items[i].n * (items[i].m + items[i].n);
    }
    std::vector<int> fresh;
    unsigned tuning = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_forced) return;
        tuning = g_tuning;
        for (int k = 0; k < 8; ++k) {
            if (by[k].empty()) continue;
            int &t = g_tuned[dev][comp ? 1 : 0][k];
            if (t) continue;
            std::vector<std::pair<double, int>> sz;
            for (int i : by[k]) sz.push_back({(double)items[i].n * items[i].n * items[i].m, i});
            std::sort(sz.begin(), sz.end());
            const BatchItem &it = items[sz[sz.size() / 2].second];
            t = measure_class(comp, it.cplx, it.R, it.m, it.n, ncu, 0, s);
            if (t) fresh.push_back(k);
        }
    }
    if (fresh.empty() || !(tuning & (JSVD_TUNE_DENSE | JSVD_TUNE_WGS))) return;
    // the sample: evenly spaced members of each class, in the batch's
    // proportions, at most 2048 matrices and 512 MiB of G and V
    double total_bytes = 0.0;
    for (int i = 0; i < cnt; ++i)
        total_bytes += 8.0 * (items[i].cplx ? 2 : 1) * ((double)items[i].m * items[i].n + (double)items[i].n * items[i].n);
    const double frac = std::min(1.0, std::min(2048.0 / cnt, (double)(512u << 20) / total_bytes));
    std::vector<int> pick;
    for (int k = 0; k < 8; ++k) {
        if (by[k].empty()) continue;
        const int want = std::max(1, (int)(frac * by[k].size() + 0.5));
        for (int j = 0; j < want; ++j) pick.push_back(by[k][(size_t)j * by[k].size() / want]);
    }
    size_t nbuf = 0;
    for (int i : pick) {
        const size_t c = items[i].cplx ? 2 : 1;
        nbuf += c * ((size_t)items[i].m * items[i].n + (size_t)items[i].n * items[i].n) + 2 * (size_t)items[i].n;
    }
    double *buf = nullptr;
    if (hipMalloc(&buf, nbuf * sizeof(double)) != hipSuccess) return;
    std::vector<BatchItem> sample;
    size_t off = 0;
    for (int i : pick) {
        const int m = items[i].m, n = items[i].n, c = items[i].cplx;
        double *G = buf + off;
        double *V = G + (size_t)(c ? 2 : 1) * m * n;
        double *e = V + (size_t)(c ? 2 : 1) * n * n;
        sample.push_back(make_batch_item(m, n, c, G, c ? G + (size_t)m * n : nullptr, m, V,
                                         c ? V + (size_t)n * n : nullptr, n, e, e + n));
        off += (size_t)(c ? 2 : 1) * ((size_t)m * n + (size_t)n * n) + 2 * (size_t)n;
    }
    hipEvent_t a = nullptr, b = nullptr;
    bool ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int k = 0; k < 8; ++k) t_trial[k] = g_tuned[dev][comp ? 1 : 0][k];
    }
    t_trial_on = true;
    auto span = [&]() {
        float best = -1.f;
        for (int rep = 0; ok && rep < 2; ++rep) {
            const float ms = sample_span(sample, flags, buf, nbuf, a, b, s);
            if (ms < 0.f) ok = false;
            else if (best < 0.f || ms < best) best = ms;
        }
        return best;
    };
    (void)span();   // warm-up
    float best = span();
    std::sort(fresh.begin(), fresh.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    for (int k : fresh) {
        if (!ok) break;
        const BatchItem &it = items[by[k][0]];
        const int cur = t_trial[k];
        int keep = cur;
        for (const BatchSched &sc : class_candidates(comp, it.cplx, it.R, tuning)) {
            const int v = sched_pack(sc);
            if (v == cur || !ok) continue;
            t_trial[k] = v;
            const float ms = span();
            if (ok && ms > 0.f && ms < 0.99f * best) {
                best = ms;
                keep = v;
            }
        }
        t_trial[k] = keep;
    }
    t_trial_on = false;
    if (ok) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int k : fresh) g_tuned[dev][comp ? 1 : 0][k] = t_trial[k];
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
}

BatchSched batch_sched_of(int m, int n, int cplx, unsigned flags)
{
    const int R = batch_rows(m, n, cplx);
    if (!R) return BatchSched{0, 0, 0};
    return class_sched((flags & JSVD_COMPENSATED) != 0, cplx, R, m, n, nullptr, false);
}

int batch_threads_of(int m, int n, int cplx, unsigned flags) { return batch_sched_of(m, n, cplx, flags).nt; }

int batch_set_sched(int nt, int dense, int wpc)
{
    if (nt != 0 && nt != 128 && nt != 256 && nt != 512) return JSVD_EINVAL;
    if (dense < 0 || dense > 1 || wpc < 0 || wpc > 64) return JSVD_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_forced = nt ? sched_pack(BatchSched{nt, dense, wpc}) : 0;
    return JSVD_OK;
}

int batch_set_threads(int nt) { return batch_set_sched(nt, 0, 0); }

int batch_set_tuning(unsigned what)
{
    if (what & ~(unsigned)(JSVD_TUNE_DENSE | JSVD_TUNE_WGS)) return JSVD_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuning = what;
    memset(g_tuned, 0, sizeof(g_tuned));
    return JSVD_OK;
}

struct BatchLaunch {
    void *dmem;
    BatchItem *host;   // pinned; results land here
    int count;
    int dev;
    int nside;         // class streams checked out of the pool for this launch
    hipStream_t side[8];
};

// Streams of the classes (default priority): the classes of a batch run side
// by side, forked from the caller's stream and joined back into it, so that
// one class's longest matrices overlap the others' instead of adding up.
// Each launch checks its side streams out of a per-device pool and returns
// them once it has completed, so launches in flight at the same time (two
// callers, or two group slots of a server) never queue one's classes behind
// the other's persistent kernels on a shared stream.
static std::mutex g_stream_mu;
static std::vector<hipStream_t> g_stream_pool[kMaxDev];

static bool take_streams(int dev, int k, hipStream_t *out)
{
    if (dev < 0 || dev >= kMaxDev) return false;
    std::lock_guard<std::mutex> lk(g_stream_mu);
    std::vector<hipStream_t> &pool = g_stream_pool[dev];
    int got = 0;
    while (got < k && !pool.empty()) {
        out[got++] = pool.back();
        pool.pop_back();
    }
    while (got < k) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (int i = 0; i < got; ++i) pool.push_back(out[i]);
            return false;
        }
        out[got++] = st;
    }
    return true;
}

static void give_streams(int dev, int k, const hipStream_t *st)
{
    std::lock_guard<std::mutex> lk(g_stream_mu);
    for (int i = 0; i < k; ++i) g_stream_pool[dev].push_back(st[i]);
}

// the launch has completed (its side streams were joined into the caller's
// stream, which has passed the join): its streams go back to the pool
void batch_done(BatchLaunch *bl)
{
    if (!bl || bl->nside == 0) return;
    give_streams(bl->dev, bl->nside, bl->side);
    bl->nside = 0;
}

BatchLaunch *batch_launch(const BatchItem *items, int cnt, int max_sweeps, unsigned flags, hipStream_t s, bool tune)
{
    if (cnt <= 0) return nullptr;
    const bool comp = (flags & JSVD_COMPENSATED) != 0;
    if (tune) batch_tune(items, cnt, flags, s);
    BatchLaunch *bl = new (std::nothrow) BatchLaunch;
    if (!bl) return nullptr;
    bl->count = cnt;
    bl->dmem = nullptr;
    bl->host = nullptr;
    bl->dev = 0;
    bl->nside = 0;
    // per class, longest first: cost ~ c n^2 (m + n) per sweep
    auto cost = [&](int i) {
        return (items[i].cplx ? 2.0 : 1.0) * items[i].n * (double)items[i].n * (items[i].m + items[i].n);
    };
    std::vector<int> order(cnt);
    for (int i = 0; i < cnt; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int ka = class_index(items[a].cplx, items[a].R), kb = class_index(items[b].cplx, items[b].R);
        if (ka != kb) return ka > kb;   // complex before real, larger R first
        return cost(a) > cost(b);
    });
    int first[9], ncls = 0, cls_of[8];
    for (int i = 0; i < cnt; ++i) {
        const int k = class_index(items[order[i]].cplx, items[order[i]].R);
        if (ncls == 0 || cls_of[ncls - 1] != k) {
            cls_of[ncls] = k;
            first[ncls++] = i;
        }
    }
    first[ncls] = cnt;
    const size_t oItems = 0;
    const size_t oOrder = (sizeof(BatchItem) * cnt + 255) & ~(size_t)255;
    const size_t oCtl = oOrder + ((sizeof(int) * cnt + 255) & ~(size_t)255);
    const size_t bytes = oCtl + 256 * (size_t)ncls;
    if (hipMalloc(&bl->dmem, bytes) != hipSuccess) {
        delete bl;
        return nullptr;
    }
    if (hipHostMalloc((void **)&bl->host, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(bl->dmem);
        delete bl;
        return nullptr;
    }
    char *h = (char *)bl->host;
    memcpy(h + oItems, items, sizeof(BatchItem) * cnt);
    memcpy(h + oOrder, order.data(), sizeof(int) * cnt);
    for (int c = 0; c < ncls; ++c) {
        BatchCtl ctl;
        ctl.next = 0;
        ctl.count = first[c + 1] - first[c];
        ctl.max_sweeps = max_sweeps;
        ctl.nosort = iter_nosort(flags);
        ctl.nogs = (flags & JSVD_NO_GS) ? 1 : 0;
        memcpy(h + oCtl + 256 * (size_t)c, &ctl, sizeof(ctl));
    }
    char *dm = (char *)bl->dmem;
    int dev = 0;
    const int ncu = current_device_ncu(&dev);
    bool ok = hipMemcpyAsync(dm, h, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    // the first class on the caller's stream, the others side by side on
    // class streams forked from it (one stream fewer to share the process's
    // hardware queues)
    hipStream_t *cs = bl->side;
    hipEvent_t fork = nullptr, join[8] = {};
    bl->dev = dev;
    const bool side = ncls > 1 && take_streams(dev, ncls - 1, cs);
    if (side) bl->nside = ncls - 1;
    if (side) {
        ok = ok && hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess &&
             hipEventRecord(fork, s) == hipSuccess;
    }
    for (int c = 0; ok && c < ncls; ++c) {
        const BatchItem &it0 = items[order[first[c]]];
        const BatchSched sc = class_sched(comp, it0.cplx, it0.R, it0.m, it0.n, s, false);
        hipStream_t ls = s;
        if (side && c > 0) {
            ls = cs[c - 1];
            ok = hipStreamWaitEvent(ls, fork, 0) == hipSuccess;
        }
        ok = ok && launch_class(comp, it0.cplx, it0.R, sc, (BatchItem *)(dm + oItems),
                                (const int *)(dm + oOrder) + first[c], (BatchCtl *)(dm + oCtl + 256 * (size_t)c),
                                first[c + 1] - first[c], ncu, ls) == hipSuccess;
        if (side && c > 0 && ok) {
            ok = hipEventCreateWithFlags(&join[c], hipEventDisableTiming) == hipSuccess &&
                 hipEventRecord(join[c], ls) == hipSuccess && hipStreamWaitEvent(s, join[c], 0) == hipSuccess;
        }
    }
    if (fork) (void)hipEventDestroy(fork);
    for (int c = 0; c < 8; ++c)
        if (join[c]) (void)hipEventDestroy(join[c]);
    ok = ok && hipMemcpyAsync(bl->host, dm, sizeof(BatchItem) * cnt, hipMemcpyDeviceToHost, s) == hipSuccess;
    if (!ok) {
        // nothing may still use the buffers when they are freed
        (void)hipStreamSynchronize(s);
        for (int c = 0; c < bl->nside; ++c) (void)hipStreamSynchronize(cs[c]);
        batch_release(bl);
        return nullptr;
    }
    return bl;
}

const BatchItem *batch_results(const BatchLaunch *bl) { return bl->host; }

void batch_release(BatchLaunch *bl)
{
    if (!bl) return;
    batch_done(bl);
    if (bl->dmem) (void)hipFree(bl->dmem);
    if (bl->host) (void)hipHostFree(bl->host);
    delete bl;
}

// ---------------------------------------------------------------------------
// The allocation-free batched call: its per-matrix records, the processing
// order and the classes' work-queue counters live in a file-scope device
// array instead of a hipMalloc'ed buffer, staged through file-scope host
// arrays.  Its address is looked up once per device (the array's name is a
// host-side stand-in, not a device address).

constexpr size_t kNaItemsOff = 0;
constexpr size_t kNaOrderOff = (sizeof(BatchItem) * kNoAllocMaxCount + 255) & ~(size_t)255;
constexpr size_t kNaCtlOff = kNaOrderOff + ((sizeof(int) * kNoAllocMaxCount + 255) & ~(size_t)255);
constexpr size_t kNoAllocBytes = kNaCtlOff + 256 * 8;
static_assert(kNoAllocBytes <= 930 * 1024, "the size the header states");

static __device__ __align__(256) char scratch[kNoAllocBytes];

static std::mutex g_na_mu;                 // one call at a time in the process
static char *g_na_dev[kMaxDev];            // the array's address on each device
alignas(256) static char g_na_host[kNoAllocBytes];

// the device address of `scratch` on the current device (looked up on the
// first call on that device); nullptr on failure.  Caller holds g_na_mu.
static char *noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDev) return nullptr;
    if (!g_na_dev[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_na_dev[dev] = (char *)ptr;
    }
    return g_na_dev[dev];
}

// Run the items (all batched shapes, count <= kNoAllocMaxCount) class by
// class on stream s, without allocating; their status and sweeps come back
// in items.  Synchronises.
int batch_run_noalloc(BatchItem *items, int cnt, int max_sweeps, unsigned flags, hipStream_t s)
{
    if (cnt < 0 || cnt > kNoAllocMaxCount) return JSVD_EINVAL;
    if (cnt == 0) return JSVD_OK;
    const bool comp = (flags & JSVD_COMPENSATED) != 0;
    std::lock_guard<std::mutex> lk(g_na_mu);
    int dev = 0;
    const int ncu = current_device_ncu(&dev);
    char *dm = noalloc_scratch(dev);
    if (!dm) return JSVD_EDEVICE;
    BatchItem *hitems = (BatchItem *)(g_na_host + kNaItemsOff);
    int *horder = (int *)(g_na_host + kNaOrderOff);
    memcpy(hitems, items, sizeof(BatchItem) * cnt);
    // per class (complex first, more rows first), longest first; ties by index
    auto cost = [&](int i) {
        return (hitems[i].cplx ? 2.0 : 1.0) * hitems[i].n * (double)hitems[i].n * (hitems[i].m + hitems[i].n);
    };
    for (int i = 0; i < cnt; ++i) horder[i] = i;
    std::sort(horder, horder + cnt, [&](int a, int b) {
        const int ka = class_index(hitems[a].cplx, hitems[a].R), kb = class_index(hitems[b].cplx, hitems[b].R);
        if (ka != kb) return ka > kb;
        const double ca = cost(a), cb = cost(b);
        if (ca != cb) return ca > cb;
        return a < b;
    });
    int first[9], ncls = 0, cls_of[8];
    for (int i = 0; i < cnt; ++i) {
        const int k = class_index(hitems[horder[i]].cplx, hitems[horder[i]].R);
        if (ncls == 0 || cls_of[ncls - 1] != k) {
            cls_of[ncls] = k;
            first[ncls++] = i;
        }
    }
    first[ncls] = cnt;
    for (int c = 0; c < ncls; ++c) {
        BatchCtl ctl;
        memset(&ctl, 0, sizeof(ctl));
        ctl.next = 0;   // the class's work queue starts at zero on every call
        ctl.count = first[c + 1] - first[c];
        ctl.max_sweeps = max_sweeps;
        ctl.nosort = iter_nosort(flags);
        ctl.nogs = (flags & JSVD_NO_GS) ? 1 : 0;
        memcpy(g_na_host + kNaCtlOff + 256 * (size_t)c, &ctl, sizeof(ctl));
    }
    bool ok = hipMemcpyAsync(dm + kNaItemsOff, hitems, sizeof(BatchItem) * cnt, hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemcpyAsync(dm + kNaOrderOff, horder, sizeof(int) * cnt, hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync(dm + kNaCtlOff, g_na_host + kNaCtlOff, 256 * (size_t)ncls, hipMemcpyHostToDevice, s) ==
                  hipSuccess;
    // the classes one after another on the caller's stream (no class streams:
    // creating one may allocate)
    for (int c = 0; ok && c < ncls; ++c) {
        const BatchItem &it0 = hitems[horder[first[c]]];
        const BatchSched sc = class_sched(comp, it0.cplx, it0.R, it0.m, it0.n, s, false);
        ok = launch_class(comp, it0.cplx, it0.R, sc, (BatchItem *)(dm + kNaItemsOff),
                          (const int *)(dm + kNaOrderOff) + first[c], (BatchCtl *)(dm + kNaCtlOff + 256 * (size_t)c),
                          first[c + 1] - first[c], ncu, s) == hipSuccess;
    }
    ok = ok && hipMemcpyAsync(hitems, dm + kNaItemsOff, sizeof(BatchItem) * cnt, hipMemcpyDeviceToHost, s) ==
                   hipSuccess;
    ok = (hipStreamSynchronize(s) == hipSuccess) && ok;
    if (!ok) return JSVD_EDEVICE;
    for (int i = 0; i < cnt; ++i) {
        items[i].status = hitems[i].status;
        items[i].sweeps = hitems[i].sweeps;
        items[i].transformations = hitems[i].transformations;
    }
    return JSVD_OK;
}

} // namespace jsvd

using namespace jsvd;

namespace {

// Matrices of a batch outside the batched kernel's tile (more than 512 rows):
// each on a state of its own, up to kPlainRuns of them at once on streams of
// the pool, side by side with the batched launch on the caller's stream.  A
// sweep is enqueued as soon as the previous one is seen done (one sweep is a
// captured graph of K steps, and every step spreads its pairs over the whole
// GPU; a second and third matrix fill the gaps between one's steps and
// sweeps).  Each matrix goes through the same load, sweeps and finalisation
// as jsvd_gesvj, so its result is the same bits.
constexpr int kPlainRuns = 4;

struct PlainRun {
    jsvd_state st = nullptr;
    hipEvent_t ev = nullptr;
    int idx = -1;        // matrix of the batch, -1 = free
    int finishing = 0;   // 0 sweeping, 1 converged output enqueued, 2 output after the sweep limit
};

struct PlainBatch {
    const int *m, *n, *is_complex;
    double *const *G_re, *const *G_im;
    const size_t *ldg;
    double *const *V_re, *const *V_im;
    const size_t *ldv;
    double *const *sv_e, *const *sv_f;
    int max_sweeps;
    unsigned flags;
    int *sweeps, *status;
    int64_t *transformations;
};

// start matrix i on run r (its stream waits for `ready`, the caller's inputs)
int plain_start(const PlainBatch &b, int i, PlainRun &r, hipStream_t st, hipEvent_t ready)
{
    const int c = b.is_complex ? (b.is_complex[i] != 0) : 0;
    r.idx = i;
    r.finishing = 0;
    int rc = jsvd_state_create(b.m[i], b.n[i], c, &r.st);
    if (rc != JSVD_OK) return rc;
    r.st->max_sweeps = b.max_sweeps;
    rc = state_set_flags(r.st, b.flags);
    if (rc == JSVD_OK && hipStreamWaitEvent(st, ready, 0) != hipSuccess) rc = JSVD_EDEVICE;
    if (rc == JSVD_OK) rc = state_load_async(r.st, b.G_re[i], c ? b.G_im[i] : nullptr, b.ldg[i], st);
    if (rc == JSVD_OK) rc = state_sweep_async(r.st, st);
    if (rc == JSVD_OK && hipEventRecord(r.ev, st) != hipSuccess) rc = JSVD_EDEVICE;
    return rc;
}

// advance run r if its stream has passed the last recorded point; returns
// whether anything happened, and sets *done_status once the matrix is done
bool plain_service(const PlainBatch &b, PlainRun &r, hipStream_t st, int *done_status, int *done_sweeps)
{
    constexpr int kRunning = 1 << 20;
    *done_status = kRunning;
    const hipError_t q = hipEventQuery(r.ev);
    if (q == hipErrorNotReady) return false;
    const int i = r.idx;
    const int c = b.is_complex ? (b.is_complex[i] != 0) : 0;
    if (q != hipSuccess) {
        *done_status = JSVD_EDEVICE;
    } else if (!r.finishing) {
        const DevScalars &h = state_staged(r.st);
        *done_sweeps = (int)h.C;
        if (!h.stop) {
            if (state_sweep_async(r.st, st) != JSVD_OK || hipEventRecord(r.ev, st) != hipSuccess)
                *done_status = JSVD_EDEVICE;
        } else if (h.status != 0) {
            *done_status = h.status;
        } else {
            r.finishing = h.converged ? 1 : 2;
            if (state_finish_async(r.st, h.converged != 0, b.G_re[i], c ? b.G_im[i] : nullptr, b.ldg[i], b.V_re[i],
                                   c ? b.V_im[i] : nullptr, b.ldv[i], b.sv_e[i], b.sv_f[i], (double *)nullptr,
                                   st) != JSVD_OK ||
                hipEventRecord(r.ev, st) != hipSuccess)
                *done_status = JSVD_EDEVICE;
        }
    } else {
        *done_status = r.finishing == 1 ? JSVD_OK : JSVD_NOT_CONVERGED;
        *done_sweeps = (int)state_staged(r.st).C;
    }
    return true;
}

// every matrix of `list`, at most kPlainRuns at once and at most half the
// free device memory in states (one at a time beyond that); blocks until all
// are done; returns the first negative status
int plain_concurrent(const PlainBatch &b, const std::vector<int> &list, hipStream_t caller)
{
    if (list.empty()) return JSVD_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return JSVD_EDEVICE;
    const int k = std::min<int>(kPlainRuns, (int)list.size());
    hipStream_t streams[kPlainRuns];
    if (!take_streams(dev, k, streams)) return JSVD_EDEVICE;
    PlainRun runs[kPlainRuns];
    hipEvent_t ready = nullptr;
    bool ok = hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess &&
              hipEventRecord(ready, caller) == hipSuccess;
    for (int j = 0; j < k && ok; ++j)
        ok = hipEventCreateWithFlags(&runs[j].ev, hipEventDisableTiming) == hipSuccess;
    size_t free_b = 0, total_b = 0;
    if (ok && hipMemGetInfo(&free_b, &total_b) != hipSuccess) ok = false;
    const size_t budget = free_b / 2;
    int rc_all = JSVD_OK;
    size_t next = 0, in_use = 0;
    int active = 0;
    auto finish = [&](PlainRun &r, hipStream_t st, int status, int sw) {
        (void)hipStreamSynchronize(st);
        in_use -= state_bytes(r.st->m, r.st->n, r.st->cplx);
        jsvd_state_destroy(r.st);
        r.st = nullptr;
        b.status[r.idx] = status;
        if (b.sweeps) b.sweeps[r.idx] = sw;
        if (b.transformations) b.transformations[r.idx] = -1;   // not counted on this path
        if (status < 0 && rc_all == JSVD_OK) rc_all = status;
        r.idx = -1;
        --active;
    };
    if (!ok) {
        for (int i : list) b.status[i] = JSVD_EDEVICE;
        rc_all = JSVD_EDEVICE;
        next = list.size();
    }
    while (next < list.size() || active > 0) {
        bool progressed = false;
        for (int j = 0; j < k; ++j) {
            PlainRun &r = runs[j];
            if (r.idx < 0) {
                if (next >= list.size()) continue;
                const int i = list[next];
                const size_t fp = state_bytes(b.m[i], b.n[i], b.is_complex ? (b.is_complex[i] != 0) : 0);
                if (active > 0 && in_use + fp > budget) continue;
                ++next;
                ++active;
                progressed = true;
                const int rc = plain_start(b, i, r, streams[j], ready);
                if (r.st) in_use += fp;
                if (rc != JSVD_OK) {
                    if (r.st) {
                        finish(r, streams[j], rc, 0);
                    } else {
                        b.status[i] = rc;
                        if (b.sweeps) b.sweeps[i] = 0;
                        if (b.transformations) b.transformations[i] = -1;
                        if (rc < 0 && rc_all == JSVD_OK) rc_all = rc;
                        r.idx = -1;
                        --active;
                    }
                }
                continue;
            }
            int st_done = 0, sw = 0;
            if (!plain_service(b, r, streams[j], &st_done, &sw)) continue;
            progressed = true;
            if (st_done != (1 << 20)) finish(r, streams[j], st_done, sw);
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (int j = 0; j < k; ++j) {
        (void)hipStreamSynchronize(streams[j]);
        if (runs[j].ev) (void)hipEventDestroy(runs[j].ev);
    }
    if (ready) (void)hipEventDestroy(ready);
    give_streams(dev, k, streams);
    return rc_all;
}

} // namespace

extern "C" int jsvd_batched_tune(int count, const int *m, const int *n, const int *is_complex, unsigned flags,
                                 void *stream)
{
    if (count < 0 || (count > 0 && (!m || !n))) return JSVD_EINVAL;
    if (!iter_flags_valid(flags, JSVD_NO_PERMUTE | JSVD_PERMUTE | JSVD_COMPENSATED | JSVD_NO_GS)) return JSVD_EINVAL;
    std::vector<BatchItem> items;
    for (int i = 0; i < count; ++i) {
        const int c = is_complex ? (is_complex[i] != 0) : 0;
        if (n[i] < 1 || m[i] < n[i]) return JSVD_EINVAL;
        if (!batch_rows(m[i], n[i], c)) continue;
        items.push_back(make_batch_item(m[i], n[i], c, nullptr, nullptr, (size_t)m[i], nullptr, nullptr, (size_t)n[i],
                                        nullptr, nullptr));
    }
    if (!items.empty()) batch_tune(items.data(), (int)items.size(), flags, (hipStream_t)stream);
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? JSVD_OK : JSVD_EDEVICE;
}

extern "C" int jsvd_batched_set_launch(int threads_per_matrix) { return batch_set_threads(threads_per_matrix); }

extern "C" int jsvd_batched_set_schedule(int threads_per_matrix, int dense, int workgroups_per_cu)
{
    return batch_set_sched(threads_per_matrix, dense, workgroups_per_cu);
}

extern "C" int jsvd_batched_set_tuning(unsigned candidates) { return batch_set_tuning(candidates); }

extern "C" int jsvd_batched_schedule_of(int m, int n, int is_complex, unsigned flags, int *threads_per_matrix,
                                        int *dense, int *workgroups_per_cu)
{
    if (n < 1 || m < n || !threads_per_matrix || !dense || !workgroups_per_cu) return JSVD_EINVAL;
    const BatchSched b = batch_sched_of(m, n, is_complex != 0, flags);
    *threads_per_matrix = b.nt;
    *dense = b.dense;
    *workgroups_per_cu = b.wpc;
    return JSVD_OK;
}

extern "C" int jsvd_batched_launch_of(int m, int n, int is_complex, unsigned flags)
{
    if (n < 1 || m < n) return JSVD_EINVAL;
    return batch_threads_of(m, n, is_complex != 0, flags);
}

extern "C" int jsvd_gesvj_batched(int count, const int *m, const int *n, const int *is_complex,
                                  double *const *G_re, double *const *G_im, const size_t *ldg,
                                  double *const *V_re, double *const *V_im, const size_t *ldv,
                                  double *const *sv_e, double *const *sv_f, int max_sweeps, int *sweeps,
                                  int *status, int64_t *transformations, unsigned flags, void *stream)
{
    if (count < 0) return JSVD_EINVAL;
    if (count == 0) return JSVD_OK;
    if (!m || !n || !G_re || !ldg || !V_re || !ldv || !sv_e || !sv_f || !status) return JSVD_EINVAL;
    if (!iter_flags_valid(flags, JSVD_NO_PERMUTE | JSVD_PERMUTE | JSVD_COMPENSATED | JSVD_NO_GS)) return JSVD_EINVAL;
    for (int i = 0; i < count; ++i) {
        const int c = is_complex ? is_complex[i] : 0;
        if (n[i] < 1 || m[i] < n[i] || !G_re[i] || !V_re[i] || !sv_e[i] || !sv_f[i] || ldg[i] < (size_t)m[i] ||
            ldv[i] < (size_t)n[i])
            return JSVD_EINVAL;
        if (c && (!G_im || !V_im || !G_im[i] || !V_im[i])) return JSVD_EINVAL;
    }
    if (max_sweeps <= 0) max_sweeps = 128;
    hipStream_t s = (hipStream_t)stream;
    std::vector<BatchItem> items;
    std::vector<int> plain, item_of(count, -1);
    items.reserve(count);
    for (int i = 0; i < count; ++i) {
        const int c = is_complex ? (is_complex[i] != 0) : 0;
        if (!batch_rows(m[i], n[i], c)) {
            plain.push_back(i);
            continue;
        }
        item_of[i] = (int)items.size();
        items.push_back(make_batch_item(m[i], n[i], c, G_re[i], c ? G_im[i] : nullptr, ldg[i], V_re[i],
                                        c ? V_im[i] : nullptr, ldv[i], sv_e[i], sv_f[i]));
    }
    int rc_all = JSVD_OK;
    BatchLaunch *bl = nullptr;
    if (!items.empty()) {
        bl = batch_launch(items.data(), (int)items.size(), max_sweeps, flags, s);
        if (!bl) return JSVD_EDEVICE;
    }
    // matrices outside the batched kernel's tile, beside the batched launch
    const PlainBatch pb{m, n, is_complex, G_re, G_im, ldg, V_re, V_im, ldv, sv_e, sv_f, max_sweeps, flags,
                        sweeps, status, transformations};
    rc_all = plain_concurrent(pb, plain, s);
    if (bl) {
        if (hipStreamSynchronize(s) != hipSuccess) {
            batch_release(bl);
            return JSVD_EDEVICE;
        }
        const BatchItem *res = batch_results(bl);
        for (int i = 0; i < count; ++i) {
            if (item_of[i] < 0) continue;
            const BatchItem &it = res[item_of[i]];
            status[i] = it.status;
            if (sweeps) sweeps[i] = it.sweeps;
            if (transformations) transformations[i] = it.transformations;
            if (it.status < 0 && rc_all == JSVD_OK) rc_all = it.status;
        }
        batch_release(bl);
    }
    return rc_all;
}

extern "C" int jsvd_gesvj_batched_noalloc(int count, const int *m, const int *n, const int *is_complex,
                                          double *const *G_re, double *const *G_im, const size_t *ldg,
                                          double *const *V_re, double *const *V_im, const size_t *ldv,
                                          double *const *sv_e, double *const *sv_f, int max_sweeps, int *sweeps,
                                          int *status, int64_t *transformations, unsigned flags, void *stream)
{
    if (count < 0 || count > kNoAllocMaxCount) return JSVD_EINVAL;
    if (count == 0) return JSVD_OK;
    if (!m || !n || !G_re || !ldg || !V_re || !ldv || !sv_e || !sv_f || !status) return JSVD_EINVAL;
    if (!iter_flags_valid(flags, JSVD_NO_PERMUTE | JSVD_PERMUTE | JSVD_COMPENSATED | JSVD_NO_GS)) return JSVD_EINVAL;
    for (int i = 0; i < count; ++i) {
        const int c = is_complex ? is_complex[i] : 0;
        if (n[i] < 1 || m[i] < n[i] || !G_re[i] || !V_re[i] || !sv_e[i] || !sv_f[i] || ldg[i] < (size_t)m[i] ||
            ldv[i] < (size_t)n[i])
            return JSVD_EINVAL;
        if (c && (!G_im || !V_im || !G_im[i] || !V_im[i])) return JSVD_EINVAL;
        // only the batched kernel's shapes: the plain path would allocate a state
        if (!batch_rows(m[i], n[i], c != 0)) return JSVD_EINVAL;
    }
    if (max_sweeps <= 0) max_sweeps = 128;
    // the records are built in a file-scope array too (no heap allocation)
    static BatchItem items[kNoAllocMaxCount];
    static std::mutex items_mu;
    std::lock_guard<std::mutex> lk(items_mu);
    for (int i = 0; i < count; ++i) {
        const int c = is_complex ? (is_complex[i] != 0) : 0;
        items[i] = make_batch_item(m[i], n[i], c, G_re[i], c ? G_im[i] : nullptr, ldg[i], V_re[i],
                                   c ? V_im[i] : nullptr, ldv[i], sv_e[i], sv_f[i]);
    }
    const int rc = batch_run_noalloc(items, count, max_sweeps, flags, (hipStream_t)stream);
    if (rc != JSVD_OK) return rc;
    int rc_all = JSVD_OK;
    for (int i = 0; i < count; ++i) {
        status[i] = items[i].status;
        if (sweeps) sweeps[i] = items[i].sweeps;
        if (transformations) transformations[i] = items[i].transformations;
        if (items[i].status < 0 && rc_all == JSVD_OK) rc_all = items[i].status;
    }
    return rc_all;
}
