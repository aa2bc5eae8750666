// batched.hip -- many independent SVDs of uneven sizes in one persistent
// launch (the batched form of Alg. zvjsvd, arXiv:2202.08361).
//
// One workgroup of 512 threads (8 wavefronts) owns one matrix at a time and
// runs its whole SVD: initial scaling, sweeps of round-robin steps, the
// convergence test and the finalisation.  Within a step each wavefront takes
// pivot pairs (one pair per wavefront at a time, the same canonical sums as
// every other launch shape, so each matrix's result is bit-for-bit the one
// jsvd_gesvj gives); a workgroup barrier separates the steps, so no step ever
// needs the host or a grid-wide synchronisation.  Workgroups pull matrices
// from an atomic queue ordered by decreasing cost (longest first), which
// balances the uneven sizes.  G and V are iterated in place in the caller's
// buffers; the final sort is an in-place cycle permutation through LDS.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/jsvd.h"
#include "evd2_core.hpp"
#include "batch.hpp"
#include "kernels.hpp"
#include "pair.hpp"

namespace jsvd {

constexpr int kBT = 512;           // threads per workgroup
constexpr int kBWaves = kBT / 64;  // wavefronts per workgroup
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

struct BatchSmem {
    double e[kBMaxN], f[kBMaxN];
    int rank[kBMaxN], inv[kBMaxN];
    double tmp[2 * (kBMaxRowsR + kBMaxN)];
    double wM[kBWaves];
    unsigned long long wt[kBWaves], wsw[kBWaves];
    double red[kBWaves];
    int item;
};

// block-wide max of a non-negative value (exact)
__device__ __forceinline__ double block_max(double x, double *red)
{
    x = wave_max(x);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < kBWaves; ++w) r = fmax(r, red[w]);
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

template <bool CPLX, int R, bool COMP>
__device__ void svd_workgroup(BatchItem &it, int max_sweeps, int nosort, int nogs, BatchSmem &sm)
{
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
    const double M0 = block_max(mx, sm.red);
    if (!(M0 <= 1.79769313486231570815e308) || M0 == 0.0) {
        if (tid == 0) {
            it.status = (M0 == 0.0) ? JSVD_EZERO : JSVD_ENONFINITE;
            it.sweeps = 0;
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
    __syncthreads();

    const int N = n + (n & 1), K = N - 1, npairs = N / 2;
    int C = 0;
    bool converged = false;
    long long k = 0;
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
                    if (rescale)
                        for (int i = lane; i < m; i += 64) {
                            Gpr[i] = scal2(Gpr[i], sp);
                            if (CPLX) Gpi[i] = scal2(Gpi[i], sp);
                        }
                    continue;
                }
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
    }
}

template <bool COMP>
__global__ __launch_bounds__(kBT) void batched_kernel(BatchItem *items, const int *order, BatchCtl *ctl)
{
    __shared__ BatchSmem sm;
    const int count = ctl->count;
    for (;;) {
        if (threadIdx.x == 0) sm.item = (int)atomicAdd(&ctl->next, 1u);
        __syncthreads();
        const int idx = sm.item;
        __syncthreads();
        if (idx >= count) return;
        BatchItem it = items[order[idx]];
        switch ((it.cplx ? 100 : 0) + it.R) {
        case 1: svd_workgroup<false, 1, COMP>(it, ctl->max_sweeps, ctl->nosort, ctl->nogs, sm); break;
        case 2: svd_workgroup<false, 2, COMP>(it, ctl->max_sweeps, ctl->nosort, ctl->nogs, sm); break;
        case 4: svd_workgroup<false, 4, COMP>(it, ctl->max_sweeps, ctl->nosort, ctl->nogs, sm); break;
        case 8: svd_workgroup<false, 8, COMP>(it, ctl->max_sweeps, ctl->nosort, ctl->nogs, sm); break;
        case 101: svd_workgroup<true, 1, COMP>(it, ctl->max_sweeps, ctl->nosort, ctl->nogs, sm); break;
        case 102: svd_workgroup<true, 2, COMP>(it, ctl->max_sweeps, ctl->nosort, ctl->nogs, sm); break;
        case 104: svd_workgroup<true, 4, COMP>(it, ctl->max_sweeps, ctl->nosort, ctl->nogs, sm); break;
        case 108: svd_workgroup<true, 8, COMP>(it, ctl->max_sweeps, ctl->nosort, ctl->nogs, sm); break;
        default: break;
        }
        if (threadIdx.x == 0) {
            items[order[idx]].status = it.status;
            items[order[idx]].sweeps = it.sweeps;
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

struct BatchLaunch {
    void *dmem;
    BatchItem *host;   // pinned; results land here
    int count;
};

BatchLaunch *batch_launch(const BatchItem *items, int cnt, int max_sweeps, unsigned flags, hipStream_t s)
{
    if (cnt <= 0) return nullptr;
    BatchLaunch *bl = new (std::nothrow) BatchLaunch;
    if (!bl) return nullptr;
    bl->count = cnt;
    bl->dmem = nullptr;
    bl->host = nullptr;
    // longest first: cost ~ c n^2 (m + n) per sweep
    std::vector<int> order(cnt);
    for (int i = 0; i < cnt; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const double ca = (items[a].cplx ? 2.0 : 1.0) * items[a].n * (double)items[a].n * (items[a].m + items[a].n);
        const double cb = (items[b].cplx ? 2.0 : 1.0) * items[b].n * (double)items[b].n * (items[b].m + items[b].n);
        return ca > cb;
    });
    const size_t oItems = 0;
    const size_t oOrder = (sizeof(BatchItem) * cnt + 255) & ~(size_t)255;
    const size_t oCtl = oOrder + ((sizeof(int) * cnt + 255) & ~(size_t)255);
    const size_t bytes = oCtl + 256;
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
    BatchCtl ctl;
    ctl.next = 0;
    ctl.count = cnt;
    ctl.max_sweeps = max_sweeps;
    ctl.nosort = (flags & JSVD_NO_PERMUTE) ? 1 : 0;
    ctl.nogs = (flags & JSVD_NO_GS) ? 1 : 0;
    memcpy(h + oCtl, &ctl, sizeof(ctl));
    char *dm = (char *)bl->dmem;
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 256;
    bool ok = hipMemcpyAsync(dm, h, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    if (ok) {
        const int grid = std::min(cnt, 2 * ncu);
        if (flags & JSVD_COMPENSATED)
            hipLaunchKernelGGL(batched_kernel<true>, dim3(grid), dim3(kBT), 0, s, (BatchItem *)(dm + oItems),
                               (const int *)(dm + oOrder), (BatchCtl *)(dm + oCtl));
        else
            hipLaunchKernelGGL(batched_kernel<false>, dim3(grid), dim3(kBT), 0, s, (BatchItem *)(dm + oItems),
                               (const int *)(dm + oOrder), (BatchCtl *)(dm + oCtl));
        ok = hipGetLastError() == hipSuccess &&
             hipMemcpyAsync(bl->host, dm, sizeof(BatchItem) * cnt, hipMemcpyDeviceToHost, s) == hipSuccess;
    }
    if (!ok) {
        (void)hipStreamSynchronize(s);
        batch_release(bl);
        return nullptr;
    }
    return bl;
}

const BatchItem *batch_results(const BatchLaunch *bl) { return bl->host; }

void batch_release(BatchLaunch *bl)
{
    if (!bl) return;
    if (bl->dmem) (void)hipFree(bl->dmem);
    if (bl->host) (void)hipHostFree(bl->host);
    delete bl;
}

} // namespace jsvd

using namespace jsvd;

extern "C" int jsvd_gesvj_batched(int count, const int *m, const int *n, const int *is_complex,
                                  double *const *G_re, double *const *G_im, const size_t *ldg,
                                  double *const *V_re, double *const *V_im, const size_t *ldv,
                                  double *const *sv_e, double *const *sv_f, int max_sweeps, int *sweeps,
                                  int *status, unsigned flags, void *stream)
{
    if (count < 0) return JSVD_EINVAL;
    if (count == 0) return JSVD_OK;
    if (!m || !n || !G_re || !ldg || !V_re || !ldv || !sv_e || !sv_f || !status) return JSVD_EINVAL;
    if (flags & ~(JSVD_NO_PERMUTE | JSVD_COMPENSATED | JSVD_NO_GS)) return JSVD_EINVAL;
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
    if (!items.empty()) {
        BatchLaunch *bl = batch_launch(items.data(), (int)items.size(), max_sweeps, flags, s);
        if (!bl) return JSVD_EDEVICE;
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
            if (it.status < 0 && rc_all == JSVD_OK) rc_all = it.status;
        }
        batch_release(bl);
    }
    // matrices outside the batched kernel's tile: the plain path, one by one
    for (int i : plain) {
        const int c = is_complex ? is_complex[i] : 0;
        int sw = 0;
        const int rc = jsvd_gesvj(m[i], n[i], G_re[i], c ? G_im[i] : nullptr, ldg[i], V_re[i],
                                  c ? V_im[i] : nullptr, ldv[i], sv_e[i], sv_f[i], nullptr, max_sweeps, &sw,
                                  flags, stream);
        status[i] = rc;
        if (sweeps) sweeps[i] = sw;
        if (rc < 0 && rc_all == JSVD_OK) rc_all = rc;
    }
    return rc_all;
}
