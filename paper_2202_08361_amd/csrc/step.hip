// step.hip -- one parallel step of the one-sided Jacobi SVD on gfx950
// (arXiv:2202.08361, Alg. zvjsvd phases: column norms, scaled dot-products
// (Alg. zdpscl), convergence test (Alg. cvg) and scaled Gram matrices
// (Alg. Gram), batched 2x2 EVD (Listing 1), rotations (Alg. zjrot), with the
// step-start rescaling check of Sect. 3.2), plus initialisation, end-of-sweep
// bookkeeping and finalisation (Sect. 4.2.1).
//
// Mapping: one workgroup of W threads per pivot pair; the column pair lives
// in registers between the phases, so a step reads and writes each column of
// G and V once (16 c n (m + n) bytes per fully transformed step, c = 1 real,
// 2 complex).  The step index, M~ and the counters live on the device.  Each
// workgroup logs its pair's outcome; the next step (its workgroup 0), or a
// fold kernel before the scalars are read, folds a step into them
// (fold.hpp), so consecutive steps need no host involvement, no workgroup
// waits on another, and the steps can be captured in a graph.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "evd2_core.hpp"
#include "kernels.hpp"
#include "pair.hpp"
#include "fold.hpp"

namespace jsvd {

template <int W, bool COMP, typename T>
struct StepSmem {
    T norm[4 * W];
    T dot[(COMP ? 8 : 2) * W];
    T mx1[2 * (W / 64)];
    T mx2[W / 64];
};

template <bool CPLX, int W, int R, bool COMP, typename T>
__global__ __launch_bounds__(W) void step_kernel(SvdDescT<T> d, StepSlot slot, StepSlot prev)
{
    __shared__ StepSmem<W, COMP, T> sm;
    DevScalars *sc = d.sc;
    PairParam *const prm = slot.prm;
    const int t = threadIdx.x;
    const int l = blockIdx.x;
    if (*(volatile int *)&sc->stop) {
        // a stopped iteration: the step does nothing, and its log slot says so
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

    // the G pair and (short columns) the V pair, loaded before anything
    // else: the loads of V do not depend on the pair's outcome
    constexpr bool kVEarly = R <= 4 && W <= 256;
    T xr[2][R], xi[2][R], vr[2][R], vi[2][R];
    if (valid) {
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
        if constexpr (kVEarly) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = t + W * j;
                const bool in = i < n;
                vr[0][j] = in ? Vpr[i] : T(0);
                vr[1][j] = in ? Vqr[i] : T(0);
                if (CPLX) {
                    vi[0][j] = in ? Vpi[i] : T(0);
                    vi[1][j] = in ? Vqi[i] : T(0);
                }
            }
        }
    }

    // floor(lg M~) of this step, which is all the rescaling check needs:
    // after another step whose fold is due, from its slot (and workgroup 0
    // does that fold), else from the device scalars
    int eMt;
    if (prev.prm) {
        const T Mp = (T)bits2d(prev.hdr->Mt_bits);
        const bool rp = (CPLX ? SvdFp<T>::round_cplx : SvdFp<T>::round_real) - getexp(Mp) < 0;
        const T Mp2 = rp ? scal2(Mp, d.lgbound - getexp(Mp) - 1) : Mp;
        eMt = max(getexp(Mp2), step_max_exp(pkey, k - 1));
        if (l == 0) {
            const unsigned long long Mt_bits = fold_step<W, T>(d, prev.prm, prev.mx, npairs);
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

    // step-start rescaling check, Sect. 3.2: s_(k) < 0 => scale by 2^{s_[k]}
    const int sr = (CPLX ? SvdFp<T>::round_cplx : SvdFp<T>::round_real) - eMt;
    const bool rescale = sr < 0;
    const int sp = rescale ? (d.lgbound - eMt - 1) : 0;

    PairParam pp;
    pp.pq = p | (q << 16);
    pp.flag = 0;
    pp.c = 1.0;
    pp.C = 0.0;
    pp.S = 0.0;
    T Mblk = T(0);

    if (!valid) {
        // the column sitting out this step (odd n): only the rescaling applies
        if (rescale) {
            for (int i = t; i < m; i += W) {
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
    if (rescale) {
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                xr[c][j] = scal2(xr[c][j], sp);
                if (CPLX) xi[c][j] = scal2(xi[c][j], sp);
            }
    }

    const PairDecisionT<T> dc = pair_core<CPLX, W, R, COMP>(xr, xi, d.ups, d.nosort, d.nogs, sm.norm, sm.dot, sm.mx1);
    const bool transform = dc.transform;
    const int pbit = dc.pbit;
    const NormT<T> np_ = dc.np, nq_ = dc.nq;

    // ---- rotation (Alg. zjrot) or Gram-Schmidt step (eq. GS) or swap of
    // the G pair, then the rotation or swap of the V pair
    T *const Dp_r = pbit ? Gqr : Gpr;   // destination of x_p'
    T *const Dq_r = pbit ? Gpr : Gqr;   // destination of x_q'
    T *const Dp_i = pbit ? Gqi : Gpi;
    T *const Dq_i = pbit ? Gpi : Gqi;
    T *const Ep_r = pbit ? Vqr : Vpr;
    T *const Eq_r = pbit ? Vpr : Vqr;
    T *const Ep_i = pbit ? Vqi : Vpi;
    T *const Eq_i = pbit ? Vpi : Vqi;
    if (transform) {
        const T Mx = transform_regs<CPLX, R>(xr, xi, dc);
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
        if constexpr (!kVEarly) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = t + W * j;
                const bool in = i < n;
                vr[0][j] = in ? Vpr[i] : T(0);
                vr[1][j] = in ? Vqr[i] : T(0);
                if (CPLX) {
                    vi[0][j] = in ? Vpi[i] : T(0);
                    vi[1][j] = in ? Vqi[i] : T(0);
                }
            }
        }
        (void)rot_regs<CPLX, R>(vr, vi, dc.c, dc.C, dc.S);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = t + W * j;
            if (i < n) {
                Ep_r[i] = vr[0][j];
                Eq_r[i] = vr[1][j];
                if (CPLX) {
                    Ep_i[i] = vi[0][j];
                    Eq_i[i] = vi[1][j];
                }
            }
        }
        T mm[1] = {Mx};
        group_max<W, 1, valu_trees<R>()>(mm, sm.mx2);
        Mblk = mm[0];
        pp.flag = 1 | (pbit ? 2 : 0) | (dc.gs ? 4 : 0);
        pp.c = dc.c;
        pp.C = dc.C;
        pp.S = dc.S;
    } else if (pbit || rescale) {
        // swap (or only store the rescaled columns)
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
        if (pbit) {
            pp.flag = 2;
            if constexpr (kVEarly) {
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int i = t + W * j;
                    if (i < n) {
                        Vpr[i] = vr[1][j];
                        Vqr[i] = vr[0][j];
                        if (CPLX) {
                            Vpi[i] = vi[1][j];
                            Vqi[i] = vi[0][j];
                        }
                    }
                }
            } else {
                for (int i = t; i < n; i += W) {
                    const T a = Vpr[i], b = Vqr[i];
                    Vpr[i] = b;
                    Vqr[i] = a;
                    if (CPLX) {
                        const T ai = Vpi[i], bi = Vqi[i];
                        Vpi[i] = bi;
                        Vqi[i] = ai;
                    }
                }
            }
        }
    }
    // ---- the pair's outcome for the fold of this step (done by the next
    // step or a fold kernel), and its norms
    if (t == 0) {
        prm[l] = pp;
        slot.mx[l] = (double)Mblk;
        if (transform && Mblk > T(0)) step_max_add(slot.mxkey, k, getexp(Mblk));
        const T ep = np_.zero ? T(-INFINITY) : (T)np_.e;
        const T eq = nq_.zero ? T(-INFINITY) : (T)nq_.e;
        const int dp = pbit ? q : p, dq = pbit ? p : q;
        d.e[dp] = ep;
        d.f[dp] = np_.zero ? T(1) : np_.f;
        d.e[dq] = eq;
        d.f[dq] = nq_.zero ? T(1) : nq_.f;
    }
}

// ---------------------------------------------------------------------------
// dispatch over (complex, W, R, compensated dot-products; these exist in
// double precision only)
template <bool CPLX, int W, int R, typename T>
static hipError_t launch_step_t(const SvdDescT<T> &d, const StepSlot &slot, const StepSlot &prev, hipStream_t s)
{
    const int N = d.n + (d.n & 1);
    const unsigned blocks = (unsigned)(N / 2);
    if (d.comp) {
        if constexpr (sizeof(T) == sizeof(double))
            hipLaunchKernelGGL((step_kernel<CPLX, W, R, true, T>), dim3(blocks), dim3(W), 0, s, d, slot, prev);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((step_kernel<CPLX, W, R, false, T>), dim3(blocks), dim3(W), 0, s, d, slot, prev);
    }
    return hipGetLastError();
}

template <bool CPLX, int W, typename T>
static hipError_t launch_step_w(const SvdDescT<T> &d, const StepSlot &slot, const StepSlot &prev, hipStream_t s)
{
    const int R = (d.m + W - 1) / W;
    if (R <= 1) return launch_step_t<CPLX, W, 1>(d, slot, prev, s);
    if (R <= 2) return launch_step_t<CPLX, W, 2>(d, slot, prev, s);
    if (R <= 4) return launch_step_t<CPLX, W, 4>(d, slot, prev, s);
    if (R <= 8) return launch_step_t<CPLX, W, 8>(d, slot, prev, s);
    if constexpr (!CPLX && W == 1024)
        if (R <= 16) return launch_step_t<CPLX, W, 16>(d, slot, prev, s);
    return hipErrorInvalidValue;
}

// largest supported m for a workgroup size
int step_max_rows(int cplx, int W) { return W * ((!cplx && W == 1024) ? 16 : 8); }

int state_max_rows() { return 1 << 24; }

int step_auto_threads(int m, int n)
{
    (void)n;
    if (m <= 256) return 64;
    if (m <= 1024) return 256;
    if (m <= 2048) return 512;
    return 1024;
}

template <typename T>
hipError_t launch_step(const SvdDescT<T> &d, int threads, StepSlot slot, StepSlot prev, hipStream_t s)
{
    // columns longer than the register tile of the largest workgroup: the
    // pair is streamed from memory (sstep.hip)
    if (d.m > step_max_rows(d.cplx, 1024)) return launch_stream_step(d, slot, prev, s);
    if (threads <= 0) threads = step_auto_threads(d.m, d.n);
    if (d.m > step_max_rows(d.cplx, threads)) return hipErrorInvalidValue;
    if (d.cplx) {
        switch (threads) {
        case 64: return launch_step_w<true, 64>(d, slot, prev, s);
        case 128: return launch_step_w<true, 128>(d, slot, prev, s);
        case 256: return launch_step_w<true, 256>(d, slot, prev, s);
        case 512: return launch_step_w<true, 512>(d, slot, prev, s);
        case 1024: return launch_step_w<true, 1024>(d, slot, prev, s);
        }
    } else {
        switch (threads) {
        case 64: return launch_step_w<false, 64>(d, slot, prev, s);
        case 128: return launch_step_w<false, 128>(d, slot, prev, s);
        case 256: return launch_step_w<false, 256>(d, slot, prev, s);
        case 512: return launch_step_w<false, 512>(d, slot, prev, s);
        case 1024: return launch_step_w<false, 1024>(d, slot, prev, s);
        }
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// end of sweep: convergence when a whole sweep neither transformed nor swapped
__global__ void sweep_end_kernel(DevScalars *sc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    // a persistent sweep that gave up is redone step by step; it does not count
    if (sc->stop || sc->loop_redo) return;
    sc->sweeps += 1;
    if (sc->T == 0 && sc->SW == 0) {
        sc->converged = 1;
        sc->stop = 1;
    } else {
        sc->C += 1;
        if (sc->C >= sc->max_sweeps) sc->stop = 1;
    }
    sc->T_prev = sc->T;
    sc->SW_prev = sc->SW;
    sc->GS_prev = sc->GS;
    sc->T = 0;
    sc->SW = 0;
    sc->GS = 0;
}

hipError_t launch_sweep_end(DevScalars *sc, hipStream_t s)
{
    hipLaunchKernelGGL(sweep_end_kernel, dim3(1), dim3(64), 0, s, sc);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// initialisation
template <bool CPLX, typename T>
__global__ __launch_bounds__(256) void maxabs_kernel(int m, int n, const T *Ar, const T *Ai, long long lda,
                                                     unsigned long long *out)
{
    // M~_0 = max |component|, NaN turned into Inf (Sect. 3.2)
    T mx = T(0);
    const int j = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
        mx = fmax(mx, fmin(fabs(Ar[(size_t)j * lda + i]), T(INFINITY)));
        if (CPLX) mx = fmax(mx, fmin(fabs(Ai[(size_t)j * lda + i]), T(INFINITY)));
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) atomicMax(out, d2bits((double)mx));
}

// s_0 = s_[0] of eq. (skn) from M~_0 (device side, so the load needs no host round trip);
// a non-finite or zero M~_0 stops the state with its status
template <typename T>
__global__ void init_scalars_kernel(SvdDescT<T> d, const unsigned long long *maxbits, int max_sweeps)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const T M0 = (T)bits2d(*maxbits);
    DevScalars *sc = d.sc;
    sc->Mt_bits = 0;
    sc->k = 0;
    sc->T = 0;
    sc->SW = 0;
    sc->last_t = 0;
    sc->sweeps = 0;
    sc->C = 0;
    sc->T_prev = 0;
    sc->SW_prev = 0;
    sc->GS = 0;
    sc->GS_prev = 0;
    sc->rescaled = 0;
    sc->converged = 0;
    sc->max_sweeps = max_sweeps;
    // (loop_epoch keeps counting across loads: it tags the column flags of
    // the persistent sweeps, which are never cleared)
    sc->loop_ok = 0;
    sc->loop_redo = 0;
    sc->loop_sweeps = 0;
    sc->skipped = 0;
    if (!(M0 < T(INFINITY)) || M0 == T(0)) {
        sc->status = (M0 == T(0)) ? -3 : -2;
        sc->stop = 1;
        sc->s = 0;
        return;
    }
    const int s0 = d.lgbound - getexp(M0) - 1;
    sc->status = 0;
    sc->stop = 0;
    sc->s = s0;
    sc->Mt_bits = d2bits((double)scal2(M0, s0));
}

template <bool CPLX, typename T>
__global__ __launch_bounds__(256) void init_scale_kernel(SvdDescT<T> d, const T *Ar, const T *Ai, long long lda)
{
    if (d.sc->status != 0) return;
    const int s0 = d.sc->s;
    const int j = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < d.m; i += gridDim.x * 256) {
        d.Gr[(size_t)j * d.ldg + i] = scal2(Ar[(size_t)j * lda + i], s0);
        if (CPLX) d.Gi[(size_t)j * d.ldg + i] = scal2(Ai[(size_t)j * lda + i], s0);
    }
    for (int i = blockIdx.x * 256 + threadIdx.x; i < d.n; i += gridDim.x * 256) {
        d.Vr[(size_t)j * d.ldv + i] = (i == j) ? T(1) : T(0);
        if (CPLX) d.Vi[(size_t)j * d.ldv + i] = T(0);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        d.e[j] = T(-INFINITY);
        d.f[j] = T(1);
    }
}

static unsigned row_blocks(int m) { return (unsigned)min(64, (m + 255) / 256); }

template <typename T>
hipError_t launch_maxabs(const SvdDescT<T> &d, const T *Ar, const T *Ai, long long lda, unsigned long long *maxbits,
                         hipStream_t s)
{
    // reduces M~_0 into *maxbits, which the caller has zeroed
    dim3 grid(row_blocks(d.m), d.n);
    if (d.cplx)
        hipLaunchKernelGGL((maxabs_kernel<true, T>), grid, dim3(256), 0, s, d.m, d.n, Ar, Ai, lda, maxbits);
    else
        hipLaunchKernelGGL((maxabs_kernel<false, T>), grid, dim3(256), 0, s, d.m, d.n, Ar, Ai, lda, maxbits);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_scale(const SvdDescT<T> &d, const T *Ar, const T *Ai, long long lda,
                             const unsigned long long *maxbits, int max_sweeps, hipStream_t s)
{
    hipLaunchKernelGGL((init_scalars_kernel<T>), dim3(1), dim3(64), 0, s, d, maxbits, max_sweeps);
    dim3 grid(row_blocks(d.m), d.n);
    if (d.cplx)
        hipLaunchKernelGGL((init_scale_kernel<true, T>), grid, dim3(256), 0, s, d, Ar, Ai, lda);
    else
        hipLaunchKernelGGL((init_scale_kernel<false, T>), grid, dim3(256), 0, s, d, Ar, Ai, lda);
    return hipGetLastError();
}

// clear a 64-bit word on the stream (a kernel rather than a memset, so the
// sequence may be captured in a graph)
__global__ void zero_u64_kernel(unsigned long long *p) { if (threadIdx.x == 0) *p = 0ull; }

hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// finalisation
// Column norms of all columns (1024 threads per column, the canonical order:
// thread t = lane t, rows t, t+1024, ... in order).
template <bool CPLX, typename T>
__global__ __launch_bounds__(1024) void colnorm_kernel(SvdDescT<T> d, T *e_out, T *f_out)
{
    __shared__ T red[2 * 1024];
    __shared__ T mx1[16];
    const int j = blockIdx.x, t = threadIdx.x;
    const T *xr = d.Gr + (size_t)j * d.ldg;
    const T *xi = CPLX ? d.Gi + (size_t)j * d.ldg : nullptr;
    T mx[1] = {T(0)};
    for (int i = t; i < d.m; i += 1024) {
        mx[0] = fmax(mx[0], fabs(xr[i]));
        if (CPLX) mx[0] = fmax(mx[0], fabs(xi[i]));
    }
    group_max<1024, 1>(mx, mx1);
    if (mx[0] == T(0)) {
        if (t == 0) {
            e_out[j] = T(-INFINITY);
            f_out[j] = T(1);
        }
        return;
    }
    const int E = getexp(mx[0]);
    T s[2] = {T(0), T(0)};
    for (int i = t; i < d.m; i += 1024) {
        const T yr = scal2(xr[i], -E);
        s[0] = fma(yr, yr, s[0]);
        if (CPLX) {
            const T yi = scal2(xi[i], -E);
            s[1] = fma(yi, yi, s[1]);
        }
    }
    group_tree_sum<1024, 2>(s, red);
    const NormT<T> nn = norm_from_sums(E, s[0], s[1], CPLX);
    if (t == 0) {
        e_out[j] = (T)nn.e;
        f_out[j] = nn.f;
    }
}

// stable descending rank of sigma_j = (e_j, f_j)
template <typename T>
__global__ __launch_bounds__(256) void rank_kernel(int n, const T *e, const T *f, int *rank)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const T ej = e[j], fj = f[j];
    int r = 0;
    for (int i = 0; i < n; ++i) {
        const T ei = e[i], fi = f[i];
        const bool gt = ei > ej || (ei == ej && fi > fj);
        const bool eqb = (ei == ej && fi == fj) && i < j;
        r += (gt || eqb) ? 1 : 0;
    }
    rank[j] = r;
}

template <bool CPLX, typename T>
__global__ __launch_bounds__(256) void final_write_kernel(SvdDescT<T> d, const T *e, const T *f, const int *rank,
                                                          T *Ur, T *Ui, long long ldu, T *Vr, T *Vi, long long ldv,
                                                          T *sv_e, T *sv_f, T *sv)
{
    const int s = d.sc->s;
    const int j = blockIdx.x;
    const int dst = rank[j];
    const T ej = e[j], fj = f[j];
    const bool zero = isinf(ej);
    const int E = zero ? 0 : (int)ej;
    for (int i = threadIdx.x; i < d.m; i += 256) {
        const T xr = d.Gr[(size_t)j * d.ldg + i];
        Ur[(size_t)dst * ldu + i] = zero ? T(0) : scal2(xr, -E) / fj;
        if (CPLX) {
            const T xi = d.Gi[(size_t)j * d.ldg + i];
            Ui[(size_t)dst * ldu + i] = zero ? T(0) : scal2(xi, -E) / fj;
        }
    }
    for (int i = threadIdx.x; i < d.n; i += 256) {
        Vr[(size_t)dst * ldv + i] = d.Vr[(size_t)j * d.ldv + i];
        if (CPLX) Vi[(size_t)dst * ldv + i] = d.Vi[(size_t)j * d.ldv + i];
    }
    if (threadIdx.x == 0) {
        sv_e[dst] = zero ? T(-INFINITY) : ej - (T)s;
        sv_f[dst] = fj;
        if (sv) sv[dst] = zero ? T(0) : scal2(fj, E - s);
    }
}

template <typename T>
hipError_t launch_final_write(const SvdDescT<T> &d, const int *rank, T *Ur, T *Ui, long long ldu, T *Vr, T *Vi,
                              long long ldv, T *sv_e, T *sv_f, T *sv, hipStream_t st)
{
    if (d.cplx)
        hipLaunchKernelGGL((final_write_kernel<true, T>), dim3(d.n), dim3(256), 0, st, d, d.e, d.f, rank, Ur, Ui,
                           ldu, Vr, Vi, ldv, sv_e, sv_f, sv);
    else
        hipLaunchKernelGGL((final_write_kernel<false, T>), dim3(d.n), dim3(256), 0, st, d, d.e, d.f, rank, Ur, Ui,
                           ldu, Vr, Vi, ldv, sv_e, sv_f, sv);
    return hipGetLastError();
}

// non-converged exit: current column norms, backscaled, in column order
template <typename T>
__global__ __launch_bounds__(256) void colnorm_out_kernel(int n, const T *e, const T *f, const DevScalars *sc,
                                                          T *sv_e, T *sv_f, T *sv)
{
    const int s = sc->s;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const bool zero = isinf(e[j]);
    sv_e[j] = zero ? T(-INFINITY) : e[j] - (T)s;
    sv_f[j] = f[j];
    if (sv) sv[j] = zero ? T(0) : scal2(f[j], (int)e[j] - s);
}

template <typename T>
hipError_t launch_colnorms_raw(const SvdDescT<T> &d, hipStream_t st)
{
    if (d.cplx)
        hipLaunchKernelGGL((colnorm_kernel<true, T>), dim3(d.n), dim3(1024), 0, st, d, d.e, d.f);
    else
        hipLaunchKernelGGL((colnorm_kernel<false, T>), dim3(d.n), dim3(1024), 0, st, d, d.e, d.f);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_colnorm_out(const SvdDescT<T> &d, T *sv_e, T *sv_f, T *sv, hipStream_t st)
{
    hipLaunchKernelGGL((colnorm_out_kernel<T>), dim3((d.n + 255) / 256), dim3(256), 0, st, d.n, d.e, d.f, d.sc,
                       sv_e, sv_f, sv);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rank(const SvdDescT<T> &d, int *rank, hipStream_t st)
{
    hipLaunchKernelGGL((rank_kernel<T>), dim3((d.n + 255) / 256), dim3(256), 0, st, d.n, d.e, d.f, rank);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// layout helpers (Sect. SM5)
template <typename T>
__global__ __launch_bounds__(256) void copy2d_kernel(int m, const T *src, long long lds, T *dst, long long ldd)
{
    const int j = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256)
        dst[(size_t)j * ldd + i] = src[(size_t)j * lds + i];
}

template <typename T>
hipError_t launch_copy2d(int m, int n, const T *src, long long lds, T *dst, long long ldd, hipStream_t s)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL((copy2d_kernel<T>), dim3(row_blocks(m), n), dim3(256), 0, s, m, src, lds, dst, ldd);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void split_kernel(int m, const double *Z, long long ldz, double *Xr,
                                                    double *Xi, long long ldx)
{
    const int j = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
        Xr[(size_t)j * ldx + i] = Z[(size_t)j * ldz + 2 * (size_t)i];
        Xi[(size_t)j * ldx + i] = Z[(size_t)j * ldz + 2 * (size_t)i + 1];
    }
}

__global__ __launch_bounds__(256) void merge_kernel(int m, const double *Xr, const double *Xi, long long ldx,
                                                    double *Z, long long ldz)
{
    const int j = blockIdx.y;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
        Z[(size_t)j * ldz + 2 * (size_t)i] = Xr[(size_t)j * ldx + i];
        Z[(size_t)j * ldz + 2 * (size_t)i + 1] = Xi[(size_t)j * ldx + i];
    }
}

hipError_t launch_split(int m, int n, const double *Z, long long ldz, double *Xr, double *Xi, long long ldx,
                        hipStream_t s)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(split_kernel, dim3(row_blocks(m), n), dim3(256), 0, s, m, Z, ldz, Xr, Xi, ldx);
    return hipGetLastError();
}

hipError_t launch_merge(int m, int n, const double *Xr, const double *Xi, long long ldx, double *Z,
                        long long ldz, hipStream_t s)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(merge_kernel, dim3(row_blocks(m), n), dim3(256), 0, s, m, Xr, Xi, ldx, Z, ldz);
    return hipGetLastError();
}

// the two working precisions
#define JSVD_STEP_INST(T)                                                                                         \
    template hipError_t launch_maxabs<T>(const SvdDescT<T> &, const T *, const T *, long long, unsigned long long *, \
                                         hipStream_t);                                                            \
    template hipError_t launch_init_scale<T>(const SvdDescT<T> &, const T *, const T *, long long,                  \
                                             const unsigned long long *, int, hipStream_t);                       \
    template hipError_t launch_step<T>(const SvdDescT<T> &, int, StepSlot, StepSlot, hipStream_t);                 \
    template hipError_t launch_colnorms_raw<T>(const SvdDescT<T> &, hipStream_t);                                  \
    template hipError_t launch_rank<T>(const SvdDescT<T> &, int *, hipStream_t);                                   \
    template hipError_t launch_final_write<T>(const SvdDescT<T> &, const int *, T *, T *, long long, T *, T *,      \
                                              long long, T *, T *, T *, hipStream_t);                             \
    template hipError_t launch_colnorm_out<T>(const SvdDescT<T> &, T *, T *, T *, hipStream_t);                    \
    template hipError_t launch_copy2d<T>(int, int, const T *, long long, T *, long long, hipStream_t);
JSVD_STEP_INST(double)
JSVD_STEP_INST(float)
#undef JSVD_STEP_INST

} // namespace jsvd
