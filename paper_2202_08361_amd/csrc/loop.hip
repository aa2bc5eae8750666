// loop.hip -- a whole sweep of the one-sided Jacobi SVD (Alg. zvjsvd: K
// round-robin steps) in one persistent launch, for columns of up to 1024
// rows.
//
// One workgroup per pair slot l (n/2 of them, all resident at once; one
// wavefront up to 256 rows, four up to 1024) runs the
// K steps of the sweep.  In the circle method a column of step k + 1 comes
// from slot l - 1, l or l + 1 of step k, so there is no need for a barrier
// between steps: each column carries a flag, the step it is ready for, and a
// workgroup starts its pair of step k as soon as both of its columns are
// ready (agent-scope acquire), then publishes them for step k + 1
// (agent-scope release).  The pair's arithmetic is that of the fused step
// kernel (pair_core, transform_regs, rot_regs), so the sweep gives the same
// bits as K steps.
//
// What a step needs from all pairs of the step before is M~, for the
// rescaling check of Sect. 3.2.  The launch is used only when no rescaling
// can happen in the sweep: every component of G stays below ||G||_F, the
// rotations change ||G||_F by a factor within 1 + 16 eps per step, and a
// bound B >= (1 + 32 eps K) ||G_k0||_F is computed before the sweep
// (frob_cols_kernel, loop_check_kernel).  If max(M~_k0, B) < 2^(round + 1)
// then M~ stays below the threshold for the whole sweep and every check
// says "no rescaling", exactly as the steps would decide it.  Otherwise
// the caller runs the sweep step by step.
//
// L2-local mode (64-thread workgroups, at most four per compute unit of one
// XCC, n <= 256; columns of up to 1024 real / 512 complex rows at 8 or 16
// rows per lane, the same canonical sums): the launch has one workgroup per pair slot on every
// XCC, and only
// those that land on one XCC (the first one to arrive names it) take the
// slots; the others end at once.  Those workgroups share one L2, which is
// then the point of coherence for everything the sweep exchanges: columns
// are read with L2-coherent loads (past the compute unit's L1), written with
// plain stores (the L1 writes through), and a column's flag is stored once
// the stores before it have completed in the L2 (a wait on the vector memory
// counter).  No L2 write-back or invalidation is needed on either side,
// which halves the latency of a column's hand-over (measured on a ring of
// workgroups: 670 against 1390 ns).  Should fewer workgroups than slots land
// on the XCC, the waits run out of budget and the sweep is redone step by
// step like any other that gives up.
//
// A pair whose two columns have not changed since it last met, one sweep
// earlier (the per-column step of the last change, kept up to date by the
// sweep like the large-column steps keep it), had no transformation and no
// swap then, and its columns are the same now: its workgroup computes and
// stores nothing for it and only passes the columns on.  (The columns are
// loaded anyway, together with the two last-change steps: loading those
// first would add a memory round trip to every step.)
//
// Every wait is bounded (a wall-clock budget); a workgroup that runs out of
// it raises an abort flag that every other one sees, so the launch always
// ends.  The counts and the max-norm are kept per workgroup and folded once
// at the end (loop_fold_kernel): integer sums and an exact max, so the
// order does not matter.  An aborted sweep is marked for a redo from the
// snapshot taken before it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "evd2_core.hpp"
#include "kernels.hpp"
#include "pair.hpp"

namespace jsvd {

// wait until column c is ready for step offset `want` (flag >= want), then
// acquire (L2-local mode: the column's loads are L2-coherent and only have to
// stay after the flag's); false on abort or when the budget runs out
template <bool LOCAL>
__device__ __forceinline__ bool loop_wait(const LoopArgs &a, int c, unsigned long long want)
{
    unsigned long long v = __hip_atomic_load(a.ver + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v < want) {
        const unsigned long long t0 = wall_clock64();
        for (unsigned it = 1;; ++it) {
            __builtin_amdgcn_s_sleep(2);
            v = __hip_atomic_load(a.ver + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v >= want) break;
            if (wall_clock64() - t0 >= a.budget) {
                __hip_atomic_store(a.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
            if ((it & 7) == 0 && __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                return false;
        }
    }
    if constexpr (LOCAL)
        asm volatile("" ::: "memory");
    else
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// both columns of a pair (q < 0: p only) ready for step offset `want`, with
// one outcome for the whole workgroup: in a workgroup of several wavefronts
// the first one waits and the others take its outcome from LDS, so that no
// two wavefronts can see different ones (a barrier later in the step would
// then never be reached by all of them)
template <int W, bool LOCAL>
__device__ __forceinline__ bool loop_wait_pair(const LoopArgs &a, int p, int q, unsigned long long want, int *ok_lds)
{
    if constexpr (W == 64) {
        return loop_wait<LOCAL>(a, p, want) && (q < 0 || loop_wait<LOCAL>(a, q, want));
    } else {
        static_assert(!LOCAL, "the L2-local mode has one wavefront per workgroup");
        if (threadIdx.x < 64) {
            const bool ok = loop_wait<false>(a, p, want) && (q < 0 || loop_wait<false>(a, q, want));
            if (threadIdx.x == 0) *ok_lds = ok ? 1 : 0;
        }
        // the first wavefront's acquire (after its wait) has invalidated the
        // caches this compute unit reads through; the barrier orders the other
        // wavefronts' loads after it
        __syncthreads();
        return *(volatile int *)ok_lds != 0;
    }
}

// a store that is coherent at agent scope (relaxed atomic); in the L2-local
// mode a plain store (the L1 writes through to the shared L2)
template <bool LOCAL, typename T>
__device__ __forceinline__ void col_store(T *p, T v)
{
    if constexpr (LOCAL)
        *p = v;
    else
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// a column element as published by another workgroup: after the acquire a
// plain load; in the L2-local mode an L2-coherent one (relaxed atomic at
// agent scope, which does not hit in the L1)
template <bool LOCAL, typename T>
__device__ __forceinline__ T col_load(T *p)
{
    if constexpr (LOCAL)
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}

// the XCC this wavefront runs on (hardware register XCC_ID, bits 3:0)
__device__ __forceinline__ unsigned xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u; }

// publish columns p and q (q < 0: p only) as ready for step offset `val`,
// after everything this wavefront wrote before
// (the workgroup barrier first makes every wavefront's stores complete in
// the L2; the agent-scope release of the first wavefront then writes the
// L2 back once for all of them)
// (L2-local mode, one wavefront: the wait for the vector memory counter
// makes every store of the wavefront complete in the L2 first)
template <bool LOCAL>
__device__ __forceinline__ void loop_publish(const LoopArgs &a, int p, int q, unsigned long long val)
{
    if constexpr (LOCAL) {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0); expcnt and lgkmcnt not waited on
        asm volatile("" ::: "memory");
        if (threadIdx.x == 0) {
            __hip_atomic_store(a.ver + p, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (q >= 0) __hip_atomic_store(a.ver + q, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0) {
            __hip_atomic_store(a.ver + p, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (q >= 0) __hip_atomic_store(a.ver + q, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <bool CPLX, int W, int R, bool COMP, bool LOCAL, typename T>
__global__ __launch_bounds__(W) void loop_kernel(SvdDescT<T> d, LoopArgs a)
{
    static_assert(!LOCAL || W == 64, "the L2-local mode has one wavefront per workgroup");
    // rows of V per thread: V has n <= 256 rows wherever a wavefront holds a
    // pair slot (64-thread workgroups run for n <= 256 only), so a 64-thread
    // workgroup with more G rows per lane keeps four of V's
    constexpr int RV = (W == 64 && R > 4) ? 4 : R;
    // the reduction scratch of pair_core (a workgroup of one wavefront
    // reduces in registers alone)
    __shared__ T red[W > 64 ? (COMP ? 12 : 6) * W : 1];
    __shared__ T mxs[W > 64 ? 4 * (W / 64) : 1];
    __shared__ int wait_ok;
    T *const red_norm = W > 64 ? red : (T *)nullptr;
    T *const red_dot = W > 64 ? red + 4 * W : (T *)nullptr;
    T *const mxs_p = W > 64 ? mxs : (T *)nullptr;
    const int t = threadIdx.x;
    DevScalars *sc = d.sc;
    LoopAcc acc;
    acc.t = acc.sw = acc.gs = acc.tlast = acc.sk = 0;
    acc.M = 0.0;
    acc.done = 0;
    // the scalars do not change during the launch: every workgroup reads the same
    if (sc->stop) {
        if (!LOCAL && t == 0) a.acc[blockIdx.x] = acc;
        return;
    }
    const int m = d.m, n = d.n;
    const int N = n + (n & 1), K = N - 1;
    int l = blockIdx.x;
    if constexpr (LOCAL) {
        // the first workgroup to arrive names its XCC; the workgroups on that
        // XCC take the pair slots in the order they arrive, the rest end here
        int got = 0x7fffffff;
        if (t == 0) {
            const unsigned x = xcc_id() + 1u;
            const unsigned named = atomicCAS(a.claim + 1, 0u, x);
            if (named == 0u || named == x) got = (int)atomicAdd(a.claim, 1u);
        }
        l = __builtin_amdgcn_readlane(got, 0);
        if (l >= N / 2) return;
    }
    const long long k0 = sc->k;
    const unsigned long long epoch = (unsigned long long)(unsigned)sc->loop_epoch << 32;
    T Mrun = T(0);
    int steps = 0;
    for (int j = 0; j < K; ++j) {
        const long long k = k0 + j;
        int p, q;
        const bool valid = rr_pair(n, k, l, &p, &q);
        // the columns of step offset 0 are current from the launch boundary
        if (j > 0 && !loop_wait_pair<W, LOCAL>(a, p, valid ? q : -1, epoch | (unsigned)j, &wait_ok)) break;
        if (!valid) {
            // the column sitting out this step (odd n): nothing to compute
            loop_publish<LOCAL>(a, p, -1, epoch | (unsigned)(j + 1));
            ++steps;
            continue;
        }
        // the steps of the columns' last changes, loaded beside the columns
        // (a load before the columns' would add its latency to every step)
        const long long lm_p = col_load<LOCAL>(d.lastmod + p), lm_q = col_load<LOCAL>(d.lastmod + q);
        T *const Gpr = d.Gr + (size_t)p * d.ldg;
        T *const Gqr = d.Gr + (size_t)q * d.ldg;
        T *const Gpi = CPLX ? d.Gi + (size_t)p * d.ldg : nullptr;
        T *const Gqi = CPLX ? d.Gi + (size_t)q * d.ldg : nullptr;
        T *const Vpr = d.Vr + (size_t)p * d.ldv;
        T *const Vqr = d.Vr + (size_t)q * d.ldv;
        T *const Vpi = CPLX ? d.Vi + (size_t)p * d.ldv : nullptr;
        T *const Vqi = CPLX ? d.Vi + (size_t)q * d.ldv : nullptr;
        T xr[2][R], xi[2][R], vr[2][RV], vi[2][RV];
#pragma unroll
        for (int jj = 0; jj < R; ++jj) {
            const int i = t + W * jj;
            const bool in = i < m;
            xr[0][jj] = in ? col_load<LOCAL>(Gpr + i) : T(0);
            xr[1][jj] = in ? col_load<LOCAL>(Gqr + i) : T(0);
            if (CPLX) {
                xi[0][jj] = in ? col_load<LOCAL>(Gpi + i) : T(0);
                xi[1][jj] = in ? col_load<LOCAL>(Gqi + i) : T(0);
            }
        }
#pragma unroll
        for (int jj = 0; jj < RV; ++jj) {
            const int i = t + W * jj;
            const bool inv = i < n;
            vr[0][jj] = inv ? col_load<LOCAL>(Vpr + i) : T(0);
            vr[1][jj] = inv ? col_load<LOCAL>(Vqr + i) : T(0);
            if (CPLX) {
                vi[0][jj] = inv ? col_load<LOCAL>(Vpi + i) : T(0);
                vi[1][jj] = inv ? col_load<LOCAL>(Vqi + i) : T(0);
            }
        }
        // both columns unchanged since the pair last met (K steps ago, when it
        // changed neither): the same outcome, no change, so nothing to compute
        if (lm_p < k - K && lm_q < k - K) {
            ++acc.sk;
            loop_publish<LOCAL>(a, p, q, epoch | (unsigned)(j + 1));
            ++steps;
            continue;
        }
        // no rescaling in this sweep (checked before the launch)
        const PairDecisionT<T> dc = pair_core<CPLX, W, R, COMP>(xr, xi, d.ups, d.nosort, d.nogs, red_norm, red_dot, mxs_p);
        const int pbit = dc.pbit;
        T *const Dp_r = pbit ? Gqr : Gpr;
        T *const Dq_r = pbit ? Gpr : Gqr;
        T *const Dp_i = pbit ? Gqi : Gpi;
        T *const Dq_i = pbit ? Gpi : Gqi;
        T *const Ep_r = pbit ? Vqr : Vpr;
        T *const Eq_r = pbit ? Vpr : Vqr;
        T *const Ep_i = pbit ? Vqi : Vpi;
        T *const Eq_i = pbit ? Vpi : Vqi;
        if (dc.transform) {
            // this thread's max-norm; the workgroup's is taken once, at the end
            Mrun = fmax(Mrun, transform_regs<CPLX, R>(xr, xi, dc));
            (void)rot_regs<CPLX, RV>(vr, vi, dc.c, dc.C, dc.S);
            ++acc.t;
            if (dc.gs) ++acc.gs;
            if (j == K - 1) acc.tlast = 1;
        } else if (pbit) {
            ++acc.sw;
        }
        if (dc.transform || pbit) {
            // agent-coherent stores: the release below then has fewer dirty
            // L2 lines to write back (measured 6.9 -> 5.5 us per 256 x 256
            // real step); ordering still comes from the release / acquire
#pragma unroll
            for (int jj = 0; jj < R; ++jj) {
                const int i = t + W * jj;
                if (i < m) {
                    col_store<LOCAL>(Dp_r + i, xr[0][jj]);
                    col_store<LOCAL>(Dq_r + i, xr[1][jj]);
                    if (CPLX) {
                        col_store<LOCAL>(Dp_i + i, xi[0][jj]);
                        col_store<LOCAL>(Dq_i + i, xi[1][jj]);
                    }
                }
            }
#pragma unroll
            for (int jj = 0; jj < RV; ++jj) {
                const int i = t + W * jj;
                if (i < n) {
                    col_store<LOCAL>(Ep_r + i, vr[0][jj]);
                    col_store<LOCAL>(Eq_r + i, vr[1][jj]);
                    if (CPLX) {
                        col_store<LOCAL>(Ep_i + i, vi[0][jj]);
                        col_store<LOCAL>(Eq_i + i, vi[1][jj]);
                    }
                }
            }
        }
        if (t == 0 && (dc.transform || pbit)) {
            // the step of the last change of both columns (read with the
            // columns by their next owners)
            col_store<LOCAL>(d.lastmod + p, k);
            col_store<LOCAL>(d.lastmod + q, k);
        }
        if (t == 0) {
            const NormT<T> np_ = dc.np, nq_ = dc.nq;
            const int dp = pbit ? q : p, dq = pbit ? p : q;
            d.e[dp] = np_.zero ? T(-INFINITY) : (T)np_.e;
            d.f[dp] = np_.zero ? T(1) : np_.f;
            d.e[dq] = nq_.zero ? T(-INFINITY) : (T)nq_.e;
            d.f[dq] = nq_.zero ? T(1) : nq_.f;
        }
        loop_publish<LOCAL>(a, p, q, epoch | (unsigned)(j + 1));
        ++steps;
    }
    // the max-norm of the rotated columns over the workgroup (an exact max)
    if constexpr (W == 64) {
        Mrun = wave_max(Mrun);
    } else {
        T mm[1] = {Mrun};
        group_max<W, 1>(mm, mxs);
        Mrun = mm[0];
    }
    if (t == 0) {
        acc.M = (double)Mrun;
        acc.done = steps;
        a.acc[l] = acc;
    }
}

// The end of a persistent sweep: the counts and the max-norm of all
// workgroups folded into the device scalars as the K step folds would have
// done it (no rescaling happened), the step index advanced by K, the flag
// epoch advanced.  An aborted sweep (some workgroup ran out of its wait
// budget) changes no scalar but the redo mark.  One workgroup.
template <typename T>
__global__ __launch_bounds__(256) void loop_fold_kernel(SvdDescT<T> d, LoopArgs a, int npairs, int K)
{
    __shared__ double sM[4];
    __shared__ long long sc4[4][6];
    DevScalars *sc = d.sc;
    // the slot claims of an L2-local launch start from zero in the next one
    if (a.local && threadIdx.x == 0) {
        a.claim[0] = 0u;
        a.claim[1] = 0u;
    }
    if (sc->stop) return;
    const int t = threadIdx.x;
    double M = 0.0;
    long long tt = 0, sw = 0, gg = 0, tl = 0, short_ = 0, sk = 0;
    for (int l = t; l < npairs; l += 256) {
        const LoopAcc x = a.acc[l];
        M = fmax(M, x.M);
        tt += x.t;
        sw += x.sw;
        gg += x.gs;
        tl += x.tlast;
        sk += x.sk;
        short_ += (x.done != K) ? 1 : 0;
    }
    M = wave_max(M);
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) {
        tt += __shfl_xor(tt, h, 64);
        sw += __shfl_xor(sw, h, 64);
        gg += __shfl_xor(gg, h, 64);
        tl += __shfl_xor(tl, h, 64);
        sk += __shfl_xor(sk, h, 64);
        short_ += __shfl_xor(short_, h, 64);
    }
    if ((t & 63) == 0) {
        sM[t >> 6] = M;
        sc4[t >> 6][0] = tt;
        sc4[t >> 6][1] = sw;
        sc4[t >> 6][2] = gg;
        sc4[t >> 6][3] = tl;
        sc4[t >> 6][4] = short_;
        sc4[t >> 6][5] = sk;
    }
    __syncthreads();
    if (t != 0) return;
    for (int w = 1; w < 4; ++w) {
        sM[0] = fmax(sM[0], sM[w]);
        for (int c = 0; c < 6; ++c) sc4[0][c] += sc4[w][c];
    }
    const bool aborted = *a.abort != 0 || sc4[0][4] != 0;
    *a.abort = 0;
    sc->loop_epoch += 1;
    if (aborted) {
        sc->loop_redo = 1;
        return;
    }
    const T Mt = (T)bits2d(sc->Mt_bits);
    sc->Mt_bits = d2bits((double)fmax(Mt, (T)sM[0]));
    sc->T += sc4[0][0];
    sc->SW += sc4[0][1];
    sc->GS += sc4[0][2];
    sc->last_t = sc4[0][3];
    sc->skipped += sc4[0][5];
    sc->k += K;
    sc->loop_sweeps += 1;
}

// Per column j: sum_i (g_ij 2^-E)^2 (both parts of a complex column), with
// E = floor(lg M~): every component is at most M~, so each term is below 4.
// One wavefront per column, lanes over rows, a fixed tree (the sum is used
// as a bound only).
template <bool CPLX, typename T>
__global__ __launch_bounds__(64) void frob_cols_kernel(SvdDescT<T> d, double *colsq)
{
    const int j = blockIdx.x, t = threadIdx.x;
    const double Mt = bits2d(d.sc->Mt_bits);
    const int E = Mt > 0.0 ? getexp(Mt) : 0;
    const T *gr = d.Gr + (size_t)j * d.ldg;
    const T *gi = CPLX ? d.Gi + (size_t)j * d.ldg : nullptr;
    double s = 0.0;
    for (int i = t; i < d.m; i += 64) {
        const double x = scal2((double)gr[i], -E);
        s = fma(x, x, s);
        if (CPLX) {
            const double y = scal2((double)gi[i], -E);
            s = fma(y, y, s);
        }
    }
    s = wave_tree_sum(s);
    if (t == 0) colsq[j] = s;
}

// loop_ok: max(M~, B) < 2^(round + 1) with B an upper bound of
// (1 + 32 eps K) ||G||_F (rounding of the sums covered by the factors below,
// underflowed squares by an absolute term).  One workgroup.
template <typename T>
__global__ __launch_bounds__(256) void loop_check_kernel(SvdDescT<T> d, const double *colsq)
{
    __shared__ double part[4];
    DevScalars *sc = d.sc;
    const int t = threadIdx.x;
    double s = 0.0;
    for (int j = t; j < d.n; j += 256) s += colsq[j];
    s = wave_tree_sum(s);
    if ((t & 63) == 0) part[t >> 6] = s;
    __syncthreads();
    if (t != 0) return;
    const double tot = ((part[0] + part[1]) + (part[2] + part[3])) * (1.0 + 0x1p-30) +
                       (double)d.m * d.n * (d.cplx ? 2.0 : 1.0) * 0x1p-1000;
    const double Mt = bits2d(sc->Mt_bits);
    const int E = Mt > 0.0 ? getexp(Mt) : 0;
    // ||G||_F grows by at most a factor 1 + 16 eps per step (the rotation
    // with the computed parameters, Lemmas l:rt and l:ct, and the rounding
    // of cos phi); over the K steps of a sweep by at most 1 + 32 eps K
    const int K = d.n + (d.n & 1) - 1;
    const double eps = sizeof(T) == sizeof(double) ? 0x1p-53 : 0x1p-24;
    const double F = 1.0 + 32.0 * eps * K + 0x1p-30;
    const double B = scal2(sqrt(tot) * F, E);
    const double top = fmax(Mt, B);
    // the check of Sect. 3.2 rescales iff floor(lg M~) > round, i.e. M~ >= 2^(round + 1)
    const int round = d.cplx ? SvdFp<T>::round_cplx : SvdFp<T>::round_real;
    sc->loop_ok = top < scal2(1.0, round + 1) ? 1 : 0;
}

__global__ void loop_clear_kernel(DevScalars *sc)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->loop_redo = 0;
}

// ---------------------------------------------------------------------------
// Launch shape of a persistent sweep: one 64-thread workgroup per pair slot
// up to 256 rows (R = 1, 2, 4 rows per lane), one 256-thread workgroup up to
// 1024 rows (R = 2, 4), the same canonical sums either way.
struct LoopShape {
    int W, R;
};

static LoopShape loop_shape(int m, bool local)
{
    if (m <= 64) return {64, 1};
    if (m <= 128) return {64, 2};
    if (m <= 256) return {64, 4};
    // L2-local mode: one wavefront per slot throughout (its XCD has one SIMD
    // per slot), with more rows per lane
    if (local) return {64, m <= 512 ? 8 : 16};
    if (m <= 512) return {256, 2};
    return {256, 4};
}

int loop_max_rows() { return 1024; }

template <bool CPLX, bool COMP, typename T>
static const void *loop_fn_c(LoopShape sh, bool local)
{
    if (sh.W == 64) {
        if (local) {
            if (sh.R <= 1) return (const void *)loop_kernel<CPLX, 64, 1, COMP, true, T>;
            if (sh.R <= 2) return (const void *)loop_kernel<CPLX, 64, 2, COMP, true, T>;
            if (sh.R <= 4) return (const void *)loop_kernel<CPLX, 64, 4, COMP, true, T>;
            if (sh.R <= 8) return (const void *)loop_kernel<CPLX, 64, 8, COMP, true, T>;
            // a complex pair at 16 rows per lane is slower on one wavefront
            // than spread over four (1000 x 199: 45.5 against 36.9 ms)
            if constexpr (CPLX)
                return nullptr;
            else
                return (const void *)loop_kernel<CPLX, 64, 16, COMP, true, T>;
        }
        if (sh.R <= 1) return (const void *)loop_kernel<CPLX, 64, 1, COMP, false, T>;
        if (sh.R <= 2) return (const void *)loop_kernel<CPLX, 64, 2, COMP, false, T>;
        return (const void *)loop_kernel<CPLX, 64, 4, COMP, false, T>;
    }
    if (local) return nullptr;
    if (sh.R <= 2) return (const void *)loop_kernel<CPLX, 256, 2, COMP, false, T>;
    return (const void *)loop_kernel<CPLX, 256, 4, COMP, false, T>;
}

template <typename T>
static const void *loop_fn_of(const SvdDescT<T> &d, LoopShape sh, bool local)
{
    if constexpr (sizeof(T) == sizeof(double)) {
        if (d.comp) return d.cplx ? loop_fn_c<true, true, T>(sh, local) : loop_fn_c<false, true, T>(sh, local);
    } else {
        if (d.comp) return nullptr;
    }
    return d.cplx ? loop_fn_c<true, false, T>(sh, local) : loop_fn_c<false, false, T>(sh, local);
}

// XCCs of the device: an L2-local launch has one workgroup per slot on each
constexpr int kXcc = 8;

// every pair slot's workgroup resident at once
template <typename T>
bool loop_fits(const SvdDescT<T> &d, int ncu)
{
    if (d.m > loop_max_rows()) return false;
    const LoopShape sh = loop_shape(d.m, false);
    const void *fn = loop_fn_of(d, sh, false);
    if (!fn) return false;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, sh.W, 0) != hipSuccess || per_cu < 1) return false;
    const int npairs = (d.n + (d.n & 1)) / 2;
    return (long long)per_cu * ncu >= npairs;
}

// every pair slot's 64-thread workgroup resident on one XCC, at most one
// wavefront per SIMD (four per compute unit), so that no two slots share a
// SIMD's issue
template <typename T>
bool loop_fits_local(const SvdDescT<T> &d, int ncu)
{
    if (d.m > loop_max_rows() || d.n > 256 || ncu % kXcc != 0) return false;
    const LoopShape sh = loop_shape(d.m, true);
    if (sh.W != 64) return false;
    const void *fn = loop_fn_of(d, sh, true);
    if (!fn) return false;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, sh.W, 0) != hipSuccess || per_cu < 1) return false;
    const int npairs = (d.n + (d.n & 1)) / 2;
    const int cus = ncu / kXcc;
    return npairs <= 4 * cus && (long long)per_cu * cus >= npairs;
}

template <typename T>
hipError_t launch_loop_sweep(const SvdDescT<T> &d, const LoopArgs &a, hipStream_t s)
{
    const int N = d.n + (d.n & 1), npairs = N / 2, K = N - 1;
    if (d.m > loop_max_rows()) return hipErrorInvalidValue;
    const LoopShape sh = loop_shape(d.m, a.local != 0);
    const void *fn = loop_fn_of(d, sh, a.local != 0);
    if (!fn) return hipErrorInvalidValue;
    SvdDescT<T> dd = d;
    LoopArgs aa = a;
    void *args[] = {(void *)&dd, (void *)&aa};
    const int grid = a.local ? kXcc * npairs : npairs;
    hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(sh.W), args, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((loop_fold_kernel<T>), dim3(1), dim3(256), 0, s, d, a, npairs, K);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_loop_check(const SvdDescT<T> &d, double *colsq, hipStream_t s)
{
    if (d.cplx)
        hipLaunchKernelGGL((frob_cols_kernel<true, T>), dim3(d.n), dim3(64), 0, s, d, colsq);
    else
        hipLaunchKernelGGL((frob_cols_kernel<false, T>), dim3(d.n), dim3(64), 0, s, d, colsq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((loop_check_kernel<T>), dim3(1), dim3(256), 0, s, d, (const double *)colsq);
    return hipGetLastError();
}

hipError_t launch_loop_clear(DevScalars *sc, hipStream_t s)
{
    hipLaunchKernelGGL(loop_clear_kernel, dim3(1), dim3(64), 0, s, sc);
    return hipGetLastError();
}

template bool loop_fits<double>(const SvdDescT<double> &, int);
template bool loop_fits<float>(const SvdDescT<float> &, int);
template bool loop_fits_local<double>(const SvdDescT<double> &, int);
template bool loop_fits_local<float>(const SvdDescT<float> &, int);
template hipError_t launch_loop_sweep<double>(const SvdDescT<double> &, const LoopArgs &, hipStream_t);
template hipError_t launch_loop_sweep<float>(const SvdDescT<float> &, const LoopArgs &, hipStream_t);
template hipError_t launch_loop_check<double>(const SvdDescT<double> &, double *, hipStream_t);
template hipError_t launch_loop_check<float>(const SvdDescT<float> &, double *, hipStream_t);

} // namespace jsvd
