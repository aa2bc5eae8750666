// gstep.hip -- the parallel Jacobi step for large columns (arXiv:2202.08361,
// Alg. zvjsvd phases; the same arithmetic, bit for bit, as step.hip).
//
// Per step:
//
// * gpair_kernel: one workgroup per pivot pair.  The G column pair is read
//   once into registers; norms, scaled dot-product (Alg. zdpscl),
//   convergence test (Alg. cvg), Gram matrix (Alg. Gram), 2x2 EVD
//   (Listing 1) and rotation (Alg. zjrot) run on it there, and it is written
//   once.  Two workgroups per compute unit overlap one pair's reductions and
//   EVD with the other's memory traffic.  The pair's outcome (rotation,
//   permutation, max-norm) goes to the step's slot of an outcome log.
// * the fold of a step into the device scalars (M~, counts, s, k): done at
//   the start of the next such step (its workgroups derive k and the exponent
//   of M~ from the logged step, its workgroup 0 updates the scalars), or by
//   fold_kernel when the scalars are read.  The only atomic is one relaxed
//   max per rotating workgroup into the step's max-norm key; no workgroup
//   waits on another.
//
// V is not touched per step.  Its rows never mix, so the rotations of up to
// a log's worth of consecutive steps are applied to it in one pass
// (vacc_kernel), on a row-major V staged row by row in LDS: every element
// gets the same operations in the same order as with a per-step update,
// while V crosses HBM once per flush instead of once per step.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "evd2_core.hpp"
#include "kernels.hpp"
#include "pair.hpp"
#include "fold.hpp"

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
    if (COMP) return 2;
    if (sizeof(T) == sizeof(float) && !CPLX && R <= 32) return 4;
    return 2;
}

// rows t + W j (j < R) of the pair's columns into registers, 0 beyond m
template <bool CPLX, int W, int R, typename T>
__device__ __forceinline__ void gpair_load(T (&xr)[2][R], T (&xi)[2][R], const T *Gpr, const T *Gqr, const T *Gpi,
                                           const T *Gqi, int m, int t)
{
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
}

// G part of the step: one workgroup of W = 256 threads per pivot pair, the
// pair held in registers from its load to its store.  Several workgroups
// share a compute unit, so one computes (reductions, EVD) while the others
// wait on their loads or stores.  The outcome of the pair (rotation,
// permutation, max-norm of the rotated columns) goes to the log slot.
//
// The step index and M~ come from the device scalars, or, after another
// step of this kind (prev.prm set), from that step: k + 1, and floor(lg M~)
// = max(floor(lg 2^{s_[k]} M~_k), floor(lg M)) from its header and its
// max-norm key, while workgroup 0 folds that step into the device scalars
// (fold_step: the exact M~ and the counts).  So no kernel runs between two
// steps.
template <bool CPLX, int W, int R, bool COMP, typename T>
__global__ __launch_bounds__(W, (gpair_wgs_per_cu<T, CPLX, R, COMP>() * W / 256)) void gpair_kernel(SvdDescT<T> d,
                                                                                                      StepSlot slot,
                                                                                                      StepSlot prev)
{
    __shared__ T red[(COMP ? 12 : 6) * W];
    __shared__ T mxs[4 * (W / 64)];
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
    // A pair whose two columns have not changed since it last met, one sweep
    // (K steps) earlier: its norms, dot-product and decision are the same bits
    // as at that meeting, which left both columns as they were (neither
    // rotated nor swapped them).  It is not read again, unless this step
    // rescales every column.
    const long long K = (long long)(n + (n & 1)) - 1;
    const bool unchanged = valid && d.lastmod[p] < k - K && d.lastmod[q] < k - K;
    T xr[2][R], xi[2][R];
    if (valid && !unchanged) gpair_load<CPLX, W, R>(xr, xi, Gpr, Gqr, Gpi, Gqi, m, t);
    // floor(lg M~) of this step, which is all the rescaling check needs
    int eMt;
    if (prev.prm) {
        const T Mp = (T)bits2d(prev.hdr->Mt_bits);
        const bool rp = (CPLX ? SvdFp<T>::round_cplx : SvdFp<T>::round_real) - getexp(Mp) < 0;
        const T Mp2 = rp ? scal2(Mp, d.lgbound - getexp(Mp) - 1) : Mp;
        eMt = max(getexp(Mp2), step_max_exp(pkey, k - 1));
        // the previous step's fold: the exact M~ of this step, the counts
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
    const int sr = (CPLX ? SvdFp<T>::round_cplx : SvdFp<T>::round_real) - eMt;
    const bool rescale = sr < 0;
    const int sp = rescale ? (d.lgbound - eMt - 1) : 0;
    PairParam pp;
    pp.pq = p | (q << 16);
    pp.flag = 0;
    pp.c = 1.0;
    pp.C = 0.0;
    pp.S = 0.0;
    double pmx = 0.0;
    if (!valid) {
        // the column sitting out (odd n): only the rescaling applies
        if (rescale) {
            for (int i = t; i < m; i += W) {
                Gpr[i] = scal2(Gpr[i], sp);
                if (CPLX) Gpi[i] = scal2(Gpi[i], sp);
            }
            if (t == 0) d.lastmod[p] = k;
        }
        if (t == 0) {
            prm[l] = pp;
            slot.mx[l] = pmx;
        }
    } else if (unchanged && !rescale) {
        // the outcome of the pair's last meeting: nothing to do
        if (t == 0) {
            pp.flag = 8;
            prm[l] = pp;
            slot.mx[l] = pmx;
        }
    } else {
        if (unchanged) gpair_load<CPLX, W, R>(xr, xi, Gpr, Gqr, Gpi, Gqi, m, t);
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
            group_max<W, 1, valu_trees<R>()>(mm, mxs + 2 * (W / 64));
            pmx = mm[0];
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
            if (t == 0) {
                d.lastmod[p] = k;
                d.lastmod[q] = k;
            }
        }
        if (t == 0) {
            prm[l] = pp;
            slot.mx[l] = pmx;
            if ((pp.flag & 1) && pmx > 0.0) step_max_add(slot.mxkey, k, getexp((T)pmx));
            const int dp = pbit ? q : p, dq = pbit ? p : q;
            d.e[dp] = dc.np.zero ? T(-INFINITY) : (T)dc.np.e;
            d.f[dp] = dc.np.zero ? T(1) : dc.np.f;
            d.e[dq] = dc.nq.zero ? T(-INFINITY) : (T)dc.nq.e;
            d.f[dq] = dc.nq.zero ? T(1) : dc.nq.f;
        }
    }
}


// every column's last change := the step about to run
template <typename T>
__global__ void lastmod_reset_kernel(SvdDescT<T> d, StepSlot prev)
{
    const long long k = prev.prm ? prev.hdr->k + 1 : *(volatile long long *)&d.sc->k;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < d.n; j += gridDim.x * blockDim.x) d.lastmod[j] = k;
}

template <typename T>
hipError_t launch_lastmod_reset(const SvdDescT<T> &d, StepSlot prev, hipStream_t s)
{
    const int blocks = (d.n + 255) / 256;
    hipLaunchKernelGGL((lastmod_reset_kernel<T>), dim3(blocks < 64 ? blocks : 64), dim3(256), 0, s, d, prev);
    return hipGetLastError();
}
template hipError_t launch_lastmod_reset<double>(const SvdDescT<double> &, StepSlot, hipStream_t);
template hipError_t launch_lastmod_reset<float>(const SvdDescT<float> &, StepSlot, hipStream_t);

// the fold of one step as a kernel of its own: the G kernel's workgroups do
// not see each other's outcomes before that launch has ended
template <typename T>
__global__ __launch_bounds__(kFoldW) void fold_kernel(SvdDescT<T> d, const PairParam *prm, const double *pmx)
{
    if (*(volatile int *)&d.sc->stop) return;
    (void)fold_step<kFoldW, T>(d, prm, pmx, (d.n + (d.n & 1)) / 2);
}

// outcomes of this thread's pairs l = t + W u in one step (only what V needs)
template <int PPT, typename T>
struct VaccPairs {
    T c[PPT], C[PPT], S[PPT];
    int p[PPT], q[PPT], f[PPT];
};

// The loads are unconditional (a pair beyond the step's count reads the
// slot's first entry and is masked out), so that every step issues the same
// loads and the compiler can wait for the previous step's only.
template <bool CPLX, int PPT, typename T>
__device__ __forceinline__ void vacc_load(VaccPairs<PPT, T> &o, const PairParam *pl, int np, int t, int W)
{
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
        const int l = t + W * u;
        // the 32-byte outcome as two 16-byte loads: (c, C), (S, pq, flag)
        const uint4 *const P = reinterpret_cast<const uint4 *>(pl + (l < np ? l : 0));
        const uint4 a = P[0], b = P[1];
        const int pq = (int)b.z, f = (int)b.w;
        // rotation or swap only (bit 2 marks a Gram-Schmidt rotation, which V
        // takes as any other; bit 3 a pair that was not read: no change)
        o.f[u] = l < np ? (f & 3) : 0;
        o.p[u] = pq & 0xFFFF;
        o.q[u] = pq >> 16;
        o.c[u] = (T)__hiloint2double((int)a.y, (int)a.x);
        o.C[u] = (T)__hiloint2double((int)a.w, (int)a.z);
        o.S[u] = CPLX ? (T)__hiloint2double((int)b.y, (int)b.x) : T(0);
    }
}

// Deferred V update: nsteps logged steps (step j's outcomes at plog + j
// stride) applied to B rows of the row-major V (row i at Vr + i ldv) per
// workgroup, staged in LDS as sm[(plane B + r) n + column].  Within a step
// the pairs are disjoint, so each thread updates its pairs' two columns in
// all staged rows, with the per-element formulas of the column update: a
// rotation (flag & 1; the swap of the permutation, flag & 2, exchanges the
// destination columns), or a plain exchange.  One barrier per step.  The
// next step's outcomes are loaded while the current step is applied.
template <bool CPLX, int PPT, typename T>
__global__ __launch_bounds__(1024) void vacc_kernel(SvdDescT<T> d, const PairParam *plog, long long stride,
                                                    int nsteps, int B)
{
    if (*(volatile int *)&d.sc->stop) return;
    constexpr int RB = PPT >= 4 ? 1 : 2;   // staged rows updated together
    extern __shared__ __align__(16) unsigned char vacc_lds[];
    T *const sm = (T *)vacc_lds;
    const int n = d.n, t = threadIdx.x, W = blockDim.x;
    const int np = (n + 1) / 2;
    const int row0 = blockIdx.x * B;
    const int nb = min(B, n - row0);
    for (int r = 0; r < nb; ++r) {
        const T *vr = d.Vr + (size_t)(row0 + r) * d.ldv;
        const T *vi = CPLX ? d.Vi + (size_t)(row0 + r) * d.ldv : nullptr;
        for (int j = t; j < n; j += W) {
            sm[r * n + j] = vr[j];
            if (CPLX) sm[(B + r) * n + j] = vi[j];
        }
    }
    VaccPairs<PPT, T> cur, nxt;
    vacc_load<CPLX, PPT, T>(cur, plog, np, t, W);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        // the next step's outcomes (the last step reloads its own, unused)
        vacc_load<CPLX, PPT, T>(nxt, plog + (size_t)(s + 1 < nsteps ? s + 1 : s) * stride, np, t, W);
        // RB rows at a time: first every value the thread's pairs need from
        // them (the pairs of a step are disjoint, so none of these loads
        // depends on a store of the step), then the updates
        for (int r0 = 0; r0 < nb; r0 += RB) {
            T a[PPT][RB][4];   // p, q (real parts), then p, q (imaginary parts)
#pragma unroll
            for (int u = 0; u < PPT; ++u)
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) {
                    if (cur.f[u] == 0 || r0 + rr >= nb) continue;
                    const T *const R = sm + (r0 + rr) * n;
                    a[u][rr][0] = R[cur.p[u]];
                    a[u][rr][1] = R[cur.q[u]];
                    if (CPLX) {
                        const T *const I = sm + (B + r0 + rr) * n;
                        a[u][rr][2] = I[cur.p[u]];
                        a[u][rr][3] = I[cur.q[u]];
                    }
                }
#pragma unroll
            for (int u = 0; u < PPT; ++u)
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) {
                    const int f = cur.f[u];
                    if (f == 0 || r0 + rr >= nb) continue;
                    const int p = cur.p[u], q = cur.q[u];
                    const int ep = (f & 2) ? q : p, eq = (f & 2) ? p : q;
                    const T c = cur.c[u], C = cur.C[u], S = cur.S[u];
                    const T pr = a[u][rr][0], qr = a[u][rr][1];
                    T *const R = sm + (r0 + rr) * n;
                    if (CPLX) {
                        const T pi = a[u][rr][2], qi = a[u][rr][3];
                        T *const I = sm + (B + r0 + rr) * n;
                        if (f & 1) {
                            R[ep] = fma(qr, C, fma(-qi, S, pr)) * c;
                            I[ep] = fma(qr, S, fma(qi, C, pi)) * c;
                            R[eq] = fma(pr, -C, fma(-pi, S, qr)) * c;
                            I[eq] = fma(pr, S, fma(pi, -C, qi)) * c;
                        } else {
                            R[p] = qr;
                            R[q] = pr;
                            I[p] = qi;
                            I[q] = pi;
                        }
                    } else if (f & 1) {
                        R[ep] = fma(qr, C, pr) * c;
                        R[eq] = fma(pr, -C, qr) * c;
                    } else {
                        R[p] = qr;
                        R[q] = pr;
                    }
                }
        }
        lds_barrier();
        cur = nxt;
    }
    for (int r = 0; r < nb; ++r) {
        T *const vr = d.Vr + (size_t)(row0 + r) * d.ldv;
        T *const vi = CPLX ? d.Vi + (size_t)(row0 + r) * d.ldv : nullptr;
        for (int j = t; j < n; j += W) {
            vr[j] = sm[r * n + j];
            if (CPLX) vi[j] = sm[(B + r) * n + j];
        }
    }
}

// In-place transpose of the n x n matrix V (each plane): switches V between
// the column-major layout (the fused step kernel, the caller) and the
// row-major one of the deferred update.  32 x 32 tiles; workgroup (bj, bi,
// plane) with bi <= bj exchanges tile (bi, bj) with the transpose of tile
// (bj, bi), a diagonal tile with its own transpose.
template <typename T>
__global__ __launch_bounds__(256) void vtrans_kernel(T *Vr, T *Vi, int n, long long ld)
{
    const int bi = blockIdx.y, bj = blockIdx.x;
    if (bi > bj) return;
    T *const P = blockIdx.z ? Vi : Vr;
    __shared__ T ta[32][33], tb[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // ta[c][r] = X(32 bi + r, 32 bj + c), tb[c][r] = X(32 bj + r, 32 bi + c); X(i, j) at P[i + j ld]
    for (int c = ty; c < 32; c += 8) {
        const int i = bi * 32 + tx, j = bj * 32 + c;
        if (i < n && j < n) ta[c][tx] = P[i + (size_t)j * ld];
        const int i2 = bj * 32 + tx, j2 = bi * 32 + c;
        if (bi != bj && i2 < n && j2 < n) tb[c][tx] = P[i2 + (size_t)j2 * ld];
    }
    __syncthreads();
    // X'(32 bj + r, 32 bi + c) = X(32 bi + c, 32 bj + r) = ta[r][c], and the mirror from tb
    for (int c = ty; c < 32; c += 8) {
        const int i = bj * 32 + tx, j = bi * 32 + c;
        if (i < n && j < n) P[i + (size_t)j * ld] = ta[tx][c];
        const int i2 = bi * 32 + tx, j2 = bj * 32 + c;
        if (bi != bj && i2 < n && j2 < n) P[i2 + (size_t)j2 * ld] = tb[tx][c];
    }
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
static hipError_t launch_gpair_t(const SvdDescT<T> &d, StepSlot slot, StepSlot prev, int R, hipStream_t s)
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
                                       slot, prev);                                                             \
                    return hipGetLastError();                                                                   \
                }                                                                                               \
            }                                                                                                   \
            hipLaunchKernelGGL((gpair_kernel<CPLX, kPW, r, false, T>), dim3(npairs), dim3(kPW), 0, s, d, slot,  \
                               prev);                                                                           \
            return hipGetLastError();                                                                           \
        }                                                                                                       \
        break;
        JSVD_GP(1) JSVD_GP(2) JSVD_GP(4) JSVD_GP(8) JSVD_GP(16) JSVD_GP(32) JSVD_GP(64)
#undef JSVD_GP
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_gpair(const SvdDescT<T> &d, StepSlot slot, StepSlot prev, hipStream_t s)
{
    const int R = gpair_rows(d.m, d.cplx, sizeof(T) == sizeof(float));
    if (R == 0) return hipErrorInvalidValue;
    return d.cplx ? launch_gpair_t<true>(d, slot, prev, R, s) : launch_gpair_t<false>(d, slot, prev, R, s);
}

template <typename T>
hipError_t launch_fold(const SvdDescT<T> &d, const PairParam *prm, const double *mx, hipStream_t s)
{
    hipLaunchKernelGGL((fold_kernel<T>), dim3(1), dim3(kFoldW), 0, s, d, prm, mx);
    return hipGetLastError();
}

// the LDS the deferred update may take (more than the default 64 KiB needs
// the kernel attribute, set by vacc_prepare on the current device)
constexpr int kVaccMaxLds = 128 << 10;

// rows of V per workgroup of the deferred update: for real rows 64 KiB of
// LDS (two workgroups per compute unit) when that holds at least two rows,
// else 128 KiB; for complex rows 128 KiB, which halves the workgroups that
// each re-read every logged step's outcomes (measured: single precision
// complex 4096^2 66.1 -> 61.6 us per step; real rows lose 4 % that way);
// 0 when a row does not fit
static int vacc_rows(int n, int cplx, size_t es)
{
    const size_t row = es * (size_t)n * (cplx ? 2 : 1);
    int B = (int)((size_t)(64 << 10) / row);
    if (B < 2 || cplx) B = (int)((size_t)kVaccMaxLds / row);
    return B < n ? B : n;
}

int vacc_supported(int n, int cplx, bool fp32)
{
    return vacc_rows(n, cplx, fp32 ? sizeof(float) : sizeof(double)) >= 1;
}

template <bool CPLX, int PPT, typename T>
static hipError_t vacc_allow_lds()
{
    return hipFuncSetAttribute((const void *)vacc_kernel<CPLX, PPT, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kVaccMaxLds);
}

template <bool CPLX, typename T>
static hipError_t vacc_prepare_t()
{
    constexpr bool F32 = sizeof(T) == sizeof(float);
    hipError_t e = vacc_allow_lds<CPLX, 1, T>();
    if (e == hipSuccess) e = vacc_allow_lds<CPLX, 2, T>();
    if constexpr (!CPLX || F32)
        if (e == hipSuccess) e = vacc_allow_lds<CPLX, 4, T>();
    if constexpr (!CPLX && F32)
        if (e == hipSuccess) e = vacc_allow_lds<CPLX, 8, T>();
    return e;
}

hipError_t vacc_prepare(int cplx, bool fp32)
{
    if (fp32) return cplx ? vacc_prepare_t<true, float>() : vacc_prepare_t<false, float>();
    return cplx ? vacc_prepare_t<true, double>() : vacc_prepare_t<false, double>();
}

template <bool CPLX, int PPT, typename T>
static hipError_t launch_vacc_k(const SvdDescT<T> &d, const PairParam *plog, long long stride, int nsteps, int B,
                                int W, hipStream_t s)
{
    const size_t lds = sizeof(T) * (size_t)B * d.n * (CPLX ? 2 : 1);
    if (lds > (size_t)kVaccMaxLds) return hipErrorInvalidValue;
    hipLaunchKernelGGL((vacc_kernel<CPLX, PPT, T>), dim3((d.n + B - 1) / B), dim3(W), lds, s, d, plog, stride, nsteps,
                       B);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_vacc(const SvdDescT<T> &d, const PairParam *plog, long long stride, int nsteps, hipStream_t s)
{
    if (nsteps <= 0) return hipSuccess;
    const int B = vacc_rows(d.n, d.cplx, sizeof(T));
    if (B < 1) return hipErrorInvalidValue;
    const int np = (d.n + 1) / 2;
    const int W = np >= 1024 ? 1024 : ((np + 63) / 64) * 64;
    const int ppt = (np + W - 1) / W;
    // pairs per thread: n <= m rows, and m is at most 8192 (real) / 4096
    // (complex) rows in double precision, twice that in single precision
    constexpr bool F32 = sizeof(T) == sizeof(float);
    if (d.cplx) {
        if (ppt <= 1) return launch_vacc_k<true, 1, T>(d, plog, stride, nsteps, B, W, s);
        if (ppt <= 2) return launch_vacc_k<true, 2, T>(d, plog, stride, nsteps, B, W, s);
        if constexpr (F32)
            if (ppt <= 4) return launch_vacc_k<true, 4, T>(d, plog, stride, nsteps, B, W, s);
    } else {
        if (ppt <= 1) return launch_vacc_k<false, 1, T>(d, plog, stride, nsteps, B, W, s);
        if (ppt <= 2) return launch_vacc_k<false, 2, T>(d, plog, stride, nsteps, B, W, s);
        if (ppt <= 4) return launch_vacc_k<false, 4, T>(d, plog, stride, nsteps, B, W, s);
        if constexpr (F32)
            if (ppt <= 8) return launch_vacc_k<false, 8, T>(d, plog, stride, nsteps, B, W, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_vtrans(const SvdDescT<T> &d, hipStream_t s)
{
    const int nt = (d.n + 31) / 32;
    hipLaunchKernelGGL((vtrans_kernel<T>), dim3(nt, nt, d.cplx ? 2 : 1), dim3(256), 0, s, d.Vr, d.Vi, d.n, d.ldv);
    return hipGetLastError();
}

template hipError_t launch_gpair<double>(const SvdDescT<double> &, StepSlot, StepSlot, hipStream_t);
template hipError_t launch_gpair<float>(const SvdDescT<float> &, StepSlot, StepSlot, hipStream_t);
template hipError_t launch_fold<double>(const SvdDescT<double> &, const PairParam *, const double *, hipStream_t);
template hipError_t launch_fold<float>(const SvdDescT<float> &, const PairParam *, const double *, hipStream_t);
template hipError_t launch_vacc<double>(const SvdDescT<double> &, const PairParam *, long long, int, hipStream_t);
template hipError_t launch_vacc<float>(const SvdDescT<float> &, const PairParam *, long long, int, hipStream_t);
template hipError_t launch_vtrans<double>(const SvdDescT<double> &, hipStream_t);
template hipError_t launch_vtrans<float>(const SvdDescT<float> &, hipStream_t);

} // namespace jsvd
