// gstep.hip -- pipelined form of the parallel Jacobi step for large columns
// (arXiv:2202.08361, Alg. zvjsvd phases; same arithmetic, bit for bit, as
// step.hip).
//
// The step is split into two kernels:
//
// * gstep_kernel: a persistent grid of one 256-thread workgroup per compute
//   unit walks the pivot pairs of the step.  While the current pair is in
//   registers (norms, scaled dot-product, Gram matrix, 2x2 EVD, rotation of
//   the G columns), the next pair is already streaming into LDS through the
//   direct global->LDS loads of gfx950 (global_load_lds_dwordx4), so HBM
//   stays busy during the reductions and the EVD.  The rotation of each pair
//   (cos phi, e^{i alpha} tan phi, the permutation and whether to rotate or
//   swap) is written to a small parameter array.
// * vrot_kernel: a fully occupied streaming kernel applies those parameters
//   to the column pairs of V.
//
// Tile layout in LDS: [column p re | column q re | (column p im | column q im)],
// each `ldt` doubles (ldt = R * 256, rows >= m ignored); the prefetch moves
// whole 1 KiB chunks (64 lanes x 16 bytes), so the workspace leading
// dimension is a multiple of 128 doubles and no chunk leaves its column.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "evd2_core.hpp"
#include "kernels.hpp"
#include "pair.hpp"

namespace jsvd {

constexpr int kGW = 256;   // threads per workgroup of the pipelined kernel

typedef __attribute__((address_space(3))) void lds_void;

// Issue the asynchronous copy of the column pair (p, q) into the LDS tile.
template <bool CPLX>
__device__ __forceinline__ void prefetch_pair(const SvdDesc &d, int p, int q, int m, int ldt, double *tile)
{
    constexpr int NCOL = CPLX ? 4 : 2;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int chunks = (m + 127) >> 7;               // 128 doubles per chunk
    for (int c = wv; c < NCOL * chunks; c += kGW / 64) {
        const int col = c / chunks, ch = c - col * chunks;
        const double *base = (col & 2) ? d.Gi : d.Gr;
        const int j = (col & 1) ? q : p;
        const double *src = base + (size_t)j * d.ldg + ch * 128 + lane * 2;
        double *dst = tile + col * ldt + ch * 128;
        __builtin_amdgcn_global_load_lds((const void *)src, (lds_void *)dst, 16, 0, 0);
    }
}

template <bool CPLX, int R>
__global__ __launch_bounds__(kGW, 1) void gstep_kernel(SvdDesc d, PairParam *prm)
{
    constexpr int W = kGW;
    constexpr int NCOL = CPLX ? 4 : 2;
    extern __shared__ double smem[];
    double *const tile = smem;                               // NCOL * ldt doubles
    constexpr int ldt = R * W;
    double *const red = smem + NCOL * ldt;                   // 6 * W doubles
    double *const mxs = red + 6 * W;                         // 12 doubles

    DevScalars *sc = d.sc;
    if (*(volatile int *)&sc->stop) return;
    const long long k = *(volatile long long *)&sc->k;
    const double Mt = bits2d(*(volatile unsigned long long *)&sc->Mt_bits);
    const int m = d.m, n = d.n;
    const int t = threadIdx.x;
    const int npairs = (n + (n & 1)) / 2;
    const int sr = (CPLX ? 1020 : 1022) - getexp(Mt);
    const bool rescale = sr < 0;
    const int sp = rescale ? (d.lgbound - getexp(Mt) - 1) : 0;

    double Mblk = 0.0;
    unsigned long long tcount = 0, swcount = 0;

    int l = blockIdx.x;
    {
        int p, q;
        if (l < npairs && rr_pair(n, k, l, &p, &q)) prefetch_pair<CPLX>(d, p, q, m, ldt, tile);
    }
    for (; l < npairs; l += gridDim.x) {
        int p, q;
        const bool valid = rr_pair(n, k, l, &p, &q);
        // the tile of this pair has landed (and the previous pair's stores are done)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        double xr[2][R], xi[2][R];
        if (valid) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int i = t + W * j;
                const bool in = i < m;
                xr[0][j] = in ? tile[i] : 0.0;
                xr[1][j] = in ? tile[ldt + i] : 0.0;
                if (CPLX) {
                    xi[0][j] = in ? tile[2 * ldt + i] : 0.0;
                    xi[1][j] = in ? tile[3 * ldt + i] : 0.0;
                }
            }
        }
        __syncthreads();
        // start the next pair's tile while this one is processed
        {
            int p2, q2;
            const int l2 = l + gridDim.x;
            if (l2 < npairs && rr_pair(n, k, l2, &p2, &q2)) prefetch_pair<CPLX>(d, p2, q2, m, ldt, tile);
        }
        PairParam pp;
        pp.p = p;
        pp.q = q;
        pp.flag = 0;
        pp.c = 1.0;
        pp.C = 0.0;
        pp.S = 0.0;
        if (!valid) {
            // the column sitting out (odd n): only the rescaling applies
            if (rescale) {
                double *Gp = d.Gr + (size_t)p * d.ldg;
                double *Gpi = CPLX ? d.Gi + (size_t)p * d.ldg : nullptr;
                for (int i = t; i < m; i += W) {
                    Gp[i] = scal2(Gp[i], sp);
                    if (CPLX) Gpi[i] = scal2(Gpi[i], sp);
                }
            }
            if (t == 0) prm[l] = pp;
            continue;
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
        const PairDecision dc = pair_core<CPLX, W, R>(xr, xi, d.ups, d.nosort, red, red + 4 * W, mxs);
        const bool transform = dc.transform;
        const int pbit = dc.pbit;
        const Norm np_ = dc.np, nq_ = dc.nq;

        double *const Gpr = d.Gr + (size_t)p * d.ldg;
        double *const Gqr = d.Gr + (size_t)q * d.ldg;
        double *const Gpi = CPLX ? d.Gi + (size_t)p * d.ldg : nullptr;
        double *const Gqi = CPLX ? d.Gi + (size_t)q * d.ldg : nullptr;
        double *const Dp_r = pbit ? Gqr : Gpr;
        double *const Dq_r = pbit ? Gpr : Gqr;
        double *const Dp_i = pbit ? Gqi : Gpi;
        double *const Dq_i = pbit ? Gpi : Gqi;
        if (transform) {
            const double Mx = rot_regs<CPLX, R>(xr, xi, dc.c, dc.C, dc.S);
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
            Mblk = fmax(Mblk, Mx);   // thread-local; reduced once at the end
            ++tcount;
            pp.flag = 1 | (pbit ? 2 : 0);
            pp.c = dc.c;
            pp.C = dc.C;
            pp.S = dc.S;
        } else if (pbit || rescale) {
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
                ++swcount;
                pp.flag = 2;
            }
        }
        if (t == 0) {
            prm[l] = pp;
            const int dp = pbit ? q : p, dq = pbit ? p : q;
            d.e[dp] = np_.zero ? -INFINITY : (double)np_.e;
            d.f[dp] = np_.zero ? 1.0 : np_.f;
            d.e[dq] = nq_.zero ? -INFINITY : (double)nq_.e;
            d.f[dq] = nq_.zero ? 1.0 : nq_.f;
        }
    }

    // ---- end of step: block max of the transformed columns, then the last
    // workgroup folds the step into the device scalars
    __syncthreads();
    double mm[1] = {Mblk};
    group_max<W, 1>(mm, mxs + 8);
    if (t == 0) {
        if (tcount) {
            atomicMax(&sc->M_step, d2bits(mm[0]));
            atomicAdd(&sc->t_step, tcount);
        }
        if (swcount) atomicAdd(&sc->sw_step, swcount);
        __threadfence();
        const unsigned long long prev = atomicAdd(&sc->done, 1ull);
        if (prev == (unsigned long long)gridDim.x - 1) {
            __threadfence();
            const double Mt2 = rescale ? scal2(Mt, sp) : Mt;
            const double Ms = bits2d(atomicExch(&sc->M_step, 0ull));
            sc->Mt_bits = d2bits(fmax(Mt2, Ms));
            const long long tt = (long long)atomicExch(&sc->t_step, 0ull);
            const long long sw = (long long)atomicExch(&sc->sw_step, 0ull);
            sc->T += tt;
            sc->SW += sw;
            sc->last_t = tt;
            if (rescale) {
                sc->s += sp;
                sc->rescaled += 1;
            }
            atomicExch(&sc->done, 0ull);
            sc->k = k + 1;
            __threadfence();
        }
    }
}

// V column pairs: rotate (flag & 1) and/or swap (flag & 2) with the step's
// parameters; 2 rows per thread, grid (pairs, row blocks).
template <bool CPLX>
__global__ __launch_bounds__(256) void vrot_kernel(SvdDesc d, const PairParam *prm)
{
    if (*(volatile int *)&d.sc->stop) return;
    const PairParam pp = prm[blockIdx.x];
    if (pp.flag == 0) return;
    const int n = d.n;
    const int i0 = blockIdx.y * 512 + threadIdx.x;
    double *const Vpr = d.Vr + (size_t)pp.p * d.ldv;
    double *const Vqr = d.Vr + (size_t)pp.q * d.ldv;
    double *const Vpi = CPLX ? d.Vi + (size_t)pp.p * d.ldv : nullptr;
    double *const Vqi = CPLX ? d.Vi + (size_t)pp.q * d.ldv : nullptr;
    const bool swap = (pp.flag & 2) != 0;
    double *const Ep_r = swap ? Vqr : Vpr;
    double *const Eq_r = swap ? Vpr : Vqr;
    double *const Ep_i = swap ? Vqi : Vpi;
    double *const Eq_i = swap ? Vpi : Vqi;
    const double c = pp.c, C = pp.C, S = pp.S;
    double pr[2], qr[2], pi[2] = {0, 0}, qi[2] = {0, 0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = i0 + 256 * u;
        const bool in = i < n;
        pr[u] = in ? Vpr[i] : 0.0;
        qr[u] = in ? Vqr[i] : 0.0;
        if (CPLX) {
            pi[u] = in ? Vpi[i] : 0.0;
            qi[u] = in ? Vqi[i] : 0.0;
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

template <bool CPLX, int R>
static size_t gstep_shm()
{
    constexpr int NCOL = CPLX ? 4 : 2;
    return sizeof(double) * ((size_t)NCOL * R * kGW + 6 * kGW + 12);
}

template <bool CPLX, int R>
static hipError_t gstep_prepare_t()
{
    // more than 64 KiB of dynamic LDS must be allowed explicitly (set before any capture)
    return hipFuncSetAttribute((const void *)gstep_kernel<CPLX, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)gstep_shm<CPLX, R>());
}

template <bool CPLX, int R>
static hipError_t launch_gstep_t(const SvdDesc &d, PairParam *prm, int grid, hipStream_t s)
{
    const size_t shm = gstep_shm<CPLX, R>();
    hipLaunchKernelGGL((gstep_kernel<CPLX, R>), dim3(grid), dim3(kGW), shm, s, d, prm);
    return hipGetLastError();
}

hipError_t gstep_prepare(int m, int cplx)
{
    switch (cplx ? -gstep_rows(m, 1) : gstep_rows(m, 0)) {
    case -1: return gstep_prepare_t<true, 1>();
    case -2: return gstep_prepare_t<true, 2>();
    case -4: return gstep_prepare_t<true, 4>();
    case -8: return gstep_prepare_t<true, 8>();
    case -16: return gstep_prepare_t<true, 16>();
    case 1: return gstep_prepare_t<false, 1>();
    case 2: return gstep_prepare_t<false, 2>();
    case 4: return gstep_prepare_t<false, 4>();
    case 8: return gstep_prepare_t<false, 8>();
    case 16: return gstep_prepare_t<false, 16>();
    case 32: return gstep_prepare_t<false, 32>();
    }
    return hipSuccess;
}

// rows per thread of the pipelined kernel for m rows (0 = not supported)
int gstep_rows(int m, int cplx)
{
    const int R = (m + kGW - 1) / kGW;
    const int rmax = cplx ? 16 : 32;
    if (R > rmax) return 0;
    int r = 1;
    while (r < R) r *= 2;
    return r;
}

hipError_t launch_gstep(const SvdDesc &d, PairParam *prm, int grid, hipStream_t s)
{
    const int R = gstep_rows(d.m, d.cplx);
    const int npairs = (d.n + (d.n & 1)) / 2;
    if (grid > npairs) grid = npairs;
    hipError_t e = hipErrorInvalidValue;
    if (d.cplx) {
        switch (R) {
        case 1: e = launch_gstep_t<true, 1>(d, prm, grid, s); break;
        case 2: e = launch_gstep_t<true, 2>(d, prm, grid, s); break;
        case 4: e = launch_gstep_t<true, 4>(d, prm, grid, s); break;
        case 8: e = launch_gstep_t<true, 8>(d, prm, grid, s); break;
        case 16: e = launch_gstep_t<true, 16>(d, prm, grid, s); break;
        }
    } else {
        switch (R) {
        case 1: e = launch_gstep_t<false, 1>(d, prm, grid, s); break;
        case 2: e = launch_gstep_t<false, 2>(d, prm, grid, s); break;
        case 4: e = launch_gstep_t<false, 4>(d, prm, grid, s); break;
        case 8: e = launch_gstep_t<false, 8>(d, prm, grid, s); break;
        case 16: e = launch_gstep_t<false, 16>(d, prm, grid, s); break;
        case 32: e = launch_gstep_t<false, 32>(d, prm, grid, s); break;
        }
    }
    if (e != hipSuccess) return e;
    dim3 vgrid(npairs, (d.n + 511) / 512);
    if (d.cplx)
        hipLaunchKernelGGL(vrot_kernel<true>, vgrid, dim3(256), 0, s, d, prm);
    else
        hipLaunchKernelGGL(vrot_kernel<false>, vgrid, dim3(256), 0, s, d, prm);
    return hipGetLastError();
}

} // namespace jsvd
