// kernels.hpp -- internal launch interface between the C ABI (capi.cpp) and
// the HIP kernels.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/jsvd.h"

namespace jsvd {

// Iteration flags: only the bits in `allowed`, and not both JSVD_PERMUTE and
// JSVD_NO_PERMUTE.
inline bool iter_flags_valid(unsigned flags, unsigned allowed)
{
    return (flags & ~allowed) == 0 && !((flags & JSVD_PERMUTE) && (flags & JSVD_NO_PERMUTE));
}

// 1 (apply U, the default) unless the EVD's sorting permutation is asked for.
inline int iter_nosort(unsigned flags) { return (flags & JSVD_PERMUTE) ? 0 : 1; }

// the EVD's streams moved without arithmetic (the memory ceiling of launch_evd2
// at batches of 2^22 and more)
hipError_t launch_evd2_stream(size_t r, const double *a11, const double *a22, const double *ar, const double *ai,
                              double *cs, double *cr, double *ci, double *l1, double *l2, int32_t *zp,
                              hipStream_t s);
hipError_t launch_evd2(size_t r, const double *a11, const double *a22, const double *ar,
                       const double *ai, double *cs, double *cr, double *ci, double *l1,
                       double *l2, int32_t *zp, unsigned flags, hipStream_t s);

// single precision batched EVD: `widest` matrices per lane at most (1, 2 or
// 4; fewer when a stream's alignment does not allow the wider accesses)
hipError_t launch_sevd2(size_t r, const float *a11, const float *a22, const float *ar, const float *ai, float *cs,
                        float *cr, float *ci, float *l1, float *l2, int32_t *zp, unsigned flags, int widest,
                        hipStream_t s);

// Device-resident scalars of one SVD (updated only by kernels).
struct DevScalars {
    unsigned long long Mt_bits;   // M~_k as the bit pattern of a non-negative double
    long long k;                  // global step counter
    long long T;                  // transformations in the current sweep
    long long SW;                 // swaps without transformation in the current sweep
    long long last_t;             // transformations of the last completed step
    long long sweeps;             // sweeps completed
    long long C;                  // sweeps that found a transformation or a swap
    long long T_prev;             // transformations of the last completed sweep
    long long SW_prev;            // swaps without transformation of the last completed sweep
    long long GS;                 // Gram-Schmidt transformations in the current sweep (counted in T)
    long long GS_prev;            // Gram-Schmidt transformations of the last completed sweep
    int s;                        // effective scaling exponent
    int rescaled;                 // step-start downscalings
    int converged;                // a sweep without transformation and swap was seen
    int stop;                     // set when converged or the sweep limit is reached
    int max_sweeps;
    int status;                   // init status: 0, or -2 (non-finite), -3 (zero)
    int loop_ok;                  // the next sweep may run as one persistent launch (loop.hip)
    int loop_epoch;               // persistent sweeps launched (tags the column flags)
    int loop_redo;                // the last persistent sweep gave up: redo it step by step
    long long loop_sweeps;        // sweeps completed as persistent launches
    long long skipped;            // pairs of large-column steps not read: unchanged since they last met
};

// Problem description shared by the SVD kernels, for the working precision T
// (double, or float for the single precision variant).  Device scalars that
// hold a value of the working precision (M~, the max-norms) keep it as a
// double: a float converts to double and back exactly.
template <typename T>
struct SvdDescT {
    int m, n;
    int cplx;
    int nosort;            // ignore the permutation of the EVD during the iteration (the default)
    int comp;              // compensated scaled dot-products (Alg. zdpsclcs / ddpsclcs; double only)
    int nogs;              // always rotate (no Gram-Schmidt replacement, eq. GScond)
    T *Gr, *Gi;            // working iteration matrix
    long long ldg;
    T *Vr, *Vi;            // accumulated right transformations
    long long ldv;
    T *e, *f;              // column norms of the last step (e as a value of type T)
    DevScalars *sc;
    int lgbound;           // floor(lg(nu/(varsigma m))) of eq. (skn), nu = DBL_MAX or FLT_MAX
    T ups;                 // fl(sqrt(m)) eps, eps = 2^-53 or 2^-24
    // per column, the step that last changed it (read and kept by the
    // large-column G kernel only; other steps leave it stale, and the host
    // resets it before the G kernel runs again)
    long long *lastmod;
};
using SvdDesc = SvdDescT<double>;
using SvdDescF = SvdDescT<float>;

// outcome of one pivot pair, written by the G kernels for the end-of-step
// fold and the (deferred) V update: 32 bytes, read by the V update as two
// 16-byte loads (the max-norm of the rotated columns, which only the fold
// reads, is kept beside, in the slot's mx array)
struct alignas(16) PairParam {
    double c, C, S;   // cos phi, e^{i alpha} tan phi
    int pq;           // the pair: p | q << 16
    int flag;         // bit 0: transform (rotation of V, counted), bit 1: swap the columns
                      // (permutation P), bit 2: G took the Gram-Schmidt step of eq. (GS),
                      // bit 3: not read, unchanged since its last meeting (counted)
};
static_assert(sizeof(PairParam) == 32, "PairParam is two 16-byte loads");

// index and M~ of a large-column step, for the step after it
struct StepHdr {
    long long k;
    unsigned long long Mt_bits;
};

// one slot of the outcome log of the large-column steps: the pair outcomes,
// the max |component| of each pair's rotated columns (0 if not rotated),
// the step header, and the key of the max-norm of its rotated columns
// ((k << 12) | (floor(lg M) + 1075), an atomic max over the workgroups)
struct StepSlot {
    PairParam *prm;
    double *mx;
    StepHdr *hdr;
    unsigned long long *mxkey;
};

// step for large columns (gstep.hip): rows per thread of the G kernel for m
// (0 = not supported); one step on G into a log slot (V untouched).  With a
// previous slot (prev.prm != nullptr) the step starts from that step's
// outcomes, whose fold into the device scalars is then also done; without,
// from the device scalars as they are.  launch_fold folds a slot's step
// into the device scalars (for the last step before they are read).  The
// deferred V update applies nsteps logged steps (step j's outcomes at plog +
// j stride) to the row-major V; the in-place transpose switches V between
// its column-major and row-major layouts.
int gpair_rows(int m, int cplx, bool fp32 = false);
int vacc_supported(int n, int cplx, bool fp32);
hipError_t vacc_prepare(int cplx, bool fp32);   // once per state, on its device, outside graph capture
template <typename T>
hipError_t launch_gpair(const SvdDescT<T> &d, StepSlot slot, StepSlot prev, hipStream_t s);
template <typename T>
hipError_t launch_fold(const SvdDescT<T> &d, const PairParam *prm, const double *mx, hipStream_t s);
// every column's last change set to the step about to run (k from the
// previous slot when its fold is still due, else from the device scalars):
// no pair of the large-column steps is skipped before a whole sweep of them
// has met it
template <typename T>
hipError_t launch_lastmod_reset(const SvdDescT<T> &d, StepSlot prev, hipStream_t s);
template <typename T>
hipError_t launch_vacc(const SvdDescT<T> &d, const PairParam *plog, long long stride, int nsteps, hipStream_t s);
template <typename T>
hipError_t launch_vtrans(const SvdDescT<T> &d, hipStream_t s);

// batched scaled dot-products (dot.hip): rows per thread for m (0 = not
// supported) and the launch (one workgroup per column pair)
int dot_rows(int m, int cplx);
hipError_t launch_dot(int npairs, int m, const double *Qr, const double *Qi, const double *Pr, const double *Pi,
                      long long ld, const double *eq, const double *fq, const double *ep, const double *fp,
                      double *zr, double *zi, bool comp, hipStream_t s);

// batched widened-exponent Frobenius norms (nrmf.hip, Alg. rnF): one
// workgroup per column; lanes a power of two <= 1024
hipError_t launch_nrmf(int ncols, int m, const double *Xr, const double *Xi, long long ld, int lanes, double *e2,
                       double *f2, double *e, double *f, hipStream_t s);

// initialisation: M~_0 into *maxbits (zeroed by the caller), then
// G <- 2^{s_0} A copied into the workspace and V <- I
template <typename T>
hipError_t launch_maxabs(const SvdDescT<T> &d, const T *Ar, const T *Ai, long long lda, unsigned long long *maxbits,
                         hipStream_t s);
template <typename T>
hipError_t launch_init_scale(const SvdDescT<T> &d, const T *Ar, const T *Ai, long long lda,
                             const unsigned long long *maxbits, int max_sweeps, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s);
// one parallel step of the fused kernel (G and V in one workgroup per pair);
// threads = 0 picks automatically.  Its outcomes go to the log slot `slot`;
// with a previous slot (prev.prm != nullptr) the step starts from that
// step's outcomes and also folds them into the device scalars, as the
// large-column step does.
template <typename T>
hipError_t launch_step(const SvdDescT<T> &d, int threads, StepSlot slot, StepSlot prev, hipStream_t s);
int step_max_rows(int cplx, int W);
// rows of a state: beyond step_max_rows(cplx, 1024) the step streams the
// pair from memory (sstep.hip)
int state_max_rows();
template <typename T>
hipError_t launch_stream_step(const SvdDescT<T> &d, StepSlot slot, StepSlot prev, hipStream_t s);
int step_auto_threads(int m, int n);
// end-of-sweep bookkeeping (1 thread)
hipError_t launch_sweep_end(DevScalars *sc, hipStream_t s);

// ---------------------------------------------------------------------------
// a whole sweep in one persistent launch (loop.hip), for m <= 256
struct LoopAcc {                  // one workgroup's share of the sweep's fold
    long long t, sw, gs, tlast;   // transformations, swaps, Gram-Schmidt steps, transformations of the last step
    long long sk;                 // pairs not read: unchanged since they last met
    double M;                     // max-norm of the transformed columns
    int done;                     // steps completed (K unless the launch gave up)
    int pad;
};
struct LoopArgs {
    unsigned long long *ver;      // per column: (epoch << 32) | the step offset it is ready for
    LoopAcc *acc;                 // per workgroup
    unsigned *abort;              // raised by a workgroup whose wait ran out of budget
    unsigned long long budget;    // wall-clock ticks a workgroup may wait for one column
    // L2-local mode (nonzero): every pair slot's workgroup on one XCC, columns
    // and flags exchanged through that XCC's L2 without cache maintenance;
    // claim[0] counts the slots taken, claim[1] names the XCC (its id + 1)
    int local;
    unsigned *claim;
};
// the persistent sweep applies to this state (m <= 256, every pair slot resident at once)
template <typename T>
bool loop_fits(const SvdDescT<T> &d, int ncu);
// the sweep may run in the L2-local mode (every slot's workgroup on one XCC,
// one wavefront per SIMD there)
template <typename T>
bool loop_fits_local(const SvdDescT<T> &d, int ncu);
// longest columns of a persistent sweep
int loop_max_rows();
// the persistent sweep and its fold into the device scalars
template <typename T>
hipError_t launch_loop_sweep(const SvdDescT<T> &d, const LoopArgs &a, hipStream_t s);
// loop_ok for the next sweep: no rescaling can happen in it (column sums of
// squares into colsq, n doubles)
template <typename T>
hipError_t launch_loop_check(const SvdDescT<T> &d, double *colsq, hipStream_t s);
hipError_t launch_loop_clear(DevScalars *sc, hipStream_t s);
// finalisation: norms of all columns into d.e/d.f, their descending ranks,
// then U = G diag(2^-e)/f and V permuted into the caller's buffers
template <typename T>
hipError_t launch_colnorms_raw(const SvdDescT<T> &d, hipStream_t s);
template <typename T>
hipError_t launch_rank(const SvdDescT<T> &d, int *rank, hipStream_t s);
template <typename T>
hipError_t launch_final_write(const SvdDescT<T> &d, const int *rank, T *Ur, T *Ui, long long ldu, T *Vr, T *Vi,
                              long long ldv, T *sv_e, T *sv_f, T *sv, hipStream_t s);
// non-converged exit: the current norms, backscaled, in column order
template <typename T>
hipError_t launch_colnorm_out(const SvdDescT<T> &d, T *sv_e, T *sv_f, T *sv, hipStream_t s);
// strided 2D copy (device to device), and 2D scaling by 2^e
template <typename T>
hipError_t launch_copy2d(int m, int n, const T *src, long long lds, T *dst, long long ldd, hipStream_t s);
hipError_t launch_split(int m, int n, const double *Z, long long ldz, double *Xr, double *Xi,
                        long long ldx, hipStream_t s);
hipError_t launch_merge(int m, int n, const double *Xr, const double *Xi, long long ldx, double *Z,
                        long long ldz, hipStream_t s);

} // namespace jsvd
