// capi.cpp -- the C ABI (include/jsvd.h) over the gfx950 kernels: argument
// validation, device workspace, the sweep loop of Alg. zvjsvd
// (arXiv:2202.08361, Sect. 4.3) with hipGraph-captured sweeps, and the
// finalisation.  No exception crosses the ABI.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <limits>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/jsvd.h"
#include "kernels.hpp"
#include "state.hpp"

using namespace jsvd;

#define HIPCHK(x)                                 \
    do {                                          \
        if ((x) != hipSuccess) return JSVD_EDEVICE; \
    } while (0)

// floor(lg(nu / (varsigma m))) of eq. (skn) by integer arithmetic:
// real (varsigma = 2): 1022 - floor(lg m);
// complex (varsigma = 4 sqrt 2): 1021 - floor(lg m) - [m^2 > 2^(2 floor(lg m) + 1)].
static int lg_bound(int m, int cplx)
{
    int a = 0;
    while ((2LL << a) <= (long long)m) ++a;
    if (!cplx) return 1022 - a;
    const unsigned long long mm = (unsigned long long)m * (unsigned long long)m;
    return 1021 - a - (mm > (1ULL << (2 * a + 1)) ? 1 : 0);
}

// The same bound for nu = FLT_MAX = (2^24 - 1) 2^104, evaluated as its
// definition, the largest k with 2^k varsigma m <= nu: nu lies only 2^-24
// (relative) below 2^128, so closed forms like those above can be off by one
// once m approaches that resolution.  The comparisons are exact in double for
// m < 2^26: real 2 m 2^k <= nu, complex (4 sqrt 2 m 2^k)^2 = 32 m^2 2^2k <= nu^2.
static int lg_bound_f32(int m, int cplx)
{
    const double nu24 = 16777215.0;
    for (int k = 160;; --k) {
        const bool fits = cplx ? ldexp(32.0 * (double)m * (double)m, 2 * k) <= ldexp(nu24 * nu24, 208)
                               : ldexp(2.0 * (double)m, k) <= ldexp(nu24, 104);
        if (fits) return k;
    }
}

static long long round_up(long long x, long long a) { return (x + a - 1) / a * a; }

// matrices per lane of the single precision EVD kernel, the fastest of 1, 2
// and 4 measured on MI355X for batches beyond the caches: two (8-byte
// accesses) for the real, one for the complex variant
static int sevd2_lanes_for(bool cplx) { return cplx ? 1 : 2; }

extern "C" int jsvd_version(void) { return (JSVD_VERSION_MAJOR << 16) | JSVD_VERSION_MINOR; }

extern "C" const char *jsvd_strerror(int status)
{
    switch (status) {
    case JSVD_OK: return "ok";
    case JSVD_NOT_CONVERGED: return "not converged within the sweep limit";
    case JSVD_EINVAL: return "invalid argument";
    case JSVD_ENONFINITE: return "input holds Inf or NaN";
    case JSVD_EZERO: return "input is the zero matrix";
    case JSVD_ENOMEM: return "out of memory";
    case JSVD_EDEVICE: return "HIP runtime error";
    case JSVD_EAGAIN: return "request not admitted now";
    case JSVD_ENOTFOUND: return "unknown ticket";
    }
    return "unknown status";
}

// ---------------------------------------------------------------------------
// batched EVD
extern "C" int jsvd_evd2_batched(size_t r, const double *a11, const double *a22, const double *a21_re,
                                 const double *a21_im, double *cos_phi, double *ctan_re, double *ctan_im,
                                 double *lambda1, double *lambda2, int32_t *zp, unsigned flags, void *stream)
{
    if (flags & ~3u) return JSVD_EINVAL;
    if (r == 0) return JSVD_OK;
    if (!a11 || !a22 || !a21_re || !cos_phi || !ctan_re) return JSVD_EINVAL;
    if ((a21_im == nullptr) != (ctan_im == nullptr)) return JSVD_EINVAL;
    if (r > (size_t)1 << 40) return JSVD_EINVAL;
    if (launch_evd2(r, a11, a22, a21_re, a21_im, cos_phi, ctan_re, ctan_im, lambda1, lambda2, zp, flags,
                    (hipStream_t)stream) != hipSuccess)
        return JSVD_EDEVICE;
    return JSVD_OK;
}

extern "C" int jsvd_evd2_stream_ceiling(size_t r, const double *a11, const double *a22, const double *a21_re,
                                        const double *a21_im, double *cos_phi, double *ctan_re, double *ctan_im,
                                        double *lambda1, double *lambda2, int32_t *zp, void *stream)
{
    if (r == 0) return JSVD_OK;
    if (!a11 || !a22 || !a21_re || !cos_phi || !ctan_re || !lambda1 || !lambda2 || !zp) return JSVD_EINVAL;
    if ((a21_im == nullptr) != (ctan_im == nullptr)) return JSVD_EINVAL;
    if (r > (size_t)1 << 40) return JSVD_EINVAL;
    if (launch_evd2_stream(r, a11, a22, a21_re, a21_im, cos_phi, ctan_re, ctan_im, lambda1, lambda2, zp,
                           (hipStream_t)stream) != hipSuccess)
        return JSVD_EDEVICE;
    return JSVD_OK;
}

extern "C" int jsvd_evd2_batched_f32(size_t r, const float *a11, const float *a22, const float *a21_re,
                                     const float *a21_im, float *cos_phi, float *ctan_re, float *ctan_im,
                                     float *lambda1, float *lambda2, int32_t *zp, unsigned flags, void *stream)
{
    if (flags & ~3u) return JSVD_EINVAL;
    if (r == 0) return JSVD_OK;
    if (!a11 || !a22 || !a21_re || !cos_phi || !ctan_re) return JSVD_EINVAL;
    if ((a21_im == nullptr) != (ctan_im == nullptr)) return JSVD_EINVAL;
    if (r > (size_t)1 << 40) return JSVD_EINVAL;
    if (launch_sevd2(r, a11, a22, a21_re, a21_im, cos_phi, ctan_re, ctan_im, lambda1, lambda2, zp, flags,
                     sevd2_lanes_for(a21_im != nullptr), (hipStream_t)stream) != hipSuccess)
        return JSVD_EDEVICE;
    return JSVD_OK;
}

// ---------------------------------------------------------------------------
// state
static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct StateLayout {
    long long ldg, ldv, vstride;
    size_t oG, oV, oE, oF, oR, oS, oM, oP, oQ, oX, oH, oT;
    size_t oLV, oLA, oLC, oLB, oLZ;   // persistent sweeps (m <= 1024): flags, folds, sums, abort, snapshot
    size_t total;
};

// states whose sweeps may run as one persistent launch
static bool loop_candidate_shape(int m) { return m <= loop_max_rows(); }

// es: bytes per element of the working precision
static StateLayout state_layout(int m, int n, int cplx, size_t es)
{
    StateLayout L;
    // columns of the working G start on 1 KiB boundaries
    L.ldg = round_up(m, (long long)(1024 / es));
    L.ldv = round_up(n, 64);
    const int c = cplx ? 2 : 1;
    size_t off = 0;
    L.oG = off; off = align_up(off + es * (size_t)L.ldg * n * c);
    L.oV = off; off = align_up(off + es * (size_t)L.ldv * n * c);
    L.oE = off; off = align_up(off + es * (size_t)n);
    L.oF = off; off = align_up(off + es * (size_t)n);
    L.oR = off; off = align_up(off + sizeof(int) * (size_t)(n + 1));
    L.oS = off; off = align_up(off + sizeof(DevScalars));
    L.oM = off; off = align_up(off + sizeof(unsigned long long));
    // the outcome log: kVlogSlots slots of the step's pair outcomes
    L.vstride = round_up((long long)(n + 1) / 2, 4LL);
    L.oP = off; off = align_up(off + sizeof(PairParam) * (size_t)L.vstride * kVlogSlots);
    L.oQ = off; off = align_up(off + sizeof(double) * (size_t)L.vstride * kVlogSlots);
    L.oH = off; off = align_up(off + sizeof(StepHdr) * (size_t)kVlogSlots);
    L.oX = off; off = align_up(off + sizeof(unsigned long long) * (size_t)kVlogSlots);
    // per column, the step that last changed it (large-column steps)
    L.oT = off; off = align_up(off + sizeof(long long) * (size_t)n);
    L.oLV = L.oLA = L.oLC = L.oLB = L.oLZ = 0;
    if (loop_candidate_shape(m)) {
        const size_t npairs = (size_t)(n + 1) / 2;
        L.oLV = off; off = align_up(off + sizeof(unsigned long long) * (size_t)n);
        L.oLA = off; off = align_up(off + sizeof(LoopAcc) * npairs);
        L.oLC = off; off = align_up(off + sizeof(double) * (size_t)n);
        L.oLB = off; off = align_up(off + sizeof(unsigned));
        // the snapshot: G, V, e and f, one contiguous block from oG to oR
        L.oLZ = off; off = align_up(off + (L.oR - L.oG));
    }
    L.total = off;
    return L;
}

size_t jsvd::state_bytes(int m, int n, int cplx, bool fp32)
{
    return state_layout(m, n, cplx, fp32 ? sizeof(float) : sizeof(double)).total;
}

// the descriptor of the state's working precision
template <typename T>
static SvdDescT<T> &desc_of(jsvd_state st);
template <>
SvdDescT<double> &desc_of<double>(jsvd_state st) { return st->d; }
template <>
SvdDescT<float> &desc_of<float>(jsvd_state st) { return st->df; }

template <typename T>
static void fill_desc(SvdDescT<T> &d, int m, int n, int cplx, char *b, const StateLayout &L, int lgbound, T ups)
{
    d.m = m;
    d.n = n;
    d.cplx = cplx;
    d.nosort = 1;
    d.comp = 0;
    d.nogs = 0;
    d.Gr = (T *)(b + L.oG);
    d.Gi = cplx ? d.Gr + (size_t)L.ldg * n : nullptr;
    d.ldg = L.ldg;
    d.Vr = (T *)(b + L.oV);
    d.Vi = cplx ? d.Vr + (size_t)L.ldv * n : nullptr;
    d.ldv = L.ldv;
    d.e = (T *)(b + L.oE);
    d.f = (T *)(b + L.oF);
    d.sc = (DevScalars *)(b + L.oS);
    d.lgbound = lgbound;
    d.ups = ups;
    d.lastmod = (long long *)(b + L.oT);
}

static int state_create(int m, int n, int is_complex, bool fp32, jsvd_state *out)
{
    if (!out) return JSVD_EINVAL;
    *out = nullptr;
    if (n < 1 || m < n) return JSVD_EINVAL;
    if (m > state_max_rows()) return JSVD_EINVAL;
    jsvd_state st = new (std::nothrow) jsvd_state_s;
    if (!st) return JSVD_ENOMEM;
    memset(st, 0, sizeof(*st));
    st->m = m;
    st->n = n;
    st->cplx = is_complex != 0;
    st->fp32 = fp32 ? 1 : 0;
    st->max_sweeps = 128;
    if (hipGetDevice(&st->device) != hipSuccess) {
        delete st;
        return JSVD_EDEVICE;
    }
    if (hipDeviceGetAttribute(&st->ncu, hipDeviceAttributeMultiprocessorCount, st->device) != hipSuccess ||
        st->ncu <= 0)
        st->ncu = 256;
    const StateLayout L = state_layout(m, n, st->cplx, fp32 ? sizeof(float) : sizeof(double));
    if (hipMalloc(&st->mem, L.total) != hipSuccess) {
        delete st;
        return JSVD_ENOMEM;
    }
    st->mem_bytes = L.total;
    if (vacc_prepare(st->cplx, fp32) != hipSuccess) {
        (void)hipFree(st->mem);
        delete st;
        return JSVD_EDEVICE;
    }
    if (hipHostMalloc((void **)&st->host, 512, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(st->mem);
        delete st;
        return JSVD_ENOMEM;
    }
    static_assert(sizeof(DevScalars) <= 256, "staging layout");
    char *b = (char *)st->mem;
    if (fp32)
        fill_desc<float>(st->df, m, n, st->cplx, b, L, lg_bound_f32(m, st->cplx), ldexpf(sqrtf((float)m), -24));
    else
        fill_desc<double>(st->d, m, n, st->cplx, b, L, lg_bound(m, st->cplx), ldexp(sqrt((double)m), -53));
    st->sc = (DevScalars *)(b + L.oS);
    st->rank = (int *)(b + L.oR);
    st->maxbits = (unsigned long long *)(b + L.oM);
    st->vlog = (PairParam *)(b + L.oP);
    st->vmx = (double *)(b + L.oQ);
    st->vhdr = (StepHdr *)(b + L.oH);
    st->vkey = (unsigned long long *)(b + L.oX);
    st->vlog_stride = L.vstride;
    st->vlog_n = 0;
    st->vbase = 0;
    st->vlast = -1;
    st->v_layout = V_EITHER;
    // the device scalars start from zero (loop_epoch included)
    if (hipMemset(st->sc, 0, sizeof(DevScalars)) != hipSuccess) {
        jsvd_state_destroy(st);
        return JSVD_EDEVICE;
    }
    if (loop_candidate_shape(m)) {
        st->loop_cand = 1;
        st->loop.ver = (unsigned long long *)(b + L.oLV);
        st->loop.acc = (LoopAcc *)(b + L.oLA);
        st->loop.abort = (unsigned *)(b + L.oLB);
        // the slot claims of an L2-local launch, in the abort flag's block
        st->loop.claim = st->loop.abort + 1;
        st->loop.local = 0;
        st->loop_local_allow = 1;
        st->colsq = (double *)(b + L.oLC);
        st->snap = b + L.oLZ;
        st->snap_bytes = L.oR - L.oG;
        // a wait for one column may take 0.25 s (wall clock) before the sweep gives up
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, st->device) != hipSuccess || khz <= 0)
            khz = 100000;
        st->loop.budget = (unsigned long long)khz * 250ull;
        // column flags of epoch 0, a lowered abort flag and scalars of epoch 0
        // (outside any graph)
        if (hipMemset(b + L.oLV, 0, L.oLC - L.oLV) != hipSuccess || hipMemset(b + L.oLB, 0, 256) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess) {
            jsvd_state_destroy(st);
            return JSVD_EDEVICE;
        }
    }
    *out = st;
    return JSVD_OK;
}

extern "C" int jsvd_state_create(int m, int n, int is_complex, jsvd_state *out)
{
    return state_create(m, n, is_complex, false, out);
}

extern "C" int jsvd_state_create_f32(int m, int n, int is_complex, jsvd_state *out)
{
    return state_create(m, n, is_complex, true, out);
}

extern "C" void jsvd_state_destroy(jsvd_state st)
{
    if (!st) return;
    if (st->graph) (void)hipGraphExecDestroy(st->graph);
    if (st->graph_def) (void)hipGraphDestroy(st->graph_def);
    if (st->loop_graph) (void)hipGraphExecDestroy(st->loop_graph);
    if (st->loop_graph_def) (void)hipGraphDestroy(st->loop_graph_def);
    if (st->mem) (void)hipFree(st->mem);
    if (st->host) (void)hipHostFree(st->host);
    delete st;
}

static int push_scalars(jsvd_state st, const DevScalars &h, hipStream_t s)
{
    *st->host = h;
    HIPCHK(hipMemcpyAsync(st->sc, st->host, sizeof(DevScalars), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return JSVD_OK;
}

static int pull_scalars(jsvd_state st, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(st->host, st->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return JSVD_OK;
}

static unsigned long long dbits(double x)
{
    unsigned long long b;
    memcpy(&b, &x, 8);
    return b;
}

static double bitsd(unsigned long long b)
{
    double x;
    memcpy(&x, &b, 8);
    return x;
}

// a state of the precision T
template <typename T>
static bool is_prec(jsvd_state st)
{
    return st && (st->fp32 != 0) == (sizeof(T) == sizeof(float));
}

// The load is stream-ordered: M~_0 is reduced on the device, s_0 and the
// status are derived there too, and nothing waits for the host.
template <typename T>
static int load_async_t(jsvd_state st, const T *G_re, const T *G_im, size_t ldg, hipStream_t s)
{
    if (!is_prec<T>(st) || !G_re || ldg < (size_t)st->m) return JSVD_EINVAL;
    if ((G_im != nullptr) != (st->cplx != 0)) return JSVD_EINVAL;
    const SvdDescT<T> &d = desc_of<T>(st);
    HIPCHK(launch_zero_u64(st->maxbits, s));
    HIPCHK(launch_maxabs(d, G_re, G_im, (long long)ldg, st->maxbits, s));
    HIPCHK(launch_init_scale(d, G_re, G_im, (long long)ldg, st->maxbits, st->max_sweeps, s));
    // whether the first sweep may run as one persistent launch
    if (st->loop_cand) HIPCHK(launch_loop_check(d, st->colsq, s));
    // V = I: the same in either layout, nothing logged, the scalars current,
    // no step keys (k starts again from 0)
    HIPCHK(hipMemsetAsync(st->vkey, 0, sizeof(unsigned long long) * kVlogSlots, s));
    st->vlog_n = 0;
    st->vlast = -1;
    st->v_layout = V_EITHER;
    st->lastmod_valid = 0;
    return JSVD_OK;
}

int jsvd::state_load_async(jsvd_state st, const double *G_re, const double *G_im, size_t ldg, hipStream_t s)
{
    return load_async_t<double>(st, G_re, G_im, ldg, s);
}

int jsvd::state_load_async(jsvd_state st, const float *G_re, const float *G_im, size_t ldg, hipStream_t s)
{
    return load_async_t<float>(st, G_re, G_im, ldg, s);
}

template <typename T>
static int load_t(jsvd_state st, const T *G_re, const T *G_im, size_t ldg, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    int rc = load_async_t<T>(st, G_re, G_im, ldg, s);
    if (rc != JSVD_OK) return rc;
    rc = pull_scalars(st, s);
    if (rc != JSVD_OK) return rc;
    return st->host->status;
}

extern "C" int jsvd_state_load(jsvd_state st, const double *G_re, const double *G_im, size_t ldg, void *stream)
{
    return load_t<double>(st, G_re, G_im, ldg, stream);
}

extern "C" int jsvd_state_load_f32(jsvd_state st, const float *G_re, const float *G_im, size_t ldg, void *stream)
{
    return load_t<float>(st, G_re, G_im, ldg, stream);
}

extern "C" int jsvd_state_set_launch(jsvd_state st, int threads_per_pair)
{
    if (!st) return JSVD_EINVAL;
    const int t = threads_per_pair;
    if (t != 0 && t != 64 && t != 128 && t != 256 && t != 512 && t != 1024) return JSVD_EINVAL;
    if (t != 0 && st->m > step_max_rows(st->cplx, t)) return JSVD_EINVAL;
    st->threads = t;
    return JSVD_OK;
}

static constexpr unsigned kIterFlags = JSVD_NO_PERMUTE | JSVD_PERMUTE | JSVD_COMPENSATED | JSVD_NO_GS;
static constexpr unsigned kIterFlagsF32 = JSVD_NO_PERMUTE | JSVD_PERMUTE | JSVD_NO_GS;

// the iteration flags a state accepts (the compensated dot-products are
// double precision only)
static unsigned iter_flags_of(jsvd_state st) { return st->fp32 ? kIterFlagsF32 : kIterFlags; }

static void apply_flags(jsvd_state st, unsigned flags)
{
    // a pair's earlier decision holds only under the same flags
    if (flags != st->flags) st->lastmod_valid = 0;
    st->flags = flags;
    const int nosort = iter_nosort(flags);
    const int comp = (flags & JSVD_COMPENSATED) ? 1 : 0;
    const int nogs = (flags & JSVD_NO_GS) ? 1 : 0;
    st->d.nosort = st->df.nosort = nosort;
    st->d.comp = st->df.comp = comp;
    st->d.nogs = st->df.nogs = nogs;
}

extern "C" int jsvd_state_set_flags(jsvd_state st, unsigned flags)
{
    if (!st || !iter_flags_valid(flags, iter_flags_of(st))) return JSVD_EINVAL;
    apply_flags(st, flags);
    return JSVD_OK;
}

int jsvd::state_set_flags(jsvd_state st, unsigned flags) { return jsvd_state_set_flags(st, flags); }

static int state_threads(jsvd_state st)
{
    return st->threads ? st->threads : step_auto_threads(st->m, st->n);
}

// one step: for long columns (and no forced workgroup size) the G kernel and
// the fold, with V updated from the outcome log (deferred), otherwise the
// fused one-workgroup-per-pair kernel
static bool uses_gpair(jsvd_state st)
{
    return st->threads == 0 && gpair_rows(st->m, st->cplx, st->fp32 != 0) != 0 && st->m > 256 &&
           vacc_supported(st->n, st->cplx, st->fp32 != 0);
}

// apply the logged steps to V (row-major while anything is logged)
template <typename T>
static hipError_t flush_vlog_t(jsvd_state st, hipStream_t s)
{
    if (st->vlog_n == 0) return hipSuccess;
    const int nsteps = st->vlog_n;
    st->vlog_n = 0;
    return launch_vacc(desc_of<T>(st), st->vlog + (size_t)st->vbase * st->vlog_stride, st->vlog_stride, nsteps, s);
}

static hipError_t flush_vlog(jsvd_state st, hipStream_t s)
{
    return st->fp32 ? flush_vlog_t<float>(st, s) : flush_vlog_t<double>(st, s);
}

// V in the layout `want` (V_COLS or V_ROWS) with every logged step applied
// once it is column-major
static hipError_t set_v_layout(jsvd_state st, int want, hipStream_t s)
{
    if (st->v_layout == V_EITHER || st->v_layout == want) {
        st->v_layout = want;
        return want == V_COLS ? flush_vlog(st, s) : hipSuccess;
    }
    hipError_t e = flush_vlog(st, s);
    if (e != hipSuccess) return e;
    e = st->fp32 ? launch_vtrans(st->df, s) : launch_vtrans(st->d, s);
    if (e != hipSuccess) return e;
    st->v_layout = want;
    return hipSuccess;
}

static int path_layout(jsvd_state st) { return uses_gpair(st) ? V_ROWS : V_COLS; }

static StepSlot slot_of(jsvd_state st, int j)
{
    StepSlot z;
    z.prm = st->vlog + (size_t)j * st->vlog_stride;
    z.mx = st->vmx + (size_t)j * st->vlog_stride;
    z.hdr = st->vhdr + j;
    z.mxkey = st->vkey + j;
    return z;
}

// the device scalars up to date: the fold of the last large-column step,
// which the next such step would otherwise do
static hipError_t settle(jsvd_state st, hipStream_t s)
{
    if (st->vlast < 0) return hipSuccess;
    const StepSlot z = slot_of(st, st->vlast);
    st->vlast = -1;
    return st->fp32 ? launch_fold(st->df, z.prm, z.mx, s) : launch_fold(st->d, z.prm, z.mx, s);
}

// one step on a state whose V is in the path's layout.  Each step continues
// from the previous one's slot (if its fold is still due) and logs its
// outcomes to a slot of its own.  On the large-column path that is the next
// slot of the outcome log, and a full log is applied to V; the fused kernel
// (V rotated in the step, no V update pending) alternates between slots 0
// and 1.
template <typename T>
static hipError_t launch_one_step_t(jsvd_state st, hipStream_t s, bool defer = false)
{
    const SvdDescT<T> &d = desc_of<T>(st);
    StepSlot prev;
    prev.prm = nullptr;
    prev.mx = nullptr;
    prev.hdr = nullptr;
    prev.mxkey = nullptr;
    if (!uses_gpair(st)) {
        if (st->vlast >= 0) prev = slot_of(st, st->vlast);
        const int jf = st->vlast == 0 ? 1 : 0;
        const hipError_t e = launch_step(d, state_threads(st), slot_of(st, jf), prev, s);
        if (e != hipSuccess) return e;
        st->vlast = jf;
        st->lastmod_valid = 0;   // this kernel changes columns without recording it
        return hipSuccess;
    }
    const int j = st->vbase + st->vlog_n;
    if (st->vlast == j) {
        // the last step was a fused one logged in the slot this step fills
        const hipError_t e = settle(st, s);
        if (e != hipSuccess) return e;
    }
    if (st->vlast >= 0) prev = slot_of(st, st->vlast);
    if (!st->lastmod_valid) {
        const hipError_t e = launch_lastmod_reset(d, prev, s);
        if (e != hipSuccess) return e;
        st->lastmod_valid = 1;
    }
    const hipError_t e = launch_gpair(d, slot_of(st, j), prev, s);
    if (e != hipSuccess) return e;
    st->vlast = j;
    if (++st->vlog_n == kVlogSteps && !defer) return flush_vlog_t<T>(st, s);
    return hipSuccess;
}

static hipError_t launch_one_step(jsvd_state st, hipStream_t s)
{
    return st->fp32 ? launch_one_step_t<float>(st, s) : launch_one_step_t<double>(st, s);
}

extern "C" int jsvd_step(jsvd_state st, void *stream)
{
    if (!st) return JSVD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(set_v_layout(st, path_layout(st), s));
    HIPCHK(launch_one_step(st, s));
    return JSVD_OK;
}

static int sweep_steps(int n) { return n + (n & 1) - 1; }

static hipError_t loop_check(jsvd_state st, hipStream_t s)
{
    return st->fp32 ? launch_loop_check(st->df, st->colsq, s) : launch_loop_check(st->d, st->colsq, s);
}

// Pair slots up to which a persistent sweep beats the step-by-step one
// (measured, whole SVDs: n = 256: 1.35-1.41x, n = 300: 1.21-1.23x, n = 384:
// 1.06-1.13x, n = 512: 0.86-0.99x, n = 1024: 0.53x).  Each step of the
// persistent sweep writes back and invalidates caches per workgroup, and
// with more workgroups that costs more than the launch boundary it saves.
constexpr int kLoopMaxPairs = 192;

// The sweep of this state may run as one persistent launch: a state with
// the loop's workspace (automatic launch shape) of at most kLoopMaxPairs
// pair slots, all resident at once.
static bool loop_usable(jsvd_state st)
{
    if (!st->loop_cand || st->threads != 0 || st->loop.budget == 0) return false;
    if ((st->n + 1) / 2 > kLoopMaxPairs) return false;
    return st->fp32 ? loop_fits(st->df, st->ncu) : loop_fits(st->d, st->ncu);
}

// The persistent sweep of this state runs in the L2-local mode: allowed, no
// L2-local sweep of the state has given up, and the slots' workgroups fit on
// one XCC with one wavefront per SIMD.
static int loop_local_now(jsvd_state st)
{
    if (!st->loop_local_allow || st->loop_local_failed) return 0;
    return (st->fp32 ? loop_fits_local(st->df, st->ncu) : loop_fits_local(st->d, st->ncu)) ? 1 : 0;
}

// Capture a persistent sweep: the snapshot of G, V, e and f it can be redone
// from, the sweep with its fold, the check for the sweep after it, and the
// end-of-sweep bookkeeping (which skips a sweep that gave up).
static int build_loop_graph(jsvd_state st)
{
    st->loop.local = loop_local_now(st);
    if (st->loop_graph && st->loop_graph_flags == st->flags && st->loop_graph_budget == st->loop.budget &&
        st->loop_graph_local == st->loop.local)
        return JSVD_OK;
    if (st->loop_graph) {
        (void)hipGraphExecDestroy(st->loop_graph);
        st->loop_graph = nullptr;
    }
    if (st->loop_graph_def) {
        (void)hipGraphDestroy(st->loop_graph_def);
        st->loop_graph_def = nullptr;
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return JSVD_EDEVICE;
    int rc = JSVD_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = JSVD_EDEVICE;
    } else {
        char *gbase = st->fp32 ? (char *)st->df.Gr : (char *)st->d.Gr;
        if (hipMemcpyAsync(st->snap, gbase, st->snap_bytes, hipMemcpyDeviceToDevice, cs) != hipSuccess ||
            (st->fp32 ? launch_loop_sweep(st->df, st->loop, cs) : launch_loop_sweep(st->d, st->loop, cs)) !=
                hipSuccess ||
            loop_check(st, cs) != hipSuccess || launch_sweep_end(st->sc, cs) != hipSuccess)
            rc = JSVD_EDEVICE;
        if (hipStreamEndCapture(cs, &g) != hipSuccess && rc == JSVD_OK) rc = JSVD_EDEVICE;
    }
    (void)hipStreamDestroy(cs);
    if (rc == JSVD_OK && (!g || hipGraphInstantiate(&st->loop_graph, g, nullptr, nullptr, 0) != hipSuccess))
        rc = JSVD_EDEVICE;
    if (rc != JSVD_OK) {
        if (g) (void)hipGraphDestroy(g);
        st->loop_graph = nullptr;
        return rc;
    }
    st->loop_graph_def = g;
    st->loop_graph_flags = st->flags;
    st->loop_graph_budget = st->loop.budget;
    st->loop_graph_local = st->loop.local;
    return JSVD_OK;
}

// Capture the K steps of a sweep, the update of V from the steps still
// logged, and the end-of-sweep bookkeeping.  The log is empty when the
// capture starts and when the graph ends.  On the large-column path each
// full half of the log is applied to V on a second stream (vs), beside the
// steps that fill the other half: a step only waits for the update of the
// half it is about to overwrite, issued a half earlier, and the sweep's end
// waits for the last update.  The events made here (evs) live until the
// capture has ended.
static int capture_sweep(jsvd_state st, hipStream_t cs, hipStream_t vs, std::vector<hipEvent_t> &evs)
{
    const int K = sweep_steps(st->n);
    if (!uses_gpair(st)) {
        for (int k = 0; k < K; ++k)
            if (launch_one_step(st, cs) != hipSuccess) return JSVD_EDEVICE;
        if (flush_vlog(st, cs) != hipSuccess || settle(st, cs) != hipSuccess) return JSVD_EDEVICE;
        // whether the next sweep may run as one persistent launch
        if (st->loop_cand && loop_check(st, cs) != hipSuccess) return JSVD_EDEVICE;
        return launch_sweep_end(st->sc, cs) == hipSuccess ? JSVD_OK : JSVD_EDEVICE;
    }
    auto event = [&](hipEvent_t *e) {
        *e = nullptr;
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return false;
        evs.push_back(*e);
        return true;
    };
    // the logged steps of the current half, applied on vs after what cs has issued
    bool forked = false;
    auto update_on_vs = [&](hipEvent_t *done) {
        hipEvent_t f;
        if (!event(&f) || hipEventRecord(f, cs) != hipSuccess || hipStreamWaitEvent(vs, f, 0) != hipSuccess)
            return false;
        forked = true;
        if (flush_vlog(st, vs) != hipSuccess) return false;
        return done == nullptr || (event(done) && hipEventRecord(*done, vs) == hipSuccess);
    };
    hipEvent_t done[2] = {nullptr, nullptr};
    for (int k = 0; k < K; ++k) {
        const hipError_t e = st->fp32 ? launch_one_step_t<float>(st, cs, true) : launch_one_step_t<double>(st, cs, true);
        if (e != hipSuccess) return JSVD_EDEVICE;
        if (st->vlog_n < kVlogSteps) continue;
        if (!update_on_vs(&done[st->vbase / kVlogSteps])) return JSVD_EDEVICE;
        st->vbase = kVlogSteps - st->vbase;
        hipEvent_t &w = done[st->vbase / kVlogSteps];
        if (w) {
            if (hipStreamWaitEvent(cs, w, 0) != hipSuccess) return JSVD_EDEVICE;
            w = nullptr;
        }
    }
    if (st->vlog_n > 0 && !update_on_vs(nullptr)) return JSVD_EDEVICE;
    st->vbase = 0;
    if (forked) {
        hipEvent_t j;
        if (!event(&j) || hipEventRecord(j, vs) != hipSuccess || hipStreamWaitEvent(cs, j, 0) != hipSuccess)
            return JSVD_EDEVICE;
    }
    if (settle(st, cs) != hipSuccess) return JSVD_EDEVICE;
    // whether the next sweep may run as one persistent launch
    if (st->loop_cand && loop_check(st, cs) != hipSuccess) return JSVD_EDEVICE;
    return launch_sweep_end(st->sc, cs) == hipSuccess ? JSVD_OK : JSVD_EDEVICE;
}

static int build_graph(jsvd_state st)
{
    const int thr = st->threads;
    if (st->graph && st->graph_threads == thr && st->graph_flags == st->flags) return JSVD_OK;
    if (st->graph) {
        (void)hipGraphExecDestroy(st->graph);
        st->graph = nullptr;
    }
    if (st->graph_def) {
        (void)hipGraphDestroy(st->graph_def);
        st->graph_def = nullptr;
    }
    hipStream_t cs = nullptr, vs = nullptr;
    std::vector<hipEvent_t> evs;
    int rc = JSVD_OK;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&vs, hipStreamNonBlocking) != hipSuccess)
        rc = JSVD_EDEVICE;
    hipGraph_t g = nullptr;
    if (rc == JSVD_OK) {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = JSVD_EDEVICE;
        } else {
            rc = capture_sweep(st, cs, vs, evs);
            st->vlog_n = 0;
            st->vbase = 0;
            st->vlast = -1;
            // a failed capture still has to be ended
            if (hipStreamEndCapture(cs, &g) != hipSuccess && rc == JSVD_OK) rc = JSVD_EDEVICE;
        }
    }
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    if (vs) (void)hipStreamDestroy(vs);
    if (cs) (void)hipStreamDestroy(cs);
    if (rc == JSVD_OK && (!g || hipGraphInstantiate(&st->graph, g, nullptr, nullptr, 0) != hipSuccess))
        rc = JSVD_EDEVICE;
    if (rc != JSVD_OK) {
        if (g) (void)hipGraphDestroy(g);
        st->graph = nullptr;
        return rc;
    }
    st->graph_def = g;
    st->graph_threads = thr;
    st->graph_flags = st->flags;
    return JSVD_OK;
}

// The per-column steps of the last change, reset (every column "changed
// now") unless they are current: enqueued outside any graph.
static hipError_t lastmod_ensure(jsvd_state st, hipStream_t s)
{
    if (st->lastmod_valid) return hipSuccess;
    StepSlot none;
    none.prm = nullptr;
    none.mx = nullptr;
    none.hdr = nullptr;
    none.mxkey = nullptr;
    const hipError_t e = st->fp32 ? launch_lastmod_reset(st->df, none, s) : launch_lastmod_reset(st->d, none, s);
    if (e == hipSuccess) st->lastmod_valid = 1;
    return e;
}

extern "C" int jsvd_sweep(jsvd_state st, void *stream)
{
    if (!st) return JSVD_EINVAL;
    // V in the path's layout, the log empty and the scalars current, as the
    // captured sweep expects
    HIPCHK(set_v_layout(st, path_layout(st), (hipStream_t)stream));
    HIPCHK(flush_vlog(st, (hipStream_t)stream));
    HIPCHK(settle(st, (hipStream_t)stream));
    // the last-change steps are reset here, outside the graph: inside it the
    // reset would run again at every replay and no pair would ever be skipped
    if (uses_gpair(st)) HIPCHK(lastmod_ensure(st, (hipStream_t)stream));
    const int rc = build_graph(st);
    if (rc != JSVD_OK) return rc;
    HIPCHK(hipGraphLaunch(st->graph, (hipStream_t)stream));
    return JSVD_OK;
}

int jsvd::state_sweep_async(jsvd_state st, hipStream_t s)
{
    const int rc = jsvd_sweep(st, s);
    if (rc != JSVD_OK) return rc;
    HIPCHK(hipMemcpyAsync(st->host, st->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    return JSVD_OK;
}

const DevScalars &jsvd::state_staged(jsvd_state st) { return *st->host; }

template <typename T>
static int finish_async_t(jsvd_state st, bool converged, T *U_re, T *U_im, size_t ldu, T *V_re, T *V_im, size_t ldv,
                          T *sv_e, T *sv_f, T *sv, hipStream_t s)
{
    if (!is_prec<T>(st)) return JSVD_EINVAL;
    const SvdDescT<T> &d = desc_of<T>(st);
    HIPCHK(set_v_layout(st, V_COLS, s));
    HIPCHK(settle(st, s));
    if (converged) {
        HIPCHK(launch_colnorms_raw(d, s));
        HIPCHK(launch_rank(d, st->rank, s));
        HIPCHK(launch_final_write(d, st->rank, U_re, U_im, (long long)ldu, V_re, V_im, (long long)ldv, sv_e, sv_f,
                                  sv, s));
        return JSVD_OK;
    }
    HIPCHK(launch_copy2d(d.m, d.n, (const T *)d.Gr, d.ldg, U_re, (long long)ldu, s));
    if (st->cplx) HIPCHK(launch_copy2d(d.m, d.n, (const T *)d.Gi, d.ldg, U_im, (long long)ldu, s));
    HIPCHK(launch_copy2d(d.n, d.n, (const T *)d.Vr, d.ldv, V_re, (long long)ldv, s));
    if (st->cplx) HIPCHK(launch_copy2d(d.n, d.n, (const T *)d.Vi, d.ldv, V_im, (long long)ldv, s));
    HIPCHK(launch_colnorms_raw(d, s));
    HIPCHK(launch_colnorm_out(d, sv_e, sv_f, sv, s));
    return JSVD_OK;
}

int jsvd::state_finish_async(jsvd_state st, bool converged, double *U_re, double *U_im, size_t ldu, double *V_re,
                             double *V_im, size_t ldv, double *sv_e, double *sv_f, double *sv, hipStream_t s)
{
    return finish_async_t<double>(st, converged, U_re, U_im, ldu, V_re, V_im, ldv, sv_e, sv_f, sv, s);
}

int jsvd::state_finish_async(jsvd_state st, bool converged, float *U_re, float *U_im, size_t ldu, float *V_re,
                             float *V_im, size_t ldv, float *sv_e, float *sv_f, float *sv, hipStream_t s)
{
    return finish_async_t<float>(st, converged, U_re, U_im, ldu, V_re, V_im, ldv, sv_e, sv_f, sv, s);
}

extern "C" int jsvd_state_query(jsvd_state st, jsvd_info *out, void *stream)
{
    if (!st || !out) return JSVD_EINVAL;
    HIPCHK(settle(st, (hipStream_t)stream));
    const int rc = pull_scalars(st, (hipStream_t)stream);
    if (rc != JSVD_OK) return rc;
    const DevScalars &h = *st->host;
    out->steps = h.k;
    out->sweeps = h.C;
    out->T = h.T;
    out->last_t = h.last_t;
    out->swaps = h.SW;
    out->s = h.s;
    out->rescaled = h.rescaled;
    out->Mt = bitsd(h.Mt_bits);
    out->converged = h.converged;
    out->status = h.status;
    out->last_sweep_T = h.T_prev;
    out->last_sweep_swaps = h.SW_prev;
    out->gs = h.GS;
    out->last_sweep_gs = h.GS_prev;
    out->loop_sweeps = h.loop_sweeps;
    out->loop_redos = st->loop_redos;
    out->local_sweeps = st->loop_local_sweeps;
    out->skipped_pairs = h.skipped;
    return JSVD_OK;
}

template <typename T>
static int save_t(jsvd_state st, T *G_re, T *G_im, size_t ldg, T *V_re, T *V_im, size_t ldv, T *e, T *f,
                  int32_t *s_out, double *Mt, int64_t *step, void *stream)
{
    if (!is_prec<T>(st)) return JSVD_EINVAL;
    if (G_re && ldg < (size_t)st->m) return JSVD_EINVAL;
    if (V_re && ldv < (size_t)st->n) return JSVD_EINVAL;
    if (st->cplx && ((G_re && !G_im) || (V_re && !V_im))) return JSVD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const SvdDescT<T> &d = desc_of<T>(st);
    if (G_re) {
        HIPCHK(launch_copy2d(d.m, d.n, (const T *)d.Gr, d.ldg, G_re, (long long)ldg, s));
        if (st->cplx) HIPCHK(launch_copy2d(d.m, d.n, (const T *)d.Gi, d.ldg, G_im, (long long)ldg, s));
    }
    if (V_re) {
        HIPCHK(set_v_layout(st, V_COLS, s));
        HIPCHK(launch_copy2d(d.n, d.n, (const T *)d.Vr, d.ldv, V_re, (long long)ldv, s));
        if (st->cplx) HIPCHK(launch_copy2d(d.n, d.n, (const T *)d.Vi, d.ldv, V_im, (long long)ldv, s));
    }
    if (e) HIPCHK(hipMemcpyAsync(e, d.e, sizeof(T) * d.n, hipMemcpyDeviceToDevice, s));
    if (f) HIPCHK(hipMemcpyAsync(f, d.f, sizeof(T) * d.n, hipMemcpyDeviceToDevice, s));
    HIPCHK(settle(st, s));
    const int rc = pull_scalars(st, s);
    if (rc != JSVD_OK) return rc;
    if (s_out) *s_out = st->host->s;
    if (Mt) *Mt = bitsd(st->host->Mt_bits);
    if (step) *step = st->host->k;
    return JSVD_OK;
}

extern "C" int jsvd_state_save(jsvd_state st, double *G_re, double *G_im, size_t ldg, double *V_re,
                               double *V_im, size_t ldv, double *e, double *f, int32_t *s_out, double *Mt,
                               int64_t *step, void *stream)
{
    return save_t<double>(st, G_re, G_im, ldg, V_re, V_im, ldv, e, f, s_out, Mt, step, stream);
}

extern "C" int jsvd_state_save_f32(jsvd_state st, float *G_re, float *G_im, size_t ldg, float *V_re, float *V_im,
                                   size_t ldv, float *e, float *f, int32_t *s_out, double *Mt, int64_t *step,
                                   void *stream)
{
    return save_t<float>(st, G_re, G_im, ldg, V_re, V_im, ldv, e, f, s_out, Mt, step, stream);
}

template <typename T>
static int restore_t(jsvd_state st, const T *G_re, const T *G_im, size_t ldg, const T *V_re, const T *V_im,
                     size_t ldv, int32_t s_in, double Mt, int64_t step, void *stream)
{
    if (!is_prec<T>(st) || !G_re || !V_re || ldg < (size_t)st->m || ldv < (size_t)st->n) return JSVD_EINVAL;
    if (st->cplx && (!G_im || !V_im)) return JSVD_EINVAL;
    // M~ must be a finite non-negative value of the working precision
    if (!(Mt >= 0.0 && Mt <= (double)std::numeric_limits<T>::max()) || (double)(T)Mt != Mt || step < 0)
        return JSVD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const SvdDescT<T> &d = desc_of<T>(st);
    HIPCHK(launch_copy2d(d.m, d.n, G_re, (long long)ldg, d.Gr, d.ldg, s));
    if (st->cplx) HIPCHK(launch_copy2d(d.m, d.n, G_im, (long long)ldg, d.Gi, d.ldg, s));
    HIPCHK(launch_copy2d(d.n, d.n, V_re, (long long)ldv, d.Vr, d.ldv, s));
    if (st->cplx) HIPCHK(launch_copy2d(d.n, d.n, V_im, (long long)ldv, d.Vi, d.ldv, s));
    // the restored V and scalars replace the logged steps too (and k may
    // go back: no step keys)
    HIPCHK(hipMemsetAsync(st->vkey, 0, sizeof(unsigned long long) * kVlogSlots, s));
    st->vlog_n = 0;
    st->vlast = -1;
    st->v_layout = V_COLS;
    st->lastmod_valid = 0;
    // the pushed scalars start the persistent sweeps' flag epochs again at 0,
    // so the flags are cleared with them
    if (st->loop_cand) HIPCHK(hipMemsetAsync(st->loop.ver, 0, sizeof(unsigned long long) * (size_t)st->n, s));
    DevScalars h;
    memset(&h, 0, sizeof(h));
    h.Mt_bits = dbits(Mt);
    h.s = s_in;
    h.k = step;
    h.max_sweeps = st->max_sweeps;
    return push_scalars(st, h, s);
}

extern "C" int jsvd_state_restore(jsvd_state st, const double *G_re, const double *G_im, size_t ldg,
                                  const double *V_re, const double *V_im, size_t ldv, int32_t s_in, double Mt,
                                  int64_t step, void *stream)
{
    return restore_t<double>(st, G_re, G_im, ldg, V_re, V_im, ldv, s_in, Mt, step, stream);
}

extern "C" int jsvd_state_restore_f32(jsvd_state st, const float *G_re, const float *G_im, size_t ldg,
                                      const float *V_re, const float *V_im, size_t ldv, int32_t s_in, double Mt,
                                      int64_t step, void *stream)
{
    return restore_t<float>(st, G_re, G_im, ldg, V_re, V_im, ldv, s_in, Mt, step, stream);
}

template <typename T>
static int finalize_t(jsvd_state st, T *U_re, T *U_im, size_t ldu, T *V_re, T *V_im, size_t ldv, T *sv_e, T *sv_f,
                      T *sv, void *stream)
{
    if (!is_prec<T>(st) || !U_re || !V_re || !sv_e || !sv_f || ldu < (size_t)st->m || ldv < (size_t)st->n)
        return JSVD_EINVAL;
    if (st->cplx && (!U_im || !V_im)) return JSVD_EINVAL;
    return finish_async_t<T>(st, true, U_re, U_im, ldu, V_re, V_im, ldv, sv_e, sv_f, sv, (hipStream_t)stream);
}

extern "C" int jsvd_state_finalize(jsvd_state st, double *U_re, double *U_im, size_t ldu, double *V_re,
                                   double *V_im, size_t ldv, double *sv_e, double *sv_f, double *sv,
                                   void *stream)
{
    return finalize_t<double>(st, U_re, U_im, ldu, V_re, V_im, ldv, sv_e, sv_f, sv, stream);
}

extern "C" int jsvd_state_finalize_f32(jsvd_state st, float *U_re, float *U_im, size_t ldu, float *V_re,
                                       float *V_im, size_t ldv, float *sv_e, float *sv_f, float *sv, void *stream)
{
    return finalize_t<float>(st, U_re, U_im, ldu, V_re, V_im, ldv, sv_e, sv_f, sv, stream);
}

// ---------------------------------------------------------------------------
// the whole SVD
// Sweeps on a loaded state until it stops (converged, or the sweep limit),
// one graph launch per sweep, synchronising after each: the device decides
// convergence.  Where the device has found that no rescaling can happen in
// the next sweep, the sweep runs as one persistent launch (loop.hip); one
// that gives up is redone step by step from the snapshot taken before it.
int jsvd::state_next_sweep_async(jsvd_state st, hipStream_t s, bool allow_persistent, bool *persistent)
{
    *persistent = false;
    if (allow_persistent && loop_usable(st) && st->host->loop_ok) {
        const int rc = build_loop_graph(st);
        if (rc != JSVD_OK) return rc;
        // a persistent sweep rotates V's columns in place (V column-major); the
        // large-column steps keep V row-major, so a switch between the two
        // transposes V once
        HIPCHK(set_v_layout(st, V_COLS, s));
        HIPCHK(settle(st, s));
        // the sweep reads and keeps the last-change steps (outside its graph,
        // as for the large-column steps)
        HIPCHK(lastmod_ensure(st, s));
        HIPCHK(hipGraphLaunch(st->loop_graph, s));
        HIPCHK(hipMemcpyAsync(st->host, st->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
        *persistent = true;
        return JSVD_OK;
    }
    return state_sweep_async(st, s);
}

int jsvd::state_after_persistent_async(jsvd_state st, hipStream_t s, bool *redone)
{
    *redone = false;
    const bool gave_up = st->host->loop_redo != 0;
    if (st->loop.local) {
        // an L2-local sweep that gave up (too few of its workgroups on the
        // XCC, say) is not tried again on this state
        if (gave_up)
            st->loop_local_failed = 1;
        else
            st->loop_local_sweeps++;
    }
    if (!gave_up) return JSVD_OK;
    // the sweep that gave up recorded part of its changes: the record starts over
    st->lastmod_valid = 0;
    char *gbase = st->fp32 ? (char *)st->df.Gr : (char *)st->d.Gr;
    HIPCHK(hipMemcpyAsync(gbase, st->snap, st->snap_bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_loop_clear(st->sc, s));
    const int rc = state_sweep_async(st, s);
    if (rc != JSVD_OK) return rc;
    st->loop_redos++;
    *redone = true;
    return JSVD_OK;
}

static int iterate(jsvd_state st, hipStream_t s)
{
    HIPCHK(set_v_layout(st, loop_usable(st) ? V_COLS : path_layout(st), s));
    HIPCHK(flush_vlog(st, s));
    HIPCHK(settle(st, s));
    HIPCHK(hipMemcpyAsync(st->host, st->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    while (!st->host->stop) {
        bool as_loop = false, redone = false;
        int rc = state_next_sweep_async(st, s, true, &as_loop);
        if (rc != JSVD_OK) return rc;
        HIPCHK(hipStreamSynchronize(s));
        if (!as_loop) continue;
        rc = state_after_persistent_async(st, s, &redone);
        if (rc != JSVD_OK) return rc;
        if (redone) HIPCHK(hipStreamSynchronize(s));
    }
    return JSVD_OK;
}

extern "C" int jsvd_state_set_loop_wait(jsvd_state st, double seconds)
{
    if (!st || !(seconds >= 0.0 && seconds <= 60.0)) return JSVD_EINVAL;
    if (!st->loop_cand) return JSVD_OK;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, st->device) != hipSuccess || khz <= 0)
        khz = 100000;
    const double ticks = seconds * 1e3 * khz;
    // a positive wait of less than one tick still allows persistent sweeps
    st->loop.budget = seconds == 0.0 ? 0ull : (ticks < 1.0 ? 1ull : (unsigned long long)ticks);
    return JSVD_OK;
}

extern "C" int jsvd_state_set_loop_local(jsvd_state st, int allow)
{
    if (!st || (allow != 0 && allow != 1)) return JSVD_EINVAL;
    st->loop_local_allow = allow;
    st->loop_local_failed = 0;
    return JSVD_OK;
}

extern "C" int jsvd_state_iterate(jsvd_state st, void *stream)
{
    if (!st) return JSVD_EINVAL;
    return iterate(st, (hipStream_t)stream);
}

template <typename T>
static int gesvj_on_state(jsvd_state st, T *G_re, T *G_im, size_t ldg, T *V_re, T *V_im, size_t ldv, T *sv_e,
                          T *sv_f, T *sv, int *sweeps, hipStream_t s)
{
    int rc = load_async_t<T>(st, G_re, G_im, ldg, s);
    if (rc != JSVD_OK) return rc;
    rc = iterate(st, s);
    if (rc != JSVD_OK) return rc;
    const DevScalars h = *st->host;
    if (sweeps) *sweeps = (int)h.C;
    if (h.status != 0) return h.status;
    rc = finish_async_t<T>(st, h.converged != 0, G_re, G_im, ldg, V_re, V_im, ldv, sv_e, sv_f, sv, s);
    if (rc != JSVD_OK) return rc;
    HIPCHK(hipStreamSynchronize(s));
    return h.converged ? JSVD_OK : JSVD_NOT_CONVERGED;
}

template <typename T>
static int gesvj_t(int m, int n, T *G_re, T *G_im, size_t ldg, T *V_re, T *V_im, size_t ldv, T *sv_e, T *sv_f,
                   T *sv, int max_sweeps, int *sweeps, unsigned flags, void *stream)
{
    constexpr bool F32 = sizeof(T) == sizeof(float);
    if (n < 1 || m < n || !G_re || !V_re || !sv_e || !sv_f || ldg < (size_t)m || ldv < (size_t)n)
        return JSVD_EINVAL;
    if ((G_im == nullptr) != (V_im == nullptr)) return JSVD_EINVAL;
    if (!iter_flags_valid(flags, F32 ? kIterFlagsF32 : kIterFlags)) return JSVD_EINVAL;
    jsvd_state st = nullptr;
    int rc = state_create(m, n, G_im != nullptr, F32, &st);
    if (rc != JSVD_OK) return rc;
    st->max_sweeps = max_sweeps > 0 ? max_sweeps : 128;
    apply_flags(st, flags);
    rc = gesvj_on_state<T>(st, G_re, G_im, ldg, V_re, V_im, ldv, sv_e, sv_f, sv, sweeps, (hipStream_t)stream);
    jsvd_state_destroy(st);
    return rc;
}

extern "C" int jsvd_gesvj(int m, int n, double *G_re, double *G_im, size_t ldg, double *V_re, double *V_im,
                          size_t ldv, double *sv_e, double *sv_f, double *sv, int max_sweeps, int *sweeps,
                          unsigned flags, void *stream)
{
    return gesvj_t<double>(m, n, G_re, G_im, ldg, V_re, V_im, ldv, sv_e, sv_f, sv, max_sweeps, sweeps, flags,
                           stream);
}

extern "C" int jsvd_gesvj_f32(int m, int n, float *G_re, float *G_im, size_t ldg, float *V_re, float *V_im,
                              size_t ldv, float *sv_e, float *sv_f, float *sv, int max_sweeps, int *sweeps,
                              unsigned flags, void *stream)
{
    return gesvj_t<float>(m, n, G_re, G_im, ldg, V_re, V_im, ldv, sv_e, sv_f, sv, max_sweeps, sweeps, flags,
                          stream);
}

// ---------------------------------------------------------------------------
// batched scaled dot-products
extern "C" int jsvd_dot_scaled_batched(int npairs, int m, const double *Q_re, const double *Q_im,
                                       const double *P_re, const double *P_im, size_t ld, const double *eq,
                                       const double *fq, const double *ep, const double *fp, double *z_re,
                                       double *z_im, unsigned flags, void *stream)
{
    if (flags & ~JSVD_COMPENSATED) return JSVD_EINVAL;
    if (npairs < 0 || m < 1 || ld < (size_t)m) return JSVD_EINVAL;
    const bool cplx = Q_im != nullptr;
    if ((P_im != nullptr) != cplx || (z_im != nullptr && !cplx) || (cplx && !z_im)) return JSVD_EINVAL;
    if (npairs == 0) return JSVD_OK;
    if (!Q_re || !P_re || !eq || !fq || !ep || !fp || !z_re) return JSVD_EINVAL;
    if (dot_rows(m, cplx) == 0) return JSVD_EINVAL;
    HIPCHK(launch_dot(npairs, m, Q_re, Q_im, P_re, P_im, (long long)ld, eq, fq, ep, fp, z_re, z_im,
                      (flags & JSVD_COMPENSATED) != 0, (hipStream_t)stream));
    return JSVD_OK;
}

// ---------------------------------------------------------------------------
// batched widened-exponent Frobenius norms
extern "C" int jsvd_nrmf_batched(int ncols, int m, const double *X_re, const double *X_im, size_t ld, int lanes,
                                 double *e2, double *f2, double *e, double *f, void *stream)
{
    if (ncols < 0 || m < 0 || lanes < 1 || lanes > 1024 || (lanes & (lanes - 1))) return JSVD_EINVAL;
    if (ncols == 0) return JSVD_OK;
    if (!X_re || !e || !f || ld < (size_t)(m > 0 ? m : 1)) return JSVD_EINVAL;
    if (m > 0 && (size_t)ncols * ld > ((size_t)1 << 40)) return JSVD_EINVAL;
    HIPCHK(launch_nrmf(ncols, m, X_re, X_im, (long long)ld, lanes, e2, f2, e, f, (hipStream_t)stream));
    return JSVD_OK;
}

// ---------------------------------------------------------------------------
// layout helpers
extern "C" int jsvd_split(int m, int n, const double *Z, size_t ldz, double *X_re, double *X_im, size_t ldx,
                          void *stream)
{
    if (m < 0 || n < 0 || !Z || !X_re || !X_im || ldz < 2 * (size_t)m || ldx < (size_t)m) return JSVD_EINVAL;
    HIPCHK(launch_split(m, n, Z, (long long)ldz, X_re, X_im, (long long)ldx, (hipStream_t)stream));
    return JSVD_OK;
}

extern "C" int jsvd_merge(int m, int n, const double *X_re, const double *X_im, size_t ldx, double *Z, size_t ldz,
                          void *stream)
{
    if (m < 0 || n < 0 || !Z || !X_re || !X_im || ldz < 2 * (size_t)m || ldx < (size_t)m) return JSVD_EINVAL;
    HIPCHK(launch_merge(m, n, X_re, X_im, (long long)ldx, Z, (long long)ldz, (hipStream_t)stream));
    return JSVD_OK;
}
