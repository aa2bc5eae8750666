// capi.cpp -- the C ABI (include/jsvd.h) over the gfx950 kernels: argument
// validation, device workspace, the sweep loop of Alg. zvjsvd
// (arXiv:2202.08361, Sect. 4.3) with hipGraph-captured sweeps, and the
// finalisation.  No exception crosses the ABI.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

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
    long long ldg, ldv;
    size_t oG, oV, oE, oF, oR, oS, oM, oP, total;
};

static StateLayout state_layout(int m, int n, int cplx)
{
    StateLayout L;
    // columns of the working G are whole 1 KiB chunks (the LDS prefetch moves 128 doubles at a time)
    L.ldg = round_up(m, 128);
    L.ldv = round_up(n, 64);
    const int c = cplx ? 2 : 1;
    size_t off = 0;
    L.oG = off; off = align_up(off + sizeof(double) * (size_t)L.ldg * n * c);
    L.oV = off; off = align_up(off + sizeof(double) * (size_t)L.ldv * n * c);
    L.oE = off; off = align_up(off + sizeof(double) * (size_t)n);
    L.oF = off; off = align_up(off + sizeof(double) * (size_t)n);
    L.oR = off; off = align_up(off + sizeof(int) * (size_t)(n + 1));
    L.oS = off; off = align_up(off + sizeof(DevScalars));
    L.oM = off; off = align_up(off + sizeof(unsigned long long));
    L.oP = off; off = align_up(off + sizeof(PairParam) * (size_t)((n + 1) / 2 + 1));
    L.total = off;
    return L;
}

size_t jsvd::state_bytes(int m, int n, int cplx) { return state_layout(m, n, cplx).total; }

extern "C" int jsvd_state_create(int m, int n, int is_complex, jsvd_state *out)
{
    if (!out) return JSVD_EINVAL;
    *out = nullptr;
    if (n < 1 || m < n) return JSVD_EINVAL;
    if (m > step_max_rows(is_complex != 0, 1024)) return JSVD_EINVAL;
    jsvd_state st = new (std::nothrow) jsvd_state_s;
    if (!st) return JSVD_ENOMEM;
    memset(st, 0, sizeof(*st));
    st->m = m;
    st->n = n;
    st->cplx = is_complex != 0;
    st->max_sweeps = 128;
    if (hipGetDevice(&st->device) != hipSuccess) {
        delete st;
        return JSVD_EDEVICE;
    }
    if (hipDeviceGetAttribute(&st->ncu, hipDeviceAttributeMultiprocessorCount, st->device) != hipSuccess ||
        st->ncu <= 0)
        st->ncu = 256;
    const StateLayout L = state_layout(m, n, st->cplx);
    if (hipMalloc(&st->mem, L.total) != hipSuccess) {
        delete st;
        return JSVD_ENOMEM;
    }
    st->mem_bytes = L.total;
    if (hipHostMalloc((void **)&st->host, 512, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(st->mem);
        delete st;
        return JSVD_ENOMEM;
    }
    static_assert(sizeof(DevScalars) <= 256, "staging layout");
    char *b = (char *)st->mem;
    SvdDesc &d = st->d;
    d.m = m;
    d.n = n;
    d.cplx = st->cplx;
    d.nosort = 0;
    d.comp = 0;
    d.Gr = (double *)(b + L.oG);
    d.Gi = st->cplx ? d.Gr + (size_t)L.ldg * n : nullptr;
    d.ldg = L.ldg;
    d.Vr = (double *)(b + L.oV);
    d.Vi = st->cplx ? d.Vr + (size_t)L.ldv * n : nullptr;
    d.ldv = L.ldv;
    d.e = (double *)(b + L.oE);
    d.f = (double *)(b + L.oF);
    d.sc = (DevScalars *)(b + L.oS);
    d.lgbound = lg_bound(m, st->cplx);
    d.ups = ldexp(sqrt((double)m), -53);
    st->rank = (int *)(b + L.oR);
    st->maxbits = (unsigned long long *)(b + L.oM);
    st->prm = (PairParam *)(b + L.oP);
    *out = st;
    return JSVD_OK;
}

extern "C" void jsvd_state_destroy(jsvd_state st)
{
    if (!st) return;
    if (st->graph) (void)hipGraphExecDestroy(st->graph);
    if (st->graph_def) (void)hipGraphDestroy(st->graph_def);
    if (st->mem) (void)hipFree(st->mem);
    if (st->host) (void)hipHostFree(st->host);
    delete st;
}

static int push_scalars(jsvd_state st, const DevScalars &h, hipStream_t s)
{
    *st->host = h;
    HIPCHK(hipMemcpyAsync(st->d.sc, st->host, sizeof(DevScalars), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return JSVD_OK;
}

static int pull_scalars(jsvd_state st, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(st->host, st->d.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
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

// The load is stream-ordered: M~_0 is reduced on the device, s_0 and the
// status are derived there too, and nothing waits for the host.
int jsvd::state_load_async(jsvd_state st, const double *G_re, const double *G_im, size_t ldg, hipStream_t s)
{
    if (!st || !G_re || ldg < (size_t)st->m) return JSVD_EINVAL;
    if ((G_im != nullptr) != (st->cplx != 0)) return JSVD_EINVAL;
    HIPCHK(launch_zero_u64(st->maxbits, s));
    HIPCHK(launch_maxabs(st->d, G_re, G_im, (long long)ldg, st->maxbits, s));
    HIPCHK(launch_init_scale(st->d, G_re, G_im, (long long)ldg, st->maxbits, st->max_sweeps, s));
    return JSVD_OK;
}

extern "C" int jsvd_state_load(jsvd_state st, const double *G_re, const double *G_im, size_t ldg, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    int rc = state_load_async(st, G_re, G_im, ldg, s);
    if (rc != JSVD_OK) return rc;
    rc = pull_scalars(st, s);
    if (rc != JSVD_OK) return rc;
    return st->host->status;
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

static constexpr unsigned kIterFlags = JSVD_NO_PERMUTE | JSVD_COMPENSATED;

static void apply_flags(jsvd_state st, unsigned flags)
{
    st->flags = flags;
    st->d.nosort = (flags & JSVD_NO_PERMUTE) ? 1 : 0;
    st->d.comp = (flags & JSVD_COMPENSATED) ? 1 : 0;
}

extern "C" int jsvd_state_set_flags(jsvd_state st, unsigned flags)
{
    if (!st || (flags & ~kIterFlags)) return JSVD_EINVAL;
    apply_flags(st, flags);
    return JSVD_OK;
}

int jsvd::state_set_flags(jsvd_state st, unsigned flags) { return jsvd_state_set_flags(st, flags); }

static int state_threads(jsvd_state st)
{
    return st->threads ? st->threads : step_auto_threads(st->m, st->n);
}

// one step: for long columns (and no forced workgroup size) the G kernel and
// the V kernel, otherwise the fused one-workgroup-per-pair kernel
static bool uses_gpair(jsvd_state st)
{
    return st->threads == 0 && gpair_rows(st->m, st->cplx) != 0 && st->m > 256;
}

static hipError_t launch_one_step(jsvd_state st, hipStream_t s)
{
    if (uses_gpair(st)) return launch_gpair(st->d, st->prm, s);
    return launch_step(st->d, state_threads(st), s);
}

extern "C" int jsvd_step(jsvd_state st, void *stream)
{
    if (!st) return JSVD_EINVAL;
    HIPCHK(launch_one_step(st, (hipStream_t)stream));
    return JSVD_OK;
}

static int sweep_steps(int n) { return n + (n & 1) - 1; }

// Capture the K steps of a sweep and the end-of-sweep bookkeeping.
static int capture_sweep(jsvd_state st, hipStream_t cs)
{
    const int K = sweep_steps(st->n);
    for (int k = 0; k < K; ++k)
        if (launch_one_step(st, cs) != hipSuccess) return JSVD_EDEVICE;
    return launch_sweep_end(st->d, cs) == hipSuccess ? JSVD_OK : JSVD_EDEVICE;
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
    hipStream_t cs = nullptr;
    int rc = JSVD_OK;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) rc = JSVD_EDEVICE;
    hipGraph_t g = nullptr;
    if (rc == JSVD_OK) {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = JSVD_EDEVICE;
        } else {
            rc = capture_sweep(st, cs);
            // a failed capture still has to be ended
            if (hipStreamEndCapture(cs, &g) != hipSuccess && rc == JSVD_OK) rc = JSVD_EDEVICE;
        }
    }
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

extern "C" int jsvd_sweep(jsvd_state st, void *stream)
{
    if (!st) return JSVD_EINVAL;
    const int rc = build_graph(st);
    if (rc != JSVD_OK) return rc;
    HIPCHK(hipGraphLaunch(st->graph, (hipStream_t)stream));
    return JSVD_OK;
}

int jsvd::state_sweep_async(jsvd_state st, hipStream_t s)
{
    const int rc = jsvd_sweep(st, s);
    if (rc != JSVD_OK) return rc;
    HIPCHK(hipMemcpyAsync(st->host, st->d.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    return JSVD_OK;
}

const DevScalars &jsvd::state_staged(jsvd_state st) { return *st->host; }

int jsvd::state_finish_async(jsvd_state st, bool converged, double *U_re, double *U_im, size_t ldu,
                             double *V_re, double *V_im, size_t ldv, double *sv_e, double *sv_f, double *sv,
                             hipStream_t s)
{
    const SvdDesc &d = st->d;
    if (converged) {
        HIPCHK(launch_colnorms_raw(d, s));
        HIPCHK(launch_rank(d, st->rank, s));
        HIPCHK(launch_final_write(d, st->rank, U_re, U_im, (long long)ldu, V_re, V_im, (long long)ldv, sv_e, sv_f,
                                  sv, s));
        return JSVD_OK;
    }
    HIPCHK(launch_copy2d(d.m, d.n, d.Gr, d.ldg, U_re, (long long)ldu, s));
    if (st->cplx) HIPCHK(launch_copy2d(d.m, d.n, d.Gi, d.ldg, U_im, (long long)ldu, s));
    HIPCHK(launch_copy2d(d.n, d.n, d.Vr, d.ldv, V_re, (long long)ldv, s));
    if (st->cplx) HIPCHK(launch_copy2d(d.n, d.n, d.Vi, d.ldv, V_im, (long long)ldv, s));
    HIPCHK(launch_colnorms_raw(d, s));
    HIPCHK(launch_colnorm_out(d, sv_e, sv_f, sv, s));
    return JSVD_OK;
}

extern "C" int jsvd_state_query(jsvd_state st, jsvd_info *out, void *stream)
{
    if (!st || !out) return JSVD_EINVAL;
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
    return JSVD_OK;
}

extern "C" int jsvd_state_save(jsvd_state st, double *G_re, double *G_im, size_t ldg, double *V_re,
                               double *V_im, size_t ldv, double *e, double *f, int32_t *s_out, double *Mt,
                               int64_t *step, void *stream)
{
    if (!st) return JSVD_EINVAL;
    if (G_re && ldg < (size_t)st->m) return JSVD_EINVAL;
    if (V_re && ldv < (size_t)st->n) return JSVD_EINVAL;
    if (st->cplx && ((G_re && !G_im) || (V_re && !V_im))) return JSVD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const SvdDesc &d = st->d;
    if (G_re) {
        HIPCHK(launch_copy2d(d.m, d.n, d.Gr, d.ldg, G_re, (long long)ldg, s));
        if (st->cplx) HIPCHK(launch_copy2d(d.m, d.n, d.Gi, d.ldg, G_im, (long long)ldg, s));
    }
    if (V_re) {
        HIPCHK(launch_copy2d(d.n, d.n, d.Vr, d.ldv, V_re, (long long)ldv, s));
        if (st->cplx) HIPCHK(launch_copy2d(d.n, d.n, d.Vi, d.ldv, V_im, (long long)ldv, s));
    }
    if (e) HIPCHK(hipMemcpyAsync(e, d.e, sizeof(double) * d.n, hipMemcpyDeviceToDevice, s));
    if (f) HIPCHK(hipMemcpyAsync(f, d.f, sizeof(double) * d.n, hipMemcpyDeviceToDevice, s));
    const int rc = pull_scalars(st, s);
    if (rc != JSVD_OK) return rc;
    if (s_out) *s_out = st->host->s;
    if (Mt) *Mt = bitsd(st->host->Mt_bits);
    if (step) *step = st->host->k;
    return JSVD_OK;
}

extern "C" int jsvd_state_restore(jsvd_state st, const double *G_re, const double *G_im, size_t ldg,
                                  const double *V_re, const double *V_im, size_t ldv, int32_t s_in, double Mt,
                                  int64_t step, void *stream)
{
    if (!st || !G_re || !V_re || ldg < (size_t)st->m || ldv < (size_t)st->n) return JSVD_EINVAL;
    if (st->cplx && (!G_im || !V_im)) return JSVD_EINVAL;
    if (!(Mt >= 0.0 && Mt <= 1.79769313486231570815e308) || step < 0) return JSVD_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const SvdDesc &d = st->d;
    HIPCHK(launch_copy2d(d.m, d.n, G_re, (long long)ldg, d.Gr, d.ldg, s));
    if (st->cplx) HIPCHK(launch_copy2d(d.m, d.n, G_im, (long long)ldg, d.Gi, d.ldg, s));
    HIPCHK(launch_copy2d(d.n, d.n, V_re, (long long)ldv, d.Vr, d.ldv, s));
    if (st->cplx) HIPCHK(launch_copy2d(d.n, d.n, V_im, (long long)ldv, d.Vi, d.ldv, s));
    DevScalars h;
    memset(&h, 0, sizeof(h));
    h.Mt_bits = dbits(Mt);
    h.s = s_in;
    h.k = step;
    h.max_sweeps = st->max_sweeps;
    return push_scalars(st, h, s);
}

extern "C" int jsvd_state_finalize(jsvd_state st, double *U_re, double *U_im, size_t ldu, double *V_re,
                                   double *V_im, size_t ldv, double *sv_e, double *sv_f, double *sv,
                                   void *stream)
{
    if (!st || !U_re || !V_re || !sv_e || !sv_f || ldu < (size_t)st->m || ldv < (size_t)st->n)
        return JSVD_EINVAL;
    if (st->cplx && (!U_im || !V_im)) return JSVD_EINVAL;
    return state_finish_async(st, true, U_re, U_im, ldu, V_re, V_im, ldv, sv_e, sv_f, sv, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// the whole SVD
static int gesvj_on_state(jsvd_state st, double *G_re, double *G_im, size_t ldg, double *V_re, double *V_im,
                          size_t ldv, double *sv_e, double *sv_f, double *sv, int *sweeps, hipStream_t s)
{
    int rc = state_load_async(st, G_re, G_im, ldg, s);
    if (rc != JSVD_OK) return rc;
    // one graph-launched sweep at a time; the device decides convergence
    for (;;) {
        rc = state_sweep_async(st, s);
        if (rc != JSVD_OK) return rc;
        HIPCHK(hipStreamSynchronize(s));
        if (st->host->stop) break;
    }
    const DevScalars h = *st->host;
    if (sweeps) *sweeps = (int)h.C;
    if (h.status != 0) return h.status;
    rc = state_finish_async(st, h.converged != 0, G_re, G_im, ldg, V_re, V_im, ldv, sv_e, sv_f, sv, s);
    if (rc != JSVD_OK) return rc;
    HIPCHK(hipStreamSynchronize(s));
    return h.converged ? JSVD_OK : JSVD_NOT_CONVERGED;
}

extern "C" int jsvd_gesvj(int m, int n, double *G_re, double *G_im, size_t ldg, double *V_re, double *V_im,
                          size_t ldv, double *sv_e, double *sv_f, double *sv, int max_sweeps, int *sweeps,
                          unsigned flags, void *stream)
{
    if (n < 1 || m < n || !G_re || !V_re || !sv_e || !sv_f || ldg < (size_t)m || ldv < (size_t)n)
        return JSVD_EINVAL;
    if ((G_im == nullptr) != (V_im == nullptr)) return JSVD_EINVAL;
    if (flags & ~kIterFlags) return JSVD_EINVAL;
    jsvd_state st = nullptr;
    int rc = jsvd_state_create(m, n, G_im != nullptr, &st);
    if (rc != JSVD_OK) return rc;
    st->max_sweeps = max_sweeps > 0 ? max_sweeps : 128;
    apply_flags(st, flags);
    rc = gesvj_on_state(st, G_re, G_im, ldg, V_re, V_im, ldv, sv_e, sv_f, sv, sweeps, (hipStream_t)stream);
    jsvd_state_destroy(st);
    return rc;
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
