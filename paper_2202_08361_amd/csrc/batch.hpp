// batch.hpp -- the persistent batched SVD launch (batched.hip) as used by the
// C ABI and the server.  Internal; not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace jsvd {

// One matrix of a batched launch (device pointers; status/sweeps are outputs).
struct BatchItem {
    int m, n, cplx, R;
    double *Gr, *Gi;
    long long ldg;
    double *Vr, *Vi;
    long long ldv;
    double *sv_e, *sv_f;
    int lgbound;
    double ups;
    int status, sweeps;
    long long transformations;   // pairs transformed over the whole iteration
};

// rows-per-lane class of the batched kernel for an m x n matrix (0: too large)
int batch_rows(int m, int n, int cplx);
BatchItem make_batch_item(int m, int n, int cplx, double *Gr, double *Gi, size_t ldg, double *Vr, double *Vi,
                          size_t ldv, double *sv_e, double *sv_f);

// The launch schedule of a class (real or complex, rows per lane): threads
// per matrix, the dense (four waves per SIMD) instance or the default one,
// and workgroups per CU of the persistent grid (0: as many as fit).
struct BatchSched {
    int nt;
    int dense;
    int wpc;
};

// Measured once per process and device for the classes of these items
// (batch_tune) among the candidates batch_set_tuning allows, forced for all
// (batch_set_sched / batch_set_threads, nt = 0: measured), and the current
// choice for one shape (nt = 0: not a batched shape).
void batch_tune(const BatchItem *items, int count, unsigned flags, hipStream_t s);
int batch_set_sched(int nt, int dense, int wpc);
int batch_set_threads(int threads);
int batch_set_tuning(unsigned what);
BatchSched batch_sched_of(int m, int n, int cplx, unsigned flags);
int batch_threads_of(int m, int n, int cplx, unsigned flags);

struct BatchLaunch;
// Enqueue one persistent launch over the items (all batch_rows() != 0) and the
// copy of their outcomes to pinned host memory; nullptr on failure.  With
// tune, classes whose launch shape has not been measured in this process
// are measured first (which synchronises the stream); without, they take the
// default shape.
BatchLaunch *batch_launch(const BatchItem *items, int count, int max_sweeps, unsigned flags, hipStream_t s,
                          bool tune = true);
// The outcomes (valid once the stream has passed the launch); batch_done
// hands the launch's class streams back for other launches once the stream
// has passed it; release (which also does that) frees the rest.
const BatchItem *batch_results(const BatchLaunch *bl);
void batch_done(BatchLaunch *bl);
void batch_release(BatchLaunch *bl);

// The allocation-free variant: the items (all batched shapes, at most
// kNoAllocMaxCount) run class after class on stream s with the launch
// records in a file-scope device array; status and sweeps come back in the
// items.  Synchronises.  Calls in one process are serialised by a lock.
constexpr int kNoAllocMaxCount = 8192;
int batch_run_noalloc(BatchItem *items, int count, int max_sweeps, unsigned flags, hipStream_t s);

} // namespace jsvd
