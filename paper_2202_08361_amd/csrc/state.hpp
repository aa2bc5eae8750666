// state.hpp -- the device-resident SVD state behind jsvd_state and the
// stream-ordered operations the C ABI and the server are built from.
// Internal; not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/jsvd.h"
#include "kernels.hpp"

struct jsvd_state_s {
    int m, n, cplx;
    int fp32;          // single precision state: float G, V and norms (descriptor df)
    int threads;       // forced workgroup size (0 = automatic)
    int max_sweeps;
    int device;
    int ncu;           // compute units (persistent grid size)
    void *mem;         // the single device allocation
    size_t mem_bytes;
    jsvd::SvdDesc d;     // double precision descriptor (fp32 == 0)
    jsvd::SvdDescF df;   // single precision descriptor (fp32 != 0)
    jsvd::DevScalars *sc;  // the device scalars (either descriptor's sc)
    int *rank;
    unsigned long long *maxbits;
    double *vmx;             // the slots' max-norms of the rotated columns (vlog_stride each)
    jsvd::PairParam *vlog;   // outcome log of the large-column steps: kVlogSlots slots of vlog_stride
    jsvd::StepHdr *vhdr;     // the header of each slot
    unsigned long long *vkey;  // the max-norm key of each slot (zeroed by a load or restore)
    long long vlog_stride;
    int vlog_n;              // logged steps not yet applied to V (slots vbase ...)
    int vbase;               // first slot of the half of the log being filled (0 outside a captured sweep)
    int vlast;               // slot of the last step when its fold is still due, else -1
    int v_layout;            // V_COLS, V_ROWS, or V_EITHER (V = I after a load)
    jsvd::DevScalars *host;  // pinned staging for the scalars
    hipGraphExec_t graph;
    hipGraph_t graph_def;
    int graph_threads;
    unsigned flags;          // iteration flags (JSVD_PERMUTE, JSVD_COMPENSATED, JSVD_NO_GS)
    unsigned graph_flags;    // flags the captured sweep was built with
    // whole sweeps as one persistent launch (loop.hip; states with m <= 256)
    int loop_cand;           // the state has the loop's workspace (m <= 256)
    jsvd::LoopArgs loop;     // column flags, per-workgroup folds, abort flag, wait budget
    double *colsq;           // per-column sums of squares of the bound check
    char *snap;              // G, V, e, f as they were before the last persistent sweep
    size_t snap_bytes;
    hipGraphExec_t loop_graph;
    hipGraph_t loop_graph_def;
    unsigned loop_graph_flags;
    unsigned long long loop_graph_budget;
    int loop_graph_local;    // the captured persistent sweep is an L2-local launch
    long long loop_redos;    // persistent sweeps that gave up and were redone step by step
    int loop_local_allow;    // persistent sweeps may run in the L2-local mode (default)
    int loop_local_failed;   // an L2-local sweep gave up: the state keeps the spread mode
    long long loop_local_sweeps;   // persistent sweeps that ran in the L2-local mode
    int lastmod_valid;       // the per-column last-change steps are current (only large-column steps and persistent sweeps ran since their reset)
};

namespace jsvd {

// Steps of the outcome log: V is updated once per this many large-column
// steps, and whenever it is read.
constexpr int kVlogSteps = 32;
// Slots of the log: two halves, so that a captured sweep can update V from
// one half on a second stream while its steps fill the other.
constexpr int kVlogSlots = 2 * kVlogSteps;

// Layouts of the n x n V workspace: column-major (the fused step kernel and
// every output), row-major (the deferred update of the large-column steps),
// or either (V = I).
enum { V_COLS = 0, V_ROWS = 1, V_EITHER = 2 };

// Bytes of device memory a state for this problem allocates (fp32: the
// single precision state).
size_t state_bytes(int m, int n, int cplx, bool fp32 = false);

// Set the iteration flags (JSVD_PERMUTE, JSVD_COMPENSATED, JSVD_NO_GS) of a state.
int state_set_flags(jsvd_state st, unsigned flags);

// Enqueue the load of G (M~_0, s_0, G_1 = 2^{s_0} G, V_1 = I); a non-finite or
// zero G leaves the state stopped with that status.  The double overloads
// need a double precision state, the float ones a single precision state.
int state_load_async(jsvd_state st, const double *G_re, const double *G_im, size_t ldg, hipStream_t s);
int state_load_async(jsvd_state st, const float *G_re, const float *G_im, size_t ldg, hipStream_t s);
// Enqueue one sweep (a graph of K steps and the end-of-sweep bookkeeping)
// followed by the copy of the scalars into the state's pinned staging area.
int state_sweep_async(jsvd_state st, hipStream_t s);
// Enqueue the next sweep as jsvd_state_iterate runs it: where
// allow_persistent, the state admits it and the staged scalars (those of the
// sweep before, so not right after a load) say that no rescaling can happen
// in it, as one persistent launch (*persistent = true), else step by step;
// then the copy of the scalars.
int state_next_sweep_async(jsvd_state st, hipStream_t s, bool allow_persistent, bool *persistent);
// Once a persistent sweep so enqueued has completed (its scalars staged):
// if it gave up, restore the state from the copy taken before it and
// enqueue the sweep step by step with the copy of the scalars (*redone).
int state_after_persistent_async(jsvd_state st, hipStream_t s, bool *redone);
// The scalars staged by the last state_sweep_async (valid once the stream
// has passed that point).
const DevScalars &state_staged(jsvd_state st);
// Enqueue the output: for a converged state U = G diag(2^-e)/f and V sorted
// by descending sigma, else the scaled iteration matrix, V and the current
// column norms.
int state_finish_async(jsvd_state st, bool converged, double *U_re, double *U_im, size_t ldu, double *V_re,
                       double *V_im, size_t ldv, double *sv_e, double *sv_f, double *sv, hipStream_t s);
int state_finish_async(jsvd_state st, bool converged, float *U_re, float *U_im, size_t ldu, float *V_re,
                       float *V_im, size_t ldv, float *sv_e, float *sv_f, float *sv, hipStream_t s);

} // namespace jsvd
