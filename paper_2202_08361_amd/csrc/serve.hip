// serve.hip -- continuous-batching SVD server (jsvd_serve_*).
//
// A worker thread owns the device side.  Submitted requests wait in a FIFO
// queue; the worker admits them while a slot is free and the HBM budget
// covers their footprint, and keeps every admitted request's iteration state
// on the device:
//
// * small requests (the batched kernel's tile: m, n <= 512) are admitted in
//   groups while enough of them wait; a group is one persistent batched
//   launch (one workgroup per matrix, the whole SVD on the device, in place
//   in the caller's buffers) on the slot's stream.  One workgroup per matrix
//   spends little of the GPU per matrix but is slow for each one, so with
//   few small requests waiting they are admitted one by one, like large
//   ones;
// * larger requests get a device-resident jsvd_state on their slot's stream
//   and advance one graph-launched sweep at a time; after each sweep the
//   device's convergence flags are staged to pinned memory and checked by the
//   worker without blocking (events), then the next sweep or the finalisation
//   is enqueued.  While such a request is the only one on the device, its
//   sweeps run as persistent launches where jsvd_state_iterate would (a
//   persistent launch needs all its workgroups resident; next to other
//   requests' kernels it could wait out its budget), with the same redo of a
//   sweep that gives up.
//
// Slots run on separate streams, so admitted requests overlap on the device
// while new ones are admitted as slots and memory free up.  Freeing device
// memory waits for the whole device, so nothing is freed while work is in
// flight if it can be helped: a finished large request's state (with its
// captured sweep) is kept for the next request of its shape, within the HBM
// budget, and a finished group's launch record is released once the device
// is idle.  Every request's
// result is exactly the one jsvd_gesvj computes for it alone (the kernels
// are the same and their arithmetic does not depend on what else runs).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/jsvd.h"
#include "batch.hpp"
#include "kernels.hpp"
#include "state.hpp"

using namespace jsvd;

namespace {

using Clock = std::chrono::steady_clock;

struct Ticket {
    jsvd_request req;
    int phase;  // 0 queued, 1 active, 2 done
    int status, sweeps;
    Clock::time_point t_submit, t_admit;
    size_t footprint;
    bool small;
};

enum SlotKind { SLOT_FREE, SLOT_BIG, SLOT_GROUP };

struct Slot {
    SlotKind kind = SLOT_FREE;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    jsvd_state st = nullptr;
    uint64_t ticket = 0;
    int finishing = 0;
    bool persistent = false;   // the sweep in flight is a persistent launch
    BatchLaunch *bl = nullptr;
    std::vector<uint64_t> group;
    size_t footprint = 0;
    bool heavy = false;   // a large request (counted against max_large)
};

constexpr int kMaxGroup = 512;
// small requests waiting before they are admitted as a batched group
constexpr int kGroupMin = 32;
// large requests on the device at once unless configured: one such request
// already spreads its steps over the whole GPU, a second one fills the gaps
// between them; more only compete for the caches
constexpr int kDefaultLarge = 2;
constexpr int kMaxIdleStates = 8;    // finished states kept for reuse
constexpr int kMaxHeldLaunches = 64;  // finished group launches kept before a release

size_t footprint_of(const jsvd_request &r, bool small)
{
    const size_t c = r.is_complex ? 2 : 1;
    if (small) return 8 * c * ((size_t)r.m * r.n + (size_t)r.n * r.n);
    return state_bytes(r.m, r.n, r.is_complex);
}

} // namespace

struct jsvd_server_s {
    jsvd_serve_config cfg;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Ticket> tickets;
    uint64_t next_ticket = 1;
    std::vector<Slot> slots;
    size_t hbm_in_use = 0;
    int active = 0;
    int active_large = 0;
    bool stopping = false;
    std::thread worker;
    uint64_t submitted = 0, completed = 0, rejected = 0;
    uint64_t persistent_sweeps = 0, persistent_redos = 0;
    std::vector<double> lat_ns, qlat_ns, svc_ns;
    Clock::time_point t_create;
    // worker thread only: states of finished large requests (oldest first),
    // their bytes, and finished group launches not yet released
    std::vector<jsvd_state> idle;
    size_t idle_bytes = 0;
    std::vector<BatchLaunch *> held;
};

// a kept state of this shape, or a new one; kept states are freed (oldest
// first) while they would push the server past its budget
static int take_state(jsvd_server sv, const jsvd_request &r, jsvd_state *out)
{
    for (size_t i = 0; i < sv->idle.size(); ++i) {
        jsvd_state st = sv->idle[i];
        if (st->m == r.m && st->n == r.n && st->cplx == (r.is_complex != 0) && !st->fp32) {
            sv->idle.erase(sv->idle.begin() + (long)i);
            sv->idle_bytes -= st->mem_bytes;
            *out = st;
            return JSVD_OK;
        }
    }
    size_t in_use;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        in_use = sv->hbm_in_use;
    }
    while (!sv->idle.empty() && in_use + sv->idle_bytes > sv->cfg.hbm_budget_bytes) {
        sv->idle_bytes -= sv->idle.front()->mem_bytes;
        jsvd_state_destroy(sv->idle.front());
        sv->idle.erase(sv->idle.begin());
    }
    return jsvd_state_create(r.m, r.n, r.is_complex, out);
}

// a finished request's state: kept for reuse, or freed
static void put_state(jsvd_server sv, jsvd_state st)
{
    if ((int)sv->idle.size() >= kMaxIdleStates) {
        sv->idle_bytes -= sv->idle.front()->mem_bytes;
        jsvd_state_destroy(sv->idle.front());
        sv->idle.erase(sv->idle.begin());
    }
    sv->idle.push_back(st);
    sv->idle_bytes += st->mem_bytes;
}

static void release_held(jsvd_server sv)
{
    for (BatchLaunch *bl : sv->held) batch_release(bl);
    sv->held.clear();
}

static double percentile(std::vector<double> &v, double p)
{
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k];
}

// caller holds sv->mu
static void complete_locked(jsvd_server sv, uint64_t id, int status, int sweeps)
{
    auto it = sv->tickets.find(id);
    if (it == sv->tickets.end()) return;
    Ticket &t = it->second;
    t.phase = 2;
    t.status = status;
    t.sweeps = sweeps;
    const auto now = Clock::now();
    sv->lat_ns.push_back((double)std::chrono::duration_cast<std::chrono::nanoseconds>(now - t.t_submit).count());
    sv->svc_ns.push_back((double)std::chrono::duration_cast<std::chrono::nanoseconds>(now - t.t_admit).count());
    sv->completed++;
}

static void free_slot_locked(jsvd_server sv, Slot &s)
{
    if (s.kind == SLOT_BIG && s.heavy) sv->active_large--;
    s.heavy = false;
    sv->hbm_in_use -= s.footprint;
    s.footprint = 0;
    s.kind = SLOT_FREE;
    s.group.clear();
    s.finishing = 0;
    s.ticket = 0;
    sv->active--;
}

// advance one slot if its stream has passed the last recorded point
static bool service_slot(jsvd_server sv, Slot &s)
{
    if (s.kind == SLOT_FREE) return false;
    const hipError_t q = hipEventQuery(s.ev);
    if (q == hipErrorNotReady) return false;
    if (s.kind == SLOT_GROUP) {
        const BatchItem *res = q == hipSuccess ? batch_results(s.bl) : nullptr;
        std::lock_guard<std::mutex> lk(sv->mu);
        for (size_t i = 0; i < s.group.size(); ++i)
            complete_locked(sv, s.group[i], res ? res[i].status : JSVD_EDEVICE, res ? res[i].sweeps : 0);
        if (q == hipSuccess) batch_done(s.bl);   // its class streams serve other launches now
        sv->held.push_back(s.bl);   // its results are read; released with the others
        s.bl = nullptr;
        free_slot_locked(sv, s);
        sv->cv_done.notify_all();
        return true;
    }
    // a large request: the stream has passed the last sweep (or the finalisation)
    constexpr int kRunning = 1 << 20;   // not a status: more work was enqueued
    int done_status = kRunning;
    int done_sweeps = 0;
    if (q != hipSuccess) {
        done_status = JSVD_EDEVICE;
    } else if (!s.finishing) {
        bool redone = false;
        if (s.persistent) {
            // a persistent sweep that gave up is redone step by step first
            s.persistent = false;
            if (state_after_persistent_async(s.st, s.stream, &redone) != JSVD_OK ||
                (redone && hipEventRecord(s.ev, s.stream) != hipSuccess))
                done_status = JSVD_EDEVICE;
            if (redone) {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->persistent_redos++;
            }
        }
        const DevScalars &h = state_staged(s.st);
        if (done_status != kRunning || redone) {
            // the redo's scalars are read once it has run
        } else if (!h.stop) {
            bool alone;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                alone = sv->active == 1;
            }
            if (state_next_sweep_async(s.st, s.stream, alone, &s.persistent) != JSVD_OK ||
                hipEventRecord(s.ev, s.stream) != hipSuccess)
                done_status = JSVD_EDEVICE;
            if (s.persistent) {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->persistent_sweeps++;
            }
        } else if (h.status != 0) {
            done_status = h.status;
        } else {
            jsvd_request r;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                r = sv->tickets[s.ticket].req;
            }
            s.finishing = h.converged ? 1 : 2;
            if (state_finish_async(s.st, h.converged != 0, r.G_re, r.is_complex ? r.G_im : nullptr, r.ldg, r.V_re,
                                   r.is_complex ? r.V_im : nullptr, r.ldv, r.sv_e, r.sv_f, nullptr,
                                   s.stream) != JSVD_OK ||
                hipEventRecord(s.ev, s.stream) != hipSuccess)
                done_status = JSVD_EDEVICE;
        }
    } else {
        done_status = s.finishing == 1 ? JSVD_OK : JSVD_NOT_CONVERGED;
        done_sweeps = (int)state_staged(s.st).C;
    }
    if (done_status == kRunning) return true;
    (void)hipStreamSynchronize(s.stream);
    if (done_status == JSVD_EDEVICE) jsvd_state_destroy(s.st);
    else put_state(sv, s.st);
    s.st = nullptr;
    std::lock_guard<std::mutex> lk(sv->mu);
    complete_locked(sv, s.ticket, done_status, done_sweeps);
    free_slot_locked(sv, s);
    sv->cv_done.notify_all();
    return true;
}

// admit queued requests while slots and budget allow; returns whether any was admitted
static bool admit(jsvd_server sv)
{
    std::vector<uint64_t> group;
    uint64_t big = 0;   // a request admitted alone (large, or small with few waiting)
    bool heavy = false;
    size_t fp_total = 0;
    int slot_idx = -1;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->queue.empty()) return false;
        for (size_t i = 0; i < sv->slots.size(); ++i)
            if (sv->slots[i].kind == SLOT_FREE) {
                slot_idx = (int)i;
                break;
            }
        if (slot_idx < 0) return false;
        const size_t budget = sv->cfg.hbm_budget_bytes;
        const int large_cap = sv->cfg.max_large > 0 ? sv->cfg.max_large : kDefaultLarge;
        Ticket &front = sv->tickets[sv->queue.front()];
        int waiting_small = 0;
        for (uint64_t id : sv->queue)
            if (sv->tickets[id].small && ++waiting_small >= kGroupMin) break;
        const bool cap_reached = sv->active_large >= large_cap;
        if (!front.small && !cap_reached) {
            // a large request, alone on its own state
            if (sv->hbm_in_use + front.footprint > budget && sv->active > 0) return false;
            big = sv->queue.front();
            sv->queue.pop_front();
            fp_total = front.footprint;
            heavy = true;
        } else if (waiting_small < kGroupMin) {
            // few small requests: the first of them alone on its own state
            auto q = sv->queue.begin();
            while (q != sv->queue.end() && !sv->tickets[*q].small) ++q;
            if (q == sv->queue.end()) return false;
            const jsvd_request &r = sv->tickets[*q].req;
            const size_t fp = state_bytes(r.m, r.n, r.is_complex);
            if (sv->hbm_in_use + fp > budget && sv->active > 0) return false;
            big = *q;
            sv->queue.erase(q);
            fp_total = fp;
        } else {
            // continuous batching: the run of small requests at the head of the
            // queue; with a large request at the head that has to wait for one
            // of the large ones on the device, the small requests queued behind it
            const bool past_large = !front.small;
            for (auto q = sv->queue.begin(); q != sv->queue.end() && (int)group.size() < kMaxGroup;) {
                Ticket &t = sv->tickets[*q];
                if (!t.small) {
                    if (!past_large) break;
                    ++q;
                    continue;
                }
                if (sv->hbm_in_use + fp_total + t.footprint > budget && (sv->active > 0 || !group.empty())) break;
                fp_total += t.footprint;
                group.push_back(*q);
                q = sv->queue.erase(q);
            }
            if (group.empty()) return false;
        }
        const auto now = Clock::now();
        for (uint64_t id : group) {
            sv->tickets[id].phase = 1;
            sv->tickets[id].t_admit = now;
            sv->qlat_ns.push_back(
                (double)std::chrono::duration_cast<std::chrono::nanoseconds>(now - sv->tickets[id].t_submit).count());
        }
        if (big) {
            sv->tickets[big].phase = 1;
            sv->tickets[big].t_admit = now;
            sv->qlat_ns.push_back(
                (double)std::chrono::duration_cast<std::chrono::nanoseconds>(now - sv->tickets[big].t_submit).count());
        }
        Slot &s = sv->slots[slot_idx];
        s.kind = big ? SLOT_BIG : SLOT_GROUP;
        s.heavy = heavy;
        if (heavy) sv->active_large++;
        s.footprint = fp_total;
        s.ticket = big;
        s.group = group;
        s.finishing = 0;
        s.persistent = false;
        sv->hbm_in_use += fp_total;
        sv->active++;
    }
    Slot &s = sv->slots[slot_idx];
    int rc = JSVD_OK;
    if (big) {
        jsvd_request r;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            r = sv->tickets[big].req;
        }
        rc = take_state(sv, r, &s.st);
        if (rc == JSVD_OK) {
            s.st->max_sweeps = sv->cfg.max_sweeps > 0 ? sv->cfg.max_sweeps : 128;
            rc = state_set_flags(s.st, sv->cfg.flags);
        }
        if (rc == JSVD_OK) {
            rc = state_load_async(s.st, r.G_re, r.is_complex ? r.G_im : nullptr, r.ldg, s.stream);
        }
        if (rc == JSVD_OK) rc = state_sweep_async(s.st, s.stream);
        if (rc == JSVD_OK && hipEventRecord(s.ev, s.stream) != hipSuccess) rc = JSVD_EDEVICE;
    } else {
        std::vector<BatchItem> items;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (uint64_t id : group) {
                const jsvd_request &r = sv->tickets[id].req;
                items.push_back(make_batch_item(r.m, r.n, r.is_complex != 0, r.G_re, r.G_im, r.ldg, r.V_re, r.V_im,
                                                r.ldv, r.sv_e, r.sv_f));
            }
        }
        const int ms = sv->cfg.max_sweeps > 0 ? sv->cfg.max_sweeps : 128;
        // no measurement of launch shapes here: it would stall the worker, and
        // with it every request in flight (jsvd_batched_tune does it up front)
        s.bl = batch_launch(items.data(), (int)items.size(), ms, sv->cfg.flags, s.stream, false);
        if (!s.bl || hipEventRecord(s.ev, s.stream) != hipSuccess) rc = JSVD_EDEVICE;
    }
    if (rc != JSVD_OK) {
        if (s.st) {
            (void)hipStreamSynchronize(s.stream);
            jsvd_state_destroy(s.st);
            s.st = nullptr;
        }
        if (s.bl) {
            (void)hipStreamSynchronize(s.stream);
            batch_release(s.bl);
            s.bl = nullptr;
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        if (big) complete_locked(sv, big, rc, 0);
        for (uint64_t id : group) complete_locked(sv, id, rc, 0);
        free_slot_locked(sv, s);
        sv->cv_done.notify_all();
    }
    return true;
}

static void worker_main(jsvd_server sv)
{
    (void)hipSetDevice(sv->device);
    for (;;) {
        bool progressed = false;
        for (Slot &s : sv->slots) progressed |= service_slot(sv, s);
        while (admit(sv)) progressed = true;
        if (!sv->held.empty()) {
            bool idle_now;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                idle_now = sv->active == 0;
            }
            if (idle_now || (int)sv->held.size() >= kMaxHeldLaunches) release_held(sv);
        }
        std::unique_lock<std::mutex> lk(sv->mu);
        if (sv->stopping && sv->queue.empty() && sv->active == 0) break;
        if (!progressed) {
            // nothing to do right now: sleep briefly (device work in flight)
            // or until a submission arrives (idle)
            if (sv->active > 0)
                sv->cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                sv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

extern "C" int jsvd_serve_create(const jsvd_serve_config *cfg, jsvd_server *out)
{
    if (!out) return JSVD_EINVAL;
    *out = nullptr;
    if (!cfg || cfg->max_slots < 1 || cfg->max_slots > 1024 || cfg->hbm_budget_bytes == 0 ||
        !iter_flags_valid(cfg->flags, JSVD_NO_PERMUTE | JSVD_PERMUTE | JSVD_COMPENSATED | JSVD_NO_GS))
        return JSVD_EINVAL;
    jsvd_server sv = new (std::nothrow) jsvd_server_s;
    if (!sv) return JSVD_ENOMEM;
    sv->cfg = *cfg;
    if (hipGetDevice(&sv->device) != hipSuccess) {
        delete sv;
        return JSVD_EDEVICE;
    }
    sv->slots.resize(cfg->max_slots);
    for (Slot &s : sv->slots) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) {
            for (Slot &t : sv->slots) {
                if (t.stream) (void)hipStreamDestroy(t.stream);
                if (t.ev) (void)hipEventDestroy(t.ev);
            }
            delete sv;
            return JSVD_EDEVICE;
        }
    }
    sv->t_create = Clock::now();
    try {
        sv->worker = std::thread(worker_main, sv);
    } catch (...) {
        for (Slot &t : sv->slots) {
            (void)hipStreamDestroy(t.stream);
            (void)hipEventDestroy(t.ev);
        }
        delete sv;
        return JSVD_ENOMEM;
    }
    *out = sv;
    return JSVD_OK;
}

extern "C" int jsvd_serve_submit(jsvd_server sv, const jsvd_request *req, uint64_t *ticket)
{
    if (!sv || !req || !ticket) return JSVD_EINVAL;
    const jsvd_request &r = *req;
    if (r.n < 1 || r.m < r.n || !r.G_re || !r.V_re || !r.sv_e || !r.sv_f || r.ldg < (size_t)r.m ||
        r.ldv < (size_t)r.n)
        return JSVD_EINVAL;
    if (r.is_complex && (!r.G_im || !r.V_im)) return JSVD_EINVAL;
    const bool small = batch_rows(r.m, r.n, r.is_complex != 0) != 0;
    if (!small && r.m > state_max_rows()) return JSVD_EINVAL;
    const size_t fp = footprint_of(r, small);
    if (fp > sv->cfg.hbm_budget_bytes) return JSVD_EINVAL;   // could never be admitted
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) return JSVD_EINVAL;
    if (sv->cfg.max_queue > 0 && (int)sv->queue.size() >= sv->cfg.max_queue) {
        sv->rejected++;
        return JSVD_EAGAIN;
    }
    const uint64_t id = sv->next_ticket++;
    Ticket t;
    t.req = r;
    t.phase = 0;
    t.status = 0;
    t.sweeps = 0;
    t.t_submit = Clock::now();
    t.t_admit = t.t_submit;
    t.footprint = fp;
    t.small = small;
    sv->tickets.emplace(id, t);
    sv->queue.push_back(id);
    sv->submitted++;
    *ticket = id;
    sv->cv_work.notify_one();
    return JSVD_OK;
}

extern "C" int jsvd_serve_poll(jsvd_server sv, uint64_t ticket, int *done, int *status, int *sweeps)
{
    if (!sv || !done) return JSVD_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return JSVD_ENOTFOUND;
    *done = it->second.phase == 2;
    if (*done) {
        if (status) *status = it->second.status;
        if (sweeps) *sweeps = it->second.sweeps;
    }
    return JSVD_OK;
}

extern "C" int jsvd_serve_wait(jsvd_server sv, uint64_t ticket, int *status, int *sweeps)
{
    if (!sv) return JSVD_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return JSVD_ENOTFOUND;
    sv->cv_done.wait(lk, [&] { return sv->tickets[ticket].phase == 2; });
    it = sv->tickets.find(ticket);
    if (status) *status = it->second.status;
    if (sweeps) *sweeps = it->second.sweeps;
    sv->tickets.erase(it);
    return JSVD_OK;
}

extern "C" int jsvd_serve_stats_get(jsvd_server sv, jsvd_serve_stats *out)
{
    if (!sv || !out) return JSVD_EINVAL;
    std::vector<double> lat, qlat, svc;
    memset(out, 0, sizeof(*out));
    {
        // copy under the lock; the percentiles are taken outside it, so the
        // worker is held up only for the copy
        std::lock_guard<std::mutex> lk(sv->mu);
        lat = sv->lat_ns;
        qlat = sv->qlat_ns;
        svc = sv->svc_ns;
        out->submitted = sv->submitted;
        out->completed = sv->completed;
        out->rejected = sv->rejected;
        out->queue_depth = (int)sv->queue.size();
        out->active = sv->active;
        out->hbm_in_use = sv->hbm_in_use;
        out->persistent_sweeps = sv->persistent_sweeps;
        out->persistent_redos = sv->persistent_redos;
    }
    out->p50_ns = percentile(lat, 0.50);
    out->p99_ns = percentile(lat, 0.99);
    out->p50_queue_ns = percentile(qlat, 0.50);
    out->p99_queue_ns = percentile(qlat, 0.99);
    out->p50_service_ns = percentile(svc, 0.50);
    out->p99_service_ns = percentile(svc, 0.99);
    const double secs =
        std::chrono::duration_cast<std::chrono::duration<double>>(Clock::now() - sv->t_create).count();
    out->svds_per_s = secs > 0 ? (double)out->completed / secs : 0.0;
    return JSVD_OK;
}

extern "C" int jsvd_serve_load(jsvd_server sv, int *queue_depth, int *active, size_t *hbm_in_use)
{
    if (!sv) return JSVD_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (queue_depth) *queue_depth = (int)sv->queue.size();
    if (active) *active = sv->active;
    if (hbm_in_use) *hbm_in_use = sv->hbm_in_use;
    return JSVD_OK;
}

extern "C" int jsvd_serve_destroy(jsvd_server sv)
{
    if (!sv) return JSVD_EINVAL;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    release_held(sv);
    for (jsvd_state st : sv->idle) jsvd_state_destroy(st);
    sv->idle.clear();
    for (Slot &s : sv->slots) {
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.ev) (void)hipEventDestroy(s.ev);
    }
    delete sv;
    return JSVD_OK;
}
