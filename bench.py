#!/usr/bin/env python3
"""Benchmark of the MI355X Jacobi-SVD hot path (arXiv:2202.08361).

Headline workload: the stand-alone batched 2x2 EVD on 2^26 real symmetric and
2^26 complex Hermitian matrices (SoA FP64 streams, every component random
sign * 2^U(-1074,1023) * U[1,2), 1 % exact zeros, 1 % subnormal off-diagonal).
One "step" is one batch of each; the metric is EVDs per second with the
inputs resident in HBM.  The JSON line also carries the roofline of the
dominant kernel, the CPU oracle timed on the host, and the secondary
measurements: the fused Jacobi step on the large plain workloads (real
8192 x 2048, complex 4096 x 4096) against the HBM roofline, and whole-SVD
times.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
EVD_BYTES_REAL = 60      # 3 x 8 in, 4 x 8 out, 4 zp
EVD_BYTES_CPLX = 76      # 4 x 8 in, 5 x 8 out, 4 zp


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """The host's CPU model and thread counts (for the oracle baselines)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return dict(cpu_model=model, host_threads=os.cpu_count(), usable_threads=usable)


def measured_traffic(kind):
    """HBM bytes per launch of the EVD kernel from the committed hardware-counter
    record (FETCH_SIZE/WRITE_SIZE scaled by a plain copy), or None when the
    kernel sources changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "evd2_traffic.json")))
        csrc = os.path.join(ROOT, "paper_2202_08361_amd", "csrc")
        src = open(os.path.join(csrc, "evd2.hip"), "rb").read() + open(os.path.join(csrc, "evd2_core.hpp"), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["kernel_sources_sha256"]:
            return None
        return rec[kind]["bytes"]
    except (OSError, KeyError, ValueError):
        return None


def evd_kernel_name(r, cplx):
    """The EVD kernel the library launches for a 16-byte aligned batch of r."""
    v = "v1" if r >= (1 << 22) else "v2"
    return f"evd2_kernel_{v}<{'true' if cplx else 'false'}, false, false>"


def _rocpd_rows(db, sql):
    import sqlite3
    con = sqlite3.connect(db)
    try:
        return con.execute(sql).fetchall()
    finally:
        con.close()


def trace_summary(db):
    """Markdown table of a rocprofv3 --kernel-trace --stats database."""
    rows = _rocpd_rows(db, "select name, total_calls, total_duration, average, percentage from top_kernels")
    out = ["| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for name, calls, total, avg, pct in rows:
        out.append(f"| `{name[:110]}` | {calls} | {total:.1f} | {avg:.2f} | {pct:.2f} |")
    return "\n".join(out)


def last_call_table(db, pattern):
    """The dispatches of the last call into kernels whose names contain
    `pattern`: the last group of such dispatches that overlap in time (the
    classes of one batched call run on concurrent streams; the tuner's
    measurement launches before it run one after another)."""
    rows = _rocpd_rows(db, "select name, start, end, grid_x, workgroup_x, vgpr_count, accum_vgpr_count, "
                           "lds_size from kernels order by start")
    rows = [r for r in rows if pattern in r[0]]
    if not rows:
        raise SystemExit(f"no dispatch of a kernel matching {pattern!r}")
    groups, end = [], None
    for r in rows:
        if end is None or r[1] >= end:
            groups.append([])
            end = r[2]
        groups[-1].append(r)
        end = max(end, r[2])
    last = groups[-1]
    t0 = min(r[1] for r in last)
    span = (max(r[2] for r in last) - t0) / 1e3
    out = [f"Last call: {len(last)} dispatches on concurrent streams, span {span:.1f} us "
           f"(first start to last end).", "",
           "| kernel | workgroups | threads | VGPRs (arch + acc) | LDS B | start us | duration us |",
           "|---|---|---|---|---|---|---|"]
    for nm, st, en, gx, wx, vg, ag, lds in last:
        out.append(f"| `{nm[:90]}` | {gx // max(wx, 1)} | {wx} | {vg} + {ag} | {lds} | {(st - t0) / 1e3:.1f} | "
                   f"{(en - st) / 1e3:.1f} |")
    return "\n".join(out)


def _union_ns(spans, a, b):
    """Length of the union of the intervals (start, end), sorted by start,
    clipped to [a, b)."""
    tot, cs, ce = 0, None, None
    for s_, e_ in spans:
        s_, e_ = max(s_, a), min(e_, b)
        if e_ <= s_:
            continue
        if ce is None or s_ > ce:
            if ce is not None:
                tot += ce - cs
            cs, ce = s_, e_
        else:
            ce = max(ce, e_)
    if ce is not None:
        tot += ce - cs
    return tot


def busy_table(db, window_s=5.0, families=12):
    """How busy the device was over a kernel trace: the union of all kernel
    intervals (any stream) as a fraction of the span from the first start to
    the last end, overall and per window, and the summed kernel time per
    kernel family (template arguments dropped; kernels on concurrent
    streams overlap, so the sum may exceed the span)."""
    rows = _rocpd_rows(db, "select name, start, end from kernels order by start")
    if not rows:
        raise SystemExit("no kernel dispatches in the trace")
    spans = [(r[1], r[2]) for r in rows]
    t0, t1 = rows[0][1], max(r[2] for r in rows)
    out = [f"{len(rows)} dispatches over {(t1 - t0) / 1e9:.2f} s; device busy "
           f"{_union_ns(spans, t0, t1) / max(t1 - t0, 1):.3f} of it.", "",
           "| window s | busy |", "|---|---|"]
    w = int(window_s * 1e9)
    a = t0
    while a < t1:
        b = min(a + w, t1)
        out.append(f"| {(a - t0) / 1e9:.1f}–{(b - t0) / 1e9:.1f} | {_union_ns(spans, a, b) / (b - a):.3f} |")
        a = b
    fam = {}
    for nm, st, en in rows:
        key = nm.replace("void ", "").split("<")[0].split("(")[0]
        fam[key] = fam.get(key, 0) + (en - st)
    out += ["", "| kernel family | summed time s |", "|---|---|"]
    for key, v in sorted(fam.items(), key=lambda x: -x[1])[:families]:
        out.append(f"| `{key}` | {v / 1e9:.2f} |")
    return "\n".join(out)


def counters_table(fetch_db, write_db, calib_mib, last_of=None):
    """Per kernel: the mean FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of one
    counter run each, and the HBM bytes per dispatch after scaling each
    counter by what it reads for the plain device copy of calib_mib MiB."""
    q = "select kernel_name, value from counters_collection order by dispatch_id"
    fetch, write = _rocpd_rows(fetch_db, q), _rocpd_rows(write_db, q)
    moved = calib_mib * 1024.0

    def per_kernel(rows):
        acc = {}
        for nm, v in rows:
            acc.setdefault(nm, []).append(v)
        return acc
    fk, wk = per_kernel(fetch), per_kernel(write)
    if last_of:
        # only the last dispatch of each matching kernel (that of the timed call)
        for acc in (fk, wk):
            for nm in acc:
                if last_of in nm:
                    acc[nm] = acc[nm][-1:]
    # the calibration copy is the run's first plain device copy
    cf = [v for nm, v in fetch if "copyBuffer" in nm][:1]
    cw = [v for nm, v in write if "copyBuffer" in nm][:1]
    if not cf or not cw:
        raise SystemExit("no plain copy in the counter databases (run with --calib-copy)")
    f_scale, w_scale = moved / cf[-1], moved / cw[-1]
    out = ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled MB per dispatch |", "|---|---|---|---|---|"]
    for nm in sorted(fk, key=lambda n: -sum(fk[n]) * f_scale - sum(wk.get(n, [0.0])) * w_scale):
        if "copyBuffer" in nm or nm not in wk:
            continue
        f = sum(fk[nm]) / len(fk[nm])
        w = sum(wk[nm]) / len(wk[nm])
        out.append(f"| `{nm[:100]}` | {len(fk[nm])} | {f:.1f} | {w:.1f} | {(f * f_scale + w * w_scale) * 1024 / 1e6:.3f} |")
    out.append(f"\nCalibration: the plain device copy of {calib_mib} MiB reads as FETCH_SIZE {cf[-1]:.1f} KiB and "
               f"WRITE_SIZE {cw[-1]:.1f} KiB; scale factors {f_scale:.4f} and {w_scale:.4f}.")
    return "\n".join(out)


def traffic_from(fetch_db, write_db, calib_mib, r=1 << 26):
    """HBM bytes per launch of the EVD kernels from one FETCH_SIZE and one
    WRITE_SIZE run (KiB per dispatch), each scaled by what the same counter
    reads for the plain device copy of calib_mib MiB in the same run."""
    import hashlib
    q = "select kernel_name, grid_size, value from counters_collection order by dispatch_id"
    fetch, write = _rocpd_rows(fetch_db, q), _rocpd_rows(write_db, q)
    moved = calib_mib * 1024.0   # KiB read and written by the copy

    def pick(rows, key, first=False):
        vals = [v for (nm, g, v) in rows if key in nm]
        if not vals:
            raise SystemExit(f"no dispatch of {key} in the counter database")
        return vals[0] if first else vals[-1]
    # the calibration copy is the run's first plain device copy (it runs
    # before anything else; later copies, such as the stream-ceiling
    # reference, have other sizes)
    f_scale = moved / pick(fetch, "copyBuffer", first=True)
    w_scale = moved / pick(write, "copyBuffer", first=True)
    csrc = os.path.join(ROOT, "paper_2202_08361_amd", "csrc")
    src = open(os.path.join(csrc, "evd2.hip"), "rb").read() + open(os.path.join(csrc, "evd2_core.hpp"), "rb").read()
    rec = dict(kernel_sources_sha256=hashlib.sha256(src).hexdigest(), fetch_scale=f_scale, write_scale=w_scale,
               r=r, calib_copy_mib=calib_mib)
    md = ["| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled bytes | algorithmic bytes |", "|---|---|---|---|---|"]
    for kind, cplx, alg in (("real", False, EVD_BYTES_REAL), ("complex", True, EVD_BYTES_CPLX)):
        name = evd_kernel_name(r, cplx)
        fk, wk = pick(fetch, name), pick(write, name)
        byts = (fk * f_scale + wk * w_scale) * 1024.0
        rec[kind] = dict(kernel=name, fetch_kib=fk, write_kib=wk, bytes=byts)
        md.append(f"| `{name}` | {fk:.1f} | {wk:.1f} | {byts:.4g} | {alg * r:.4g} |")
    md.append(f"\nCalibration: the plain device copy of {calib_mib} MiB reads as FETCH_SIZE "
              f"{pick(fetch, 'copyBuffer', True):.1f} KiB and WRITE_SIZE {pick(write, 'copyBuffer', True):.1f} KiB; "
              f"scale factors {f_scale:.4f} and {w_scale:.4f}.")
    return rec, "\n".join(md)


def evd_workload(torch, J, inputs, r, K, W):
    dev = {}
    for cplx in (False, True):
        a = inputs.evd_batch(r, cplx)
        ins = [None if x is None else torch.from_numpy(x).cuda() for x in a]
        out = dict(cos=torch.empty(r, dtype=torch.float64, device="cuda"),
                   ctan_re=torch.empty(r, dtype=torch.float64, device="cuda"),
                   lambda1=torch.empty(r, dtype=torch.float64, device="cuda"),
                   lambda2=torch.empty(r, dtype=torch.float64, device="cuda"),
                   zp=torch.empty(r, dtype=torch.int32, device="cuda"))
        if cplx:
            out["ctan_im"] = torch.empty(r, dtype=torch.float64, device="cuda")
        dev[cplx] = (ins, out, a)
    torch.cuda.synchronize()
    for _ in range(W):
        for cplx in (False, True):
            J.evd2_batched(*dev[cplx][0], out=dev[cplx][1])
    torch.cuda.synchronize()
    ev = {c: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
          for c in (False, True)}
    t0 = time.perf_counter()
    for k in range(K):
        for cplx in (False, True):
            s, e = ev[cplx][k]
            s.record()
            J.evd2_batched(*dev[cplx][0], out=dev[cplx][1])
            e.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dur = {c: sum(s.elapsed_time(e) for s, e in ev[c]) / K * 1e-3 for c in (False, True)}
    return wall, dur, dev


def evd_ceiling(torch, J, dev, r, K):
    """The memory-system ceiling of the EVD kernels on this device: the same
    streams moved without arithmetic (jsvd_evd2_stream_ceiling, same launch
    shape and access hints), and a plain device copy of the complex EVD's
    bytes (half read, half written), each timed with HIP events over K
    launches after one warm-up."""
    res = {}
    for cplx, nb in ((False, EVD_BYTES_REAL), (True, EVD_BYTES_CPLX)):
        ins, out, _ = dev[cplx]
        J.evd2_stream_ceiling(*ins, out=out)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for a, b in evs:
            a.record()
            J.evd2_stream_ceiling(*ins, out=out)
            b.record()
        torch.cuda.synchronize()
        t = sum(a.elapsed_time(b) for a, b in evs) / K * 1e-3
        res["stream_complex" if cplx else "stream_real"] = dict(avg_launch_ms=round(t * 1e3, 4),
                                                               GBs=round(nb * r / t / 1e9, 1))
    half = EVD_BYTES_CPLX * r // 2
    src = torch.empty(half // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for a, b in evs:
        a.record()
        dst.copy_(src)
        b.record()
    torch.cuda.synchronize()
    t = sum(a.elapsed_time(b) for a, b in evs) / K * 1e-3
    res["plain_copy"] = dict(bytes=2 * half, avg_launch_ms=round(t * 1e3, 4), GBs=round(2 * half / t / 1e9, 1))
    del src, dst
    torch.cuda.empty_cache()
    return res


EVD_BYTES_REAL_F32 = 32      # 3 x 4 in, 4 x 4 out, 4 zp
EVD_BYTES_CPLX_F32 = 40      # 4 x 4 in, 5 x 4 out, 4 zp


def evd_f32(torch, J, inputs, r, K, W):
    """The single precision batched EVD on the same recipe over the float32
    range: EVDs/s over both kernels and each kernel against the HBM roofline."""
    dur = {}
    for cplx in (False, True):
        a = inputs.evd_batch_f32(r, cplx)
        ins = [None if x is None else torch.from_numpy(x).cuda() for x in a]
        out = None
        for _ in range(W):
            out = J.evd2_batched_f32(*ins, out=out)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for s, e in evs:
            s.record()
            J.evd2_batched_f32(*ins, out=out)
            e.record()
        torch.cuda.synchronize()
        dur[cplx] = sum(s.elapsed_time(e) for s, e in evs) / K * 1e-3
        del ins, out
        torch.cuda.empty_cache()
    tot = dur[False] + dur[True]
    res = dict(r=r, evd_per_s=2.0 * r / tot)
    for cplx, nb in ((False, EVD_BYTES_REAL_F32), (True, EVD_BYTES_CPLX_F32)):
        ach = nb * r / dur[cplx] / 1e9
        res["complex" if cplx else "real"] = dict(avg_launch_ms=round(dur[cplx] * 1e3, 4), achieved_GBs=round(ach, 1),
                                                  frac=round(ach / HBM_PEAK_GBS, 4), bytes_per_launch=nb * r)
    return res


VLOG_STEPS = 32   # steps of the outcome log: V is updated once per this many large-column steps


def step_roofline(torch, J, inputs, m, n, cplx, flags=0, fp32=False, streamed=False):
    """Time the Jacobi step on a freshly loaded state (every pair transforms):
    one outcome log's worth of steps (VLOG_STEPS) after a first log as warm-up,
    so that the timed block holds exactly one update of V; fp32: the single
    precision state on the same columns rounded to float."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 77 + int(cplx))
    Ar, Ai = inputs.random_columns(m, n, g, cplx)
    dt = torch.float32 if fp32 else torch.float64
    st = J.State(m, n, cplx, fp32=fp32)
    st.set_flags(flags)
    st.load(J.to_device_fortran(Ar, dtype=dt), J.to_device_fortran(Ai, dtype=dt) if cplx else None)
    for _ in range(VLOG_STEPS):
        st.step()
    T0 = st.query()["T"]
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(VLOG_STEPS):
        st.step()
    b.record()
    torch.cuda.synchronize()
    q = st.query()
    t = a.elapsed_time(b) * 1e-3 / VLOG_STEPS
    c = 2 if cplx else 1
    es = 4 if fp32 else 8
    tr = (q["T"] - T0) / VLOG_STEPS
    # (i) the per-step unit of the step's definition: every transformed pair's
    # G and V columns read and written once, 16 c n (m + n) bytes in double
    # precision when all n/2 pairs transform
    frac_tr = tr / (n // 2)
    b_step = 2.0 * es * c * n * (m + n) * frac_tr
    # (ii) what this implementation moves: the transformed G column pairs read
    # and written once per step, V read and written once per outcome log
    b_deferred = 2.0 * es * c * m * n * frac_tr + 2.0 * es * c * n * n / VLOG_STEPS
    st.close()
    if streamed:
        # columns longer than the register tile: each pair streamed from
        # memory, G and V pairs updated in the same launch every step
        return dict(m=m, n=n, complex=bool(cplx), dtype="f32" if fp32 else "f64", us_per_step=t * 1e6,
                    transformed_per_step=tr, pairs=n // 2, bytes_per_step=b_step, achieved_GBs=b_step / t / 1e9,
                    frac=b_step / t / 1e9 / HBM_PEAK_GBS,
                    frac_unit="G and V pairs of every transformed pair read and written once per step "
                              "(the kernel reads the G pair three more times for its sums)")
    return dict(m=m, n=n, complex=bool(cplx), dtype="f32" if fp32 else "f64", us_per_step=t * 1e6,
                transformed_per_step=tr, pairs=n // 2, v_update_every=VLOG_STEPS,
                bytes_per_step_g_and_v=b_step, GBs_g_and_v=b_step / t / 1e9,
                frac_g_and_v=b_step / t / 1e9 / HBM_PEAK_GBS,
                bytes_per_step_deferred_v=b_deferred, achieved_GBs=b_deferred / t / 1e9,
                frac=b_deferred / t / 1e9 / HBM_PEAK_GBS,
                frac_unit="deferred V: G pairs read+written per step, V read+written once per "
                          f"{VLOG_STEPS} steps (frac_g_and_v: G and V every step)")


def nrmf_rate(torch, J, inputs, m, n, cplx, K=10, lanes=1024):
    """Alg. rnF over every column of an m x n matrix (Gaussian columns): time
    per launch with HIP events on the launch stream, algorithmic bytes = the
    matrix read once plus 32 bytes written per column."""
    import ctypes
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 99 + int(cplx))
    Ar, Ai = inputs.random_columns(m, n, g, cplx)
    dr = J.to_device_fortran(Ar)
    di = J.to_device_fortran(Ai) if cplx else None
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    st = torch.cuda.current_stream()
    args = [n, m, ctypes.c_void_p(dr.data_ptr()), ctypes.c_void_p(di.data_ptr()) if cplx else None, m, lanes] + \
        [ctypes.c_void_p(o.data_ptr()) for o in outs] + [ctypes.c_void_p(st.cuda_stream)]
    L = J.lib()
    for _ in range(2):
        assert L.jsvd_nrmf_batched(*args) == 0
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for a, b in evs:
        a.record(st)
        L.jsvd_nrmf_batched(*args)
        b.record(st)
    torch.cuda.synchronize()
    t = sum(a.elapsed_time(b) for a, b in evs) / K * 1e-3
    byts = 8.0 * (2 if cplx else 1) * m * n + 32.0 * n
    return dict(m=m, n=n, complex=bool(cplx), lanes=lanes, us_per_launch=t * 1e6, algorithmic_bytes=byts,
                achieved_GBs=byts / t / 1e9, frac=byts / t / 1e9 / HBM_PEAK_GBS)


def sweep_time(torch, J, inputs, m, n, cplx, fp32=False):
    """One whole sweep (graph of K steps) of the large plain workloads on a fresh state."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 88 + int(cplx))
    Ar, Ai = inputs.random_columns(m, n, g, cplx)
    dt = torch.float32 if fp32 else torch.float64
    st = J.State(m, n, cplx, fp32=fp32)
    st.load(J.to_device_fortran(Ar, dtype=dt), J.to_device_fortran(Ai, dtype=dt) if cplx else None)
    st.sweep()                     # builds the graph; first sweep
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    st.sweep()
    e.record()
    torch.cuda.synchronize()
    q = st.query()
    st.close()
    K = n - 1 if n % 2 == 0 else n
    return dict(m=m, n=n, complex=bool(cplx), dtype="f32" if fp32 else "f64", ms_per_sweep=s.elapsed_time(e),
                steps=K,
                us_per_step=s.elapsed_time(e) * 1e3 / K, transformations_in_sweep=q["last_sweep_T"], swaps_in_sweep=q["last_sweep_swaps"])


_batched_cache = {}


def batched_inputs(inputs, count):
    """The first `count` matrices of the batched workload with their prescribed
    singular values, kept for the runs that follow.  Every matrix has its own
    seeded stream, so they are generated in parallel host threads, each with a
    one-thread BLAS (the products then round the same at any worker count)."""
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    if _batched_cache.get("count", -1) >= count:
        return _batched_cache["mats"][:count], _batched_cache["sigs"][:count]
    m, n, kappa = inputs.batched_shapes(10000)
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    out = []
    with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
        for c0 in range(0, count, 1000):
            ids = range(c0, min(count, c0 + 1000))
            out += list(ex.map(lambda i: inputs.batched_matrix(i, int(m[i]), int(n[i]), float(kappa[i])), ids))
            log(f"[bench]   generated {len(out)} of {count} matrices ({time.perf_counter() - t0:.1f} s)")
    _batched_cache.update(count=count, mats=[a for a, _ in out], sigs=[sg for _, sg in out])
    return _batched_cache["mats"], _batched_cache["sigs"]


def _svd_bytes(m, n, sweeps, transformations, c=1):
    """Algorithmic bytes of one SVD in double precision: (upper) every pair of
    every step transforms, 16 c n (m + n) bytes per step over the sweeps and
    the final sweep that finds nothing to do; (moved) both G columns of every
    pair read in every step, and the transformed pairs' G columns written and
    V columns read and written."""
    K = n - 1 if n % 2 == 0 else n
    upper = 16.0 * c * n * (m + n) * K * (sweeps + 1)
    moved = 16.0 * c * m * (n // 2) * K * (sweeps + 1) + transformations * (16.0 * c * m + 32.0 * c * n)
    return upper, moved


def batched_vs_plain(torch, J, inputs, count, plain_count, flags, ab=True):
    """The first `count` matrices of the batched workload in one call, and a
    sample of `plain_count` of them (stratified by n: every k-th in the order
    of n) one by one through jsvd_gesvj.  Both are priced by the same bytes
    (_svd_bytes, from the batched call's per-matrix sweeps and
    transformation counts, which the plain path shares bit for bit)."""
    import numpy as np
    m, n, kappa = inputs.batched_shapes(10000)
    mats, sigs = batched_inputs(inputs, count)
    shapes = [(int(m[i]), int(n[i]), False) for i in range(count)]

    def run(tuning):
        # the schedule of each class present is measured once, before timing,
        # among the candidates `tuning` allows
        J.batched_set_tuning(tuning)
        t0 = time.perf_counter()
        J.batched_tune(shapes, flags=flags)
        tune_s = time.perf_counter() - t0
        sched = {}
        for (mm, nn, _) in shapes:
            rows = 64
            while rows < mm:
                rows *= 2
            t, d, w = J.batched_schedule_of(mm, nn, False, flags)
            sched[f"rows<={rows}"] = dict(threads=t, dense=d, workgroups_per_cu=w)
        dev = [(J.to_device_fortran(A), None) for A in mats]
        J.gesvj_batched([(J.to_device_fortran(mats[0]), None)], flags=flags)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = J.gesvj_batched(dev, flags=flags)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, res, sched, tune_s
    # A: threads per matrix alone (default instance, full grid); B: the
    # widened schedule (dense instances, workgroups per CU); same bits
    ta, res_a, sched_a, _ = run(0) if ab else (None, None, None, None)
    tb, res, launch, tune_s = run(J.TUNE_DENSE | J.TUNE_WGS)
    same = ab and all(a["sweeps"] == b["sweeps"] and bool(torch.equal(a["sv_f"], b["sv_f"])) and
                      bool(torch.equal(a["sv_e"], b["sv_e"])) and bool(torch.equal(a["V_re"], b["V_re"]))
                      for a, b in zip(res_a, res))
    del res_a
    errs, up, mv, sweeps = [], np.zeros(count), np.zeros(count), []
    for i, r in enumerate(res):
        sv = np.ldexp(r["sv_f"].cpu().numpy(), r["sv_e"].cpu().numpy().astype(int))
        big = sigs[i] >= 1e-6 * sigs[i][0]
        errs.append(float(np.max(np.abs(sv[big] - sigs[i][big]) / sigs[i][big])))
        up[i], mv[i] = _svd_bytes(int(m[i]), int(n[i]), r["sweeps"], r["transformations"])
        sweeps.append(r["sweeps"])
    del res
    _batched_cache["bytes_upper_%d" % flags] = up
    # the plain sample: every k-th matrix in the order of n
    by_n = np.argsort(n[:count], kind="stable")
    k = max(1, count // plain_count)
    sample = [int(i) for i in by_n[k // 2::k][:plain_count]]
    dev2 = [J.to_device_fortran(mats[i]) for i in sample]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for A in dev2:
        J.gesvj(A, flags=flags, overwrite=True)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    ps = len(sample)
    bu, bm = up.sum(), mv.sum()
    pu, pm = up[sample].sum(), mv[sample].sum()
    return dict(count=count, batched_s=tb, batched_svds_per_s=count / tb,
                plain_count=ps, plain_sample="every %d-th matrix in the order of n (n from %d to %d)"
                % (k, int(n[sample[0]]), int(n[sample[-1]])),
                plain_s=tp, plain_svds_per_s=ps / tp,
                speedup=(count / tb) / (ps / tp), max_rel_sigma_err=max(errs),
                mean_sweeps=float(np.mean(sweeps)), max_sweeps=int(max(sweeps)),
                bytes_unit="upper: 16 n (m + n) per step (every pair transforms), over sweeps + 1; "
                           "moved: G pairs read every step + transformed pairs' G written and V read+written",
                batched_bytes_upper=float(bu), batched_GBs_upper=float(bu / tb / 1e9),
                batched_frac_upper=float(bu / tb / 1e9 / HBM_PEAK_GBS),
                batched_bytes_moved=float(bm), batched_GBs_moved=float(bm / tb / 1e9),
                batched_frac_moved=float(bm / tb / 1e9 / HBM_PEAK_GBS),
                plain_GBs_upper=float(pu / tp / 1e9), plain_frac_upper=float(pu / tp / 1e9 / HBM_PEAK_GBS),
                plain_GBs_moved=float(pm / tp / 1e9), plain_frac_moved=float(pm / tp / 1e9 / HBM_PEAK_GBS),
                schedule=dict(sorted(launch.items())), tune_s=round(tune_s, 3),
                threads_only_schedule=dict(sorted(sched_a.items())) if ab else None, threads_only_s=ta,
                threads_only_svds_per_s=count / ta if ab else None, schedule_gain=ta / tb if ab else None,
                schedules_same_bits=same if ab else None,
                bit_identical_to_plain="tested (tests/test_gpu_batched.py)")


_serve_cache = {}


def serve_pool(torch, J, inputs, pool_size, flags):
    """The request pool of the serving workload: the shapes of the first
    `pool_size` requests of the stream (70 % real, n log-uniform in
    [32, 2048], m uniform in [n, 2n], kappa log-uniform in [1e2, 1e10]), each
    matrix from its own seeded stream, generated in parallel host threads
    (one-thread BLAS each), then moved to the device.  Beside each: the plain
    path's time for it alone (jsvd_gesvj on a fresh copy, after one warm-up
    solve of the pool's first matrix), and the batched launch shapes of the
    pool's small requests, measured up front."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    key = (pool_size, flags)
    if _serve_cache.get("key") == key:
        return _serve_cache
    _, cplx, m, n, kappa = inputs.serve_stream(2000.0, 60.0)
    t0 = time.perf_counter()

    def make(k):
        g = inputs.rng(inputs.CFG_SERVE, 50000 + k)
        Ar, Ai, _ = inputs.serve_matrix(int(m[k]), int(n[k]), float(kappa[k]), bool(cplx[k]), g)
        return Ar, Ai
    with threadpool_limits(1), ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        host = list(ex.map(make, range(pool_size)))
    gen_s = time.perf_counter() - t0
    pool = [(J.to_device_fortran(Ar), None if Ai is None else J.to_device_fortran(Ai)) for Ar, Ai in host]
    del host
    J.batched_tune([(int(m[k]), int(n[k]), bool(cplx[k])) for k in range(pool_size)], flags=flags)

    def fresh(k):
        Gr, Gi = pool[k]
        gr = J.fortran_empty(*Gr.shape)
        gr.copy_(Gr)
        gi = None
        if Gi is not None:
            gi = J.fortran_empty(*Gi.shape)
            gi.copy_(Gi)
        return gr, gi
    gr, gi = fresh(0)
    J.gesvj(gr, gi, flags=flags, overwrite=True)
    solo = []
    for k in range(pool_size):
        gr, gi = fresh(k)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        J.gesvj(gr, gi, flags=flags, overwrite=True)
        torch.cuda.synchronize()
        solo.append(time.perf_counter() - ts)
    small = [int(m[k]) <= 512 and int(n[k]) <= 512 for k in range(pool_size)]
    _serve_cache.update(key=key, pool=pool, fresh=fresh, solo=solo, gen_s=gen_s, small=small,
                        shapes=[(int(m[k]), int(n[k]), bool(cplx[k])) for k in range(pool_size)])
    log(f"[bench]   serving pool: {pool_size} requests generated in {gen_s:.1f} s; plain path "
        f"{sum(solo):.2f} s for all of them")
    return _serve_cache


def serving_run(torch, J, inputs, rate, duration, pool_size, flags, max_queue=32, budget=64 << 30,
                slots=16, drain_limit=120.0, max_large=0):
    """Poisson arrivals at `rate` for `duration` seconds, each request a fresh
    device copy of a pool matrix (serve_pool) submitted to the server when
    its queue holds fewer than max_queue requests (else rejected: 0 means
    no limit).  Beside the server's figures: the plain path's time for the
    same completed requests one after another (the sum of their pool
    matrices' solo times)."""
    import numpy as np
    P = serve_pool(torch, J, inputs, pool_size, flags)
    t_arr = inputs.serve_stream(rate, duration)[0]
    srv = J.Server(hbm_budget_bytes=budget, max_slots=slots, max_queue=max_queue, flags=flags, max_large=max_large)
    outstanding, rejected, submitted, done = {}, 0, 0, []
    t0 = time.perf_counter()
    next_log = 15.0
    for i, ta in enumerate(t_arr):
        while time.perf_counter() - t0 < ta:
            time.sleep(0.0002)
        if ta >= next_log:
            q, a, _ = srv.load()
            log(f"[bench]   serving {rate:g}/s: t = {ta:.0f} s, submitted {submitted}, completed {len(done)}, "
                f"rejected {rejected}, queued {q}, active {a}")
            next_log += 15.0
        if max_queue > 0 and srv.load()[0] >= max_queue:
            rejected += 1
            continue
        k = i % pool_size
        gr, gi = P["fresh"](k)
        t = srv.submit(gr, gi)
        if t is None:
            rejected += 1
            continue
        submitted += 1
        outstanding[t] = (gr, gi, k)
        if i % 64 == 0:
            for tk in [tk for tk in outstanding if srv.poll(tk)[0]]:
                srv.wait(tk)
                done.append(outstanding.pop(tk)[2])
    t_end_arrivals = time.perf_counter() - t0
    deadline = time.perf_counter() + drain_limit
    for tk in list(outstanding):
        while not srv.poll(tk)[0] and time.perf_counter() < deadline:
            time.sleep(0.001)
        if srv.poll(tk)[0]:
            srv.wait(tk)
            done.append(outstanding.pop(tk)[2])
    wall = time.perf_counter() - t0
    st = srv.stats()
    unfinished = len(outstanding)
    if unfinished == 0:
        srv.close()
    plain_s = sum(P["solo"][k] for k in done)
    return dict(offered_rate=rate, arrival_window_s=duration, offered=len(t_arr), submitted=submitted,
                rejected_backpressure=rejected, completed=st["completed"], unfinished_at_limit=unfinished,
                wall_s=wall, arrivals_s=t_end_arrivals, svds_per_s=st["completed"] / wall,
                p50_latency_ms=st["p50_ns"] / 1e6, p99_latency_ms=st["p99_ns"] / 1e6,
                p50_queue_ms=st["p50_queue_ns"] / 1e6, p99_queue_ms=st["p99_queue_ns"] / 1e6,
                p50_service_ms=st["p50_service_ns"] / 1e6, p99_service_ms=st["p99_service_ns"] / 1e6,
                completed_small=sum(1 for k in done if P["small"][k]),
                pool=pool_size, pool_generation_s=round(P["gen_s"], 1), max_queue=max_queue, slots=slots,
                flags=flags, max_large=max_large,
                plain_same_requests_s=plain_s, served_vs_plain=(plain_s / wall) if wall > 0 else None)


def svd_plain(torch, J, inputs, flags, fp32=False):
    A, sig = inputs.plain_real_256()
    dA = J.to_device_fortran(A, dtype=torch.float32 if fp32 else torch.float64)
    J.gesvj(dA, flags=flags)               # warm-up (graph build, caches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = J.gesvj(dA, flags=flags)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    import numpy as np
    sv = r["sv"].cpu().numpy().astype(np.float64)
    return dict(ms=dt * 1e3, sweeps=r["sweeps"], status=r["status"], dtype="f32" if fp32 else "f64",
                max_rel_sigma_err=float(np.max(np.abs(sv - sig) / sig)))


def svd_plain_sweeps(torch, J, inputs, persistent, shape=None, local=True):
    """The 256 x 256 workload (or an m x n x complex `shape`, sigma
    log-spaced in [1e-6, 1]) through the state API (load,
    jsvd_state_iterate, finalize), with persistent sweeps or with step-by-step
    sweeps (a zero wait budget turns persistent sweeps off): the A/B of the two
    sweep forms on the same iteration (the same bits, tested).  local=False
    keeps persistent sweeps out of the L2-local mode."""
    import numpy as np
    if shape is None:
        A, sig = inputs.plain_real_256()
        Ai, m, n, cplx = None, 256, 256, False
    else:
        m, n, cplx = shape
        g = inputs.rng(inputs.CFG_PLAIN_LARGE, 4400 + m + n)
        sig = inputs.sigma_logspace(n, 1e-6)
        A, Ai = inputs.svd_matrix(m, n, sig, g, cplx=cplx)
    dA = J.to_device_fortran(A)
    dAi = J.to_device_fortran(Ai) if cplx else None
    best, q = None, None
    for rep in range(3):
        st = J.State(m, n, cplx)
        if not persistent:
            st.set_loop_wait(0.0)
        if not local:
            st.set_loop_local(False)
        st.load(dA, dAi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.iterate()
        r = st.finalize()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        q = st.query()
        st.close()
        best = dt if best is None else min(best, dt)
    sv = r["sv"].cpu().numpy()
    K = n - 1 if n % 2 == 0 else n
    return dict(m=m, n=n, complex=bool(cplx), ms=best * 1e3, sweeps=q["sweeps"], persistent_sweeps=q["loop_sweeps"],
                l2_local_sweeps=q["local_sweeps"], redone=q["loop_redos"], us_per_step=best * 1e6 / ((q["sweeps"] + 1) * K),
                max_rel_sigma_err=float(np.max(np.abs(sv - sig) / sig)))


def svd_large(torch, J, inputs, cplx, flags):
    """The whole plain SVD of a large workload: complex 4096 x 4096 (sigma
    geometric from 1 to 1e-12) or real 8192 x 2048 (sigma log-spaced in
    [1e-8, 1]), A = U diag(sigma) V^* with Haar factors (built on the host
    first, not timed).  Wall time of jsvd_gesvj on the resident input (HIP
    events), sweeps, and the sigma error against the prescribed values: the
    rounding of A to double moves sigma_i by up to about eps sigma_max, so the
    relative error is given for sigma_i >= 1e-6 sigma_max and the absolute
    error relative to sigma_max for all.  Default flags (no permutation)."""
    import numpy as np
    t0 = time.perf_counter()
    if cplx:
        Ar, Ai, sig = inputs.plain_complex_4096()
        m = n = 4096
    else:
        (Ar, sig), Ai = inputs.plain_real_tall(), None
        m, n = Ar.shape
    gen_s = time.perf_counter() - t0
    dAr = J.to_device_fortran(Ar)
    dAi = J.to_device_fortran(Ai) if cplx else None
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    r = J.gesvj(dAr, dAi, flags=flags)
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) * 1e-3
    sv = r["sv"].cpu().numpy()
    big = sig >= 1e-6 * sig[0]
    K = n - 1 if n % 2 == 0 else n
    return {"m": m, "n": n, "complex": bool(cplx), "flags": flags, "status": r["status"], "sweeps": r["sweeps"],
            "s": round(t, 3),
            "ms_per_sweep": round(t * 1e3 / max(r["sweeps"], 1), 2), "steps": r["sweeps"] * K,
            "max_rel_sigma_err_sigma_above_1e-6": float(np.max(np.abs(sv[big] - sig[big]) / sig[big])),
            "max_abs_sigma_err_over_sigma_max": float(np.max(np.abs(sv - sig)) / sig[0]),
            "input_generation_s": round(gen_s, 1)}


def cpu_oracle_svd(inputs, sweeps_256=None, sweeps_large=None, c4_sample=96):
    """Context: the oracle (C, on the host) on the SVD workloads:
    - the whole 256 x 256 real SVD with the step's loops over pairs on every
      host thread, and one sweep of it on one thread;
    - two steps each of the real 8192 x 2048 and complex 4096 x 4096
      workloads on one thread, extrapolated to one sweep (K steps) and to the
      whole SVD with the GPU run's sweep count (the oracle's iteration is the
      same, bit for bit);
    - a sample of the batched workload (every k-th matrix in the order of n),
      one oracle SVD per host thread at a time, extrapolated to the whole
      batch by the ratio of its algorithmic bytes (16 n (m + n) per step over
      the sweeps the GPU run took) to the sample's."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    nth = oracle.omp_max_threads()
    res = dict(kind="oracle", threads=nth, **host_cpu())
    A, _ = inputs.plain_real_256()
    oracle.set_step_threads(nth)
    try:
        t0 = time.perf_counter()
        r = oracle.gesvj(A)
        res["svd_real256_s"] = round(time.perf_counter() - t0, 3)
        res["svd_real256_sweeps"] = r["sweeps"]
    finally:
        oracle.set_step_threads(1)
    st = oracle.State(A)
    st.init()
    t0 = time.perf_counter()
    for _ in range(oracle.rr_steps(256)):
        st.step()
    sw = time.perf_counter() - t0
    res["svd_real256_sweep_1thread_s"] = round(sw, 3)
    if sweeps_256:
        res["svd_real256_1thread_s_extrapolated"] = round(sw * sweeps_256, 2)
    for (m, n, c) in ((8192, 2048, False), (4096, 4096, True)):
        g = inputs.rng(inputs.CFG_PLAIN_LARGE, 77 + int(c))
        Ar, Ai = inputs.random_columns(m, n, g, c)
        st = oracle.State(Ar, Ai)
        st.init()
        t0 = time.perf_counter()
        for _ in range(2):
            st.step()
        dt = (time.perf_counter() - t0) / 2
        K = n - 1 if n % 2 == 0 else n
        tg = f"{'c' if c else 'r'}{m}x{n}"
        res[f"step_{tg}_1thread_s"] = round(dt, 4)
        res[f"sweep_{tg}_1thread_s_extrapolated"] = round(dt * K, 1)
        if sweeps_large and sweeps_large.get(tg):
            res[f"svd_{tg}_1thread_h_extrapolated"] = round(dt * K * sweeps_large[tg] / 3600.0, 1)
    cost = _batched_cache.get("bytes_upper_0")
    if cost is not None and c4_sample > 0:
        count = len(cost)
        mm, nn, _ = inputs.batched_shapes(10000)
        mats, _ = batched_inputs(inputs, count)
        by_n = np.argsort(nn[:count], kind="stable")
        k = max(1, count // c4_sample)
        sample = [int(i) for i in by_n[k // 2::k][:c4_sample]]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(nth) as ex:
            outs = list(ex.map(lambda i: oracle.gesvj(mats[i])["status"], sample))
        dt = time.perf_counter() - t0
        factor = float(cost.sum() / cost[sample].sum())
        res["batched_sample"] = dict(matrices=len(sample), every=k, all_converged=all(o == 0 for o in outs),
                                     wall_s=round(dt, 2), threads=nth, extrapolation_factor=round(factor, 2),
                                     whole_batch_s_extrapolated=round(dt * factor, 1),
                                     svds_per_s_extrapolated=round(count / (dt * factor), 2))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2r", type=int, default=26)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched", type=int, default=10000, help="matrices of the batched workload (at most 10000)")
    ap.add_argument("--no-batched-ab", action="store_true",
                    help="time the batched workload with the full schedule tuner only, not also with the "
                         "threads-per-matrix tuner")
    ap.add_argument("--batched-plain", type=int, default=200,
                    help="matrices of the plain-path sample, stratified by n")
    ap.add_argument("--oracle-batched-sample", type=int, default=96,
                    help="matrices of the batched workload the CPU oracle solves (stratified by n)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-pool", type=int, default=64)
    ap.add_argument("--serve-sustained-rate", type=float, default=3.0,
                    help="a second serving line at this rate with no queue limit (0: skip)")
    ap.add_argument("--serve-sustained-seconds", type=float, default=30.0)
    ap.add_argument("--serve-max-large", type=int, default=0,
                    help="large requests on the device at once (0: the library's default)")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB copied once by a plain device copy before the timed region "
                         "(a reference for hardware byte counters)")
    ap.add_argument("--trace-summary", metavar="DB",
                    help="print the kernel table of a rocprofv3 --kernel-trace --stats database and exit")
    ap.add_argument("--only", default="",
                    help="comma-separated name prefixes: run only the secondary lines whose names start with one "
                         "(a prefix ending in '=' names one line exactly)")
    ap.add_argument("--counters", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="print per-kernel HBM bytes per dispatch from FETCH_SIZE / WRITE_SIZE databases of runs "
                         "made with --calib-copy, and exit")
    ap.add_argument("--busy", action="store_true",
                    help="with --trace-summary: print the device's busy fraction over the trace (the union of "
                         "all kernel intervals, overall and per 5 s window) and the kernel time per family instead")
    ap.add_argument("--last-call", metavar="PATTERN",
                    help="with --trace-summary: also list the dispatches of the last call into kernels matching "
                         "PATTERN; with --counters: count only the last dispatch of each such kernel")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="derive the EVD kernels' HBM bytes per launch from FETCH_SIZE / WRITE_SIZE "
                         "databases of runs made with --calib-copy, write profiles/evd2_traffic.json, exit")
    args = ap.parse_args()
    if args.trace_summary and args.busy:
        print(busy_table(args.trace_summary))
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        if args.last_call:
            print()
            print(last_call_table(args.trace_summary, args.last_call))
        return
    if args.counters:
        print(counters_table(args.counters[0], args.counters[1], args.calib_copy or 512, args.last_call))
        return
    if args.traffic_from:
        rec, md = traffic_from(args.traffic_from[0], args.traffic_from[1], args.calib_copy or 512)
        with open(os.path.join(ROOT, "profiles", "evd2_traffic.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        print(md)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the batched EVD and the Jacobi step are single-device "
              "kernels here; sharding them across GPUs is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2202_08361_amd as J
    from paper_2202_08361_amd import inputs

    if not os.path.exists(J.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)
    if args.calib_copy:
        src = torch.ones(args.calib_copy << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    r = 1 << args.log2r
    K, W = args.steps, args.warmup
    log(f"[bench] batched EVD: r = 2^{args.log2r} real + complex, warmup {W}, steps {K}")
    wall, dur, dev = evd_workload(torch, J, inputs, r, K, W)
    value = 2.0 * r * K / wall
    ms_per_step = wall / K * 1e3
    ach_c = EVD_BYTES_CPLX * r / dur[True] / 1e9
    ach_r = EVD_BYTES_REAL * r / dur[False] / 1e9
    log(f"[bench] EVD: {value:.4g} EVD/s, {ms_per_step:.3f} ms/step; complex kernel {dur[True]*1e3:.3f} ms "
        f"({ach_c:.0f} GB/s), real kernel {dur[False]*1e3:.3f} ms ({ach_r:.0f} GB/s)")
    ceil = evd_ceiling(torch, J, dev, r, K)
    log(f"[bench] EVD ceiling: {ceil}")
    tr_c, tr_r = (measured_traffic("complex"), measured_traffic("real")) if r == 1 << 26 else (None, None)
    roofline = dict(bound="hbm", kernel=evd_kernel_name(r, True), achieved=round(ach_c, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach_c / HBM_PEAK_GBS, 4),
                    traffic=None if tr_c is None else round(tr_c / 1e9, 4), traffic_unit="GB per launch",
                    bytes_per_launch=EVD_BYTES_CPLX * r, avg_launch_ms=round(dur[True] * 1e3, 4),
                    real_kernel=dict(kernel=evd_kernel_name(r, False), achieved=round(ach_r, 1),
                                     frac=round(ach_r / HBM_PEAK_GBS, 4),
                                     traffic=None if tr_r is None else round(tr_r / 1e9, 4),
                                     bytes_per_launch=EVD_BYTES_REAL * r,
                                     avg_launch_ms=round(dur[False] * 1e3, 4)),
                    ceiling=dict(ceil, frac_of_stream_ceiling=round(ach_c / ceil["stream_complex"]["GBs"], 4),
                                 note="the same streams moved without arithmetic, and a plain copy"))
    cpu = None
    if not args.no_cpu:
        import oracle
        ns = 1 << min(args.log2r, 24)
        nth = oracle.omp_max_threads()
        t0 = time.perf_counter()
        passes = 0
        while True:
            for cplx in (False, True):
                a11, a22, ar, ai = dev[cplx][2]
                oracle.evd2_batch(a11[:ns], a22[:ns], ar[:ns], None if ai is None else ai[:ns], nthreads=nth)
            passes += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        ct = time.perf_counter() - t0
        cpu = dict(value=round(2 * ns * passes / ct, 1), unit="EVD/s", cores=nth, kind="oracle",
                   sample=f"{passes} passes over the first 2^{ns.bit_length() - 1} real + "
                          f"2^{ns.bit_length() - 1} complex matrices of the workload, OpenMP over matrices, "
                          f"{ct:.1f} s", **host_cpu())
        log(f"[bench] cpu oracle: {cpu['value']:.4g} EVD/s on {nth} threads ({ct:.1f} s)")
    del dev
    torch.cuda.empty_cache()
    extra = {}
    if not args.no_extra:
        prefixes = [x for x in args.only.split(",") if x]
        tasks = [("evd_f32", lambda: evd_f32(torch, J, inputs, r, K, W))]
        big = ((8192, 2048, False), (4096, 4096, True))

        def tag(m, n, c):
            return f"{'c' if c else 'r'}{m}x{n}"
        for (m, n, c) in big:
            tasks.append((f"step_{tag(m, n, c)}", lambda m=m, n=n, c=c: step_roofline(torch, J, inputs, m, n, c)))
        for (m, n, c) in big:
            tasks.append((f"step_{tag(m, n, c)}_compensated",
                          lambda m=m, n=n, c=c: step_roofline(torch, J, inputs, m, n, c, flags=J.COMPENSATED)))
        for (m, n, c) in big:
            tasks.append((f"step_{tag(m, n, c)}_f32",
                          lambda m=m, n=n, c=c: step_roofline(torch, J, inputs, m, n, c, fp32=True)))
        # columns beyond the register tile (the streamed step)
        for (m, n, c) in ((65536, 512, False), (32768, 512, True)):
            tasks.append((f"step_{tag(m, n, c)}_streamed",
                          lambda m=m, n=n, c=c: step_roofline(torch, J, inputs, m, n, c, streamed=True)))
        for (m, n, c) in big:
            tasks.append((f"nrmf_{tag(m, n, c)}", lambda m=m, n=n, c=c: nrmf_rate(torch, J, inputs, m, n, c)))
        for nm, fl in (("svd_real256_f32", 0), ("svd_real256_permute_f32", J.PERMUTE)):
            tasks.append((nm, lambda fl=fl: svd_plain(torch, J, inputs, fl, fp32=True)))
        for nm, fl in (("svd_real256", 0), ("svd_real256_permute", J.PERMUTE),
                       ("svd_real256_compensated", J.COMPENSATED),
                       ("svd_real256_permute_compensated", J.PERMUTE | J.COMPENSATED)):
            tasks.append((nm, lambda fl=fl: svd_plain(torch, J, inputs, fl)))
        for nm, pers in (("svd_real256_persistent_sweeps", True), ("svd_real256_stepwise_sweeps", False)):
            tasks.append((nm, lambda pers=pers: svd_plain_sweeps(torch, J, inputs, pers)))
        # the persistent sweeps spread over the device instead of on one XCC
        tasks.append(("svd_real256_persistent_spread",
                      lambda: svd_plain_sweeps(torch, J, inputs, True, local=False)))
        # mid-size matrices (the persistent sweep with 256-thread workgroups)
        for (m, n, c) in ((1024, 256, False), (1000, 300, True)):
            for nm, pers in (("persistent_sweeps", True), ("stepwise_sweeps", False)):
                tasks.append((f"svd_mid_{tag(m, n, c)}_{nm}",
                              lambda m=m, n=n, c=c, pers=pers: svd_plain_sweeps(torch, J, inputs, pers, (m, n, c))))
        for (m, n, c) in big:
            for fp32 in (False, True):
                tasks.append((f"sweep_{tag(m, n, c)}" + ("_f32" if fp32 else ""),
                              lambda m=m, n=n, c=c, fp32=fp32: sweep_time(torch, J, inputs, m, n, c, fp32=fp32)))
        for (m, n, c) in big:
            tasks.append((f"svd_{tag(m, n, c)}", lambda c=c: svd_large(torch, J, inputs, c, 0)))
        if not args.no_batched:
            for nm, fl in (("batched", 0), ("batched_permute", J.PERMUTE)):
                tasks.append((nm, lambda fl=fl: batched_vs_plain(torch, J, inputs, args.batched, args.batched_plain,
                                                                 fl, ab=not args.no_batched_ab)))
        if not args.no_serve:
            tasks.append(("serving", lambda: serving_run(torch, J, inputs, args.serve_rate, args.serve_seconds,
                                                         args.serve_pool, 0,
                                                         max_large=args.serve_max_large)))
            if args.serve_sustained_rate > 0:
                tasks.append(("serving_sustained", lambda: serving_run(
                    torch, J, inputs, args.serve_sustained_rate, args.serve_sustained_seconds, args.serve_pool, 0,
                    max_queue=0, max_large=args.serve_max_large)))
        if not args.no_cpu:
            tasks.append(("cpu_oracle_svd", lambda: cpu_oracle_svd(
                inputs, extra.get("svd_real256", {}).get("sweeps"),
                {tg: extra.get(f"svd_{tg}", {}).get("sweeps") for tg in ("r8192x2048", "c4096x4096")},
                c4_sample=args.oracle_batched_sample)))
        for nm, fn in tasks:
            # a prefix ending in '=' names one line exactly
            if prefixes and not any(nm == x[:-1] if x.endswith("=") else nm.startswith(x) for x in prefixes):
                continue
            log(f"[bench] {nm}")
            extra[nm] = fn()
            log(f"[bench]   {extra[nm]}")
    line = {
        "metric": "batched 2x2 EVDs/s",
        "value": round(value, 1),
        "unit": "EVD/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched 2x2 EVD: 2^{args.log2r} real symmetric + 2^{args.log2r} complex "
                               "Hermitian, SoA FP64, components sign*2^U(-1074,1023)*U[1,2), 1% zeros, "
                               "1% subnormal a21", "r": r},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
