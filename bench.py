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


def step_roofline(torch, J, inputs, m, n, cplx, nsteps=20, warm=2):
    """Time the fused Jacobi step on a freshly loaded state (every pair transforms)."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 77 + int(cplx))
    Ar, Ai = inputs.random_columns(m, n, g, cplx)
    st = J.State(m, n, cplx)
    st.load(J.to_device_fortran(Ar), J.to_device_fortran(Ai) if cplx else None)
    for _ in range(warm):
        st.step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nsteps)]
    for s, e in evs:
        s.record()
        st.step()
        e.record()
    torch.cuda.synchronize()
    q = st.query()
    t = sum(s.elapsed_time(e) for s, e in evs) / nsteps * 1e-3
    c = 2 if cplx else 1
    byts = 16.0 * c * n * (m + n) * (q["last_t"] / (n // 2))
    st.close()
    return dict(m=m, n=n, complex=bool(cplx), us_per_step=t * 1e6, transformed=q["last_t"], pairs=n // 2,
                algorithmic_bytes=byts, achieved_GBs=byts / t / 1e9, frac=byts / t / 1e9 / HBM_PEAK_GBS)


def svd_plain(torch, J, inputs, flags):
    A, sig = inputs.plain_real_256()
    dA = J.to_device_fortran(A)
    J.gesvj(dA, flags=flags)               # warm-up (graph build, caches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = J.gesvj(dA, flags=flags)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    import numpy as np
    sv = r["sv"].cpu().numpy()
    return dict(ms=dt * 1e3, sweeps=r["sweeps"], status=r["status"],
                max_rel_sigma_err=float(np.max(np.abs(sv - sig) / sig)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2r", type=int, default=26)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the batched EVD and the Jacobi step are single-device "
              "kernels here (how the path would shard across GPUs is described in DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2202_08361_amd as J
    from paper_2202_08361_amd import inputs

    if not os.path.exists(J.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)
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
    roofline = dict(bound="hbm", kernel="evd2_kernel_v2<complex>", achieved=round(ach_c, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach_c / HBM_PEAK_GBS, 4), traffic=None,
                    bytes_per_launch=EVD_BYTES_CPLX * r, avg_launch_ms=round(dur[True] * 1e3, 4),
                    real_kernel=dict(achieved=round(ach_r, 1), frac=round(ach_r / HBM_PEAK_GBS, 4),
                                     bytes_per_launch=EVD_BYTES_REAL * r,
                                     avg_launch_ms=round(dur[False] * 1e3, 4)))
    cpu = None
    if not args.no_cpu:
        import oracle
        ns = 1 << min(args.log2r, 23)
        nth = oracle.omp_max_threads()
        t0 = time.perf_counter()
        for cplx in (False, True):
            a11, a22, ar, ai = dev[cplx][2]
            oracle.evd2_batch(a11[:ns], a22[:ns], ar[:ns], None if ai is None else ai[:ns], nthreads=nth)
        ct = time.perf_counter() - t0
        cpu = dict(value=round(2 * ns / ct, 1), unit="EVD/s", cores=nth, kind="oracle",
                   sample=f"first 2^{ns.bit_length() - 1} real + 2^{ns.bit_length() - 1} complex matrices of the "
                          f"workload, OpenMP over matrices, {ct:.1f} s")
        log(f"[bench] cpu oracle: {cpu['value']:.4g} EVD/s on {nth} threads")
    del dev
    torch.cuda.empty_cache()
    extra = {}
    if not args.no_extra:
        for (m, n, c) in ((8192, 2048, False), (4096, 4096, True)):
            log(f"[bench] Jacobi step {m}x{n} {'complex' if c else 'real'}")
            extra[f"step_{'c' if c else 'r'}{m}x{n}"] = step_roofline(torch, J, inputs, m, n, c)
            log(f"[bench]   {extra[f'step_{chr(99) if c else chr(114)}{m}x{n}']}")
        for nm, fl in (("svd_real256_permute", 0), ("svd_real256_nopermute", J.NO_PERMUTE)):
            log(f"[bench] {nm}")
            extra[nm] = svd_plain(torch, J, inputs, fl)
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
