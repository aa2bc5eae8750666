"""GPU tests of the continuous-batching server (jsvd_serve_*): requests of
mixed sizes and types submitted while others run overlap on the device, and
each result is bit-for-bit the one the same request gives alone
(jsvd_gesvj); admission under a small HBM budget, queue backpressure,
failing requests and the latency statistics."""
import numpy as np
import pytest

from paper_2202_08361_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def J():
    import paper_2202_08361_amd as jsvd
    return jsvd


def _bits(x):
    return np.ascontiguousarray(x.cpu().numpy()).view(np.int64)


def _pool(shapes, seed):
    g = inputs.rng(inputs.CFG_SERVE, 800 + seed)
    out = []
    for (m, n, c, kappa) in shapes:
        sig = inputs.sigma_logspace(n, 1.0 / kappa)
        Ar, Ai = inputs.svd_matrix(m, n, sig, g, cplx=c, extended=False)
        out.append((Ar, Ai))
    return out


def _alone(Ar, Ai):
    return J().gesvj(J().to_device_fortran(Ar), None if Ai is None else J().to_device_fortran(Ai))


def _same(a, b):
    for k in ("U_re", "U_im", "V_re", "V_im", "sv_e", "sv_f"):
        if a[k] is None and b[k] is None:
            continue
        assert np.array_equal(_bits(a[k]), _bits(b[k])), k
    assert a["status"] == b["status"] and a["sweeps"] == b["sweeps"]


def test_serve_mix_equals_alone():
    shapes = [(40, 32, False, 1e3), (700, 600, False, 1e6), (64, 33, True, 1e4), (300, 200, True, 1e5),
              (1200, 800, False, 1e4), (100, 100, False, 1e8), (513, 513, True, 1e3), (20, 20, True, 10.0),
              (256, 128, False, 1e2), (90, 17, False, 1e5)]
    pool = _pool(shapes, 1)
    srv = J().Server(hbm_budget_bytes=4 << 30, max_slots=4)
    tickets = []
    for (Ar, Ai) in pool * 2:
        t = srv.submit(J().to_device_fortran(Ar), None if Ai is None else J().to_device_fortran(Ai))
        assert t is not None
        tickets.append(t)
    results = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(tickets) and st["p99_ns"] >= st["p50_ns"] > 0
    for (Ar, Ai), r in zip(pool * 2, results):
        _same(r, _alone(Ar, Ai))


@pytest.mark.parametrize("shapes", [
    [(256, 256, False, 1e6)],                       # a small request alone: its own state, L2-local sweeps
    [(700, 300, True, 1e4), (120, 100, False, 1e3)],   # a mid-size request (spread sweeps), then a small one
])
def test_serve_lone_requests_sweep_persistently(shapes):
    """Requests submitted one at a time, each alone on the device: their
    sweeps run as persistent launches (the server's count), and each result
    is bit for bit the one jsvd_gesvj gives."""
    pool = _pool(shapes, 7)
    srv = J().Server(hbm_budget_bytes=4 << 30, max_slots=4)
    results = []
    for (Ar, Ai) in pool:
        t = srv.submit(J().to_device_fortran(Ar), None if Ai is None else J().to_device_fortran(Ai))
        assert t is not None
        results.append(srv.wait(t))
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(pool)
    assert st["persistent_sweeps"] > 0 and st["persistent_redos"] == 0, st
    for (Ar, Ai), r in zip(pool, results):
        _same(r, _alone(Ar, Ai))


def test_serve_groups_past_a_waiting_large_request():
    # two slots, one large request at a time: the first large request runs,
    # the second waits at the head of the queue, and the 40 small requests
    # behind it (at least 32 waiting) are admitted past it as a batched group
    g = inputs.rng(inputs.CFG_SERVE, 830)
    shapes = [(700, 600, False, 1e5), (640, 513, True, 1e3)]
    for i in range(40):
        n = int(g.integers(8, 65))
        shapes.append((int(g.integers(n, 2 * n + 1)), n, bool(i % 3 == 0), 10.0 ** float(g.uniform(1, 6))))
    pool = _pool(shapes, 2)
    srv = J().Server(hbm_budget_bytes=4 << 30, max_slots=2, max_large=1)
    tickets = []
    for (Ar, Ai) in pool:
        t = srv.submit(J().to_device_fortran(Ar), None if Ai is None else J().to_device_fortran(Ai))
        assert t is not None
        tickets.append(t)
    results = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(tickets)
    for (Ar, Ai), r in zip(pool, results):
        _same(r, _alone(Ar, Ai))


def test_serve_small_budget_and_backpressure():
    pool = _pool([(200, 150, False, 1e4), (600, 520, False, 1e3), (50, 40, True, 1e2)], 2)
    # a budget that holds one large request at a time: everything still completes
    one = 2 * 8 * (600 * 520 + 520 * 520) * 2
    srv = J().Server(hbm_budget_bytes=one, max_slots=8, max_queue=3)
    tickets, rejected = [], 0
    for i in range(12):
        Ar, Ai = pool[i % 3]
        t = srv.submit(J().to_device_fortran(Ar), None if Ai is None else J().to_device_fortran(Ai))
        if t is None:
            rejected += 1
        else:
            tickets.append((t, i % 3))
    res = [(srv.wait(t), k) for t, k in tickets]
    st = srv.stats()
    srv.close()
    assert st["rejected"] == rejected and st["completed"] == len(tickets)
    for r, k in res:
        _same(r, _alone(*pool[k]))


def test_serve_failures():
    A = np.ones((30, 20), order="F")
    A[3, 3] = np.nan
    B = np.ones((600, 520), order="F")
    B[7, 9] = np.inf
    srv = J().Server(hbm_budget_bytes=1 << 30, max_slots=2)
    t1 = srv.submit(J().to_device_fortran(A))
    t2 = srv.submit(J().to_device_fortran(B))
    t3 = srv.submit(J().to_device_fortran(np.zeros((40, 10), order="F")))
    r1, r2, r3 = srv.wait(t1), srv.wait(t2), srv.wait(t3)
    srv.close()
    assert r1["status"] == J().ENONFINITE and r2["status"] == J().ENONFINITE and r3["status"] == J().EZERO
