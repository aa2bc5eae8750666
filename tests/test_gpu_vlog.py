"""GPU parity of the deferred V update of the large-column step against the
oracle, bit for bit.

On the large-column path (m > 256 rows) V is not rotated per step: the pair
outcomes of up to 32 steps are logged and applied to a row-major V in one
pass, and V is switched back to column-major (and the log applied) whenever
it is read or the fused kernel takes over.  These tests drive every way in
and out of the log: more steps than the log holds between two reads, reads
in the middle of a log, switches between the two step paths with steps
still logged, single steps before a sweep, a restore with steps logged,
steps of a stopped iteration, odd n (ragged transpose tiles), single
precision.
"""
import numpy as np
import pytest

from paper_2202_08361_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

LOG = 32   # steps of the outcome log


def J():
    import paper_2202_08361_amd as jsvd
    return jsvd


def _iv(a):
    return np.int32 if a.dtype == np.float32 else np.int64


def _bits_equal(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return a.dtype == b.dtype and a.shape == b.shape and np.array_equal(a.view(_iv(a)), b.view(_iv(b)))


def _host(t):
    return None if t is None else t.cpu().numpy()


def _dev(a):
    if a is None:
        return None
    return J().to_device_fortran(a, dtype=torch.float32 if a.dtype == np.float32 else torch.float64)


def _check(ost, sv, tag):
    assert _bits_equal(_host(sv["G_re"]), ost.Gr), tag + " G_re"
    assert _bits_equal(_host(sv["V_re"]), ost.Vr), tag + " V_re"
    if ost.cplx:
        assert _bits_equal(_host(sv["G_im"]), ost.Gi), tag + " G_im"
        assert _bits_equal(_host(sv["V_im"]), ost.Vi), tag + " V_im"
    assert sv["s"] == ost.s and sv["Mt"] == float(ost.Mt) and sv["k"] == ost.k, tag + " scalars"


def _pair(ora, m, n, cplx, seed, single=False):
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 2600 + seed)
    Ar, Ai = inputs.random_columns(m, n, g, cplx)
    if single:
        Ar = np.asfortranarray(Ar.astype(np.float32))
        Ai = np.asfortranarray(Ai.astype(np.float32)) if cplx else None
    ost = (ora.SState if single else ora.State)(Ar, Ai)
    assert ost.init() == ora.OK
    st = J().State(m, n, cplx, fp32=single)
    assert st.load(_dev(Ar), _dev(Ai)) == 0
    return ost, st


def _steps(ost, st, k):
    for _ in range(k):
        ost.step()
        st.step()


@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("m,n,cplx", [(600, 40, False), (700, 33, True), (300, 77, False), (1100, 64, True)])
def test_log_wraps(ora, single, m, n, cplx):
    """More steps than the log holds between two reads of V (the log is
    applied when full and at the read), then reads in the middle of a log."""
    ost, st = _pair(ora, m, n, cplx, m + n, single)
    _steps(ost, st, 2 * LOG + 5)
    _check(ost, st.save(), f"after {2 * LOG + 5} steps")
    for k in (1, 7, LOG - 1, LOG, LOG + 1):
        _steps(ost, st, k)
        _check(ost, st.save(), f"after {k} more steps")


@pytest.mark.parametrize("cplx", [False, True])
def test_path_switches(ora, cplx):
    """Large-column steps with steps still logged, then fused-kernel steps
    (V column-major), then large-column steps again: every switch applies
    the log and transposes V."""
    m, n = 520, 45
    ost, st = _pair(ora, m, n, cplx, 11 + int(cplx))
    _steps(ost, st, 9)                  # 9 logged steps
    st.set_launch(1024)
    _steps(ost, st, 5)                  # fused kernel: log applied, V column-major
    st.set_launch(0)
    _steps(ost, st, LOG + 3)            # a full log applied, 3 logged
    st.set_launch(512)
    _steps(ost, st, 2)
    _check(ost, st.save(), "after the switches")
    st.set_launch(0)
    _steps(ost, st, 4)
    _check(ost, st.save(), "back on the large-column path")


@pytest.mark.parametrize("cplx", [False, True])
def test_steps_then_sweep(ora, cplx):
    """Single steps leave outcomes in the log; the sweep applies them before
    its own steps, and its graph ends with an empty log."""
    m, n = 900, 24
    ost, st = _pair(ora, m, n, cplx, 21 + int(cplx))
    _steps(ost, st, 5)
    K = ora.rr_steps(n)
    for _ in range(2):
        for _ in range(K):
            ost.step()
        st.sweep()
        _check(ost, st.save(), "sweep after single steps")
        _steps(ost, st, 3)
    _check(ost, st.save(), "steps after the sweeps")


def test_restore_discards_log(ora):
    """A restore replaces G, V and the scalars: steps logged before it are
    dropped, and the steps after it continue from the restored state."""
    m, n = 640, 30
    ost, st = _pair(ora, m, n, True, 31)
    _steps(ost, st, 6)
    sv = st.save()
    _check(ost, sv, "saved")
    snap = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in sv.items()}
    ref = (ost.Gr.copy(), ost.Gi.copy(), ost.Vr.copy(), ost.Vi.copy())
    _steps(ost, st, 10)                 # logged, then dropped by the restore
    st.restore(snap["G_re"], snap["G_im"], snap["V_re"], snap["V_im"], snap["s"], snap["Mt"], snap["k"])
    ost2 = ora.State(ref[0], ref[1])
    assert ost2.init() == ora.OK
    ost2.Gr[:], ost2.Gi[:], ost2.Vr[:], ost2.Vi[:] = ref
    ost2.s, ost2.Mt, ost2.k = snap["s"], snap["Mt"], snap["k"]
    _steps(ost2, st, LOG + 2)
    _check(ost2, st.save(), "after the restore")


def test_steps_after_stop(ora):
    """A converged state (the iteration stopped): further steps change
    nothing, V included, and the SVD read afterwards is the oracle's."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 2700)
    sig = inputs.sigma_logspace(20, 1e-4)
    Ar, _ = inputs.svd_matrix(400, 20, sig, g)
    ro = ora.gesvj(Ar)
    st = J().State(400, 20, False)
    assert st.load(_dev(Ar), None) == 0
    while not st.query()["converged"]:
        st.sweep()
    sv0 = st.save()
    for _ in range(LOG + 3):
        st.step()
    sv1 = st.save()
    for k in ("G_re", "V_re"):
        assert _bits_equal(_host(sv0[k]), _host(sv1[k])), k
    out = st.finalize()
    torch.cuda.synchronize()
    assert _bits_equal(_host(out["V_re"]), ro["V_re"]) and _bits_equal(_host(out["U_re"]), ro["U_re"])
    assert _bits_equal(_host(out["sv_f"]), ro["sv_f"]) and _bits_equal(_host(out["sv_e"]), ro["sv_e"])


@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("m,n,cplx", [(2000, 33, True), (1300, 65, False), (800, 97, True)])
def test_gesvj_large_column_path(ora, single, m, n, cplx):
    """Whole SVDs on the large-column path (odd and even n, n not a multiple
    of the transpose tile): U, V, sigma and the sweep count bit for bit."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 2800 + m)
    sig = inputs.sigma_logspace(n, 1e-5)
    Ar, Ai = inputs.svd_matrix(m, n, sig, g, cplx=cplx)
    if single:
        Ar = np.asfortranarray(Ar.astype(np.float32))
        Ai = np.asfortranarray(Ai.astype(np.float32)) if cplx else None
    ro = (ora.sgesvj if single else ora.gesvj)(Ar, Ai)
    rg = J().gesvj(_dev(Ar), _dev(Ai))
    torch.cuda.synchronize()
    assert ro["status"] == rg["status"] == 0 and ro["sweeps"] == rg["sweeps"]
    for k in ("U_re", "V_re", "sv_e", "sv_f") + (("U_im", "V_im") if cplx else ()):
        assert _bits_equal(_host(rg[k]), ro[k]), k


@pytest.mark.parametrize("m,permute", [(320, True), (100, False)])
@pytest.mark.parametrize("single", [False, True])
@pytest.mark.parametrize("cplx", [False, True])
def test_rescale_inside_a_chain(ora, single, cplx, m, permute):
    """Sect. 3.2 on the large-column path (320 rows) and the fused kernel
    (100 rows): G restored with its largest components just below the
    downscaling threshold, so that a later step of an unbroken chain (whose
    step index and M~ come from the previous step's log slot and max-norm
    key, not from the device scalars) is the one that downscales.  Six steps,
    then every bit against the oracle, the downscaling count included.  (With
    or without the sorting permutation: the trajectory on which one of the
    first six steps downscales in every case.)"""
    n = 16
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 2900 + 2 * int(cplx) + int(single))
    top = (124 if cplx else 126) if single else (1020 if cplx else 1022)
    Ar, Ai = inputs.random_columns(m, n, g, cplx)
    dt = np.float32 if single else np.float64
    # the largest component at 0.98 of 2^(top+1): floor(lg M~) = top, no
    # downscaling yet; a rotation that grows it by 2 % crosses the threshold
    raw = max(np.max(np.abs(Ar)), np.max(np.abs(Ai)) if cplx else 0.0)
    scale = 0.98 * np.ldexp(1.0, top + 1) / raw
    Gr = np.asfortranarray((Ar * scale).astype(dt))
    Gi = np.asfortranarray((Ai * scale).astype(dt)) if cplx else None
    mt = float(max(np.max(np.abs(Gr)), np.max(np.abs(Gi)) if cplx else 0.0))
    assert np.isfinite(mt) and np.frexp(mt)[1] - 1 <= top
    ost = (ora.SState if single else ora.State)(Gr, Gi, permute=permute)
    assert ost.init() == ora.OK
    ost.Gr[:] = Gr
    if cplx:
        ost.Gi[:] = Gi
    ost.Vr[:] = np.eye(n, dtype=dt)
    if cplx:
        ost.Vi[:] = 0
    ost.s, ost.Mt, ost.k = 0, mt, 0
    st = J().State(m, n, cplx, fp32=single)
    if permute:
        st.set_flags(J().PERMUTE)
    eye = np.asfortranarray(np.eye(n, dtype=dt))
    st.restore(_dev(Gr), _dev(Gi), _dev(eye), _dev(np.zeros_like(eye)) if cplx else None, 0, mt, 0)
    seen = []
    for _ in range(6):
        ost.step()
        st.step()
        seen.append(ost.rescaled)
    # the first step does not downscale; one of the chained steps does
    assert seen[0] == 0 and seen[-1] >= 1, seen
    q = st.query()
    assert q["rescaled"] == ost.rescaled
    _check(ost, st.save(), "after six steps")


@pytest.mark.parametrize("m,n,cplx", [(4096, 4096, True), (8192, 2048, False)])
def test_full_size_sweep_properties(m, n, cplx):
    """One whole sweep of the large workloads through the captured sweep graph
    (K steps, the V update applied 128 / 64 times, V transposed back for the
    read): properties that hold at any size, since the oracle would need half
    an hour for this sweep.  V stays unitary, ||V^H V - I||_max <= 1e-12, and
    G = 2^s A V to 1e-12 relative in the Frobenius norm (every rotation is
    applied to G and V alike; the error is a few eps per rotation)."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 88 + int(cplx))
    Ar, Ai = inputs.random_columns(m, n, g, cplx)
    st = J().State(m, n, cplx)
    assert st.load(_dev(Ar), _dev(Ai)) == 0
    st.sweep()
    q = st.query()
    assert q["sweeps"] == 1 and q["steps"] == n - 1 and q["last_sweep_T"] > 0
    sv = st.save()
    torch.cuda.synchronize()
    dev = sv["G_re"].device
    if cplx:
        G = torch.complex(sv["G_re"], sv["G_im"])
        V = torch.complex(sv["V_re"], sv["V_im"])
        A = torch.complex(torch.from_numpy(np.ascontiguousarray(Ar)), torch.from_numpy(np.ascontiguousarray(Ai))).to(dev)
    else:
        G, V = sv["G_re"], sv["V_re"]
        A = torch.from_numpy(np.ascontiguousarray(Ar)).to(dev)
    G, V = G.contiguous(), V.contiguous()
    eye = torch.eye(n, dtype=V.dtype, device=dev)
    orth = (V.conj().transpose(0, 1).contiguous() @ V - eye).abs().max().item()
    assert orth <= 1e-12, orth
    # G carries the scaling 2^s (s near 1000 here): compare 2^-s G (exact) with A V
    Gs = G * (2.0 ** -sv["s"])
    res = torch.linalg.norm(Gs - A @ V).item() / torch.linalg.norm(A).item()
    assert res <= 1e-12, res


@pytest.mark.parametrize("cplx", [False, True])
def test_full_size_svd_workloads(cplx):
    """The whole SVD of the large workloads as the benchmark times them, with
    the default flags (no permutation): real 8192 x 2048 (A = U diag(sigma) V^T with Haar factors,
    sigma log-spaced in [1e-8, 1]) and complex 4096 x 4096 (sigma geometric
    from 1 to 1e-12).  It converges; the relative sigma error is at most 1e-10
    for sigma >= 1e-6 sigma_max (kappa <= 1e6, where that tolerance applies;
    rounding A to double already moves sigma_i by about eps sigma_max); the
    residual ||A - U diag(sigma) V^*||_F is at most 64 n eps ||A||_F; V is
    unitary within the same 64 n eps (max element of V^* V - I: the 42 / 62
    sweeps' rotations accumulate a few eps each, against 1e-12 after one
    sweep)."""
    if cplx:
        Ar, Ai, sig = inputs.plain_complex_4096()
    else:
        (Ar, sig), Ai = inputs.plain_real_tall(), None
    m, n = Ar.shape
    r = J().gesvj(_dev(Ar), _dev(Ai))
    assert r["status"] == 0, r["status"]
    sv = r["sv"].cpu().numpy()
    big = sig >= 1e-6 * sig[0]
    rel = float(np.max(np.abs(sv[big] - sig[big]) / sig[big]))
    assert rel <= 1e-10, rel
    s = r["sv"]
    if cplx:
        A = torch.complex(_dev(Ar), _dev(Ai))
        U = torch.complex(r["U_re"], r["U_im"])
        V = torch.complex(r["V_re"], r["V_im"])
    else:
        A, U, V = _dev(Ar), r["U_re"], r["V_re"]
    tol = 64 * n * np.finfo(np.float64).eps
    Vh = V.conj().transpose(0, 1).contiguous()
    res = (torch.linalg.norm(A - (U * s) @ Vh) / torch.linalg.norm(A)).item()
    assert res <= tol, res
    eye = torch.eye(n, dtype=V.dtype, device=V.device)
    orth = (Vh @ V - eye).abs().max().item()
    assert orth <= tol, orth
