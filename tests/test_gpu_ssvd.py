"""GPU parity of the single precision Jacobi step and SVD (jsvd_state_*_f32,
jsvd_gesvj_f32) against the single precision CPU oracle.

Both sides carry out the method in IEEE single arithmetic with the float
range constants (nu = FLT_MAX, eps = 2^-24, s_(k) = 126 / 124 - floor(lg M~),
s_[k] from eq. (skn) with nu = FLT_MAX, the Gram scaling with
FLT_MAX_EXP - 1, the single precision EVD) and evaluate every sum in the same
canonical 1024-lane order, so the bar is bit-for-bit equality of G, V, the
column norms, M~, s and the transformation count after every step, and of U,
V and sigma at the end of the SVD.  Both the fused step kernel (m <= 256 or a
forced workgroup size) and the G / V kernel pair (longer columns, up to
16384 real / 8192 complex rows in registers) are covered.
"""
import ctypes

import numpy as np
import pytest

from paper_2202_08361_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

f32 = np.float32


def J():
    import paper_2202_08361_amd as jsvd
    return jsvd


def _bits_equal(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    return a.dtype == b.dtype == np.float32 and a.shape == b.shape and np.array_equal(a.view(np.int32),
                                                                                        b.view(np.int32))


def _host(t):
    return None if t is None else t.cpu().numpy()


def _dev32(a):
    """Column-major float32 device copy of a float32 host array."""
    if a is None:
        return None
    m, n = a.shape
    out = J().fortran_empty(m, n, dtype=torch.float32)
    out.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return out


def _columns(m, n, cplx, seed):
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 2000 + seed)
    Ar, Ai = inputs.random_columns(m, n, g, cplx)
    return Ar.astype(np.float32), (Ai.astype(np.float32) if cplx else None)


def _check_state(ost, sv, tag):
    assert _bits_equal(_host(sv["G_re"]), ost.Gr), tag + " G_re"
    if ost.cplx:
        assert _bits_equal(_host(sv["G_im"]), ost.Gi), tag + " G_im"
    assert _bits_equal(_host(sv["V_re"]), ost.Vr), tag + " V_re"
    if ost.cplx:
        assert _bits_equal(_host(sv["V_im"]), ost.Vi), tag + " V_im"
    assert sv["s"] == ost.s and sv["Mt"] == float(ost.Mt), tag + " scalars"
    assert sv["k"] == ost.k, tag + " k"


def _pair_run(ora, m, n, cplx, steps, seed, threads=0, check_every=1, permute=False):
    Ar, Ai = _columns(m, n, cplx, seed)
    ost = ora.SState(Ar, Ai, permute=permute)
    assert ost.init() == ora.OK
    st = J().State(m, n, cplx, fp32=True)
    if threads:
        st.set_launch(threads)
    if permute:
        st.set_flags(J().PERMUTE)
    assert st.load(_dev32(Ar), _dev32(Ai)) == 0
    _check_state(ost, st.save(), f"load m={m} n={n}")
    for k in range(steps):
        ost.step()
        st.step()
        if (k + 1) % check_every == 0 or k == steps - 1:
            sv = st.save()
            _check_state(ost, sv, f"step {k} m={m} n={n} cplx={cplx} W={threads}")
            q = st.query()
            assert q["last_t"] == ost.last_t
            assert _bits_equal(_host(sv["e"]), ost.e) and _bits_equal(_host(sv["f"]), ost.f)
    return st


@pytest.mark.parametrize("m,n,cplx", [
    (16, 16, False), (70, 24, True), (100, 37, False), (256, 256, False), (97, 33, True),
    (1500, 64, False), (2100, 20, True), (4096, 8, False), (5000, 12, True), (9000, 6, False),
    (16000, 4, False), (8000, 5, True),
])
def test_sstep_bitwise(ora, m, n, cplx):
    """Every step, every bit (chains of the 1024-lane accumulation from
    m > 1024, ragged tails, odd n, the longest register tiles)."""
    K = ora.rr_steps(n)
    _pair_run(ora, m, n, cplx, steps=min(2 * K + 1, 40), seed=m + n, check_every=1 if n <= 64 else 7)


def test_sstep_permute(ora):
    _pair_run(ora, 600, 30, True, steps=35, seed=11, permute=True, check_every=5)


@pytest.mark.parametrize("cplx,m", [(False, 500), (True, 500), (False, 3000), (True, 3000)])
def test_slaunch_shapes_identical(ora, cplx, m):
    """Threads per pair 64 ... 1024 (the fused kernel) give the same bits as
    the G / V kernel pair and the oracle."""
    n = 18
    ref = None
    for W in [0] + [w for w in (64, 128, 256, 512, 1024) if w * 8 >= m]:
        st = _pair_run(ora, m, n, cplx, steps=5, seed=7, threads=W, check_every=5)
        sv = st.save()
        cur = (_host(sv["G_re"]), _host(sv["V_re"]))
        if ref is not None:
            assert _bits_equal(cur[0], ref[0]) and _bits_equal(cur[1], ref[1])
        ref = cur


@pytest.mark.parametrize("m", [100, 2000])
def test_srescale_path(ora, m):
    """Sect. 3.2 with nu = FLT_MAX: a state whose M~ exceeds nu/2 is downscaled
    at the step start, on both step kernels."""
    n = 10
    Ar, _ = _columns(m, n, False, 40)
    ost = ora.SState(Ar)
    ost.init()
    ost.Mt = f32(np.finfo(np.float32).max * f32(0.75))
    ost.Vr[:] = np.eye(n, dtype=np.float32)
    st = J().State(m, n, fp32=True)
    st.restore(_dev32(ost.Gr), None, _dev32(ost.Vr), None, ost.s, float(ost.Mt), 0)
    ost.step()
    st.step()
    q = st.query()
    assert q["rescaled"] == 1 and ost.rescaled == 1
    _check_state(ost, st.save(), "rescale")


def _gesvj_both(ora, Ar, Ai, flags=0, max_sweeps=0):
    ro = ora.sgesvj(Ar, Ai, flags=flags, max_sweeps=max_sweeps or 128)
    rg = J().gesvj(_dev32(Ar), _dev32(Ai), flags=flags, max_sweeps=max_sweeps)
    torch.cuda.synchronize()
    return ro, rg


def _check_svd(ro, rg):
    assert rg["status"] == ro["status"] and rg["sweeps"] == ro["sweeps"]
    assert _bits_equal(_host(rg["sv_e"]), ro["sv_e"]) and _bits_equal(_host(rg["sv_f"]), ro["sv_f"])
    assert _bits_equal(_host(rg["U_re"]), ro["U_re"]) and _bits_equal(_host(rg["V_re"]), ro["V_re"])
    if ro["U_im"] is not None:
        assert _bits_equal(_host(rg["U_im"]), ro["U_im"]) and _bits_equal(_host(rg["V_im"]), ro["V_im"])


@pytest.mark.parametrize("flags", [0, 8])
def test_sgesvj_plain_real_256(ora, flags):
    """The plain real 256 x 256 workload rounded to float: the whole single
    precision SVD bit for bit, sigma within 32 eps kappa of the singular
    values of the rounded matrix (computed in double)."""
    A, _ = inputs.plain_real_256()
    A = A.astype(np.float32)
    ro, rg = _gesvj_both(ora, A, None, flags)
    assert ro["status"] == 0
    _check_svd(ro, rg)
    sv = rg["sv"].cpu().numpy().astype(np.float64)
    ref = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    assert np.max(np.abs(sv - ref) / ref) <= 32 * 2.0 ** -24 * (ref[0] / ref[-1])


@pytest.mark.parametrize("m,n,cplx,kappa", [(60, 33, True, 1e3), (129, 128, False, 1e4), (7, 1, False, 1.0),
                                              (2, 2, True, 10.0), (1100, 40, False, 1e3), (700, 64, True, 1e2)])
def test_sgesvj_bitwise_shapes(ora, m, n, cplx, kappa):
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 2500 + m)
    sig = inputs.sigma_logspace(n, 1.0 / kappa)
    Ar, Ai = inputs.svd_matrix(m, n, sig, g, cplx=cplx)
    Ar = Ar.astype(np.float32)
    Ai = Ai.astype(np.float32) if cplx else None
    ro, rg = _gesvj_both(ora, Ar, Ai)
    _check_svd(ro, rg)


def test_sgesvj_failures(ora):
    A = np.ones((5, 3), dtype=np.float32, order="F")
    B = A.copy(order="F")
    B[2, 1] = np.nan
    assert J().gesvj(_dev32(B))["status"] == J().ENONFINITE
    B[2, 1] = np.inf
    assert J().gesvj(_dev32(B))["status"] == J().ENONFINITE
    assert J().gesvj(_dev32(np.zeros((5, 3), dtype=np.float32)))["status"] == J().EZERO
    Ar, _ = _columns(30, 20, False, 60)
    ro, rg = _gesvj_both(ora, Ar, None, max_sweeps=1)
    assert rg["status"] == ro["status"] == J().NOT_CONVERGED and rg["sweeps"] == 1
    assert _bits_equal(_host(rg["U_re"]), ro["U_re"]) and _bits_equal(_host(rg["sv_f"]), ro["sv_f"])
    assert _bits_equal(_host(rg["sv_e"]), ro["sv_e"])


def test_sstate_kind_checks():
    """A single precision state takes only the _f32 data calls and a double
    state only the double ones; the compensated flag is double only."""
    L = J().lib()
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(x.data_ptr())
    h32, h64 = ctypes.c_void_p(), ctypes.c_void_p()
    assert L.jsvd_state_create_f32(8, 4, 0, ctypes.byref(h32)) == 0
    assert L.jsvd_state_create(8, 4, 0, ctypes.byref(h64)) == 0
    try:
        assert L.jsvd_state_load(h32, p, None, 8, None) == J().EINVAL
        assert L.jsvd_state_load_f32(h64, p, None, 8, None) == J().EINVAL
        assert L.jsvd_state_finalize(h32, p, None, 8, p, None, 4, p, p, None, None) == J().EINVAL
        assert L.jsvd_state_finalize_f32(h64, p, None, 8, p, None, 4, p, p, None, None) == J().EINVAL
        assert L.jsvd_state_set_flags(h32, J().COMPENSATED) == J().EINVAL
        assert L.jsvd_state_set_flags(h64, J().COMPENSATED) == 0
        # M~ must be a float value for a single precision state
        assert L.jsvd_state_restore_f32(h32, p, None, 8, p, None, 4, 0, 0.1, 0, None) == J().EINVAL
        assert L.jsvd_state_restore_f32(h32, p, None, 8, p, None, 4, 0, 1e300, 0, None) == J().EINVAL
    finally:
        L.jsvd_state_destroy(h32)
        L.jsvd_state_destroy(h64)
    assert L.jsvd_gesvj_f32(8, 4, p, None, 8, p, None, 4, p, p, None, 0, None, J().COMPENSATED,
                            None) == J().EINVAL


def test_srun_to_run(ora):
    """Repeated runs of the same single precision SVD give identical bits."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 2700)
    sig = inputs.sigma_logspace(96, 1e-3)
    Ar, Ai = inputs.svd_matrix(1030, 96, sig, g, cplx=True)
    Ar, Ai = Ar.astype(np.float32), Ai.astype(np.float32)
    first = None
    for _ in range(5):
        r = J().gesvj(_dev32(Ar), _dev32(Ai))
        cur = [_host(r[k]) for k in ("U_re", "U_im", "V_re", "V_im", "sv_e", "sv_f")]
        if first is None:
            first = cur
        else:
            assert all(_bits_equal(a, b) for a, b in zip(cur, first))


@pytest.mark.parametrize("m,n,cplx", [(8192, 2048, False), (4096, 4096, True)])
def test_sstep_full_size(ora, m, n, cplx):
    """One single precision step of the large workloads (real 8192 x 2048,
    complex 4096 x 4096) on Gaussian columns: G, V, norms and scalars bit
    for bit."""
    _pair_run(ora, m, n, cplx, steps=1, seed=1)


@pytest.mark.parametrize("m,n,cplx", [(1500, 21, True), (700, 32, False), (3000, 9, False), (200, 40, True)])
def test_ssweep_graph_bitwise(ora, m, n, cplx):
    """Whole sweeps through the captured sweep graph equal K oracle steps,
    with the sweep's transformation and swap counts."""
    Ar, Ai = _columns(m, n, cplx, 80 + m)
    ost = ora.SState(Ar, Ai)
    assert ost.init() == ora.OK
    st = J().State(m, n, cplx, fp32=True)
    assert st.load(_dev32(Ar), _dev32(Ai)) == 0
    K = ora.rr_steps(n)
    for sweep in range(3):
        T = SW = 0
        for _ in range(K):
            T += ost.step()
            SW += ost.last_sw
        st.sweep()
        q = st.query()
        _check_state(ost, st.save(), f"sweep {sweep} m={m} n={n} cplx={cplx}")
        assert q["last_sweep_T"] == T and q["last_sweep_swaps"] == SW
        assert q["steps"] == ost.k
