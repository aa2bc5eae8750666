"""GPU tests of the large-column steps' skipping of unchanged pairs: a pair
whose two columns have not changed since it last met (one sweep earlier)
is not read, since its norms, dot-product and decision are those of that
meeting.  The bar stays bit-for-bit equality with the oracle, which computes
every pair: after every step of several sweeps, for whole SVDs, across a
change of launch path or of flags (which must reset the record of changes),
a restore, and in single precision.  The skipping must also happen
(jsvd_state_query's skipped_pairs)."""
import numpy as np
import pytest

from paper_2202_08361_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def J():
    import paper_2202_08361_amd as jsvd
    return jsvd


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads(ora):
    import os
    ora.set_step_threads(min(16, os.cpu_count() or 1))
    yield
    ora.set_step_threads(1)


def _bits(x):
    return np.ascontiguousarray(x.cpu().numpy() if hasattr(x, "cpu") else x).view(np.int64)


def _graded(m, n, cplx, seed, kappa=1e8):
    """Columns of very different norms: the large ones settle within a few
    sweeps while the small ones keep rotating, so many pairs stop changing."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 6100 + seed)
    sig = inputs.sigma_logspace(n, 1.0 / kappa)
    Ar, Ai = inputs.svd_matrix(m, n, sig, g, cplx=cplx)
    sc = np.logspace(0, -6, n)[None, :]
    Ar = np.asfortranarray(Ar * sc)
    Ai = np.asfortranarray(Ai * sc) if cplx else None
    return Ar, Ai


def _check(ost, sv, q, tag):
    assert np.array_equal(_bits(sv["G_re"]), ost.Gr.view(np.int64)), tag + " G_re"
    assert np.array_equal(_bits(sv["V_re"]), ost.Vr.view(np.int64)), tag + " V_re"
    if ost.cplx:
        assert np.array_equal(_bits(sv["G_im"]), ost.Gi.view(np.int64)), tag + " G_im"
        assert np.array_equal(_bits(sv["V_im"]), ost.Vi.view(np.int64)), tag + " V_im"
    assert np.array_equal(_bits(sv["e"]), ost.e.view(np.int64)), tag + " e"
    assert np.array_equal(_bits(sv["f"]), ost.f.view(np.int64)), tag + " f"
    assert sv["s"] == ost.s and sv["Mt"] == ost.Mt and sv["k"] == ost.k, tag + " scalars"
    assert q["last_t"] == ost.last_t, tag + " t"


@pytest.mark.parametrize("m,n,cplx,flags", [(600, 40, False, 0), (520, 33, True, 0), (700, 24, False, 8),
                                            (300, 31, True, 2)])
def test_skipping_steps_bitwise(ora, m, n, cplx, flags):
    """Sweeps step by step (eager steps and captured sweeps alternating),
    compared with the oracle after every step, until the oracle converges."""
    Ar, Ai = _graded(m, n, cplx, m + n)
    ost = ora.State(Ar, Ai, permute=bool(flags & 8), compensated=bool(flags & 2))
    assert ost.init() == ora.OK
    st = J().State(m, n, cplx)
    st.set_flags(flags)
    st.load(J().to_device_fortran(Ar), J().to_device_fortran(Ai) if cplx else None)
    K = ora.rr_steps(n)
    for sweep in range(60):
        T = 0
        if sweep % 2 == 0:
            for k in range(K):
                ost.step()
                T += ost.last_t
                st.step()
                _check(ost, st.save(), st.query(), f"sweep {sweep} step {k}")
        else:
            for k in range(K):
                ost.step()
                T += ost.last_t
            st.sweep()
            _check(ost, st.save(), st.query(), f"sweep {sweep}")
        if T == 0:
            break
    assert T == 0
    assert st.query()["skipped_pairs"] > 0
    st.close()


@pytest.mark.parametrize("m,n,cplx,kappa", [(800, 64, False, 1e10), (600, 48, True, 1e6)])
def test_skipping_whole_svd(ora, m, n, cplx, kappa):
    Ar, Ai = _graded(m, n, cplx, 7 * m, kappa)
    st = J().State(m, n, cplx)
    # the large-column steps (these shapes would otherwise sweep as
    # persistent launches, which read every pair)
    st.set_loop_wait(0.0)
    st.load(J().to_device_fortran(Ar), J().to_device_fortran(Ai) if cplx else None)
    st.iterate()
    info = st.query()
    r = st.finalize()
    torch.cuda.synchronize()
    st.close()
    ro = ora.gesvj(Ar, Ai)
    assert info["status"] == 0 and info["converged"] == 1 and info["sweeps"] == ro["sweeps"]
    assert info["skipped_pairs"] > 0
    for k in ("U_re", "U_im", "V_re", "V_im", "sv_e", "sv_f"):
        if ro[k] is None:
            continue
        assert np.array_equal(_bits(r[k]), _bits(ro[k])), k


def test_skipping_survives_path_and_flag_changes(ora):
    """Sweeps on the large-column path, then on the fused kernel (a forced
    launch shape, which does not record changes), then back; a flag change;
    a restore of an earlier state: the record of changes is reset each time,
    and every sweep stays the oracle's."""
    m, n = 640, 36
    Ar, _ = _graded(m, n, False, 99)
    ost = ora.State(Ar)
    assert ost.init() == ora.OK
    st = J().State(m, n, False)
    st.load(J().to_device_fortran(Ar))
    K = ora.rr_steps(n)

    def sweep_both(tag):
        for _ in range(K):
            ost.step()
        st.sweep()
        _check(ost, st.save(), st.query(), tag)
    for i in range(6):
        sweep_both(f"gpair {i}")
    st.set_launch(512)
    for i in range(2):
        sweep_both(f"fused {i}")
    st.set_launch(0)
    for i in range(3):
        sweep_both(f"gpair again {i}")
    saved = st.save()
    ost_saved = (ost.Gr.copy(), ost.Vr.copy(), ost.e.copy(), ost.f.copy(), ost.s, ost.Mt, ost.k)
    st.set_flags(J().COMPENSATED)
    ost.compensated = True
    for i in range(2):
        sweep_both(f"compensated {i}")
    st.set_flags(0)
    ost.compensated = False
    # back to the saved state on both sides, then on
    st.restore(saved["G_re"], None, saved["V_re"], None, saved["s"], saved["Mt"], saved["k"])
    ost.Gr[:], ost.Vr[:], ost.e[:], ost.f[:] = ost_saved[0], ost_saved[1], ost_saved[2], ost_saved[3]
    ost.s, ost.Mt, ost.k = ost_saved[4], ost_saved[5], ost_saved[6]
    for i in range(4):
        for _ in range(K):
            ost.step()
        st.sweep()
        sv = st.save()
        assert np.array_equal(_bits(sv["G_re"]), ost.Gr.view(np.int64)), f"after restore {i}"
        assert np.array_equal(_bits(sv["V_re"]), ost.Vr.view(np.int64)), f"after restore {i}"
    assert st.query()["skipped_pairs"] > 0
    st.close()


def test_skipping_single_precision():
    import oracle
    m, n = 520, 30
    Ar, _ = _graded(m, n, False, 5, kappa=1e4)
    ar = Ar.astype(np.float32)
    ost = oracle.SState(ar)
    assert ost.init() == oracle.OK
    st = J().State(m, n, False, fp32=True)
    st.load(J().to_device_fortran(ar, dtype=torch.float32))
    K = oracle.rr_steps(n)
    for sweep in range(40):
        T = 0
        for _ in range(K):
            ost.step()
            T += ost.last_t
        st.sweep()
        sv = st.save()
        assert np.array_equal(np.ascontiguousarray(sv["G_re"].cpu().numpy()).view(np.int32), ost.Gr.view(np.int32))
        assert np.array_equal(np.ascontiguousarray(sv["V_re"].cpu().numpy()).view(np.int32), ost.Vr.view(np.int32))
        if T == 0:
            break
    assert st.query()["skipped_pairs"] > 0
    st.close()
