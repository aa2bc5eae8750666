"""GPU tests of the persistent sweep (one launch per sweep, pairs started as
soon as their columns are out of the previous step) used by
jsvd_state_iterate and jsvd_gesvj for columns of at most 1024 rows.

The bar is bit-for-bit equality with the CPU oracle (U, V, sigma, sweep
count; the oracle reads every pair, the persistent sweep skips those whose
columns have not changed since they last met), and with the step-by-step
sweeps of the same state (forced by a
fixed launch shape, or by a zero wait budget).  Also: the sweeps did run as
persistent launches (jsvd_state_query's count), a matrix whose Frobenius
bound rules the persistent sweep out gives the same bits through the
step-by-step sweeps, and a wait budget so small that every persistent sweep
gives up (the bounded wait's own exit, forced from the host) is redone step
by step with the same bits.  Where the slots fit on one XCC (64-thread
workgroups, at most four per compute unit there) the persistent sweeps run
in the L2-local mode, and give the same bits as the spread mode
(jsvd_state_set_loop_local(st, 0))."""
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
    """The oracle's step loops on the host's threads (results do not depend on it)."""
    import os
    ora.set_step_threads(min(16, os.cpu_count() or 1))
    yield
    ora.set_step_threads(1)


def _bits(x):
    return np.ascontiguousarray(x.cpu().numpy() if hasattr(x, "cpu") else x).view(np.int64)


def _matrix(m, n, cplx, kappa, seed):
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 7100 + seed)
    sig = inputs.sigma_logspace(n, 1.0 / kappa)
    return inputs.svd_matrix(m, n, sig, g, cplx=cplx)


def _iterate(Ar, Ai, flags=0, wait=None, threads=0, local=None):
    m, n = Ar.shape
    st = J().State(m, n, Ai is not None)
    if flags:
        st.set_flags(flags)
    if threads:
        st.set_launch(threads)
    if wait is not None:
        st.set_loop_wait(wait)
    if local is not None:
        st.set_loop_local(local)
    st.load(J().to_device_fortran(Ar), None if Ai is None else J().to_device_fortran(Ai))
    st.iterate()
    q = st.query()
    out = st.finalize()
    torch.cuda.synchronize()
    st.close()
    out["info"] = q
    return out


def _local_fits(m, n, cplx=False):
    """The L2-local mode applies: n <= 256 and columns of at most 1024 real /
    512 complex rows (one 64-thread workgroup per slot, 1 to 16 rows per
    lane), every slot on one of the 8 XCCs with at most four workgroups per
    compute unit."""
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    return m <= (512 if cplx else 1024) and n <= 256 and ncu % 8 == 0 and (n + 1) // 2 <= 4 * (ncu // 8)


def _same(a, b, tag):
    for k in ("U_re", "U_im", "V_re", "V_im", "sv_e", "sv_f"):
        if a[k] is None:
            assert b[k] is None, (tag, k)
        else:
            assert np.array_equal(_bits(a[k]), _bits(b[k])), (tag, k)


@pytest.mark.parametrize("m,n,cplx,flags", [
    (256, 256, False, 0), (200, 131, False, 0), (64, 64, True, 0), (100, 37, True, 0),
    (256, 255, True, 0), (120, 80, False, 2), (90, 57, True, 2), (77, 40, False, 8),
    (60, 60, True, 8), (33, 2, False, 0), (5, 3, True, 0), (1, 1, False, 0), (130, 129, False, 4),
    # 256-thread workgroups (257 to 1024 rows)
    (300, 200, False, 0), (512, 300, True, 0), (1024, 130, False, 2), (700, 255, True, 8), (640, 97, False, 0),
    (257, 257, True, 4),
    # one wavefront at 8 and 16 rows per lane (the L2-local mode beyond 256 rows)
    (512, 256, False, 0), (1000, 199, True, 2), (1024, 256, False, 4), (384, 120, True, 0)])
def test_loop_matches_oracle_and_steps(ora, m, n, cplx, flags):
    Ar, Ai = _matrix(m, n, cplx, 1e6, m + 3 * n)
    got = _iterate(Ar, Ai, flags)
    info = got["info"]
    assert info["status"] == 0 and info["converged"] == 1
    # the sweeps ran as persistent launches and none had to be redone; in the
    # L2-local mode where the slots fit on one XCC
    assert info["loop_sweeps"] == info["sweeps"] + 1 and info["loop_redos"] == 0, info
    assert info["local_sweeps"] == (info["loop_sweeps"] if _local_fits(m, n, cplx) else 0), info
    # the pairs whose columns had not changed since they last met were not read
    if n >= 64:
        assert info["skipped_pairs"] > 0, info
    ora_flags = (ora.COMPENSATED if flags & 2 else 0) | (ora.PERMUTE if flags & 8 else 0) | \
        (ora.NO_GS if flags & 4 else 0)
    ro = ora.gesvj(Ar, Ai, flags=ora_flags)
    assert ro["status"] == 0 and ro["sweeps"] == info["sweeps"]
    for k in ("U_re", "U_im", "V_re", "V_im", "sv_e", "sv_f"):
        if ro[k] is None:
            continue
        assert np.array_equal(_bits(got[k]), _bits(ro[k])), k
    # the same state swept step by step (fixed launch shape)
    steps = _iterate(Ar, Ai, flags, threads=64 if m <= 512 else 256)
    assert steps["info"]["loop_sweeps"] == 0
    _same(got, steps, "steps")
    if _local_fits(m, n, cplx):
        # the same persistent sweeps spread over the device
        spread = _iterate(Ar, Ai, flags, local=False)
        assert spread["info"]["local_sweeps"] == 0 and spread["info"]["loop_sweeps"] == info["loop_sweeps"]
        _same(got, spread, "spread")


def test_loop_single_precision():
    Ar, Ai = _matrix(180, 150, True, 1e3, 5)
    ar, ai = Ar.astype(np.float32), Ai.astype(np.float32)
    out = []
    for wait in (None, 0.0):
        m, n = ar.shape
        st = J().State(m, n, True, fp32=True)
        if wait is not None:
            st.set_loop_wait(wait)
        st.load(J().to_device_fortran(ar, dtype=torch.float32), J().to_device_fortran(ai, dtype=torch.float32))
        st.iterate()
        q = st.query()
        r = st.finalize()
        torch.cuda.synchronize()
        st.close()
        r["info"] = q
        out.append(r)
    assert out[0]["info"]["loop_sweeps"] > 0 and out[1]["info"]["loop_sweeps"] == 0
    for k in ("U_re", "U_im", "V_re", "V_im", "sv_e", "sv_f"):
        assert np.array_equal(np.ascontiguousarray(out[0][k].cpu().numpy()).view(np.int32),
                              np.ascontiguousarray(out[1][k].cpu().numpy()).view(np.int32)), k


def test_loop_ruled_out_by_the_bound(ora):
    """Complex entries of equal magnitude in both parts: ||G||_F is sqrt(2 m n)
    times the largest component, and after the initial scaling the bound
    reaches the complex threshold, so every sweep runs step by step."""
    g = np.random.default_rng(11)
    m = n = 64
    Ar = 1.9 * g.choice([-1.0, 1.0], size=(m, n))
    Ai = 1.9 * g.choice([-1.0, 1.0], size=(m, n))
    got = _iterate(Ar, Ai)
    assert got["info"]["status"] == 0 and got["info"]["loop_sweeps"] == 0
    ro = ora.gesvj(Ar, Ai)
    assert ro["sweeps"] == got["info"]["sweeps"]
    for k in ("U_re", "U_im", "V_re", "V_im", "sv_e", "sv_f"):
        assert np.array_equal(_bits(got[k]), _bits(ro[k])), k


@pytest.mark.parametrize("m,n,cplx", [(200, 160, False), (200, 160, True), (600, 300, False), (800, 200, True)])
def test_loop_gives_up_and_is_redone(m, n, cplx):
    """A wait budget of a few microseconds: persistent sweeps give up through
    their bounded waits (forced from the host, every launch still exits)
    and are redone step by step from the copy taken before them (with
    256-thread workgroups beyond 256 rows: one outcome per workgroup)."""
    Ar, Ai = _matrix(m, n, cplx, 1e5, 40 + int(cplx) + m)
    got = _iterate(Ar, Ai, wait=1e-6)
    ref = _iterate(Ar, Ai, wait=0.0)
    assert ref["info"]["loop_sweeps"] == 0
    assert got["info"]["loop_redos"] > 0, got["info"]
    assert got["info"]["sweeps"] == ref["info"]["sweeps"]
    _same(got, ref, "redo")


@pytest.mark.parametrize("m,n,cplx", [(256, 256, False), (130, 97, True)])
def test_local_mode_gives_up_and_turns_off(m, n, cplx):
    """An L2-local sweep that gives up (a wait budget of a microsecond,
    forced from the host) is redone step by step and turns the mode off for
    the state: the later persistent sweeps are spread ones (which give up
    too, at that budget), and the bits are those of step-by-step sweeps.
    jsvd_state_set_loop_local(st, 1) turns it on again."""
    if not _local_fits(m, n, cplx):
        pytest.skip("the slots do not fit on one XCC of this device")
    Ar, Ai = _matrix(m, n, cplx, 1e5, 900 + m)
    got = _iterate(Ar, Ai, wait=1e-6)
    ref = _iterate(Ar, Ai, wait=0.0)
    assert got["info"]["loop_redos"] > 0 and got["info"]["local_sweeps"] == 0, got["info"]
    _same(got, ref, "local give-up")
    st = J().State(m, n, cplx)
    st.set_loop_wait(1e-6)
    st.load(J().to_device_fortran(Ar), J().to_device_fortran(Ai) if cplx else None)
    st.iterate()
    st.set_loop_wait(0.25)
    st.set_loop_local(True)
    st.load(J().to_device_fortran(Ar), J().to_device_fortran(Ai) if cplx else None)
    st.iterate()
    q = st.query()
    r = st.finalize()
    torch.cuda.synchronize()
    st.close()
    assert q["local_sweeps"] > 0 and q["loop_sweeps"] == q["sweeps"] + 1, q
    _same(r, ref, "local again")


def test_many_pairs_sweep_step_by_step(ora):
    """Beyond 192 pair slots the step-by-step sweep is the faster one: a
    600 x 400 state (200 slots) takes no persistent sweep and still gives the
    oracle's bits."""
    Ar, Ai = _matrix(600, 400, False, 1e4, 77)
    got = _iterate(Ar, Ai)
    assert got["info"]["status"] == 0 and got["info"]["loop_sweeps"] == 0
    ro = ora.gesvj(Ar, Ai)
    assert ro["sweeps"] == got["info"]["sweeps"]
    for k in ("U_re", "V_re", "sv_e", "sv_f"):
        assert np.array_equal(_bits(got[k]), _bits(ro[k])), k


def test_gesvj_uses_the_loop_and_matches(ora):
    """jsvd_gesvj on the 256 x 256 workload: bit for bit the oracle's SVD."""
    A, sig = inputs.plain_real_256()
    r = J().gesvj(J().to_device_fortran(A))
    torch.cuda.synchronize()
    ro = ora.gesvj(A)
    assert r["status"] == ro["status"] == 0 and r["sweeps"] == ro["sweeps"]
    for k in ("U_re", "V_re", "sv_e", "sv_f"):
        assert np.array_equal(_bits(r[k]), _bits(ro[k])), k
