"""Pins of the single precision SVD oracle (Sect. SM8: the same method over
the float range; nu = FLT_MAX, eps = 2^-24): exact integer scaling
exponents, the (e, f) norm examples and norms against 60-digit values, the
scaled dot-product within its error bound, the rotation lemmas with the
float epsilon, and whole SVDs against the prescribed singular values, the
singular values of the rounded matrix, orthogonality and the residual;
bitwise scaling invariance and real = complex with a zero imaginary part."""
import math

import numpy as np
import pytest

from paper_2202_08361_amd import inputs

mpmath = pytest.importorskip("mpmath")
mp = mpmath.mp

EPS = 2.0 ** -24
f32 = np.float32
FLT_MAX_INT = int(2 ** 128 - 2 ** 104)


def _floor_lg(x):
    return math.frexp(float(x))[1] - 1


def _lg_bound_exact(m, cplx):
    """floor(lg(nu / (varsigma m))) with nu = FLT_MAX as exact integers."""
    for k in range(200, -200, -1):
        if not cplx:
            if 2 ** k * 2 * m <= FLT_MAX_INT if k >= 0 else 2 * m <= FLT_MAX_INT * 2 ** (-k):
                return k
        else:
            lhs = (2 ** k * 4 * m) ** 2 * 2 if k >= 0 else (4 * m) ** 2 * 2
            rhs = FLT_MAX_INT ** 2 if k >= 0 else FLT_MAX_INT ** 2 * 4 ** (-k)
            if lhs <= rhs:
                return k
    raise AssertionError


@pytest.mark.parametrize("cplx", [False, True])
def test_s_lg_bound_exact(ora, cplx):
    ms = list(range(1, 1200)) + [2 ** k + d for k in range(11, 30) for d in (-1, 0, 1)] + [3037000499]
    for m in [m for m in ms if m < 2 ** 31]:
        assert ora.s_lg_bound_m(m, cplx) == _lg_bound_exact(m, cplx), m


@pytest.mark.parametrize("cplx", [False, True])
def test_s_scaling_exponents(ora, cplx):
    """s_(k) = floor(lg(nu/2)) - floor(lg M~) (real), floor(lg(nu/(4 sqrt 2)))
    - floor(lg M~) - 1 (complex); s_[k] keeps 2^s M~ <= nu/(varsigma m)."""
    g = inputs.rng(inputs.CFG_PLAIN_REAL_256, 1090)
    mp.dps = 50
    for _ in range(500):
        Mt = f32(g.uniform(1, 2) * 2.0 ** int(g.integers(-149, 127)))
        if Mt == 0 or not np.isfinite(Mt):
            continue
        m = int(g.integers(1, 100000))
        sr = ora.s_s_round(Mt, cplx)
        sq = ora.s_s_square(Mt, m, cplx)
        assert sr == (124 if cplx else 126) - _floor_lg(Mt)
        assert sq == _lg_bound_exact(m, cplx) - _floor_lg(Mt) - 1
        vs = mpmath.mpf(2) if not cplx else 4 * mpmath.sqrt(2)
        assert mpmath.mpf(float(Mt)) * mpmath.mpf(2) ** sq <= mpmath.mpf(FLT_MAX_INT) / (vs * m)
        assert mpmath.mpf(float(Mt)) * mpmath.mpf(2) ** sr <= mpmath.mpf(FLT_MAX_INT) / vs


def test_s_ef_examples(ora):
    """Sect. SM6.1 examples in float: 12 = (3, 1.5), 80 = (6, 1.25), and the
    norms of [sqrt 12]-like columns (2, 2, 2) -> (1, fl sqrt 3)."""
    assert ora.s_colnorm(np.array([12.0], dtype=np.float32)) == (f32(3), f32(1.5))
    assert ora.s_colnorm(np.array([80.0], dtype=np.float32)) == (f32(6), f32(1.25))
    e, f = ora.s_colnorm(np.array([2.0, 2.0, 2.0], dtype=np.float32))     # sqrt 12
    assert e == 1 and f == np.sqrt(f32(3))
    e, f = ora.s_colnorm(np.array([8.0, 4.0], dtype=np.float32))          # sqrt 80
    assert e == 3 and f == np.sqrt(f32(1.25))


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("m", [1, 7, 300, 1024, 1500, 5000])
def test_s_colnorm_vs_exact(ora, cplx, m):
    g = inputs.rng(inputs.CFG_PLAIN_REAL_256, 1092 + m)
    mp.dps = 40
    for scale in (1.0, 2.0 ** 100, 2.0 ** -100):
        xr = (g.uniform(-1, 1, m) * scale).astype(np.float32)
        xi = (g.uniform(-1, 1, m) * scale).astype(np.float32) if cplx else None
        e, f = ora.s_colnorm(xr, xi)
        assert 1.0 <= f < 2.0
        s = mpmath.fsum(mpmath.mpf(float(v)) ** 2 for v in xr)
        if cplx:
            s += mpmath.fsum(mpmath.mpf(float(v)) ** 2 for v in xi)
        ex = mpmath.sqrt(s)
        got = mpmath.mpf(float(f)) * mpmath.mpf(2) ** int(e)
        assert abs(got / ex - 1) <= (math.ceil(m / 1024) + 10 + 8) * EPS


@pytest.mark.parametrize("cplx", [False, True])
def test_s_dpscl_vs_exact(ora, cplx):
    g = inputs.rng(inputs.CFG_PLAIN_REAL_256, 1093)
    mp.dps = 40
    for m in (3, 200, 2500):
        qr = (g.standard_normal(m) * 1e20).astype(np.float32)
        pr = (g.standard_normal(m) * 1e-20).astype(np.float32)
        qi = (g.standard_normal(m) * 1e20).astype(np.float32) if cplx else None
        pi = (g.standard_normal(m) * 1e-20).astype(np.float32) if cplx else None
        eq, fq = ora.s_colnorm(qr, qi)
        ep, fp = ora.s_colnorm(pr, pi)
        zr, zi = ora.s_dpscl(qr, qi, pr, pi, eq, fq, ep, fp)
        Q = [mpmath.mpc(float(a), float(b)) for a, b in zip(qr, qi if cplx else np.zeros(m))]
        P = [mpmath.mpc(float(a), float(b)) for a, b in zip(pr, pi if cplx else np.zeros(m))]
        nq = mpmath.sqrt(mpmath.fsum(abs(v) ** 2 for v in Q))
        npp = mpmath.sqrt(mpmath.fsum(abs(v) ** 2 for v in P))
        ex = mpmath.fsum(mpmath.conj(a) * b for a, b in zip(Q, P)) / (nq * npp)
        absum = mpmath.fsum(abs(a) * abs(b) for a, b in zip(Q, P)) / (nq * npp)
        k = math.ceil(m / 1024) + 10 + 2 * (1 if cplx else 0) + 4
        err = abs(mpmath.mpc(float(zr), float(zi)) - ex)
        # the norms' own rounding enters through the division (a few eps of |a21'|)
        assert err <= k * EPS * absum + 2 * (math.ceil(m / 1024) + 18) * EPS * abs(ex)


def test_s_rotation_lemmas(ora):
    """Lemma l:rt in float: each element of the real rotation within (1 +- eps)^2
    of the exact product with the computed parameters; Lemma l:ct: complex
    elements within 5.656856 eps where the lemma's condition holds."""
    g = inputs.rng(inputs.CFG_PLAIN_REAL_256, 1095)
    mp.dps = 40
    l = 400
    xp, xq = (g.standard_normal(l).astype(np.float32) for _ in range(2))
    T = f32(g.uniform(-1, 1))
    c = f32(1) / np.sqrt(T * T + f32(1))
    yp, yq = xp.copy(), xq.copy()
    lib = ora.lib()
    lib.ora_s_rot(l, ora._pf(yp), None, ora._pf(yq), None, c, T, 0.0, 0)
    lo, hi = (1 - mpmath.mpf(EPS)) ** 2, (1 + mpmath.mpf(EPS)) ** 2
    for i in range(l):
        wp = (mpmath.mpf(float(xp[i])) + mpmath.mpf(float(xq[i])) * float(T)) * float(c)
        wq = (mpmath.mpf(float(xq[i])) - mpmath.mpf(float(xp[i])) * float(T)) * float(c)
        for got, want in ((yp[i], wp), (yq[i], wq)):
            if want != 0:
                assert lo <= mpmath.mpf(float(got)) / want <= hi
    xpr, xpi, xqr, xqi = (g.standard_normal(l).astype(np.float32) for _ in range(4))
    C, S = (f32(v) for v in g.uniform(-0.7, 0.7, 2))
    c = f32(1) / np.sqrt(C * C + S * S + f32(1))
    ypr, ypi, yqr, yqi = xpr.copy(), xpi.copy(), xqr.copy(), xqi.copy()
    lib.ora_s_rot(l, ora._pf(ypr), ora._pf(ypi), ora._pf(yqr), ora._pf(yqi), c, C, S, 0)
    e = mpmath.mpc(float(C), float(S))
    checked = 0
    for i in range(l):
        gp = mpmath.mpc(float(xpr[i]), float(xpi[i]))
        gq = mpmath.mpc(float(xqr[i]), float(xqi[i]))
        np_ = (gp + gq * e) * float(c)
        nq = (gq - gp * mpmath.conj(e)) * float(c)
        if abs(np_) / float(c) >= abs(float(xqr[i])):
            assert abs(mpmath.mpc(float(ypr[i]), float(ypi[i])) - np_) / abs(np_) <= 5.656856 * EPS
            checked += 1
        if abs(nq) / float(c) >= abs(float(xpr[i])):
            assert abs(mpmath.mpc(float(yqr[i]), float(yqi[i])) - nq) / abs(nq) <= 5.656856 * EPS
            checked += 1
    assert checked > l // 2


def _sv(res):
    return np.ldexp(res["sv_f"].astype(np.float64), res["sv_e"].astype(int))


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("flags", [0, 8])
def test_s_gesvj_accuracy(ora, cplx, flags):
    """Haar factors, kappa = 1e3, rounded once to float: the singular values
    within 32 eps kappa of those of the rounded matrix (computed in double),
    and of the prescribed ones; residual <= 64 n eps ||A||_F; U and V
    orthonormal to the accuracy the convergence test and the accumulated
    rotations allow."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 1106 + int(cplx))
    m, n = 96, 64
    sig = inputs.sigma_logspace(n, 1e-3)
    Ar, Ai = inputs.svd_matrix(m, n, sig, g, cplx=cplx)
    Ar32 = Ar.astype(np.float32)
    Ai32 = Ai.astype(np.float32) if cplx else None
    res = ora.sgesvj(Ar32, Ai32, flags=flags)
    assert res["status"] == ora.OK
    sv = _sv(res)
    A = Ar32.astype(np.float64) + (1j * Ai32.astype(np.float64) if cplx else 0)
    sref = np.linalg.svd(A, compute_uv=False)
    kappa = sref[0] / sref[-1]
    assert np.max(np.abs(sv - sref) / sref) <= 32 * EPS * kappa
    assert np.max(np.abs(sv - sig) / sig) <= 64 * EPS * kappa
    U = res["U_re"].astype(np.float64) + (1j * res["U_im"].astype(np.float64) if cplx else 0)
    V = res["V_re"].astype(np.float64) + (1j * res["V_im"].astype(np.float64) if cplx else 0)
    assert np.linalg.norm(A - (U * sv[None, :]) @ V.conj().T) / np.linalg.norm(A) <= 64 * n * EPS
    # U: each converged pair is orthogonal to within upsilon = sqrt(m) eps plus the
    # dot-product error; V: O(eps) per rotation, accumulated over sweeps * n of them
    assert np.linalg.norm(U.conj().T @ U - np.eye(n)) <= n * (math.sqrt(m) + 4) * EPS
    assert np.linalg.norm(V.conj().T @ V - np.eye(n)) <= 4 * n * math.sqrt(res["sweeps"] * n) * EPS


@pytest.mark.parametrize("cplx", [False, True])
def test_s_scaling_invariance(ora, cplx):
    """SVD(2^k A) in float: bitwise identical U, V, f and sweeps, e shifted by k."""
    g = inputs.rng(inputs.CFG_PLAIN_REAL_256, 1103)
    Ar, Ai = inputs.random_columns(30, 12, g, cplx)
    Ar, Ai = Ar.astype(np.float32), (Ai.astype(np.float32) if cplx else None)
    r0 = ora.sgesvj(Ar, Ai)
    for k in (-60, -7, 9, 50):
        r1 = ora.sgesvj(np.ldexp(Ar, k).astype(np.float32), None if Ai is None else np.ldexp(Ai, k).astype(np.float32))
        assert r1["sweeps"] == r0["sweeps"]
        for key in ("U_re", "V_re", "sv_f") + (("U_im", "V_im") if cplx else ()):
            assert np.array_equal(r1[key], r0[key]), (k, key)
        assert np.array_equal(r1["sv_e"], r0["sv_e"] + k)


def test_s_complex_path_on_real_input(ora):
    g = inputs.rng(inputs.CFG_PLAIN_REAL_256, 1104)
    Ar, _ = inputs.random_columns(25, 11, g)
    Ar = Ar.astype(np.float32)
    rr = ora.sgesvj(Ar)
    rc = ora.sgesvj(Ar, np.zeros_like(Ar))
    assert rr["sweeps"] == rc["sweeps"]
    assert np.array_equal(rr["sv_f"], rc["sv_f"]) and np.array_equal(rr["sv_e"], rc["sv_e"])
    assert np.all(rr["U_re"] == rc["U_re"]) and np.all(rc["U_im"] == 0)


def test_s_failure_modes(ora):
    A = np.ones((4, 3), dtype=np.float32, order="F")
    A[1, 1] = np.nan
    assert ora.sgesvj(A)["status"] == ora.ENONFINITE
    assert ora.sgesvj(np.zeros((4, 3), dtype=np.float32))["status"] == ora.EZERO
    g = inputs.rng(inputs.CFG_PLAIN_REAL_256, 1105)
    Ar, _ = inputs.random_columns(20, 10, g)
    r = ora.sgesvj(Ar.astype(np.float32), max_sweeps=1)
    assert r["status"] == ora.NOT_CONVERGED and r["sweeps"] == 1
