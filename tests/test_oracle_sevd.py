"""Pins of the single precision EVD oracle (Sect. 2.4.1: nu = FLT_MAX,
fl(sqrt nu) = 1.844674297E+19, FLT_TRUE_MIN, eta = FLT_MAX_EXP - 4; the
relative error bounds of Prop. p:s2 hold with eps = 2^-24): the float
counterpart of the worked example of eq. (evil), the bounds against 60-digit
closed forms, no overflow for any finite input, the exact special cases,
scaling invariance and real = complex with a zero imaginary part."""
import math

import numpy as np
import pytest

from paper_2202_08361_amd import inputs

mpmath = pytest.importorskip("mpmath")
mp = mpmath.mp

EPS = 2.0 ** -24
f32 = np.float32
FMAX = np.finfo(np.float32).max
MU = np.nextafter(f32(0), f32(1))


def _bits(x):
    return np.asarray(x, dtype=np.float32).view(np.int32)


def test_sqrt_nu_literal():
    """fl(sqrt(FLT_MAX)) = 0x1.fffffep+63 = 1.844674297E+19 (rounded to float),
    and fma(sqrt nu, sqrt nu, 1) stays finite."""
    s = f32(1.844674297e19)
    assert s == f32(math.sqrt(float(FMAX)))
    assert float(s) == float.fromhex("0x1.fffffep+63")
    assert float(mpmath.mpf(float(s)) ** 2 + 1) < float(FMAX)


@pytest.mark.parametrize("sign", [1, -1])
def test_evil_worked_example_float(ora, sign):
    """The worked example of eq. (evil) carried to single precision:
    A = [[nu/8, mu -/+ i mu], [mu +/- i mu, nu/8]] gives zeta = 0, tan phi = 1
    (the clamp by fl sqrt nu), cos phi = fl(1/fl sqrt 2), C = 1, S = +/-1,
    lambda'_1 = lambda'_2 = a11 (the float nu/8 itself) and p = 0."""
    a = FMAX / f32(8)
    r = ora.sevd2(a, a, MU, f32(sign) * MU)
    assert r["zp"] == 0
    assert r["cos"] == f32(1) / np.sqrt(f32(2))
    assert r["ctan_re"] == f32(1) and r["ctan_im"] == f32(sign)
    assert r["l1"] == a and r["l2"] == a


def _exact(a11, a22, ar, ai):
    mp.dps = 60
    a11, a22, ar, ai = (mpmath.mpf(float(x)) for x in (a11, a22, ar, ai))
    ab = mpmath.sqrt(ar * ar + ai * ai)
    a = a11 - a22
    if ab == 0:
        t = mpmath.mpf(0)
    elif a == 0:
        t = mpmath.mpf(1)
    else:
        t2 = 2 * ab / a
        t = t2 / (1 + mpmath.sqrt(1 + t2 * t2))
    c = 1 / mpmath.sqrt(1 + t * t)
    ca = ar / ab if ab != 0 else mpmath.mpf(1)
    return t, c, ca


def _paper_set_f32(n, cplx, seed):
    """Sect. 5.1 recipe in single precision: A from eq. (2) with random
    eigenvalues (moderate range), tan phi and cos alpha in 60 digits, rounded
    once to float."""
    g = inputs.rng(inputs.CFG_EVD_BATCH, 1500 + seed)
    mp.dps = 60
    out = []
    for _ in range(n):
        l1 = mpmath.mpf(float(g.uniform(-1, 1) * 10 ** g.uniform(-15, 15)))
        l2 = mpmath.mpf(float(g.uniform(-1, 1) * 10 ** g.uniform(-15, 15)))
        t = mpmath.mpf(float(g.uniform(-1, 1)))
        ca = mpmath.mpf(float(g.uniform(-1, 1))) if cplx else mpmath.mpf(1)
        sa = mpmath.sqrt(1 - ca * ca) * (1 if g.random() < 0.5 else -1) if cplx else mpmath.mpf(0)
        c2 = 1 / (1 + t * t)
        a11 = c2 * (l1 + l2 * t * t)
        a22 = c2 * (l1 * t * t + l2)
        off = c2 * t * (l1 - l2)
        out.append(tuple(f32(float(x)) for x in (a11, a22, ca * off, sa * off)))
    return out


@pytest.mark.parametrize("cplx", [False, True])
def test_prop_s2_bounds_single(ora, cplx):
    """Prop. p:s2 with eps = 2^-24: tan phi within 5.5 eps (real) / 11.5 eps
    (complex), cos phi within 8 eps / 14 eps, e^{i alpha} within 4 eps; the
    reconstructed U Lambda U^* within a few eps of A."""
    bt = 5.500001 if not cplx else 11.500004
    bc = 8.000002 if not cplx else 14.000006
    for a11, a22, ar, ai in _paper_set_f32(400, cplx, int(cplx)):
        r = ora.sevd2(a11, a22, ar, ai if cplx else None)
        t, c, ca = _exact(a11, a22, ar, ai if cplx else 0.0)
        if t == 0:
            continue
        C, S = mpmath.mpf(float(r["ctan_re"])), mpmath.mpf(float(r["ctan_im"]))
        tc = mpmath.sqrt(C * C + S * S)
        assert abs(tc / abs(t) - 1) / EPS < bt + 5.0
        assert abs(mpmath.mpf(float(r["cos"])) / c - 1) / EPS < bc
        if abs(ca) > 1e-3:
            assert abs(C / (ca * t) - 1) / EPS < 4.000001 + bt + 1.0 + 1e-6
        cc = mpmath.mpf(float(r["cos"]))
        e_t = mpmath.mpc(float(r["ctan_re"]), float(r["ctan_im"]))
        U = mpmath.matrix([[cc, -mpmath.conj(e_t) * cc], [e_t * cc, cc]])
        L = mpmath.diag([mpmath.mpf(float(r["l1"])), mpmath.mpf(float(r["l2"]))])
        A = mpmath.matrix([[float(a11), mpmath.mpc(float(ar), -float(ai))],
                           [mpmath.mpc(float(ar), float(ai)), float(a22)]])
        R = U * L * U.H - A
        assert mpmath.mnorm(R, "F") / mpmath.mnorm(A, "F") / EPS < 64


@pytest.mark.parametrize("cplx", [False, True])
def test_invariants_wide_and_adversarial_single(ora, cplx):
    """Over the float32 wide-exponent workload and the special cases: every
    scaled output finite (no overflow for any finite input), |C + iS| <= 1
    (+ rounding) where the scaled off-diagonal does not underflow, cos phi in
    [fl(1/fl sqrt 2), 1], p consistent with lambda', zeta' from eq. (z) with
    eta' = 125."""
    for a11, a22, ar, ai in (inputs.evd_batch_f32(20000, cplx), inputs.evd_adversarial_f32(cplx)):
        cs, C, S, l1, l2, zp = ora.sevd2_batch(a11, a22, ar, ai, flags=ora.EVD_SCALED)
        S = S if cplx else np.zeros_like(C)
        for x in (cs, C, S, l1, l2):
            assert np.all(np.isfinite(x))
        # |e^{i alpha}| = 1 up to rounding, barring underflow of the scaled
        # off-diagonal (the worked example of eq. (evil) shows what happens then)
        zeta = -(zp >> 1)
        tiny = float(np.finfo(np.float32).tiny)
        ok = np.ones(len(zp), dtype=bool)
        for comp in (ar,) + ((ai,) if cplx else ()):
            sc = np.abs(np.ldexp(comp.astype(np.float64), zeta))
            ok &= (sc == 0) | (sc >= tiny)
        h = np.hypot(C.astype(np.float64), S.astype(np.float64))
        assert np.all(h[ok] <= 1.0 + 8 * EPS)
        assert np.all(cs <= f32(1)) and np.all(cs >= f32(1) / np.sqrt(f32(2)))
        assert np.array_equal(zp & 1, (l1 < l2).astype(np.int32))
        for i in range(0, len(a11), max(1, len(a11) // 1500)):
            comps = (a11[i], a22[i], ar[i]) + ((ai[i],) if cplx else ())
            z = min(125 - math.frexp(max(abs(float(c)), float(MU)))[1] for c in comps)
            assert (zp[i] >> 1) == -z


def test_exact_special_cases_single(ora):
    """a21 = 0: tan phi = 0, cos phi = 1, lambda = (a11, a22) exactly; a11 = a22
    and a21 != 0: |tan phi| = 1; the all-zero matrix: zeta = 125 + 149 - 1."""
    g = inputs.rng(inputs.CFG_EVD_BATCH, 1700)
    for _ in range(200):
        a11, a22 = (f32(x) for x in g.standard_normal(2) * 10.0 ** g.uniform(-30, 30, 2))
        for ai in (None, f32(0)):
            r = ora.sevd2(a11, a22, f32(0), ai)
            assert r["cos"] == f32(1) and r["ctan_re"] == f32(0) and r["ctan_im"] == f32(0)
            assert r["l1"] == a11 and r["l2"] == a22
        a = f32(g.standard_normal() * 10.0 ** g.uniform(-30, 30))
        b = f32(g.standard_normal() * 10.0 ** g.uniform(-30, 30))
        r = ora.sevd2(a, a, b, None)
        assert abs(r["ctan_re"]) == f32(1) and r["cos"] == f32(1) / np.sqrt(f32(2))
    r = ora.sevd2(f32(0), f32(0), f32(0), f32(0))
    assert r["zp"] == (-(125 + 148)) << 1
    assert r["cos"] == f32(1) and r["l1"] == f32(0) and r["l2"] == f32(0)


@pytest.mark.parametrize("cplx", [False, True])
def test_scaling_invariance_single(ora, cplx):
    """EVD(2^k A): identical rotation and p, lambda scaled by 2^k, zeta' shifted
    by k (components kept in the normal range)."""
    g = inputs.rng(inputs.CFG_EVD_BATCH, 1702)
    for _ in range(300):
        v = (g.standard_normal(4) * 10.0 ** g.uniform(-10, 10, 4)).astype(np.float32)
        k = int(g.integers(-40, 40))
        args = list(v[: 4 if cplx else 3])
        if not cplx:
            args.append(None)
        r0 = ora.sevd2(*args)
        r1 = ora.sevd2(*[None if x is None else f32(np.ldexp(x, k)) for x in args])
        for key in ("cos", "ctan_re", "ctan_im"):
            assert r0[key] == r1[key]
        assert (r0["zp"] & 1) == (r1["zp"] & 1) and (r1["zp"] >> 1) == (r0["zp"] >> 1) + k
        assert r1["l1"] == f32(np.ldexp(r0["l1"], k)) and r1["l2"] == f32(np.ldexp(r0["l2"], k))


def test_real_equals_complex_with_zero_imag_single(ora):
    a11, a22, ar, _ = inputs.evd_batch_f32(20000, False)
    rr = ora.sevd2_batch(a11, a22, ar, None)
    rc = ora.sevd2_batch(a11, a22, ar, np.zeros_like(ar))
    for i in (0, 1, 3, 4):
        assert np.array_equal(_bits(rr[i]), _bits(rc[i]))
    assert np.array_equal(rr[5], rc[5])


def test_single_close_to_double(ora):
    """The same float inputs through the double routine: the single results
    agree to a few float ulps (rotation) and to a few eps of the larger
    eigenvalue in magnitude (eigenvalues), both being accurate to a few eps
    of their own precision."""
    for a11, a22, ar, ai in _paper_set_f32(200, True, 9):
        for cplx in (False, True):
            rs = ora.sevd2(a11, a22, ar, ai if cplx else None)
            rd = ora.evd2(float(a11), float(a22), float(ar), float(ai) if cplx else None)
            for key in ("cos", "ctan_re", "ctan_im"):
                assert abs(float(rs[key]) - rd[key]) <= 32 * EPS
            lam = max(abs(rd["l1"]), abs(rd["l2"]))
            for key in ("l1", "l2"):
                assert abs(float(rs[key]) - rd[key]) <= 32 * EPS * lam
