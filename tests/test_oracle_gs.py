"""Pins of the Gram-Schmidt replacement in the oracle (Sect. 3.5.1, eqs.
(GScond) and (GS); Alg. zgsscl / dgsscl; the test matrix of Sect. SM9):

* the decision of eq. (GScond) equals the exact rational comparison of the
  norm quotient with 2^eta_hat upsilon, boundaries included (strict >);
* eq. (GS) per component within its rounding bound of the exact value, and
  the new column orthogonal to the kept one (the conjugate of a21' in the
  forward case, a21' itself in the reversed one);
* real = complex with a zero imaginary part, bit for bit;
* a step on a pair with an extreme norm ratio: the larger column unchanged
  and first, the smaller one orthogonalised, one transformation counted,
  forward and reversed orders giving the same G (real data);
* the matrix of Sect. SM9 (and its single precision counterpart): every
  singular value to a few eps relative (against a 420-digit SVD), a small
  residual, while without the replacement the iteration does not converge
  (the rotation's tan(phi) underflows and changes nothing).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2202_08361_amd import inputs

mpmath = pytest.importorskip("mpmath")
mp = mpmath.mp

EPS = 2.0 ** -53
EPS_F = 2.0 ** -24


def _exact_case(e1, f1, e2, f2, ups, eta_hat, div):
    thr = Fraction(ups) * Fraction(2) ** eta_hat

    def exceeds(ea, fa, eb, fb):
        return Fraction(div(fa, fb)) * Fraction(2) ** (int(ea) - int(eb)) > thr
    if exceeds(e1, f1, e2, f2):
        return 1
    if exceeds(e2, f2, e1, f1):
        return 2
    return 0


def _ups(m):
    return math.ldexp(math.sqrt(m), -53)


def _ups_f(m):
    return float(np.float32(np.ldexp(np.sqrt(np.float32(m)), -24)))


def test_gs_case_random_and_boundaries(ora):
    """eq. (GScond) on (e, f) norms: the oracle's (e, f) comparison equals the
    exact rational one, for random norms and for quotients exactly at,
    one ulp above and one ulp below the threshold."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 3000)
    div = lambda a, b: a / b
    for _ in range(4000):
        m = int(g.integers(1, 1 << 20))
        ups = _ups(m)
        e1, e2 = float(g.integers(-1100, 1100)), float(g.integers(-1100, 1100))
        f1, f2 = float(g.uniform(1, 2)), float(g.uniform(1, 2))
        assert ora.gs_case(e1, f1, e2, f2, ups) == _exact_case(e1, f1, e2, f2, ups, 1023, div)
    # near the threshold: e1 - e2 in {et - 1, et, et + 1}
    for _ in range(3000):
        m = int(g.integers(1, 1 << 20))
        ups = _ups(m)
        eu = math.frexp(ups)[1] - 1
        d = 1023 + eu + int(g.integers(-1, 2))
        e2 = float(g.integers(-1000, 0))
        f1, f2 = float(g.uniform(1, 2)), float(g.uniform(1, 2))
        for a, b in ((e2 + d, e2), (e2, e2 + d)):
            assert ora.gs_case(a, f1, b, f2, ups) == _exact_case(a, f1, b, f2, ups, 1023, div)
    # quotient exactly 2^eta_hat upsilon (f2 = 1): not beyond; one ulp more: beyond
    for m in (1, 2, 3, 16, 1000, 4096, 8191, 65537):
        ups = _ups(m)
        eu = math.frexp(ups)[1] - 1
        fu = math.ldexp(ups, -eu)
        et = 1023 + eu
        assert ora.gs_case(float(et), fu, 0.0, 1.0, ups) == 0
        assert ora.gs_case(float(et), math.nextafter(fu, 3.0), 0.0, 1.0, ups) == 1
        assert ora.gs_case(float(et), math.nextafter(fu, 0.0), 0.0, 1.0, ups) == 0
        assert ora.gs_case(0.0, 1.0, float(et), math.nextafter(fu, 3.0), ups) == 2
        assert ora.gs_case(-5.0, 1.0, float(et - 5), math.nextafter(fu, 3.0), ups) == 2


def test_s_gs_case_random(ora):
    """The single precision decision (eta_hat = FLT_MAX_EXP - 1 = 127) against
    the exact comparison of the float quotient."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 3001)
    div = lambda a, b: float(np.float32(a) / np.float32(b))
    for _ in range(4000):
        m = int(g.integers(1, 1 << 20))
        ups = _ups_f(m)
        eu = math.frexp(ups)[1] - 1
        e2 = float(g.integers(-150, 128))
        e1 = e2 + 127 + eu + int(g.integers(-2, 3)) if g.random() < 0.7 else float(g.integers(-150, 128))
        f1, f2 = float(np.float32(g.uniform(1, 2))), float(np.float32(g.uniform(1, 2)))
        want = _exact_case(e1, f1, e2, f2, ups, 127, div)
        assert ora.s_gs_case(np.float32(e1), np.float32(f1), np.float32(e2), np.float32(f2), np.float32(ups)) == want


def _pair(g, m, cplx, ratio_exp, cos_t, scale_exp=500):
    """Columns p (large) and q (small, 2^ratio_exp times smaller) with a
    prescribed angle: q = 2^-ratio_exp (cos_t p^ + sin_t r^) for a unit r^
    orthogonal to p^."""
    p = g.standard_normal(m) + (1j * g.standard_normal(m) if cplx else 0)
    r = g.standard_normal(m) + (1j * g.standard_normal(m) if cplx else 0)
    p = p / np.linalg.norm(p)
    r = r - np.vdot(p, r) * p
    r = r / np.linalg.norm(r)
    ph = np.exp(1j * g.uniform(0, 2 * np.pi)) if cplx else 1.0
    q = np.ldexp(1.0, -ratio_exp) * (cos_t * ph * p + math.sqrt(1 - cos_t ** 2) * r)
    sp = float(np.ldexp(1.0, scale_exp))
    P = p * sp
    Q = q * sp
    return P, Q


def _split(z, cplx):
    zr = np.ascontiguousarray(np.real(z), dtype=np.float64)
    zi = np.ascontiguousarray(np.imag(z), dtype=np.float64) if cplx else None
    return zr, zi


@pytest.mark.parametrize("cplx", [False, True])
def test_gs_formula_componentwise(ora, cplx):
    """eq. (GS) as ordered by Alg. zgsscl / dgsscl: every component within
    4 eps (|y_i| + |psi| 2^(ey-ex) |x_i|) of the exact y_i - psi 2^(ey-ex)
    x_i (psi = conj(a21') fl(fy/fx) exactly from the computed factors); the
    returned max-norm is the max |component| of the new column."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 3002 + int(cplx))
    mp.dps = 60
    for trial in range(60):
        m = int(g.integers(1, 700))
        P, Q = _pair(g, m, cplx, int(g.integers(0, 1000)), float(g.uniform(-0.9, 0.9)))
        xr, xi = _split(P, cplx)
        yr, yi = _split(Q, cplx)
        ex, fx = ora.colnorm(xr, xi)
        ey, fy = ora.colnorm(yr, yi)
        zr, zi = ora.dpscl(yr, yi, xr, xi, ey, fy, ex, fx)
        nyr, nyi = yr.copy(), (yi.copy() if cplx else None)
        M = ora.gs(xr, xi, nyr, nyi, ex, fx, ey, fy, zr, -zi)
        fyx = fy / fx
        psi = (mpmath.mpf(zr) - 1j * mpmath.mpf(zi)) * mpmath.mpf(fyx)
        sc = mpmath.mpf(2) ** (int(ey) - int(ex))
        mx = 0.0
        for i in range(m):
            xv = mpmath.mpc(xr[i], xi[i] if cplx else 0.0)
            yv = mpmath.mpc(yr[i], yi[i] if cplx else 0.0)
            ref = yv - psi * sc * xv
            got = mpmath.mpc(nyr[i], nyi[i] if cplx else 0.0)
            bound = 4 * EPS * (abs(yv) + abs(psi) * sc * abs(xv)) + 2.0 ** -1070
            assert abs(got - ref) <= bound, (trial, i)
            mx = max(mx, abs(nyr[i]), abs(nyi[i]) if cplx else 0.0)
        assert M == mx


@pytest.mark.parametrize("cplx", [False, True])
def test_gs_orthogonalises(ora, cplx):
    """The new column is orthogonal to the kept one to the accuracy of the
    computed a21': |p^* q''| / (||p|| ||q''||) <= 64 (ceil(m/1024) + 10) eps /
    sin(theta), in both orders (forward: conj(a21'), reversed: a21')."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 3004 + int(cplx))
    mp.dps = 40
    for trial in range(40):
        m = int(g.integers(2, 2500))
        cos_t = float(g.uniform(-0.9, 0.9))
        P, Q = _pair(g, m, cplx, int(g.integers(980, 1040)), cos_t)
        sin_t = math.sqrt(1 - cos_t ** 2)
        bound = 64 * (math.ceil(m / 1024) + 10) * EPS / sin_t
        xr, xi = _split(P, cplx)
        yr, yi = _split(Q, cplx)
        ex, fx = ora.colnorm(xr, xi)
        ey, fy = ora.colnorm(yr, yi)
        # forward: q is the second column (g_q), a21' = q^* p
        zr, zi = ora.dpscl(yr, yi, xr, xi, ey, fy, ex, fx)
        nyr, nyi = yr.copy(), (yi.copy() if cplx else None)
        ora.gs(xr, xi, nyr, nyi, ex, fx, ey, fy, zr, -zi)
        # reversed: the small column is g_p, a21' = (large)^* (small)
        zr2, zi2 = ora.dpscl(xr, xi, yr, yi, ex, fx, ey, fy)
        ryr, ryi = yr.copy(), (yi.copy() if cplx else None)
        ora.gs(xr, xi, ryr, ryi, ex, fx, ey, fy, zr2, zi2)
        pv = mpmath.matrix([mpmath.mpc(xr[i], xi[i] if cplx else 0) for i in range(m)])
        for ar, ai in ((nyr, nyi), (ryr, ryi)):
            qv = mpmath.matrix([mpmath.mpc(ar[i], ai[i] if cplx else 0) for i in range(m)])
            dot = sum(mpmath.conj(pv[i]) * qv[i] for i in range(m))
            rel = abs(dot) / (mpmath.norm(pv) * mpmath.norm(qv))
            assert rel <= bound, (trial, float(rel), bound)


def test_gs_real_equals_complex_zero_imag(ora):
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 3006)
    for _ in range(30):
        m = int(g.integers(1, 900))
        P, Q = _pair(g, m, False, int(g.integers(0, 1100)), float(g.uniform(-0.9, 0.9)))
        xr, _ = _split(P, False)
        yr, _ = _split(Q, False)
        ex, fx = ora.colnorm(xr, None)
        ey, fy = ora.colnorm(yr, None)
        zr, _ = ora.dpscl(yr, None, xr, None, ey, fy, ex, fx)
        a = yr.copy()
        Ma = ora.gs(xr, None, a, None, ex, fx, ey, fy, zr, 0.0)
        b, bi = yr.copy(), np.zeros(m)
        Mb = ora.gs(xr, np.zeros(m), b, bi, ex, fx, ey, fy, zr, -0.0)
        assert np.array_equal(a.view(np.int64), b.view(np.int64)) and Ma == Mb
        assert np.all(bi == 0.0)


def _two_columns(g, m, ratio_exp, cos_t):
    P, Q = _pair(g, m, False, ratio_exp, cos_t)
    return np.asfortranarray(np.stack([P.real, Q.real], axis=1))


def test_gs_step_forward_reversed(ora):
    """One step on a pair whose norms differ by 2^1000 > 2^eta_hat upsilon: one
    transformation, and it is the Gram-Schmidt step; the larger column is
    first and unchanged, the smaller one is orthogonal to it; putting the
    columns in the other order gives the same G bit for bit (real data),
    and V stays orthogonal, all with the sorting permutation.  Without it
    (the default) the reversed order keeps the smaller column first; with
    NO_GS the pair is rotated instead."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 3007)
    for trial in range(20):
        m = int(g.integers(2, 600))
        A = _two_columns(g, m, 1000, float(g.uniform(-0.9, 0.9)))
        B = np.asfortranarray(A[:, ::-1])
        sa = ora.State(A, permute=True)
        sb = ora.State(B, permute=True)
        assert sa.init() == ora.OK and sb.init() == ora.OK
        big = sa.Gr[:, 0].copy()
        assert sa.step() == 1 and sa.last_gs == 1
        assert sb.step() == 1 and sb.last_gs == 1
        assert np.array_equal(sa.Gr[:, 0], big)
        assert np.array_equal(sa.Gr.view(np.int64), sb.Gr.view(np.int64))
        a = sa.Gr[:, 0] / np.max(np.abs(sa.Gr[:, 0]))
        b = sa.Gr[:, 1] / np.max(np.abs(sa.Gr[:, 1]))
        assert abs(np.dot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b)) <= 1e-13
        for st in (sa, sb):
            assert np.linalg.norm(st.Vr.T @ st.Vr - np.eye(2)) <= 4 * EPS
        sn = ora.State(B)
        sn.init()
        small_before = sn.Gr[:, 0].copy()
        sn.step()
        assert sn.last_gs == 1 and np.array_equal(sn.Gr[:, 1], big) and not np.array_equal(sn.Gr[:, 0],
                                                                                           small_before)
        sr = ora.State(A, nogs=True)
        sr.init()
        assert sr.step() == 1 and sr.last_gs == 0


@pytest.mark.parametrize("single", [False, True])
def test_sm9_matrix(ora, single):
    """Sect. SM9 (16 x 16, upsilon = 2^-51; single precision: 2^-22 and
    eta_hat = 127): the replacement is taken (the paper saw it in most
    transformations of the first sweeps), the SVD converges with every
    singular value within 8 n eps of a 420-digit SVD and a residual
    ||G - U Sigma V^T||_F <= 64 n eps ||G||_F (the paper reports 1.1e-15);
    without it the iteration never stops: 128 sweeps and no convergence."""
    n = 16
    eps = EPS_F if single else EPS
    G = inputs.sm9_matrix(127, -22, dtype=np.float32)[0] if single else inputs.sm9_matrix(1023, -51)[0]
    run = ora.sgesvj if single else ora.gesvj
    St = ora.SState if single else ora.State
    st = St(G)
    assert st.init() == ora.OK
    t = gs = 0
    for _ in range(3 * ora.rr_steps(n)):
        t += st.step()
        gs += st.last_gs
    assert 0 < gs <= t
    r = run(G)
    assert r["status"] == ora.OK
    mp.dps = 420
    A = mpmath.matrix(G.astype(np.float64).tolist())
    sref = [mpmath.mpf(x) for x in mpmath.svd_r(A, compute_uv=False)]
    sig = [mpmath.ldexp(mpmath.mpf(float(f)), int(e)) for e, f in zip(r["sv_e"], r["sv_f"])]
    for a, b in zip(sig, sref):
        assert abs(a / b - 1) <= 8 * n * eps
    U = mpmath.matrix(r["U_re"].astype(np.float64).tolist())
    V = mpmath.matrix(r["V_re"].astype(np.float64).tolist())
    R = A - U * mpmath.diag(sig) * V.T
    assert mpmath.mnorm(R, "F") <= 64 * n * eps * mpmath.mnorm(A, "F")
    Ud = r["U_re"].astype(np.float64)
    Vd = r["V_re"].astype(np.float64)
    assert np.linalg.norm(Ud.T @ Ud - np.eye(n)) <= 4 * n * eps
    assert np.linalg.norm(Vd.T @ Vd - np.eye(n)) <= 8 * n * eps
    rn = run(G, max_sweeps=128, flags=ora.NO_GS)
    assert rn["status"] == ora.NOT_CONVERGED and rn["sweeps"] == 128


@pytest.mark.parametrize("single", [False, True])
def test_sm9_complex_equals_real(ora, single):
    """The SM9 matrix as complex data with zero imaginary parts takes the
    complex Gram-Schmidt path and gives the real results bit for bit."""
    G = inputs.sm9_matrix(127, -22, dtype=np.float32)[0] if single else inputs.sm9_matrix(1023, -51)[0]
    run = ora.sgesvj if single else ora.gesvj
    rr = run(G)
    rc = run(G, np.zeros_like(G))
    iv = np.int32 if single else np.int64
    for k in ("U_re", "V_re", "sv_e", "sv_f"):
        assert np.array_equal(rr[k].view(iv), rc[k].view(iv)), k
    assert np.all(rc["U_im"] == 0) and np.all(rc["V_im"] == 0)


@pytest.mark.parametrize("single", [False, True])
def test_gs_step_complex_orders(ora, single):
    """Complex pairs (random phases) with a norm ratio beyond 2^eta_hat
    upsilon (2^1000; single precision 2^120) in both column orders: one step
    takes the Gram-Schmidt step (a21' conjugated in the forward order, as it
    is in the reversed one), leaving the larger column first (with the
    sorting permutation) and unchanged, and the two columns orthogonal."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 3008 + int(single))
    mp.dps = 40
    eps = EPS_F if single else EPS
    dt = np.float32 if single else np.float64
    for trial in range(20):
        m = int(g.integers(2, 500))
        cos_t = float(g.uniform(-0.9, 0.9))
        P, Q = _pair(g, m, True, 120 if single else 1000, cos_t, 60 if single else 500)
        bound = 64 * (math.ceil(m / 1024) + 10) * eps / math.sqrt(1 - cos_t ** 2)
        for order in (0, 1):
            cols = (P, Q) if order == 0 else (Q, P)
            Ar = np.asfortranarray(np.stack([c.real for c in cols], axis=1).astype(dt))
            Ai = np.asfortranarray(np.stack([c.imag for c in cols], axis=1).astype(dt))
            st = ora.SState(Ar, Ai, permute=True) if single else ora.State(Ar, Ai, permute=True)
            assert st.init() == ora.OK
            big = (st.Gr[:, order].copy(), st.Gi[:, order].copy())
            assert st.step() == 1 and st.last_gs == 1
            assert np.array_equal(st.Gr[:, 0], big[0]) and np.array_equal(st.Gi[:, 0], big[1])
            a = [mpmath.mpc(float(st.Gr[i, 0]), float(st.Gi[i, 0])) for i in range(m)]
            b = [mpmath.mpc(float(st.Gr[i, 1]), float(st.Gi[i, 1])) for i in range(m)]
            dot = abs(sum(mpmath.conj(x) * y for x, y in zip(a, b)))
            na = mpmath.sqrt(sum(abs(x) ** 2 for x in a))
            nb = mpmath.sqrt(sum(abs(y) ** 2 for y in b))
            assert dot / (na * nb) <= bound, (trial, order)
