"""Pins of the widened-exponent Frobenius norm (Sect. SM6, Alg. rnF) in the
oracle:

* the worked examples of Sect. SM6.1 (tests/golden/ef_examples.txt), for the
  norm and its square, for several lane counts;
* where no square or partial sum leaves the double range, every lane's
  partial sum equals the plain fma accumulation x x + r of Alg. vdp, and the
  result equals those plain sums sorted and added pairwise in ordinary
  double arithmetic, then one sqrt (the paper: the two methods agree there);
* beyond that range the result stays finite (nu 1 of length m: nu sqrt m) or
  non-zero (subnormal data) and accurate against 400-digit references, where
  plain double arithmetic overflows or underflows;
* the random-bit test vectors of Sect. SM6.4 (elements in [0, 2^xi],
  xi in {0, 1008}) within the summation bound;
* zero arrays, and complex data with a zero imaginary part = real data.
"""
import math
import os

import numpy as np
import pytest

from paper_2202_08361_amd import inputs

mpmath = pytest.importorskip("mpmath")
mp = mpmath.mp

EPS = 2.0 ** -53
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
LANES = (1, 2, 8, 64, 1024)


def _val(e, f):
    return mpmath.ldexp(mpmath.mpf(f), int(e)) if e != -math.inf else mpmath.mpf(0)


def test_sm61_examples(ora):
    """12 = (3, 1.5), sqrt(12) = (1, fl(sqrt 3)); 80 = (6, 1.25), sqrt(80) =
    (3, fl(sqrt 1.25)), whatever the lane count."""
    rows = []
    for line in open(os.path.join(GOLD, "ef_examples.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        xs, rhs = line.split("|")
        x = np.array([float(v) for v in xs.split(",")])
        e, fexpr = rhs.split()
        rows.append((x, int(e), eval(fexpr, {"sqrt": math.sqrt})))
    assert len(rows) >= 4
    for x, e, f in rows:
        sq = float(np.sum(x * x))
        e2 = math.frexp(sq)[1] - 1
        for s in LANES:
            r = ora.nrmf(x, lanes=s)
            assert (r["e"], r["f"]) == (e, f), (x, s, r)
            assert (r["e2"], r["f2"]) == (e2, math.ldexp(sq, -e2)), (x, s, r)


def _fma_exact(a, b, c):
    """fl(a b + c), correctly rounded (mpmath at 2200 bits, then one rounding)."""
    with mpmath.workprec(2200):
        return float(mpmath.mpf(a) * mpmath.mpf(b) + mpmath.mpf(c))


def _plain_lanes_exact(xr, xi, s):
    acc = [0.0] * s
    for i in range(len(xr)):
        L = i % s
        acc[L] = _fma_exact(xr[i], xr[i], acc[L])
        if xi is not None:
            acc[L] = _fma_exact(xi[i], xi[i], acc[L])
    return acc


def _moderate(g, m, cplx):
    xr = g.standard_normal(m) * np.ldexp(1.0, g.integers(-150, 150, m))
    xi = g.standard_normal(m) * np.ldexp(1.0, g.integers(-150, 150, m)) if cplx else None
    return xr, xi


@pytest.mark.parametrize("cplx", [False, True])
def test_lanes_equal_plain_fma(ora, cplx):
    """In the double range the widened-exponent lane update is the plain fma
    x x + r: lane by lane, the same value (Alg. vdp)."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 5000 + int(cplx))
    for trial in range(12):
        m = int(g.integers(1, 400))
        s = int(2 ** g.integers(0, 7))
        xr, xi = _moderate(g, m, cplx)
        le, lf = ora.nrmf_lanes(xr, xi, lanes=s)
        want = _plain_lanes_exact(xr, xi, s)
        for L in range(s):
            got = 0.0 if le[L] == -np.inf else math.ldexp(lf[L], int(le[L]))
            assert got == want[L], (trial, L, got, want[L])


@pytest.mark.parametrize("cplx", [False, True])
def test_result_equals_sorted_pairwise_plain(ora, cplx):
    """In the double range: ||x||^2 equals the plain lane sums sorted
    non-decreasingly and added pairwise (lane 2i + lane 2i+1 per level) in
    double arithmetic, and ||x|| is fl(sqrt) of it."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 5002 + int(cplx))
    for trial in range(12):
        m = int(g.integers(1, 300))
        s = int(2 ** g.integers(0, 7))
        xr, xi = _moderate(g, m, cplx)
        a = sorted(_plain_lanes_exact(xr, xi, s))
        while len(a) > 1:
            a = [a[2 * i] + a[2 * i + 1] for i in range(len(a) // 2)]
        tot = a[0]
        r = ora.nrmf(xr, xi, lanes=s)
        assert math.ldexp(r["f2"], int(r["e2"])) == tot
        nrm = math.sqrt(tot)
        assert math.ldexp(r["f"], int(r["e"])) == nrm
        assert 1.0 <= r["f"] < 2.0 and 1.0 <= r["f2"] < 2.0


def test_no_overflow_nu_ones(ora):
    """x = nu 1 of length m (Sect. SM6.1): ||x|| = nu sqrt(m) is not a double,
    yet (e, f) is finite and within the summation bound of the exact value."""
    nu = np.finfo(np.float64).max
    mp.dps = 60
    for m in (2, 3, 7, 100, 1024, 1025, 5000):
        for s in (1, 8, 1024):
            r = ora.nrmf(np.full(m, nu), lanes=s)
            assert np.isfinite(r["e"]) and np.isfinite(r["f"]) and r["e"] >= 1024
            exact = mpmath.mpf(nu) * mpmath.sqrt(m)
            rel = abs(_val(r["e"], r["f"]) / exact - 1)
            assert rel <= (math.ceil(m / s) + math.log2(s) + 3) * EPS, (m, s, float(rel))


def test_no_underflow_subnormals(ora):
    """Subnormal data: the plain sum of squares underflows to zero, the
    widened exponent keeps the norm accurate."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 5004)
    mp.dps = 60
    for trial in range(20):
        m = int(g.integers(1, 3000))
        k = g.integers(1, 1 << 40, m).astype(np.float64)
        x = np.ldexp(k, -1074) * np.where(g.random(m) < 0.5, -1.0, 1.0)
        assert float(np.sum(x * x)) == 0.0
        for s in (8, 1024):
            r = ora.nrmf(x, lanes=s)
            exact = mpmath.sqrt(mpmath.fsum(mpmath.mpf(v) ** 2 for v in x))
            rel = abs(_val(r["e"], r["f"]) / exact - 1)
            assert rel <= (math.ceil(m / s) + math.log2(s) + 3) * EPS, (trial, s, float(rel))


@pytest.mark.parametrize("xi", [0, 1008])
def test_sm64_vectors(ora, xi):
    """The random-bit vectors of Sect. SM6.4: relative error of ||x|| within
    (ceil(m/s) + lg s + 3) eps of a 400-digit value, s = 8 (the paper's AVX-512
    lanes) and 1024; at xi = 1008 the plain sum of squares overflows."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 5006 + xi)
    for trial in range(6):
        m = int(g.integers(1000, 20000))
        x = inputs.random_bit_vector(g, m, xi)
        with mpmath.workprec(2400):
            exact = mpmath.sqrt(mpmath.fsum(mpmath.mpf(v) ** 2 for v in sorted(x)))
        if xi == 1008:
            with np.errstate(over="ignore"):
                assert not np.isfinite(np.sum(x * x))
        for s in (8, 1024):
            r = ora.nrmf(x, lanes=s)
            with mpmath.workprec(2400):
                rel = abs(_val(r["e"], r["f"]) / exact - 1)
            assert rel <= (math.ceil(m / s) + math.log2(s) + 3) * EPS, (trial, s, float(rel))


def test_zero_and_empty(ora):
    for m in (0, 1, 5, 2000):
        for s in (1, 8, 1024):
            r = ora.nrmf(np.zeros(m), lanes=s)
            assert r == dict(e2=-np.inf, f2=1.0, e=-np.inf, f=1.0)
            r = ora.nrmf(np.zeros(m), np.zeros(m), lanes=s)
            assert r == dict(e2=-np.inf, f2=1.0, e=-np.inf, f=1.0)


def test_complex_zero_imag_equals_real(ora):
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 5008)
    for trial in range(20):
        m = int(g.integers(1, 3000))
        x = g.standard_normal(m) * np.ldexp(1.0, g.integers(-1070, 1020, m))
        for s in (1, 8, 1024):
            assert ora.nrmf(x, lanes=s) == ora.nrmf(x, np.zeros(m), lanes=s)
