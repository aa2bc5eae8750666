"""Pins of the oracle's compensated scaled dot-product (Sect. SM2.2,
Alg. zdpsclcs / ddpsclcs) against what the mathematics fixes: the
rounded-down product against the exact binary product, 2Sum's exactness,
the accuracy a compensated sum must reach on ill-conditioned dot-products
(where the plain sum demonstrably fails), and agreement with the plain
routine when every sum is exact."""
import math

import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")

EPS = 2.0 ** -53
TRUE_MIN = 5e-324


def exact_product_rd(a, b):
    """The largest double <= a*b, from the exact product in 2300-bit arithmetic."""
    with mpmath.workprec(2300):
        x = mpmath.mpf(a) * mpmath.mpf(b)
        if x == 0:
            return None
        c = float(x)                        # rounded to nearest
        if mpmath.mpf(c) > x:
            c = math.nextafter(c, -math.inf)
        return c


def _bits(x):
    return np.float64(x).view(np.int64)


def test_mul_rd_random_and_edges(ora):
    rng = np.random.default_rng(20220208)
    cases = []
    for _ in range(3000):
        cases.append((rng.standard_normal() * 2.0 ** rng.integers(-60, 60),
                      rng.standard_normal() * 2.0 ** rng.integers(-60, 60)))
    # products rounding into and below the subnormal range, both signs
    for _ in range(2000):
        a = rng.uniform(1, 2) * 2.0 ** rng.integers(-700, -400) * rng.choice([-1, 1])
        b = rng.uniform(1, 2) * 2.0 ** rng.integers(-700, -300) * rng.choice([-1, 1])
        cases.append((a, b))
    cases += [(TRUE_MIN, 0.5), (-TRUE_MIN, 0.5), (TRUE_MIN, -0.75), (3 * TRUE_MIN, 0.5),
              (1.0 / 3.0, 3.0), (-1.0 / 3.0, 3.0), (2.0 ** -537, 2.0 ** -537), (-(2.0 ** -537), 2.0 ** -538),
              (1.7976931348623157e308, 0.5), (0.1, 0.1), (-0.1, 0.1)]
    for a, b in cases:
        want = exact_product_rd(a, b)
        got = ora.mul_rd(a, b)
        assert want is not None
        assert _bits(got) == _bits(want), (a, b, got, want)


def test_mul_rd_signed_zero_products(ora):
    # an exact zero product keeps the sign rule of multiplication
    assert _bits(ora.mul_rd(0.0, 3.0)) == _bits(0.0)
    assert _bits(ora.mul_rd(-0.0, 3.0)) == _bits(-0.0)
    assert _bits(ora.mul_rd(0.0, -3.0)) == _bits(-0.0)
    # the mode switch does not leak into later round-to-nearest arithmetic
    assert ora.hypot(3.0, 4.0) == 5.0
    assert 0.1 + 0.2 == 0.30000000000000004


def test_product_error_term_exact(ora):
    """c = RD(x y), c' = fma(x, y, -c): c' >= 0 and c + c' = x y exactly when
    the product does not underflow (item G.)."""
    rng = np.random.default_rng(7)
    for _ in range(2000):
        x = rng.standard_normal() * 2.0 ** rng.integers(-40, 40)
        y = rng.standard_normal() * 2.0 ** rng.integers(-40, 40)
        c = ora.mul_rd(x, y)
        with mpmath.workprec(400):
            d = mpmath.mpf(x) * mpmath.mpf(y) - mpmath.mpf(c)   # what fma(x, y, -c) rounds
            c2 = float(d)
            assert c2 >= 0.0
            assert mpmath.mpf(c2) == d                          # exactly representable


def test_two_sum_exact(ora):
    rng = np.random.default_rng(8)
    for _ in range(3000):
        a = rng.standard_normal() * 2.0 ** rng.integers(-80, 80)
        b = rng.standard_normal() * 2.0 ** rng.integers(-80, 80)
        s, t = ora.two_sum(a, b)
        assert s == a + b
        with mpmath.workprec(400):
            assert mpmath.mpf(s) + mpmath.mpf(t) == mpmath.mpf(a) + mpmath.mpf(b)


def ill_conditioned_dot(m, cond_log10, rng):
    """x, y with sum |x_i y_i| / |x^T y| about 10^cond_log10: half of the
    terms are large and cancel in exact arithmetic (the recipe of generating
    a dot-product with a chosen condition number: random exponents on the
    first half, then the second half chosen to drive the running exact sum
    towards zero)."""
    half = m // 2
    b = cond_log10 / 2.0
    e = np.rint(rng.uniform(0, 1, half) * b).astype(int)
    e[0] = int(round(b)) + 1
    e[-1] = 0
    x = np.empty(m)
    y = np.empty(m)
    x[:half] = (2 * rng.uniform(0, 1, half) - 1) * 2.0 ** e
    y[:half] = (2 * rng.uniform(0, 1, half) - 1) * 2.0 ** e
    e2 = np.rint(np.linspace(b, 0, m - half)).astype(int)
    with mpmath.workprec(3000):
        acc = mpmath.fsum(mpmath.mpf(float(a)) * mpmath.mpf(float(c)) for a, c in zip(x[:half], y[:half]))
        for i in range(half, m):
            x[i] = (2 * rng.uniform() - 1) * 2.0 ** e2[i - half]
            y[i] = ((2 * rng.uniform() - 1) * 2.0 ** e2[i - half] - float(acc)) / x[i]
            acc += mpmath.mpf(float(x[i])) * mpmath.mpf(float(y[i]))
    perm = rng.permutation(m)
    return x[perm], y[perm]


def exact_dot(x, y):
    with mpmath.workprec(3000):
        return mpmath.fsum(mpmath.mpf(float(a)) * mpmath.mpf(float(b)) for a, b in zip(x, y))


@pytest.mark.parametrize("m,cond", [(100, 12), (300, 18), (1500, 24), (2500, 30)])
def test_compensated_error_bound(ora, m, cond):
    """With e = 0 and f = 1 the routine returns the compensated sum itself.
    Kahan's summation (with 2Sum) perturbs every summand by at most about
    2 eps, and the lane reduction adds at most lg(1024) = 10 roundings, so the
    error stays within (2 + 10 + slack) eps sum |x_i y_i| however much the
    terms cancel."""
    rng = np.random.default_rng(cond)
    x, y = ill_conditioned_dot(m, cond, rng)
    exact = exact_dot(x, y)
    absdot = float(np.sum(np.abs(x * y)))
    zc, _ = ora.dpscl_cs(y, None, x, None, 0.0, 1.0, 0.0, 1.0)
    assert abs(float(mpmath.mpf(zc) - exact)) <= 16 * EPS * absdot


def test_compensated_keeps_sub_ulp_terms(ora):
    """One lane (rows 0, 1024, 2048, ...) carries 2^40 followed by 1999 terms
    of 0.3 ulp(2^40): the plain sum rounds every one of them away (600 ulp
    lost); the compensated sum keeps them in t and is within one ulp.  The
    other lanes are zero, so the lane reduction is exact."""
    k = 2000
    x = np.zeros(1024 * k)
    y = np.ones(1024 * k)
    A = 2.0 ** 40
    ulp = 2.0 ** -12
    x[0] = A
    x[1024::1024] = 0.3 * ulp
    with mpmath.workprec(300):
        exact = mpmath.mpf(A) + (k - 1) * mpmath.mpf(0.3 * ulp)
    zc, _ = ora.dpscl_cs(y, None, x, None, 0.0, 1.0, 0.0, 1.0)
    zp, _ = ora.dpscl(y, None, x, None, 0.0, 1.0, 0.0, 1.0)
    assert abs(float(mpmath.mpf(zc) - exact)) <= ulp
    assert abs(float(mpmath.mpf(zp) - exact)) >= 500 * ulp


def test_compensated_cancelling_pairs_exact_zero(ora):
    """Row i and row i + 1024 (the same lane, consecutive in its chain) hold
    x_i y_i and (-x_i) y_i.  The rounded-down products differ by one ulp of
    x_i y_i, exactly compensated by their error terms (which are never
    negative), so the value stream holds -ulp and the error stream +ulp in
    every lane: the two reductions are exact mirror images and the result is
    exactly zero.  The plain fma sum leaves the rounding errors of the
    products behind."""
    rng = np.random.default_rng(12)
    xx = rng.standard_normal(1024)
    yy = rng.standard_normal(1024)
    x = np.concatenate([xx, -xx])
    y = np.concatenate([yy, yy])
    zc, _ = ora.dpscl_cs(y, None, x, None, 0.0, 1.0, 0.0, 1.0)
    zp, _ = ora.dpscl(y, None, x, None, 0.0, 1.0, 0.0, 1.0)
    assert zc == 0.0
    assert zp != 0.0


def test_compensated_complex_equals_conjugate_first_definition(ora):
    """Complex: z = g_q^* g_p / (|g_q| |g_p|); on an ill-conditioned real and
    imaginary part the compensated result is within the error bound of the
    exact value of that definition (the conjugate is taken on g_q)."""
    rng = np.random.default_rng(11)
    m = 400
    xr, yr = ill_conditioned_dot(m, 16, rng)
    xi, yi = ill_conditioned_dot(m, 16, rng)
    # q = yr + i yi; p = xr + i xi: Re(q^* p) = yr.xr + yi.xi, Im = yr.xi - yi.xr
    zr, zi = ora.dpscl_cs(yr, yi, xr, xi, 0.0, 1.0, 0.0, 1.0)
    with mpmath.workprec(3000):
        re = exact_dot(yr, xr) + exact_dot(yi, xi)
        im = exact_dot(yr, xi) - exact_dot(yi, xr)
    absre = float(np.sum(np.abs(yr * xr)) + np.sum(np.abs(yi * xi)))
    absim = float(np.sum(np.abs(yr * xi)) + np.sum(np.abs(yi * xr)))
    assert abs(float(mpmath.mpf(zr) - re)) <= 16 * EPS * absre
    assert abs(float(mpmath.mpf(zi) - im)) <= 16 * EPS * absim
    # and the sign of the imaginary part is that of g_q^* g_p, not g_p^* g_q
    if abs(float(im)) > 1e-3 * absim:
        assert np.sign(zi) == np.sign(float(im))


def test_compensated_equals_plain_when_sums_are_exact(ora):
    """Small integers: every product and partial sum is exact in both routines,
    so both return the same (exact) value, also after the scaling by 2^-e
    and the division by f_q f_p."""
    rng = np.random.default_rng(5)
    for m in (1, 7, 1024, 1025, 3000):
        for cplx in (False, True):
            qr = rng.integers(-64, 64, m).astype(float)
            pr = rng.integers(-64, 64, m).astype(float)
            qi = rng.integers(-64, 64, m).astype(float) if cplx else None
            pi = rng.integers(-64, 64, m).astype(float) if cplx else None
            eq, fq = ora.colnorm(qr, qi)
            ep, fp = ora.colnorm(pr, pi)
            if not (np.isfinite(eq) and np.isfinite(ep)):
                continue
            a = ora.dpscl(qr, qi, pr, pi, eq, fq, ep, fp)
            b = ora.dpscl_cs(qr, qi, pr, pi, eq, fq, ep, fp)
            assert a == b, (m, cplx)


def test_compensated_scaling_invariance(ora):
    """Scaling a column by 2^k moves its norm exponent by k and leaves the
    compensated scaled dot-product bit-identical."""
    rng = np.random.default_rng(6)
    m = 777
    q, qi, p, pi = (rng.standard_normal(m) for _ in range(4))
    e1q, f1q = ora.colnorm(q, qi)
    e1p, f1p = ora.colnorm(p, pi)
    z1 = ora.dpscl_cs(q, qi, p, pi, e1q, f1q, e1p, f1p)
    for k in (-600, -37, 41, 500):
        qs, qis = np.ldexp(q, k), np.ldexp(qi, k)
        eq, fq = ora.colnorm(qs, qis)
        assert (eq, fq) == (e1q + k, f1q)
        assert ora.dpscl_cs(qs, qis, p, pi, eq, fq, e1p, f1p) == z1
