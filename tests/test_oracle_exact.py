"""The oracle's exact mode (oracle/ora_exact.c): column norms (Sect. 3.2) and
scaled dot-products (Alg. zdpscl) from binary128 sums rounded once.

Pinned against exact rational arithmetic (Python fractions; an integer
square root for the correctly rounded norm), and then used as the
reference of the ordered mode: the ordered 1024-lane sums of the oracle lie
within the first-order error bound of their summation order of the exact
values, and a whole SVD in the exact mode agrees with the ordered one to
rounding."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as ora
from paper_2202_08361_amd import inputs

U = 2.0 ** -53


def _cols(m, seed, spread=40, cplx=False):
    g = np.random.default_rng(seed)
    def one():
        x = g.uniform(1.0, 2.0, m) * np.ldexp(1.0, g.integers(-spread, spread + 1, m)) * g.choice([-1.0, 1.0], m)
        x[g.random(m) < 0.05] = 0.0
        return x
    return one(), (one() if cplx else None)


def _norm_ef_rounded(S):
    """(e, f) of sqrt(S), S a positive Fraction, f in [1, 2) rounded to
    nearest even to 53 bits: exact integer arithmetic."""
    a, b = S.numerator, S.denominator
    E = (a.bit_length() - b.bit_length()) // 2 + 1
    while Fraction(4) ** E > S:
        E -= 1
    while Fraction(4) ** (E + 1) <= S:
        E += 1
    # 2^E <= sqrt(S) < 2^(E+1); N = floor(sqrt(S) 2^(52 - E))
    k = 52 - E
    X = S * Fraction(2) ** (2 * k)
    N = math.isqrt(X.numerator // X.denominator)
    lhs = 4 * X                  # compare sqrt(X) with N + 1/2
    rhs = Fraction((2 * N + 1) ** 2)
    if lhs > rhs or (lhs == rhs and N % 2 == 1):
        N += 1
    if N == 1 << 53:
        N >>= 1
        E += 1
    return float(E), N / 2.0 ** 52


@pytest.mark.parametrize("m,cplx,spread,seed", [(1, False, 0, 1), (7, True, 3, 2), (100, False, 40, 3),
                                                (1000, True, 200, 4), (3000, False, 500, 5), (257, True, 900, 6)])
def test_exact_norm_is_correctly_rounded(m, cplx, spread, seed):
    xr, xi = _cols(m, seed, spread, cplx)
    S = sum(Fraction(float(v)) ** 2 for v in xr)
    if cplx:
        S += sum(Fraction(float(v)) ** 2 for v in xi)
    assert ora.colnorm_exact(xr, xi) == _norm_ef_rounded(S)


def test_exact_norm_edges():
    # zero column; one subnormal; components near the top of the range (the
    # sum of squares overflows double, not binary128); a power of two
    assert ora.colnorm_exact(np.zeros(5)) == (-math.inf, 1.0)
    tiny = np.array([0.0, 5e-324, 0.0])
    assert ora.colnorm_exact(tiny) == (-1074.0, 1.0)
    big = np.array([1.7e308, -1.7e308, 1.1e308])
    assert ora.colnorm_exact(big) == _norm_ef_rounded(sum(Fraction(v) ** 2 for v in big))
    assert ora.colnorm_exact(np.array([0.0, -8.0])) == (3.0, 1.0)
    # 3-4-5, exact: the norm has no rounding at all
    assert ora.colnorm_exact(np.array([3.0]), np.array([4.0])) == (2.0, 1.25)


@pytest.mark.parametrize("m,cplx,seed", [(1, True, 11), (9, False, 12), (300, True, 13), (2048, False, 14),
                                         (777, True, 15)])
def test_exact_dot_is_correctly_rounded(m, cplx, seed):
    qr, qi = _cols(m, seed, 30, cplx)
    pr, pi = _cols(m, seed + 100, 30, cplx)
    eq, fq = ora.colnorm(qr, qi)
    ep, fp = ora.colnorm(pr, pi)
    # conj(g_q) g_p, exactly, then scaled by 2^-(eq+ep) and rounded once
    hr = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(qr, pr))
    hi = Fraction(0)
    if cplx:
        hr += sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(qi, pi))
        hi = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(qr, pi)) - \
            sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(qi, pr))
    sc = Fraction(2) ** -(int(eq) + int(ep))
    d = fq * fp
    want = (float(hr * sc) / d, float(hi * sc) / d if cplx else 0.0)
    assert ora.dpscl_exact(qr, qi, pr, pi, eq, fq, ep, fp) == want


def _lane_terms(m):
    P = 1
    while P < m and P < 1024:
        P *= 2
    return -(-m // P) + int(math.log2(P))


@pytest.mark.parametrize("m", [1, 10, 100, 1000, 3000, 20000])
@pytest.mark.parametrize("cplx", [False, True])
def test_ordered_norms_within_bound_of_exact(m, cplx):
    """Ordered norm: a lane sums k = ceil(m / P) prescaled squares by fma, the
    P lanes add in log2 P levels: relative error of the sum at most
    (k + log2 P) u to first order, half that after the square root, plus
    its rounding; the complex norm adds the naive hypot of two such norms
    (Alg. hypot, a few u)."""
    for seed in range(4):
        xr, xi = _cols(m, 1000 * m + seed, 60, cplx)
        e1, f1 = ora.colnorm(xr, xi)
        e2, f2 = ora.colnorm_exact(xr, xi)
        a, b = math.ldexp(f1, int(e1)), math.ldexp(f2, int(e2))
        bound = (_lane_terms(m) / 2.0 + (6.0 if cplx else 2.0)) * U
        assert abs(a - b) <= bound * b, (m, cplx, seed, (a - b) / b)


@pytest.mark.parametrize("m", [2, 64, 1000, 5000])
@pytest.mark.parametrize("cplx", [False, True])
def test_ordered_dots_within_bound_of_exact(m, cplx):
    """Ordered dot: the same summation order; error of each sum at most
    (k + log2 P + 1) u times the sum of the terms' magnitudes (fma
    accumulation, a term added per fma, complex streams of 2k terms), then the
    common division by fl(fq fp)."""
    for seed in range(4):
        qr, qi = _cols(m, 7000 + m + seed, 20, cplx)
        pr, pi = _cols(m, 8000 + m + seed, 20, cplx)
        eq, fq = ora.colnorm(qr, qi)
        ep, fp = ora.colnorm(pr, pi)
        zo = ora.dpscl(qr, qi, pr, pi, eq, fq, ep, fp)
        ze = ora.dpscl_exact(qr, qi, pr, pi, eq, fq, ep, fp)
        sc = 2.0 ** -(eq + ep) / (fq * fp)
        mag = np.sum(np.abs(qr * pr)) + (np.sum(np.abs(qi * pi)) if cplx else 0.0)
        magi = (np.sum(np.abs(qr * pi)) + np.sum(np.abs(qi * pr))) if cplx else 0.0
        k = _lane_terms(m) * (2 if cplx else 1) + 1
        assert abs(zo[0] - ze[0]) <= k * U * mag * sc + 2 * U * abs(ze[0])
        assert abs(zo[1] - ze[1]) <= k * U * magi * sc + 2 * U * abs(ze[1])


def test_exact_mode_state_uses_exact_norms():
    """A step in the exact mode leaves every column's (e, f) (n even: every
    column takes part) equal to the exact norm of the column it started from,
    and the ordered mode is back after the block."""
    m, n = 70, 12
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 31)
    Ar, Ai = inputs.random_columns(m, n, g, True)
    with ora.exact_mode():
        st = ora.State(Ar, Ai)
        assert st.init() == ora.OK
        G0r, G0i = st.Gr.copy(), st.Gi.copy()
        st.step()
    for j in range(n):
        assert (st.e[j], st.f[j]) == ora.colnorm_exact(G0r[:, j], G0i[:, j]), j
    assert ora.lib().ora_get_exact() == 0


@pytest.mark.parametrize("m,n,cplx,kappa", [(60, 40, False, 1e6), (48, 48, True, 1e4), (120, 30, False, 1e10)])
def test_exact_mode_svd_agrees_with_ordered(m, n, cplx, kappa):
    """The whole SVD in both modes: both converge, both meet the prescribed
    singular values as well as the double precision matrix allows, and they
    agree with each other within the normwise bound of a backward stable
    method, a small multiple of m u sigma_max for every singular value (the
    relative difference of the smallest ones scales with kappa: 9e-12 at
    kappa = 1e6)."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 40 + m + n)
    sig = inputs.sigma_logspace(n, 1.0 / kappa)
    Ar, Ai = inputs.svd_matrix(m, n, sig, g, cplx=cplx)
    ro = ora.gesvj(Ar, Ai)
    with ora.exact_mode():
        re = ora.gesvj(Ar, Ai)
    assert ro["status"] == re["status"] == ora.OK
    so = np.ldexp(ro["sv_f"], ro["sv_e"].astype(int))
    se = np.ldexp(re["sv_f"], re["sv_e"].astype(int))
    assert np.max(np.abs(so - se)) <= 16 * m * U * se[0]
    top = se >= 1e-2 * se[0]
    assert np.max(np.abs(so[top] - se[top]) / se[top]) <= 16 * m * U
    big = sig >= 1e-6 * sig[0]
    assert np.max(np.abs(se[big] - sig[big]) / sig[big]) < 1e-9
