"""Seeded synthetic inputs shaped like the workloads of arXiv:2202.08361.

This module holds only random-input generation: no step of the Jacobi method
or of the 2x2 EVD is computed here, and it imports neither the HIP binding nor
the CPU oracle.  Both sides of every parity test draw their inputs from here.

Workloads (the paper's own datasets are not available, so these synthetic
recipes stand in for them):

* EVD batch: SoA streams of real symmetric (a11, a22, a21) or complex
  Hermitian (a11, a22, Re a21, Im a21) 2x2 matrices; every component is
  random sign * 2^E * f with E uniform in [-1074, 1023], f uniform in [1, 2)
  (ldexp rounds E < -1022 into the subnormal range); then 1 % of the matrices
  get a subnormal off-diagonal k * 2^-1074, and 1 % of all components
  become exactly +0.
* Paper-shaped EVD accuracy set (Sect. 5.1): matrices built from prescribed
  eigenvalues and rotation through eq. (2), evaluated in high precision.
* SVD test matrices A = U diag(sigma) V^* with Haar-distributed U, V (QR of a
  Gaussian with the sign fix of the R diagonal), accumulated in extended
  precision and rounded once to double, sigma log-spaced or geometric.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 220208361

# configuration indices (also the seed offsets)
CFG_PLAIN_REAL_256 = 0
CFG_EVD_BATCH = 1
CFG_PLAIN_LARGE = 2
CFG_BATCHED = 3
CFG_SERVE = 4


def rng(cfg: int, sub: int = 0) -> np.random.Generator:
    """PCG64 stream for configuration ``cfg`` and sub-stream ``sub``."""
    ss = np.random.SeedSequence([SEED_BASE + cfg, sub])
    return np.random.Generator(np.random.PCG64(ss))


# ------------------------------------------------------------------ EVD batch
def _wide_components(g: np.random.Generator, r: int) -> np.ndarray:
    e = g.integers(-1074, 1024, size=r, dtype=np.int64)
    mant = g.integers(0, 1 << 52, size=r, dtype=np.int64)
    f = 1.0 + mant.astype(np.float64) * 2.0 ** -52          # exact: 52 random bits
    x = np.ldexp(f, e)
    sign = g.integers(0, 2, size=r, dtype=np.int8)
    return np.where(sign == 1, -x, x)


def evd_batch(r: int, cplx: bool, seed_sub: int = 0, zero_frac: float = 0.01,
              subn_frac: float = 0.01):
    """SoA inputs of the stand-alone batched EVD.  Returns (a11, a22, a21r, a21i|None)."""
    g = rng(CFG_EVD_BATCH, (1 if cplx else 0) + 2 * seed_sub)
    a11 = _wide_components(g, r)
    a22 = _wide_components(g, r)
    a21r = _wide_components(g, r)
    a21i = _wide_components(g, r) if cplx else None
    # 1 % of the matrices: subnormal off-diagonal, k * 2^-1074, k in [1, 2^52 - 1]
    sel = g.random(r) < subn_frac
    ns = int(sel.sum())
    a21r[sel] = np.ldexp(g.integers(1, 1 << 52, size=ns).astype(np.float64), -1074) * \
        np.where(g.integers(0, 2, size=ns) == 1, -1.0, 1.0)
    if cplx:
        a21i[sel] = np.ldexp(g.integers(1, 1 << 52, size=ns).astype(np.float64), -1074) * \
            np.where(g.integers(0, 2, size=ns) == 1, -1.0, 1.0)
    # 1 % of all components: exactly +0
    for a in (a11, a22, a21r) + ((a21i,) if cplx else ()):
        a[g.random(r) < zero_frac] = 0.0
    return a11, a22, a21r, a21i


def evd_adversarial(cplx: bool):
    """Hand-picked special cases: zeros of both signs, subnormals, huge
    values near the overflow threshold, equal diagonals, tiny/huge mixes."""
    nu = np.finfo(np.float64).max
    mu = np.nextafter(0.0, 1.0)
    tn = np.finfo(np.float64).tiny
    vals = [0.0, -0.0, mu, -mu, 2 * mu, 3 * mu, tn, -tn, tn / 2, 1.0, -1.0, 0.5, 3.0,
            nu, -nu, nu / 8, nu / 2, np.sqrt(nu), 1e-300, 1e300, 2.0 ** -1022, 1.0 + 2 ** -52,
            np.nextafter(nu / 8, 0), np.ldexp(1.5, -1060), 7.0, -7.0]
    g = rng(CFG_EVD_BATCH, 99)
    rows = []
    for a in vals:
        for b in vals[::3]:
            for c in vals[::2]:
                if cplx:
                    for d in (0.0, -0.0, mu, c, -c, tn):
                        rows.append((a, b, c, d))
                else:
                    rows.append((a, b, c, 0.0))
    # equal diagonals with all kinds of off-diagonals
    for a in vals:
        for c in vals:
            rows.append((a, a, c, c if cplx else 0.0))
    rows = np.array(rows, dtype=np.float64)
    g.shuffle(rows, axis=0)
    a11, a22, a21r = rows[:, 0].copy(), rows[:, 1].copy(), rows[:, 2].copy()
    a21i = rows[:, 3].copy() if cplx else None
    return a11, a22, a21r, a21i


def evd_exponent_sweep(cplx: bool):
    """Every pair of binary exponents (step 7) for the diagonal and off-diagonal."""
    es = np.arange(-1074, 1024, 7)
    E1, E2 = np.meshgrid(es, es, indexing="ij")
    E1, E2 = E1.ravel(), E2.ravel()
    g = rng(CFG_EVD_BATCH, 98)
    r = E1.size
    f = lambda: 1.0 + g.integers(0, 1 << 52, size=r).astype(np.float64) * 2.0 ** -52
    a11 = np.ldexp(f(), E1)
    a22 = -np.ldexp(f(), E1 - 3)
    a21r = np.ldexp(f(), E2) * np.where(g.random(r) < 0.5, -1, 1)
    a21i = np.ldexp(f(), E2 - 1) * np.where(g.random(r) < 0.5, -1, 1) if cplx else None
    return a11, a22, a21r, a21i


# ------------------------------------------------------------------ single precision EVD inputs
def _wide_components_f32(g: np.random.Generator, r: int) -> np.ndarray:
    """sign * 2^E * f as float32, E uniform in [-149, 127], f in [1, 2) with 23
    random fraction bits (E < -126 rounds into the subnormals)."""
    E = g.integers(-149, 128, size=r)
    f = 1.0 + g.integers(0, 1 << 23, size=r).astype(np.float64) * 2.0 ** -23
    s = np.where(g.integers(0, 2, size=r) == 1, -1.0, 1.0)
    return (s * np.ldexp(f, E)).astype(np.float32)


def evd_batch_f32(r: int, cplx: bool, seed_sub: int = 0, zero_frac: float = 0.01,
                  subn_frac: float = 0.01):
    """SoA float32 inputs of the single precision batched EVD, the same recipe
    as evd_batch over the float32 range.  Returns (a11, a22, a21r, a21i|None)."""
    g = rng(CFG_EVD_BATCH, 1000 + (1 if cplx else 0) + 2 * seed_sub)
    a11 = _wide_components_f32(g, r)
    a22 = _wide_components_f32(g, r)
    a21r = _wide_components_f32(g, r)
    a21i = _wide_components_f32(g, r) if cplx else None
    # subnormal off-diagonal, k * 2^-149, k in [1, 2^23 - 1]
    sel = g.random(r) < subn_frac
    ns = int(sel.sum())
    a21r[sel] = (np.ldexp(g.integers(1, 1 << 23, size=ns).astype(np.float64), -149) *
                 np.where(g.integers(0, 2, size=ns) == 1, -1.0, 1.0)).astype(np.float32)
    if cplx:
        a21i[sel] = (np.ldexp(g.integers(1, 1 << 23, size=ns).astype(np.float64), -149) *
                     np.where(g.integers(0, 2, size=ns) == 1, -1.0, 1.0)).astype(np.float32)
    for a in (a11, a22, a21r) + ((a21i,) if cplx else ()):
        a[g.random(r) < zero_frac] = np.float32(0.0)
    return a11, a22, a21r, a21i


def evd_adversarial_f32(cplx: bool):
    """Special float32 cases: signed zeros, subnormals, values near the overflow
    threshold, equal diagonals."""
    f = np.float32
    nu = np.finfo(np.float32).max
    mu = np.nextafter(f(0.0), f(1.0))
    tn = np.finfo(np.float32).tiny
    vals = [f(0.0), f(-0.0), mu, -mu, f(2) * mu, f(3) * mu, tn, -tn, tn / f(2), f(1.0), f(-1.0), f(0.5), f(3.0),
            nu, -nu, nu / f(8), nu / f(2), np.sqrt(nu), f(1e-38), f(1e38), f(2.0 ** -126), f(1.0 + 2 ** -23),
            np.nextafter(nu / f(8), f(0)), f(np.ldexp(1.5, -140)), f(7.0), f(-7.0)]
    g = rng(CFG_EVD_BATCH, 1099)
    rows = []
    for a in vals:
        for b in vals[::3]:
            for c in vals[::2]:
                if cplx:
                    for d in (f(0.0), f(-0.0), mu, c, -c, tn):
                        rows.append((a, b, c, d))
                else:
                    rows.append((a, b, c, f(0.0)))
    for a in vals:
        for c in vals:
            rows.append((a, a, c, c if cplx else f(0.0)))
    rows = np.array(rows, dtype=np.float32)
    g.shuffle(rows, axis=0)
    a11, a22, a21r = rows[:, 0].copy(), rows[:, 1].copy(), rows[:, 2].copy()
    a21i = rows[:, 3].copy() if cplx else None
    return a11, a22, a21r, a21i


# ------------------------------------------------------------------ SVD inputs
def haar(n: int, g: np.random.Generator, cplx: bool = False, m: int | None = None) -> np.ndarray:
    """m x n matrix with Haar-distributed orthonormal columns (QR of a Gaussian,
    R-diagonal sign fix)."""
    m = n if m is None else m
    Z = g.standard_normal((m, n))
    if cplx:
        Z = (Z + 1j * g.standard_normal((m, n))) / math.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    ph = d / np.abs(d)
    return Q * ph[None, :]


def sigma_logspace(n: int, lo: float, hi: float = 1.0) -> np.ndarray:
    """sigma_i = hi * (lo/hi)^((i-1)/(n-1)), descending."""
    if n == 1:
        return np.array([hi])
    t = np.arange(n, dtype=np.float64) / (n - 1)
    return hi * np.power(lo / hi, t)


def sigma_paper(xi: float, n: int) -> np.ndarray:
    """Sect. 5.1: sigma_i = 2^{xi (1 - (i-1)/(n-1))}, i = 1..n (ascending)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.exp2(xi * (1.0 - (i - 1) / (n - 1)))


def svd_matrix(m: int, n: int, sigma: np.ndarray, g: np.random.Generator,
               cplx: bool = False, extended: bool | None = None):
    """A = U diag(sigma) V^*, U m x n and V n x n Haar.  With ``extended``
    (default for m*n*n <= 2^27) the product is accumulated in long double and
    rounded once.  Returns (A_re, A_im|None) as Fortran-ordered float64."""
    U = haar(n, g, cplx, m)
    V = haar(n, g, cplx)
    if extended is None:
        extended = m * n * n <= (1 << 27)
    if extended and not cplx:
        Ul = U.astype(np.longdouble) * sigma.astype(np.longdouble)[None, :]
        A = np.asfortranarray((Ul @ V.T.astype(np.longdouble)).astype(np.float64))
        return A, None
    if extended and cplx:
        Ur, Ui = U.real.astype(np.longdouble), U.imag.astype(np.longdouble)
        s = sigma.astype(np.longdouble)[None, :]
        Ur, Ui = Ur * s, Ui * s
        Vr, Vi = V.real.astype(np.longdouble), V.imag.astype(np.longdouble)
        # (Ur + i Ui) (Vr - i Vi)^T
        Ar = Ur @ Vr.T + Ui @ Vi.T
        Ai = Ui @ Vr.T - Ur @ Vi.T
        return np.asfortranarray(Ar.astype(np.float64)), np.asfortranarray(Ai.astype(np.float64))
    A = (U * sigma[None, :]) @ V.conj().T
    if cplx:
        return np.asfortranarray(A.real), np.asfortranarray(A.imag)
    return np.asfortranarray(A), None


def plain_real_256(seed_sub: int = 0):
    """Plain real case: 256 x 256, sigma log-spaced in [1e-6, 1]."""
    g = rng(CFG_PLAIN_REAL_256, seed_sub)
    sig = sigma_logspace(256, 1e-6)
    A, _ = svd_matrix(256, 256, sig, g, extended=True)
    return A, sig


def plain_complex_4096(seed_sub: int = 0, n: int = 4096):
    """Plain complex case: n x n (4096), sigma geometric from 1 to 1e-12."""
    g = rng(CFG_PLAIN_LARGE, 2 * seed_sub)
    sig = sigma_logspace(n, 1e-12)
    Ar, Ai = svd_matrix(n, n, sig, g, cplx=True, extended=False)
    return Ar, Ai, sig


def plain_real_tall(seed_sub: int = 0, m: int = 8192, n: int = 2048):
    """Tall real case: 8192 x 2048, sigma log-spaced in [1e-8, 1]."""
    g = rng(CFG_PLAIN_LARGE, 2 * seed_sub + 1)
    sig = sigma_logspace(n, 1e-8)
    A, _ = svd_matrix(m, n, sig, g, extended=False)
    return A, sig


def random_columns(m: int, n: int, g: np.random.Generator, cplx: bool = False):
    """Gaussian columns (cheap stand-in where only the shape matters)."""
    Ar = np.asfortranarray(g.standard_normal((m, n)))
    Ai = np.asfortranarray(g.standard_normal((m, n))) if cplx else None
    return Ar, Ai


# ------------------------------------------------------------------ batched / serving
def batched_shapes(count: int = 10000, seed_sub: int = 0, nmin: int = 16, nmax: int = 256):
    """Uneven shapes: n uniform in [nmin, nmax], m uniform in [n, 2n], kappa
    log-uniform in [1e2, 1e8]."""
    g = rng(CFG_BATCHED, seed_sub)
    n = g.integers(nmin, nmax + 1, size=count)
    m = np.array([g.integers(k, 2 * k + 1) for k in n])
    kappa = 10.0 ** g.uniform(2.0, 8.0, size=count)
    return m.astype(np.int64), n.astype(np.int64), kappa


def batched_matrix(i: int, m: int, n: int, kappa: float, seed_sub: int = 0):
    """Matrix i of the batched workload (its own sub-stream)."""
    g = rng(CFG_BATCHED, 1000003 * (seed_sub + 1) + i)
    sig = sigma_logspace(n, 1.0 / kappa)
    A, _ = svd_matrix(m, n, sig, g, extended=(m * n * n <= (1 << 22)))
    return A, sig


def serve_stream(rate: float = 2000.0, duration: float = 60.0, seed_sub: int = 0,
                 nmin: int = 32, nmax: int = 2048, frac_real: float = 0.7):
    """Poisson arrivals: returns (t_arrival[s], is_complex, m, n, kappa)."""
    g = rng(CFG_SERVE, seed_sub)
    cnt = g.poisson(rate * duration)
    t = np.sort(g.uniform(0.0, duration, size=cnt))
    cplx = g.random(cnt) >= frac_real
    n = np.exp(g.uniform(math.log(nmin), math.log(nmax), size=cnt)).astype(np.int64)
    n = np.clip(n, nmin, nmax)
    m = np.array([g.integers(k, 2 * k + 1) for k in n], dtype=np.int64)
    kappa = 10.0 ** g.uniform(2.0, 10.0, size=cnt)
    return t, cplx, m, n, kappa


def serve_matrix(m: int, n: int, kappa: float, cplx: bool, g: np.random.Generator):
    """One serving request: cheap random orthonormal factors (QR of a Gaussian)."""
    sig = sigma_logspace(n, 1.0 / kappa)
    return svd_matrix(m, n, sig, g, cplx=cplx, extended=False) + (sig,)


# ------------------------------------------------------------------ extreme norm ratios
def sm9_matrix(hi: int = 1023, lo: int = -51, n: int = 16, dtype=np.float64, phases_seed: int | None = None):
    """The test matrix of Sect. SM9: G_ij = 2^(hi - (j-1) - |i-j|) for
    j <= n/2, 2^(lo - (j-1) - |i-j|) beyond (1-based indices); hi = eta_hat,
    lo = lg upsilon make the two column groups' norms differ by far more than
    2^eta_hat upsilon.  With phases_seed, complex: every entry times
    e^{i theta}, theta uniform (returns (re, im) then), else (G, None)."""
    G = np.zeros((n, n), order="F")
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            G[i - 1, j - 1] = 2.0 ** ((hi if j <= n // 2 else lo) - (j - 1) - abs(i - j))
    if phases_seed is None:
        return G.astype(dtype), None
    g = rng(CFG_PLAIN_LARGE, 4000 + phases_seed)
    th = g.uniform(0, 2 * np.pi, size=(n, n))
    return (np.asfortranarray((G * np.cos(th)).astype(dtype)), np.asfortranarray((G * np.sin(th)).astype(dtype)))


def split_scale_columns(m: int, n: int, g: np.random.Generator, cplx: bool, shift: int):
    """Gaussian columns (random_columns) with the second half of the columns
    scaled by 2^-shift: every pair across the halves has a norm ratio of about
    2^shift."""
    Ar, Ai = random_columns(m, n, g, cplx)
    Ar[:, n // 2:] = np.ldexp(Ar[:, n // 2:], -shift)
    if cplx:
        Ai[:, n // 2:] = np.ldexp(Ai[:, n // 2:], -shift)
    return Ar, Ai


# ------------------------------------------------------------------ Frobenius norm inputs
def random_bit_vector(g: np.random.Generator, m: int, xi: int) -> np.ndarray:
    """Sect. SM6.4: every element from 64 random bits (each bit 0 or 1 with
    equal probability), kept when finite with magnitude in [0, 2^xi], then
    its absolute value."""
    out = np.empty(0)
    while out.size < m:
        b = g.integers(0, 1 << 63, 2 * m, dtype=np.int64).view(np.float64)
        b = np.abs(b[np.isfinite(b)])
        out = np.concatenate([out, b[b <= np.ldexp(1.0, xi)]])
    return out[:m]


def wide_columns(m: int, n: int, g: np.random.Generator, cplx: bool = False, zero_frac: float = 0.02):
    """Columns over the whole double range: sign 2^E U[1, 2), E uniform in
    [-1074, 1023] per element (subnormals included), a fraction of zeros, and
    one column in eight entirely zero."""
    def part():
        E = g.integers(-1074, 1024, size=(m, n))
        x = np.ldexp(g.uniform(1.0, 2.0, size=(m, n)), E) * np.where(g.random((m, n)) < 0.5, -1.0, 1.0)
        x[g.random((m, n)) < zero_frac] = 0.0
        if n >= 8:
            x[:, ::8] = 0.0
        return np.asfortranarray(x)
    Ar = part()
    Ai = part() if cplx else None
    return Ar, Ai
