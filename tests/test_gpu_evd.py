"""GPU parity of the batched 2x2 EVD (jsvd_evd2_batched) against the CPU oracle.

The bar is bit-for-bit equality of every output (cos phi, e^{i alpha} tan phi,
lambda_1,2, the packed (zeta' << 1) | p) on the wide-exponent workload at
full size (2^26 real and 2^26 complex matrices), on an adversarial set (signed
zeros, subnormals, values near the overflow threshold, equal diagonals, the
matrix of eq. evil), on an all-exponent sweep, for every flag combination and
for both the 16-byte vector path and the scalar path (unaligned streams).
"""
import numpy as np
import pytest

from paper_2202_08361_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _run_gpu(J, a11, a22, ar, ai, flags, offset=0):
    """Launch on device copies; offset > 0 shifts every stream by `offset`
    elements inside a larger buffer (forces the unaligned scalar path)."""
    def place(x):
        if x is None:
            return None
        buf = torch.empty(x.shape[0] + offset, dtype=torch.float64, device="cuda")
        buf[offset:] = _dev(x)
        return buf[offset:]
    r = a11.shape[0]
    A = [place(x) for x in (a11, a22, ar, ai)]

    def out(dtype=torch.float64):
        return torch.empty(r + offset, dtype=dtype, device="cuda")[offset:]
    o = dict(cos=out(), ctan_re=out(), lambda1=out(), lambda2=out(), zp=out(torch.int32))
    if ai is not None:
        o["ctan_im"] = out()
    J.evd2_batched(*A, flags=flags, out=o)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def _compare(ora, a11, a22, ar, ai, flags, offset=0):
    import paper_2202_08361_amd as J
    g = _run_gpu(J, a11, a22, ar, ai, flags, offset)
    cs, cr, ci, l1, l2, zp = ora.evd2_batch(a11, a22, ar, ai, flags=flags)
    pairs = [("cos", cs), ("ctan_re", cr), ("lambda1", l1), ("lambda2", l2)]
    if ai is not None:
        pairs.append(("ctan_im", ci))
    for name, want in pairs:
        got = g[name]
        bad = np.flatnonzero(got.view(np.int64) != want.view(np.int64))
        assert bad.size == 0, (name, bad[:5], a11[bad[:3]], a22[bad[:3]], ar[bad[:3]],
                               None if ai is None else ai[bad[:3]], got[bad[:3]], want[bad[:3]])
    assert np.array_equal(g["zp"], zp)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_evd_adversarial(ora, cplx, flags):
    a11, a22, ar, ai = inputs.evd_adversarial(cplx)
    _compare(ora, a11, a22, ar, ai, flags)
    _compare(ora, a11, a22, ar, ai, flags, offset=1)


@pytest.mark.parametrize("cplx", [False, True])
def test_evd_exponent_sweep(ora, cplx):
    a11, a22, ar, ai = inputs.evd_exponent_sweep(cplx)
    _compare(ora, a11, a22, ar, ai, 0)
    _compare(ora, a11, a22, ar, ai, 1)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("r", [1, 2, 3, 255, 257, 100003])
def test_evd_ragged_sizes(ora, cplx, r):
    a11, a22, ar, ai = inputs.evd_batch(r, cplx, seed_sub=r)
    _compare(ora, a11, a22, ar, ai, 0)
    _compare(ora, a11, a22, ar, ai, 0, offset=1)


def test_evd_evil_matrix(ora):
    nu = np.finfo(np.float64).max
    mu = np.nextafter(0.0, 1.0)
    a = np.array([nu / 8, nu / 8])
    _compare(ora, a, a.copy(), np.array([mu, mu]), np.array([mu, -mu]), 0)


@pytest.mark.parametrize("cplx", [False, True])
def test_evd_full_size(ora, cplx):
    """The benchmark workload, 2^26 matrices, every output bit-for-bit."""
    r = 1 << 26
    a11, a22, ar, ai = inputs.evd_batch(r, cplx)
    _compare(ora, a11, a22, ar, ai, 0)


def test_evd_empty_and_invalid():
    import paper_2202_08361_amd as J
    L = J.lib()
    assert L.jsvd_evd2_batched(0, None, None, None, None, None, None, None, None, None, None, 0, None) == 0
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    # a21_im given without ctan_im -> EINVAL, nothing launched
    p = lambda t: None if t is None else __import__("ctypes").c_void_p(t.data_ptr())
    assert L.jsvd_evd2_batched(4, p(x), p(x), p(x), p(x), p(x), p(x), None, None, None, None, 0, None) == J.EINVAL
    assert L.jsvd_evd2_batched(4, p(x), p(x), p(x), None, p(x), p(x), None, None, None, None, 8, None) == J.EINVAL
