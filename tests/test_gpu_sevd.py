"""GPU parity of the single precision batched 2x2 EVD
(jsvd_evd2_batched_f32) against the single precision CPU oracle: every
output bit for bit on the float32 wide-exponent workload at full size
(2^26 real and 2^26 complex matrices), on ragged sizes, on the special cases
(including the float counterpart of the matrix of eq. evil), for every flag
combination and for the vector and the one-matrix-per-lane paths
(streams misaligned by one element)."""
import numpy as np
import pytest

from paper_2202_08361_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _run_gpu(a11, a22, ar, ai, flags, offset=0):
    import paper_2202_08361_amd as J

    def place(x):
        if x is None:
            return None
        buf = torch.empty(x.shape[0] + offset, dtype=torch.float32, device="cuda")
        buf[offset:] = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
        return buf[offset:]
    r = a11.shape[0]
    A = [place(x) for x in (a11, a22, ar, ai)]

    def out(dtype=torch.float32):
        return torch.empty(r + offset, dtype=dtype, device="cuda")[offset:]
    o = dict(cos=out(), ctan_re=out(), lambda1=out(), lambda2=out(), zp=out(torch.int32))
    if ai is not None:
        o["ctan_im"] = out()
    J.evd2_batched_f32(*A, flags=flags, out=o)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def _compare(ora, a11, a22, ar, ai, flags, offset=0):
    g = _run_gpu(a11, a22, ar, ai, flags, offset)
    cs, cr, ci, l1, l2, zp = ora.sevd2_batch(a11, a22, ar, ai, flags=flags)
    pairs = [("cos", cs), ("ctan_re", cr), ("lambda1", l1), ("lambda2", l2)]
    if ai is not None:
        pairs.append(("ctan_im", ci))
    for name, want in pairs:
        got = g[name]
        bad = np.flatnonzero(got.view(np.int32) != want.view(np.int32))
        assert bad.size == 0, (name, bad[:5], a11[bad[:3]], a22[bad[:3]], ar[bad[:3]],
                               None if ai is None else ai[bad[:3]], got[bad[:3]], want[bad[:3]])
    assert np.array_equal(g["zp"], zp)


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
@pytest.mark.parametrize("cplx", [False, True])
def test_sevd_wide_all_flags(ora, cplx, flags):
    a11, a22, ar, ai = inputs.evd_batch_f32(1 << 17, cplx, seed_sub=3)
    _compare(ora, a11, a22, ar, ai, flags)
    _compare(ora, a11, a22, ar, ai, flags, offset=1)


@pytest.mark.parametrize("cplx", [False, True])
def test_sevd_adversarial(ora, cplx):
    a11, a22, ar, ai = inputs.evd_adversarial_f32(cplx)
    for flags in (0, 1, 2):
        _compare(ora, a11, a22, ar, ai, flags)
        _compare(ora, a11, a22, ar, ai, flags, offset=1)


@pytest.mark.parametrize("r", [1, 2, 3, 255, 257, 511, 513, 100003])
@pytest.mark.parametrize("cplx", [False, True])
def test_sevd_ragged(ora, cplx, r):
    a11, a22, ar, ai = inputs.evd_batch_f32(r, cplx, seed_sub=5)
    _compare(ora, a11, a22, ar, ai, 0)
    _compare(ora, a11, a22, ar, ai, 0, offset=1)


def test_sevd_evil_float():
    f = np.float32
    nu = np.finfo(np.float32).max
    mu = np.nextafter(f(0), f(1))
    a = np.array([nu / f(8), nu / f(8)], dtype=np.float32)
    g = _run_gpu(a, a.copy(), np.array([mu, mu], dtype=np.float32), np.array([mu, -mu], dtype=np.float32), 0)
    assert np.all(g["zp"] == 0) and np.all(g["ctan_re"] == f(1))
    assert np.array_equal(g["ctan_im"], np.array([1, -1], dtype=np.float32))
    assert np.all(g["cos"] == f(1) / np.sqrt(f(2)))


@pytest.mark.parametrize("cplx", [False, True])
def test_sevd_full_size(ora, cplx):
    """The single precision benchmark workload, 2^26 matrices, bit for bit."""
    a11, a22, ar, ai = inputs.evd_batch_f32(1 << 26, cplx)
    _compare(ora, a11, a22, ar, ai, 0)


def test_sevd_empty_and_invalid():
    import ctypes
    import paper_2202_08361_amd as J
    L = J.lib()
    assert L.jsvd_evd2_batched_f32(0, None, None, None, None, None, None, None, None, None, None, 0, None) == 0
    x = torch.zeros(4, dtype=torch.float32, device="cuda")
    p = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    assert L.jsvd_evd2_batched_f32(4, p(x), p(x), p(x), p(x), p(x), p(x), None, None, None, None, 0,
                                   None) == J.EINVAL
    assert L.jsvd_evd2_batched_f32(4, p(x), p(x), p(x), None, p(x), p(x), None, None, None, None, 8,
                                   None) == J.EINVAL
