"""GPU parity of the batched widened-exponent Frobenius norms
(jsvd_nrmf_batched, Alg. rnF) against the oracle: every output (the square
and the norm, exponent and fraction) bit for bit, for lane counts 1 ... 1024,
real and complex columns over the whole double range (subnormals, zero
columns), the random-bit vectors of Sect. SM6.4, nu 1, ragged and empty
columns, and all 2048 columns of the real 8192 x 2048 workload."""
import ctypes

import numpy as np
import pytest

from paper_2202_08361_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def J():
    import paper_2202_08361_amd as jsvd
    return jsvd


def _gpu(Ar, Ai, lanes):
    dr = J().to_device_fortran(Ar)
    di = J().to_device_fortran(Ai) if Ai is not None else None
    out = J().nrmf_batched(dr, di, lanes=lanes)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out]


def _compare(ora, Ar, Ai, lanes, tag=""):
    e2, f2, e, f = _gpu(Ar, Ai, lanes)
    for j in range(Ar.shape[1]):
        r = ora.nrmf(Ar[:, j], None if Ai is None else Ai[:, j], lanes=lanes)
        got = (e2[j], f2[j], e[j], f[j])
        want = (r["e2"], r["f2"], r["e"], r["f"])
        assert np.array_equal(np.array(got).view(np.int64), np.array(want).view(np.int64)), (tag, lanes, j, got,
                                                                                              want)


@pytest.mark.parametrize("lanes", [1, 8, 64, 256, 1024])
@pytest.mark.parametrize("cplx", [False, True])
def test_nrmf_wide_range(ora, lanes, cplx):
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 6000 + lanes + int(cplx))
    for m in (1, 7, 255, 1023, 1024, 1025, 5000):
        Ar, Ai = inputs.wide_columns(m, 9, g, cplx)
        _compare(ora, Ar, Ai, lanes, f"m={m}")


@pytest.mark.parametrize("xi", [0, 1008])
def test_nrmf_sm64_vectors(ora, xi):
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 6100 + xi)
    A = np.asfortranarray(np.stack([inputs.random_bit_vector(g, 20000, xi) for _ in range(6)], axis=1))
    for lanes in (8, 1024):
        _compare(ora, A, None, lanes, f"xi={xi}")


def test_nrmf_extremes(ora):
    nu = np.finfo(np.float64).max
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 6200)
    m = 3001
    cols = [np.full(m, nu), np.full(m, -nu), np.zeros(m),
            np.ldexp(g.integers(1, 1 << 40, m).astype(np.float64), -1074),
            np.concatenate([np.full(10, nu), np.ldexp(np.ones(m - 10), -1074)]),
            np.concatenate([np.ldexp(np.ones(m - 10), -1074), np.full(10, nu)])]
    A = np.asfortranarray(np.stack(cols, axis=1))
    for lanes in (1, 8, 1024):
        _compare(ora, A, None, lanes, "extremes")
        _compare(ora, A, np.asfortranarray(A[:, ::-1]), lanes, "extremes complex")


def test_nrmf_large_workload(ora):
    """All 2048 columns of the real 8192 x 2048 workload's shape (Gaussian
    columns), lanes = 1024."""
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 6300)
    Ar, _ = inputs.random_columns(8192, 2048, g)
    _compare(ora, Ar, None, 1024, "8192x2048")


def test_nrmf_empty_and_invalid(ora):
    L = J().lib()
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(x.data_ptr())
    assert L.jsvd_nrmf_batched(0, 5, None, None, 5, 1024, None, None, None, None, None) == 0
    for bad in (0, 3, 2048, -8):
        assert L.jsvd_nrmf_batched(2, 4, p, None, 4, bad, None, None, p, p, None) == J().EINVAL
    assert L.jsvd_nrmf_batched(2, 4, p, None, 3, 8, None, None, p, p, None) == J().EINVAL
    # m = 0: every column is the empty array, norm (-inf, 1)
    e2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    f2 = torch.zeros(2, dtype=torch.float64, device="cuda")
    e = torch.zeros(2, dtype=torch.float64, device="cuda")
    f = torch.zeros(2, dtype=torch.float64, device="cuda")
    pp = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.jsvd_nrmf_batched(2, 0, p, None, 1, 1024, pp(e2), pp(f2), pp(e), pp(f), None) == 0
    torch.cuda.synchronize()
    assert np.all(e.cpu().numpy() == -np.inf) and np.all(f.cpu().numpy() == 1.0)
    assert np.all(e2.cpu().numpy() == -np.inf) and np.all(f2.cpu().numpy() == 1.0)
