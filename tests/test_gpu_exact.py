"""The HIP path against the oracle's exact mode (norms and dot-products from
binary128 sums rounded once): the GPU reproduces the ordered mode bit for
bit (the other tests), and here its singular values are compared with the
exact-mode iteration's within the normwise bound of a backward stable
method, 16 m u sigma_max, and to 16 m u relative for the singular values
within two decades of the largest.  Both iterations must converge and meet
the prescribed singular values."""
import numpy as np
import pytest

from paper_2202_08361_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def J():
    import paper_2202_08361_amd as jsvd
    return jsvd


@pytest.fixture(scope="module", autouse=True)
def _oracle_threads(ora):
    import os
    ora.set_step_threads(min(16, os.cpu_count() or 1))
    yield
    ora.set_step_threads(1)


def _case(name):
    if name == "real256":
        A, sig = inputs.plain_real_256()
        return A, None, sig
    m, n, cplx, kappa, seed = {"cplx96": (96, 80, True, 1e6, 5), "real400": (400, 64, False, 1e10, 6),
                               "cplx300": (300, 120, True, 1e4, 7)}[name]
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 5300 + seed)
    sig = inputs.sigma_logspace(n, 1.0 / kappa)
    Ar, Ai = inputs.svd_matrix(m, n, sig, g, cplx=cplx)
    return Ar, Ai, sig


@pytest.mark.parametrize("name", ["real256", "cplx96", "real400", "cplx300"])
def test_hip_singular_values_against_exact_mode(ora, name):
    Ar, Ai, sig = _case(name)
    m = Ar.shape[0]
    r = J().gesvj(J().to_device_fortran(Ar), None if Ai is None else J().to_device_fortran(Ai))
    torch.cuda.synchronize()
    with ora.exact_mode():
        re = ora.gesvj(Ar, Ai)
    assert r["status"] == 0 and re["status"] == ora.OK
    sh = np.ldexp(r["sv_f"].cpu().numpy(), r["sv_e"].cpu().numpy().astype(int))
    se = np.ldexp(re["sv_f"], re["sv_e"].astype(int))
    assert np.max(np.abs(sh - se)) <= 16 * m * U * se[0]
    top = se >= 1e-2 * se[0]
    assert np.max(np.abs(sh[top] - se[top]) / se[top]) <= 16 * m * U
    big = sig >= 1e-6 * sig[0]
    assert np.max(np.abs(sh[big] - sig[big]) / sig[big]) < 1e-9
