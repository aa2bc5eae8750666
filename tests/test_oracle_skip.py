"""The reading behind the skipping of unchanged pairs, checked on the oracle
(which computes every pair): in a step without rescaling, a pair whose two
columns have not changed since it last met, one sweep (K steps) earlier,
leaves both columns of G and V and their norms exactly as they were.

The pair's outcome depends only on its two columns (and the iteration's
fixed options); the previous meeting changed neither column (else the last
change would be that meeting), so the same columns give the same outcome:
no transformation and no swap.  The GPU kernels rely on this to skip such
pairs; here it is checked bit for bit, step by step, through whole
iterations, with every option of the iteration, and the number of pairs it
covered is required to be positive."""
import numpy as np
import pytest

import oracle as ora
from paper_2202_08361_amd import inputs


def _matrix(m, n, cplx, kappa, seed):
    g = inputs.rng(inputs.CFG_PLAIN_LARGE, 8800 + seed)
    sig = inputs.sigma_logspace(n, 1.0 / kappa)
    return inputs.svd_matrix(m, n, sig, g, cplx=cplx)


def _cols(st, j):
    out = [st.Gr[:, j].copy(), st.Vr[:, j].copy(), np.array([st.e[j], st.f[j]])]
    if st.cplx:
        out += [st.Gi[:, j].copy(), st.Vi[:, j].copy()]
    return out


def _same(a, b):
    return all(np.array_equal(x.view(np.int64), y.view(np.int64)) for x, y in zip(a, b))


@pytest.mark.parametrize("m,n,cplx,kappa,opts", [
    (96, 48, False, 1e6, {}),
    (64, 33, True, 1e4, {}),
    (80, 40, False, 1e8, {"permute": True}),
    (72, 36, False, 1e6, {"compensated": True}),
    (60, 30, True, 1e5, {"nogs": True}),
])
def test_unchanged_pairs_stay_unchanged(m, n, cplx, kappa, opts):
    Ar, Ai = _matrix(m, n, cplx, kappa, m + n)
    st = ora.State(Ar, Ai, **opts)
    assert st.init() == ora.OK
    K = ora.rr_steps(n)
    # as after a load: every column counts as changed at the first step
    last = np.zeros(n, dtype=np.int64)
    covered = 0
    for sweep in range(200):
        T = 0
        for _ in range(K):
            k = st.k
            pairs = []
            for l in range((n + 1) // 2):
                ok, p, q = ora.rr_pair(n, k, l)
                if ok:
                    pairs.append((p, q))
            before = [_cols(st, j) for j in range(n)]
            r0 = st.rescaled
            st.step()
            T += st.last_t
            rescaled = st.rescaled != r0
            after = [_cols(st, j) for j in range(n)]
            if not rescaled:
                for p, q in pairs:
                    if last[p] < k - K and last[q] < k - K:
                        covered += 1
                        assert _same(before[p], after[p]) and _same(before[q], after[q]), (sweep, k, p, q)
                for j in range(n):
                    if not _same(before[j][:2] + before[j][3:], after[j][:2] + after[j][3:]):
                        last[j] = k
            else:
                last[:] = k
        if T == 0:
            break
    assert T == 0, "the iteration did not converge"
    assert covered > 0
