"""Pin of the oracle's orthonormalisation against modified Gram-Schmidt
written out with explicit loops (unique result for a positive-diagonal R)."""
import numpy as np

import oracle as O
from paper_1601_07159_amd import synth


def _mgs(X, dV):
    Q = [x.copy() for x in X]
    for a in range(len(Q)):
        for b in range(a):
            Q[a] = Q[a] - dV * np.vdot(Q[b], Q[a]) * Q[b]
        Q[a] = Q[a] / np.sqrt(dV * np.vdot(Q[a], Q[a]).real)
    return np.array(Q)


def test_orthonormalize_equals_gram_schmidt():
    g = O.Grid.cubic(8, 5.0)
    X = synth.smooth_orbitals(8, 5.0, 6, seed=12, orthonormal=False)
    Q = O.orthonormalize(X, g)
    ref = _mgs(X, g.dV)
    assert np.linalg.norm(Q - ref) <= 1e-11 * np.linalg.norm(ref)
    S = g.dV * Q.reshape(6, -1).conj() @ Q.reshape(6, -1).T
    np.testing.assert_allclose(S, np.eye(6), atol=1e-13)
