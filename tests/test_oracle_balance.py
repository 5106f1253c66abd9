"""Pins of residual balancing (Boyd et al. 2011, Sec. 3.4.1) in the oracle:
for Q = 1 the iterates, residuals, tolerances and penalty equal a textbook
LASSO ADMM with the same rule; for Q > 1 the balanced solve reaches the same
optimum as the fixed-penalty one (the ridge gamma, not beta, fixes the
problem), and each change follows the rule."""

import numpy as np
import pytest

import oracle
from pin_helpers import lasso_admm_boyd_balanced, tiny_problem


@pytest.mark.parametrize("beta,every", [(40.0, 3), (0.02, 2)])
def test_single_sensor_balanced_equals_boyd(beta, every):
    """beta far too large (primal residual dominates... then dual) or far too
    small: the rule changes beta several times; every iterate matches."""
    A, y = tiny_problem(Q=1, KM=10, N=16, seed=5)
    mu, gamma, lam = 1.7, 0.4, 0.8
    p = oracle.Params(mu=mu, beta=beta, gamma=gamma, lam=lam, eps_abs=1e-6, eps_rel=1e-4,
                      max_iter=60, stop=False, balance_every=every)
    R = oracle.solve(A, y, p, record_iterates=True)
    ref = lasso_admm_boyd_balanced(A[0], y[0], mu, beta, gamma, lam, 60, 1e-6, 1e-4, every)
    changes = 0
    for k in range(60):
        zk, r, s, ep, ed, rho = ref[k]
        assert np.allclose(R.history["z"][k], zk, rtol=0, atol=1e-11)
        assert R.history["r"][k] == pytest.approx(r, rel=1e-8, abs=1e-13)
        assert R.history["s"][k] == pytest.approx(s, rel=1e-8, abs=1e-13)
        assert R.history["eps_pri"][k] == pytest.approx(ep, rel=1e-10)
        assert R.history["eps_dual"][k] == pytest.approx(ed, rel=1e-10)
        assert R.history["beta"][k] == rho
        changes += k > 0 and ref[k][5] != ref[k - 1][5]
    assert changes >= 2


def test_multi_sensor_balanced_reaches_the_same_optimum():
    A, y = tiny_problem(Q=3, KM=8, N=14, seed=21)
    base = dict(mu=1.1, gamma=0.7, lam=0.4, eps_abs=0.0, eps_rel=1e-12, max_iter=60000)
    fixed = oracle.solve(A, y, oracle.Params(beta=0.7, **base))
    bal = oracle.solve(A, y, oracle.Params(beta=50.0, balance_every=5, **base))
    assert fixed.converged and bal.converged
    assert np.linalg.norm(bal.z - fixed.z) <= 1e-9 * np.linalg.norm(fixed.z)
    b = np.array(bal.history["beta"])
    changed = np.flatnonzero(np.diff(b)) + 1        # iteration index (0-based) after which beta changed
    assert changed.size > 0
    r, s = np.array(bal.history["r"]), np.array(bal.history["s"])
    for i in changed:
        k = i                                        # decided at iteration index i (1-based k = i + 1)
        assert (k + 1) % 5 == 0
        if b[i] > b[i - 1]:
            assert r[k] > 10 * s[k]
        else:
            assert s[k] > 10 * r[k]
