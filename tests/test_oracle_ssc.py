"""Pins of the oracle's pixel elimination (Alg. 1, SSC) and of the freeze /
reinstatement bookkeeping."""

import numpy as np
import pytest

import oracle
from scenegen import make_geometry, make_scene, steering


@pytest.fixture(scope="module")
def radar_small():
    g = make_geometry(Q=3, M=2, K=16, n_side=10)
    sc = make_scene(g, 7, 5, 20.0)
    A = [steering(g, q) for q in range(g.Q)]
    lam = 0.2 * oracle.lambda_max(A, sc.y, 1.3, 0.8)
    base = dict(mu=1.3, beta=1.1, gamma=0.8, lam=lam, eps_abs=0.0, eps_rel=1e-3,
                Kp=4, eps_p=1e-4)
    return A, sc, base


def test_eps_p_zero_is_plain_sadmm_bit_for_bit(radar_small):
    """P6: zeta >= 0 always, so with eps_p = 0 SSC never removes a pixel."""
    A, sc, base = radar_small
    plain = oracle.solve(A, sc.y, oracle.Params(max_iter=60, stop=False, **base))
    pr = oracle.solve(A, sc.y, oracle.Params(max_iter=60, stop=False, prune=True,
                                             **{**base, "eps_p": 0.0}))
    assert pr.prune_events == 0
    assert np.array_equal(pr.z, plain.z) and np.array_equal(pr.X, plain.X)


def test_gate_and_window_first_prune_iteration(radar_small):
    """Alg. 1 gate: with eps_p = inf every active pixel goes at the first
    iteration k >= K_p whose primal residual is within tolerance."""
    A, sc, base = radar_small
    plain = oracle.solve(A, sc.y, oracle.Params(max_iter=80, stop=False, **base))
    r = np.array(plain.history["r"])
    ep = np.array(plain.history["eps_pri"])
    ks = [k for k in range(base["Kp"], 81) if r[k - 1] <= ep[k - 1]]
    assert ks, "gate never opened"
    k0 = ks[0]
    pr = oracle.solve(A, sc.y, oracle.Params(max_iter=80, stop=False, prune=True,
                                             **{**base, "eps_p": np.inf}))
    pruned = np.array(pr.history["pruned"])
    assert np.flatnonzero(pruned)[0] + 1 == k0
    assert pruned[k0 - 1] == A[0].shape[1] * len(A)
    assert pr.active.sum() == 0
    # before the first prune, identical trajectory
    assert np.array_equal(np.array(pr.history["r"][:k0]), r[:k0])


def test_ssc_decisions_match_bruteforce_window(radar_small):
    """Alg. 1 steps 1-2 recomputed from the recorded iterates: zeta_q = mean of
    the K_p most recent |x_q^(i) - x_q^(i-1)| (x^(0) = 0), keep zeta >= eps_p.
    Decisions within 1e-9 relative of eps_p are ties and are not asserted."""
    A, sc, base = radar_small
    Kp, eps_p = base["Kp"], base["eps_p"]
    pr = oracle.solve(A, sc.y, oracle.Params(max_iter=80, stop=False, prune=True, **base),
                      record_iterates=True)
    pruned = np.array(pr.history["pruned"])
    assert pruned.sum() > 0
    Xs = [np.zeros_like(pr.X)] + pr.history["X"]
    masks = [np.ones(pr.X.shape, bool)] + pr.history["masks"]
    n_checked = 0
    for k in range(1, 81):
        before, after = masks[k - 1], masks[k]
        assert not (after & ~before).any()            # J only shrinks
        if not pruned[k - 1]:
            assert np.array_equal(before, after)
            continue
        zeta = sum(np.abs(Xs[i] - Xs[i - 1]) for i in range(k - Kp + 1, k + 1)) / Kp
        keep = zeta >= eps_p
        sure = before & (np.abs(zeta - eps_p) > 1e-9 * eps_p)
        assert np.array_equal(after[sure], keep[sure])
        n_checked += int(sure.sum())
    assert n_checked > 0


def test_freeze_keeps_values_and_matches_plain_optimum(radar_small):
    """P7: frozen pixels keep their value; the pruned (freeze) run reaches the
    plain run's image support with NMSE far below 1e-3."""
    A, sc, base = radar_small
    b = {**base, "eps_rel": 1e-6}
    plain = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, **b))
    pr = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, prune=True, **b),
                      record_iterates=True)
    assert plain.converged and pr.converged and pr.prune_events > 0
    masks = pr.history["masks"]
    for k in range(1, len(masks)):
        gone = ~masks[k - 1]                 # eliminated before iteration k+1
        assert np.array_equal(pr.history["X"][k][gone], pr.history["X"][k - 1][gone])
    nmse = np.linalg.norm(pr.z - plain.z) ** 2 / np.linalg.norm(plain.z) ** 2
    assert nmse < 1e-6
    assert np.array_equal(np.abs(pr.z) > 0, np.abs(plain.z) > 0)


def test_zero_mode_zeroes_eliminated_pixels(radar_small):
    """The literal selector P~_q = P_q^T P_q: eliminated entries of x_q are 0."""
    A, sc, base = radar_small
    pr = oracle.solve(A, sc.y, oracle.Params(max_iter=60, stop=False, prune=True,
                                             mode="zero", **base))
    assert pr.prune_events > 0
    assert np.all(pr.X[~pr.active] == 0)


def test_kkt_reinstates_a_forced_false_prune(radar_small):
    """A pixel of the true optimum's support eliminated from the start (in every
    sensor) violates the optimality condition and is put back."""
    A, sc, base = radar_small
    b = {**base, "eps_rel": 1e-6}
    plain = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, **b))
    supp = np.flatnonzero(np.abs(plain.z) > 0)
    assert supp.size > 0
    mask0 = np.ones((len(A), A[0].shape[1]), bool)
    mask0[:, supp[:3]] = False
    noc = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, prune=True, **b), mask0=mask0)
    assert np.all(noc.z[supp[:3]] == 0)
    fix = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, prune=True, kkt=True, **b),
                       mask0=mask0)
    assert fix.converged and fix.reinstated >= 3
    assert np.all(fix.z[supp[:3]] != 0)
    nmse = np.linalg.norm(fix.z - plain.z) ** 2 / np.linalg.norm(plain.z) ** 2
    assert nmse < 1e-6


def test_kkt_judges_initial_selector_without_ssc(radar_small):
    """An initial selector that eliminates support pixels is re-checked even
    with SSC off (prune=False): the violations are reinstated and the optimum
    of the full problem is reached."""
    A, sc, base = radar_small
    b = {**base, "eps_rel": 1e-6}
    plain = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, **b))
    supp = np.flatnonzero(np.abs(plain.z) > 0)
    mask0 = np.ones((len(A), A[0].shape[1]), bool)
    mask0[:, supp[:3]] = False
    fix = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, kkt=True, **b), mask0=mask0)
    assert fix.converged and fix.reinstated >= 3 and fix.prune_events == 0
    nmse = np.linalg.norm(fix.z - plain.z) ** 2 / np.linalg.norm(plain.z) ** 2
    assert nmse < 1e-6


def test_kkt_round_cap_reports_remaining_violations(radar_small):
    """With no reinstating round allowed, a forced false prune is only checked:
    the solve ends unconverged and reports the violating pixels."""
    A, sc, base = radar_small
    b = {**base, "eps_rel": 1e-6}
    plain = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, **b))
    supp = np.flatnonzero(np.abs(plain.z) > 0)
    mask0 = np.ones((len(A), A[0].shape[1]), bool)
    mask0[:, supp[:3]] = False
    capped = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, kkt=True, kkt_rounds=0, **b),
                          mask0=mask0)
    assert not capped.converged
    assert capped.kkt_violations >= 3 and capped.reinstated == 0
    assert np.all(capped.z[supp[:3]] == 0)


def test_ssc_eliminations_are_not_judged(radar_small):
    """Without an initial selector the re-check has nothing to judge: an
    accelerated solve with kkt=True is the same run, bit for bit."""
    A, sc, base = radar_small
    b = {**base, "eps_rel": 1e-6}
    pr = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, prune=True, **b))
    pk = oracle.solve(A, sc.y, oracle.Params(max_iter=5000, prune=True, kkt=True, **b))
    assert pr.prune_events > 0 and pk.reinstated == 0
    assert pk.iters == pr.iters and np.array_equal(pk.z, pr.z)


def test_elimination_reinstated_exactly_above_the_threshold(radar_small):
    """An eliminated pixel is put back exactly when
    |g_qj| > kkt_tol * lambda (g at the unpruned optimum with that pixel
    moved to 0)."""
    from oracle.sadmm import _reinstate
    A, sc, base = radar_small
    b = {**base, "eps_rel": 1e-12}
    p = oracle.Params(max_iter=20000, **b)
    R = oracle.solve(A, sc.y, p)
    q, j = 1, int(np.argmax(np.abs(R.X[1])))
    X = R.X.copy()
    X[q, j] = 0.0
    g = oracle.kkt_gradient(A, sc.y, X, R.u, p)
    ratio = abs(g[q, j]) / b["lam"]
    assert ratio > 0
    for tol, expect in ((0.5 * ratio, 1), (2.0 * ratio, 0)):
        active = np.ones_like(R.active)
        active[q, j] = False
        back = _reinstate(A, sc.y, X, R.u, oracle.Params(kkt_tol=tol, **b), active,
                          sc.y.copy(), np.zeros((4,) + R.active.shape), check_only=True)
        assert back == expect
