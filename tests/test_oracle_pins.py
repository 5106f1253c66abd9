"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test targets a plausible mistake: a wrong threshold or sign in the
z-update, a dropped 1/Q, a swapped mu/beta/gamma, a wrong residual, a wrong
SSC window or comparison direction, a broken freeze bookkeeping.  Parameters
deliberately use mu != beta != gamma != 1.
"""

import numpy as np
import pytest

import oracle
from oracle.sadmm import _SensorSolve
from tests.pin_helpers import (cd_quadratic_l1, lasso_admm_boyd, misfit_gradient_fd,
                               prox_bruteforce, sharing_admm_replicated, sharing_reduction,
                               tiny_problem)


# ---------------------------------------------------------------- z-update (eq. (3), row 2)

@pytest.mark.parametrize("v,lam,beta", [(1.3 - 0.7j, 0.5, 2.0), (0.2 + 0.1j, 0.9, 3.0),
                                        (-2.0 + 0.0j, 1.0, 0.5), (0.4j, 0.3, 1.7)])
def test_soft_threshold_is_the_prox(v, lam, beta):
    """P1: S_{lam/beta}(v) minimises lam|z| + beta/2|z-v|^2 (brute-force 2-D search)."""
    z = oracle.soft_threshold(np.array([v]), lam / beta)[0]
    zb = prox_bruteforce(v, lam, beta)
    assert abs(z - zb) < 1e-5


def test_soft_threshold_real_axis_textbook():
    """P1: on the real axis it is sign(v) max(|v| - tau, 0)."""
    v = np.linspace(-3, 3, 61)
    tau = 0.75
    got = oracle.soft_threshold(v.astype(complex), tau)
    assert np.allclose(got.imag, 0)
    assert np.allclose(got.real, np.sign(v) * np.maximum(np.abs(v) - tau, 0), atol=1e-15)
    assert oracle.soft_threshold(np.zeros(3, complex), 0.1).tolist() == [0, 0, 0]


# ---------------------------------------------------------------- x-update (eq. (3), row 1)

@pytest.mark.parametrize("KM,N", [(12, 7), (8, 20)])
def test_sensor_solve_matches_dense_system(KM, N):
    """P2: both factor paths (direct N_q x N_q and Woodbury KM x KM) solve
    (mu A^H A + c I) x = b exactly."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((KM, N)) + 1j * rng.standard_normal((KM, N))
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    mu, c = 2.5, 0.7
    x = _SensorSolve(A, mu, c).solve(b)
    ref = np.linalg.solve(mu * A.conj().T @ A + c * np.eye(N), b)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


# ---------------------------------------------------------------- whole solver, special cases

def test_single_sensor_equals_boyd_lasso_admm():
    """P3: with Q = 1 sharing ADMM is the textbook LASSO ADMM (same iterates,
    same residuals and tolerances)."""
    A, y = tiny_problem(Q=1, KM=10, N=16, seed=5)
    mu, beta, gamma, lam = 1.7, 2.3, 0.4, 0.8
    p = oracle.Params(mu=mu, beta=beta, gamma=gamma, lam=lam, eps_abs=1e-6, eps_rel=1e-4,
                      max_iter=40, stop=False)
    R = oracle.solve(A, y, p, record_iterates=True)
    ref = lasso_admm_boyd(A[0], y[0], mu, beta, gamma, lam, 40, 1e-6, 1e-4)
    for k in range(40):
        zk, r, s, ep, ed = ref[k]
        assert np.allclose(R.history["z"][k], zk, rtol=0, atol=1e-12)
        assert R.history["r"][k] == pytest.approx(r, rel=1e-9, abs=1e-14)
        assert R.history["s"][k] == pytest.approx(s, rel=1e-9, abs=1e-14)
        assert R.history["eps_pri"][k] == pytest.approx(ep, rel=1e-12)
        assert R.history["eps_dual"][k] == pytest.approx(ed, rel=1e-12)


@pytest.mark.parametrize("Q,KM,N,seed", [(3, 8, 14, 3), (4, 6, 16, 4)])
def test_multi_sensor_iterates_and_residuals_equal_replicated_form(Q, KM, N, seed):
    """Q > 1: the oracle's iterates, residuals r and s, and tolerances eps_pri
    and eps_dual equal those of the sharing problem run as general two-block
    ADMM with the shared variable replicated per sensor (Boyd Sec. 7.3 set up
    in the form of Sec. 3, residuals and eq. (3.12) on the stacked vectors).
    Both tolerance terms are non-zero, so a missing sqrt(Q) in r, in eps_pri's
    absolute term or in eps_dual, or sqrt(N) in place of sqrt(QN), all fail."""
    A, y = tiny_problem(Q=Q, KM=KM, N=N, seed=seed)
    mu, beta, gamma = 1.3, 0.7, 0.9
    lam = 0.3 * oracle.lambda_max(A, y, mu, gamma)
    eps_abs, eps_rel = 2e-3, 3e-2
    p = oracle.Params(mu=mu, beta=beta, gamma=gamma, lam=lam, eps_abs=eps_abs, eps_rel=eps_rel,
                      max_iter=30, stop=False)
    R = oracle.solve(A, y, p, record_iterates=True)
    ref = sharing_admm_replicated(A, y, mu, beta, gamma, lam, 30, eps_abs, eps_rel)
    nz = 0
    for k in range(30):
        x, zb, r, s, ep, ed = ref[k]
        assert np.allclose(R.history["X"][k], x, rtol=0, atol=1e-12)
        assert np.allclose(R.history["z"][k], zb, rtol=0, atol=1e-12)
        assert R.history["r"][k] == pytest.approx(r, rel=1e-9, abs=1e-14)
        assert R.history["s"][k] == pytest.approx(s, rel=1e-9, abs=1e-14)
        assert R.history["eps_pri"][k] == pytest.approx(ep, rel=1e-12)
        assert R.history["eps_dual"][k] == pytest.approx(ed, rel=1e-12)
        nz += np.count_nonzero(zb)
        # |u_j| <= lam/beta after every z-update, so |z_j| <= |xbar_j| and
        # ||Z||_F <= ||X||_F: the tolerance's max is always ||X||_F
        Xk = R.history["X"][k]
        assert R.history["eps_pri"][k] == pytest.approx(
            np.sqrt(Q * N) * eps_abs + eps_rel * np.linalg.norm(Xk), rel=1e-12)
        assert np.all(np.abs(R.history["u"][k]) <= lam / beta * (1 + 1e-12))
    assert nz > 0                                   # the l1 term is active


def test_matched_filter_is_misfit_gradient_modulus():
    """The matched filter |A_q^H y_q| is the modulus of the gradient of
    1/2||y_q - A_q x||^2 at x = 0 (central differences, exact for a
    quadratic), and equals a scalar double loop over rows and pixels."""
    A, y = tiny_problem(Q=3, KM=7, N=9, seed=8)
    mf = oracle.matched_filter(A, y)
    assert mf.shape == (3, 9)
    for q in range(3):
        g = misfit_gradient_fd(A[q], y[q])
        assert np.allclose(mf[q], np.abs(g), rtol=1e-9, atol=1e-12)
        for n in range(9):
            acc = 0j
            for i in range(7):
                acc += A[q][i, n].conjugate() * y[q][i]
            assert mf[q, n] == pytest.approx(abs(acc), rel=1e-13)


def test_single_sensor_optimum_equals_coordinate_descent():
    """P3: converged Q=1 image equals complex CD-LASSO (underdetermined A)."""
    A, y = tiny_problem(Q=1, KM=8, N=20, seed=6)
    mu, beta, gamma, lam = 1.3, 0.9, 0.6, 0.5
    p = oracle.Params(mu=mu, beta=beta, gamma=gamma, lam=lam, eps_abs=0, eps_rel=1e-13,
                      max_iter=20000)
    R = oracle.solve(A, y, p)
    assert R.converged
    G = mu * A[0].conj().T @ A[0] + gamma * np.eye(20)
    s = cd_quadratic_l1(G, mu * A[0].conj().T @ y[0], lam)
    assert np.linalg.norm(R.z - s) <= 1e-9 * np.linalg.norm(s)
    assert np.count_nonzero(s) > 0


@pytest.mark.parametrize("Q,KM,N,gamma", [(3, 8, 16, 0.5), (3, 24, 12, 0.0), (4, 6, 14, 1.2)])
def test_multi_sensor_optimum_equals_reduced_lasso(Q, KM, N, gamma):
    """P4: Q * z* equals the minimiser of the single-variable problem the
    sharing problem reduces to (inf-convolution), found by coordinate descent."""
    A, y = tiny_problem(Q=Q, KM=KM, N=N, seed=Q * 100 + N)
    mu, beta = 1.4, 0.8
    H, bt = sharing_reduction(A, y, mu, gamma)
    lam = 0.3 * np.abs(bt).max()
    p = oracle.Params(mu=mu, beta=beta, gamma=gamma, lam=lam, eps_abs=0, eps_rel=1e-13,
                      max_iter=50000)
    R = oracle.solve(A, y, p)
    assert R.converged
    s = cd_quadratic_l1(H, bt, lam)
    assert np.count_nonzero(s) > 0
    assert np.linalg.norm(Q * R.z - s) <= 1e-8 * np.linalg.norm(s)


def test_he_yuan_quantity_non_increasing():
    """P5: for two-block ADMM, beta||dZ||^2 + beta Q ||du||^2 = s^2/beta + beta r^2
    never increases (He & Yuan 2015); and r, s -> 0."""
    A, y = tiny_problem(Q=4, KM=10, N=24, seed=11)
    beta = 1.9
    p = oracle.Params(mu=0.8, beta=beta, gamma=0.7, lam=0.4, eps_abs=0, eps_rel=0,
                      max_iter=300, stop=False)
    R = oracle.solve(A, y, p)
    r = np.array(R.history["r"])
    s = np.array(R.history["s"])
    hy = s ** 2 / beta + beta * r ** 2
    # skip the first step (Z^0 = 0 is not an ADMM iterate of the z-block)
    d = np.diff(hy[1:])
    assert np.all(d <= 1e-12 * hy[1:-1] + 1e-28)
    assert r[-1] < 1e-8 * r[0] and s[-1] < 1e-8 * s[0]


def test_kkt_certificate_at_optimum():
    """P8: at a tight optimum g_q = mu A^H(Ax-y) + gamma x + beta u = 0, |beta u| <= lam,
    and beta u = lam z/|z| on the support."""
    A, y = tiny_problem(Q=3, KM=10, N=18, seed=21)
    p = oracle.Params(mu=1.1, beta=0.7, gamma=0.9, lam=0.6, eps_abs=0, eps_rel=1e-13,
                      max_iter=50000)
    R = oracle.solve(A, y, p)
    assert R.converged
    g = oracle.kkt_gradient(A, y, R.X, R.u, p)
    scale = max(1.0, np.abs(p.mu * A[0].conj().T @ y[0]).max())
    assert np.abs(g).max() <= 1e-8 * scale
    bu = p.beta * R.u
    assert np.all(np.abs(bu) <= p.lam * (1 + 1e-9))
    sup = np.abs(R.z) > 0
    assert sup.any()
    assert np.allclose(bu[sup], p.lam * R.z[sup] / np.abs(R.z[sup]), atol=1e-8 * p.lam)


def test_lambda_max_boundary():
    """P9: lambda >= lambda_max gives z* = 0; slightly below gives z* != 0."""
    A, y = tiny_problem(Q=3, KM=10, N=16, seed=31)
    mu, gamma = 1.2, 0.8
    lm = oracle.lambda_max(A, y, mu, gamma)
    base = dict(mu=mu, beta=1.5, gamma=gamma, eps_abs=0, eps_rel=1e-12, max_iter=50000)
    hi = oracle.solve(A, y, oracle.Params(lam=1.001 * lm, **base))
    lo = oracle.solve(A, y, oracle.Params(lam=0.98 * lm, **base))
    assert np.abs(hi.z).max() == 0.0
    assert np.abs(lo.z).max() > 0.0


def test_lambda_max_single_sensor_and_cg_path():
    """P9: for Q = 1, lambda_max = mu max|A^H y|; the CG path equals the dense one."""
    A, y = tiny_problem(Q=1, KM=9, N=15, seed=41)
    assert oracle.lambda_max(A, y, 1.7, 0.3) == pytest.approx(
        1.7 * np.abs(A[0].conj().T @ y[0]).max(), rel=1e-10)
    A, y = tiny_problem(Q=3, KM=6, N=20, seed=42)
    d = oracle.lambda_max(A, y, 1.1, 0.6)
    c = oracle.lambda_max(A, y, 1.1, 0.6, dense_limit=0)
    assert c == pytest.approx(d, rel=1e-9)


def test_ridge_free_problem_is_degenerate_on_radar_geometry():
    """P10: with gamma = 0 and sensors whose row spaces barely intersect, the
    image is driven to zero (why the ridge is added)."""
    from scenegen import make_geometry, make_scene, steering
    g = make_geometry(Q=4, M=2, K=16, n_side=12)
    sc = make_scene(g, 0, 4, 20.0)
    A = [steering(g, q) for q in range(g.Q)]
    lam = 0.2 * oracle.lambda_max(A, sc.y, 1.0, 1.0)
    base = dict(mu=1.0, beta=1.0, lam=lam, eps_abs=0, eps_rel=0, max_iter=400, stop=False)
    z0 = oracle.solve(A, sc.y, oracle.Params(gamma=0.0, **base)).z
    z1 = oracle.solve(A, sc.y, oracle.Params(gamma=1.0, **base)).z
    assert np.linalg.norm(z0) < 1e-3 * np.linalg.norm(z1) or np.linalg.norm(z0) == 0.0
