"""Pins of the magnitude variant (Sec. II: x_q real, the image a non-negative
magnitude): the projected threshold against brute force, the real stacked
model against the complex normal equations, and the converged image against
non-negative coordinate descent (Q = 1 and the Q > 1 reduction)."""

import numpy as np
import pytest

import oracle
from pin_helpers import tiny_problem


@pytest.mark.parametrize("v,lam,beta", [(2.0, 1.0, 1.0), (-0.7, 0.3, 2.0), (0.2, 0.5, 1.0),
                                        (1.5 + 0.8j, 0.4, 1.3)])
def test_nonneg_threshold_is_the_projected_prox(v, lam, beta):
    """argmin over z >= 0 of lam z + beta/2 |z - v|^2 on a fine grid."""
    zs = np.linspace(0.0, abs(v) + 2.0, 400001)
    F = lam * zs + 0.5 * beta * np.abs(zs - v) ** 2
    zb = zs[np.argmin(F)]
    got = oracle.nonneg_threshold(np.array([v]), lam / beta)[0]
    assert got.imag == 0.0
    assert got.real == pytest.approx(zb, abs=2e-5)
    assert got.real == max(np.real(v) - lam / beta, 0.0)


def test_stacked_real_model_normal_equations():
    """[Re A; Im A]^T [Re A; Im A] = Re(A^H A) and [Re A; Im A]^T [Re y; Im y]
    = Re(A^H y), so the real x-update solves mu Re(A^H A) + c I."""
    A, y = tiny_problem(Q=2, KM=7, N=9, seed=4)
    As, ys = oracle.stack_real(A, y)
    for a, s_, yy, ysq in zip(A, As, y, ys):
        assert s_.shape == (14, 9) and not s_.imag.any() and not ysq.imag.any()
        assert np.allclose(s_.real.T @ s_.real, np.real(a.conj().T @ a), rtol=1e-13, atol=1e-13)
        assert np.allclose(s_.real.T @ ysq.real, np.real(a.conj().T @ yy), rtol=1e-13, atol=1e-13)


def cd_nonneg(H, b, lam, tol=1e-15, maxit=200000):
    """Coordinate descent for min 1/2 s^T H s - b^T s + lam sum(s), s >= 0
    (H symmetric positive definite): s_j = max(0, b_j - sum_{i!=j} H_ji s_i - lam) / H_jj."""
    n = b.size
    s = np.zeros(n)
    Hs = np.zeros(n)
    for _ in range(maxit):
        delta = 0.0
        for j in range(n):
            rho = b[j] - (Hs[j] - H[j, j] * s[j])
            new = max(0.0, rho - lam) / H[j, j]
            d = new - s[j]
            if d != 0.0:
                Hs += H[:, j] * d
                s[j] = new
                delta = max(delta, abs(d))
        if delta <= tol * max(1.0, np.abs(s).max()):
            break
    return s


def test_single_sensor_nonneg_optimum_equals_coordinate_descent():
    A, y = tiny_problem(Q=1, KM=6, N=14, seed=9)
    As, ys = oracle.stack_real(A, y)
    mu, beta, gamma = 1.2, 0.9, 0.7
    Ar = As[0].real
    G = mu * Ar.T @ Ar + gamma * np.eye(14)
    b = mu * Ar.T @ ys[0].real
    lam = 0.3 * np.abs(b).max()
    p = oracle.Params(mu=mu, beta=beta, gamma=gamma, lam=lam, eps_abs=0, eps_rel=1e-13,
                      max_iter=40000, nonneg=True)
    R = oracle.solve(As, ys, p)
    assert R.converged
    s = cd_nonneg(G, b, lam)
    assert np.count_nonzero(s) > 0 and np.count_nonzero(s) < 14
    assert not R.z.imag.any() and (R.z.real >= 0).all()
    assert np.linalg.norm(R.z.real - s) <= 1e-9 * np.linalg.norm(s)
    # the unconstrained real solution has negative entries: the projection matters
    pu = oracle.Params(mu=mu, beta=beta, gamma=gamma, lam=lam, eps_abs=0, eps_rel=1e-13,
                       max_iter=40000)
    assert (oracle.solve(As, ys, pu).z.real < -1e-6).any()


@pytest.mark.parametrize("Q,KM,N", [(3, 6, 12), (4, 5, 10)])
def test_multi_sensor_nonneg_optimum_equals_reduced_problem(Q, KM, N):
    """Q z* = the non-negative minimiser of the reduced single-variable problem
    (H = (sum_q G_q^-1)^-1, btilde = H sum_q G_q^-1 mu A_q^T y_q, real)."""
    A, y = tiny_problem(Q=Q, KM=KM, N=N, seed=Q * 31 + N)
    As, ys = oracle.stack_real(A, y)
    mu, beta, gamma = 1.1, 0.8, 0.6
    Sinv = np.zeros((N, N))
    rhs = np.zeros(N)
    for a, yy in zip(As, ys):
        Ar = a.real
        Gi = np.linalg.inv(mu * Ar.T @ Ar + gamma * np.eye(N))
        Sinv += Gi
        rhs += Gi @ (mu * Ar.T @ yy.real)
    H = np.linalg.inv(Sinv)
    H = 0.5 * (H + H.T)
    bt = H @ rhs
    lam = 0.25 * np.abs(bt).max()
    p = oracle.Params(mu=mu, beta=beta, gamma=gamma, lam=lam, eps_abs=0, eps_rel=1e-13,
                      max_iter=80000, nonneg=True)
    R = oracle.solve(As, ys, p)
    assert R.converged
    s = cd_nonneg(H, bt, lam)
    assert np.count_nonzero(s) > 0
    assert np.linalg.norm(Q * R.z.real - s) <= 1e-8 * np.linalg.norm(s)
