"""Smallest l1 weight whose optimum global image is zero -- test infrastructure.

For  min sum_q f_q(x_q) + lambda ||sum_q x_q||_1  with
f_q(x) = mu/2 ||y_q - A_q x||^2 + gamma/2 ||x||^2, the optimum has
sum_q x_q = 0 exactly when every x_q solves grad f_q(x_q) = -g for one common
g with |g_j| <= lambda.  grad f_q(x) = G_q x - mu A_q^H y_q, G_q = mu A_q^H A_q
+ gamma I, so x_q = R_q (mu A_q^H y_q - g) with R_q = G_q^{-1}, and
sum_q x_q = 0 gives

    g = sigma0 = (sum_q R_q)^{-1} sum_q R_q mu A_q^H y_q,
    lambda_max = max_j |sigma0_j|.

For Q = 1 this is mu * max|A^H y|.  Small N: dense Cholesky of G_q.  Large N:
R_q v = (1/gamma) (v - A^H (gamma/mu I + A A^H)^{-1} A v) (Woodbury) and the
outer solve by conjugate gradients on the Hermitian positive definite sum_q R_q.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _adjoint(A, w):
    return (w.conj() @ A).conj()


def lambda_max(A, y, mu: float, gamma: float, dense_limit: int = 4096,
               cg_tol: float = 1e-13, cg_maxit: int = 5000) -> float:
    Q = len(A)
    KM, N = A[0].shape
    if gamma <= 0:
        raise ValueError("lambda_max needs gamma > 0")
    rhs_q = [mu * _adjoint(A[q], y[q]) for q in range(Q)]
    if N <= dense_limit:
        S = np.zeros((N, N), dtype=np.complex128)
        rhs = np.zeros(N, dtype=np.complex128)
        for q in range(Q):
            G = mu * (A[q].conj().T @ A[q]) + gamma * np.eye(N)
            cho = sla.cho_factor(G, lower=True)
            S += sla.cho_solve(cho, np.eye(N))
            rhs += sla.cho_solve(cho, rhs_q[q])
        sigma0 = np.linalg.solve(S, rhs)
        return float(np.abs(sigma0).max())

    chos = []
    for q in range(Q):
        Wm = (gamma / mu) * np.eye(KM) + A[q] @ A[q].conj().T
        chos.append(sla.cho_factor(Wm, lower=True))

    def R(q, v):
        w = sla.cho_solve(chos[q], A[q] @ v)
        return (v - _adjoint(A[q], w)) / gamma

    def S(v):
        return sum(R(q, v) for q in range(Q))

    rhs = sum(R(q, rhs_q[q]) for q in range(Q))
    # conjugate gradients on S sigma = rhs
    x = np.zeros(N, dtype=np.complex128)
    r = rhs.copy()
    pdir = r.copy()
    rr = np.vdot(r, r).real
    nrm0 = np.sqrt(rr)
    for _ in range(cg_maxit):
        if np.sqrt(rr) <= cg_tol * nrm0:
            break
        Sp = S(pdir)
        alpha = rr / np.vdot(pdir, Sp).real
        x += alpha * pdir
        r -= alpha * Sp
        rr_new = np.vdot(r, r).real
        pdir = r + (rr_new / rr) * pdir
        rr = rr_new
    return float(np.abs(x).max())
