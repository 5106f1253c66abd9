"""FP64 oracle: plain SADMM and accelerated SADMM (ASADMM) -- test infrastructure.

Only tests, the smoke check, the benchmark's CPU-baseline leg and the scripts
that write stored reference values may use this module.

What is computed, and where it comes from
-----------------------------------------
Problem (Sec. III, eq. (2)), for Q sensors with operators A_q (KM x N) and
measurements y_q (Sec. II, eq. (1)):

    minimise  sum_q [ mu/2 ||y_q - A_q x_q||^2 + gamma/2 ||x_q||^2 ]
              + lambda * || sum_q x_q ||_1

solved with sharing ADMM (the paper's SADMM, after Boyd et al. 2011, Sec. 7.3)
in scaled form, where z is the global image at the scale of the *average*
sub-image xbar = (1/Q) sum_q x_q and u = sigma/beta is the scaled dual:

    x_q <- argmin mu/2||y_q - A_q x||^2 + gamma/2||x||^2
                  + beta/2 ||x - (x_q - xbar + z - u)||^2          (eq. (3), row 1)
    z   <- S_{lambda/beta}(xbar + u)                               (eq. (3), row 2)
    u   <- u + xbar - z                                            (eq. (3), row 3)
    P_q <- SSC(last K_p iterates, eps_p) if ||eta_pri|| <= eps_pri (eq. (3) row 4, Alg. 1)

How the printed equations are read (the paper is silent or inconsistent on
these points; each reading is the one that makes eq. (3) a convergent method):

* The beta-term of the x-update is the sharing-ADMM term x_q - xbar + z - u
  (the printed term lacks x_q and the 1/Q average).  z and u follow the sign
  that agrees between the dual update and the x-update: z = S(xbar + u).
* A ridge gamma/2 ||x_q||^2 per sensor is added (default gamma = beta).  The
  fixed points of the printed x-update are exactly this problem with
  gamma = beta; without it the problem is degenerate (the optimum image is 0
  whenever the sensors' row spaces barely intersect).  With gamma > 0 the
  optimum is unique.  x-update: (mu A^H A + (beta+gamma) I) x = mu A^H y + beta v.
* x_q is complex; S_tau(v) = v * max(0, 1 - tau/|v|), S_tau(0) = 0.
  The magnitude variant (x_q real, the image a non-negative magnitude): the
  real stacked model of stack_real, and with nonneg=True the z-update
  z = max(Re(xbar + u) - tau, 0).  Non-negativity is put on the shared image
  only: on every x_q it would make sum_q x_q >= 0 entrywise, so that
  ||sum_q x_q||_1 = sum_q sum_n x_q[n] and the problem would split into Q
  unrelated non-negative LASSO problems.
* Residuals (the paper defers them to earlier work) follow Boyd Sec. 3.3.1
  on the replicated form: r = sqrt(Q) ||xbar - z||,
  s = beta ||Z^k - Z^{k-1}||_F with Z^k[q] = x_q^k + z^k - xbar^k (Z^0 = 0),
  eps_pri = sqrt(QN) eps_abs + eps_rel max(||X||_F, ||Z^k||_F),
  eps_dual = sqrt(QN) eps_abs + eps_rel beta sqrt(Q) ||u||  (Boyd eq. (3.12)
  on the stacked vectors: Z^k is the replicated shared variable and every
  sensor holds the same scaled dual u).
* SSC (Alg. 1) runs per sensor on that sensor's iterates x_q over its active
  set J_q, with |.| the complex modulus.  zeta_q = (1/K_p) * sum of the K_p
  most recent |x_q^(i) - x_q^(i-1)| (x^(0) = 0 counts); no SSC before K_p
  differences exist; a prune does not reset the window.  The gate is the
  current iteration's r <= eps_pri.  A pixel stays active iff zeta >= eps_p
  (equality stays active), so J only shrinks.  The new selector applies from
  the next iteration.
* Eliminated pixels are frozen (default): x_q[j] keeps its last value, its
  contribution A_q[:, j] x_q[j] moves into the measurement (y'_q), and z, u
  keep updating over all N pixels.  mode="zero" takes the printed
  P~_q = P_q^T P_q literally and zeroes eliminated pixels instead.
* Start: X = 0, z = 0, u = 0, P_q = I (Sec. III).
* Order inside iteration k: x-updates (Jacobi, all sensors from iteration-k
  values) -> xbar -> z -> u -> residuals -> history ring -> stop test -> SSC.

Certificate and reinstatement: at the optimum of the unpruned problem,
g_q = mu A_q^H (A_q x_q - y_q) + gamma x_q + beta u = 0 for every q and pixel.
With `kkt=True`, a solve that starts from an initial selector (mask0: a
caller's or a learned one; its eliminations are frozen at 0) is judged after
convergence: every eliminated pixel with |g_qj| > kkt_tol * lambda -- the
selector's and those SSC removed in the restricted solve -- is put back into
J_q (history window +inf, so no new elimination for K_p iterations) and
iterating resumes.  After kkt_rounds reinstating rounds the next convergence
is only checked: remaining violations leave converged=False and their count
in kkt_violations.  SSC's eliminations in a solve that starts from the full
image are the paper's method (Alg. 1) and are not judged: such a pixel,
frozen at its settled value, keeps a gradient near lambda in its own sensor
(the drift of its per-sensor value times the large column norm) while the
image stays within round-off of the optimum, and no per-pixel test separates
that from a wrong elimination at 0 -- one-step estimates of the move
(coordinate, Schur complement, the thresholded image) certified restricted
solves whose images were far from the optimum.

Each x-update is solved directly from its definition: a Cholesky factor of
mu Ahat^H Ahat + c I when N_q <= KM, otherwise the same solve through the
Woodbury identity with a Cholesky factor of (c/mu) I + Ahat Ahat^H.  Both are
exact up to rounding; which one is used is not part of the method.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np
import scipy.linalg as sla


@dataclass
class Params:
    mu: float = 1.0
    beta: float = 1.0
    gamma: float = 1.0
    lam: float = 0.0
    eps_abs: float = 0.0
    eps_rel: float = 1e-4
    max_iter: int = 200
    stop: bool = True          # stop at the first k with r<=eps_pri and s<=eps_dual
    prune: bool = False        # False: plain SADMM (P_q = I throughout)
    Kp: int = 5
    eps_p: float = 1e-5
    mode: str = "freeze"       # "freeze" or "zero"
    kkt: bool = False
    kkt_tol: float = 1e-2      # reinstate when |g| > kkt_tol * lambda
    kkt_rounds: int = 8
    nonneg: bool = False       # z-update projected on the non-negative reals
    balance_every: int = 0     # residual balancing every this many iterations (0: off)
    balance_mu: float = 10.0   # imbalance ratio that triggers a change
    balance_tau: float = 2.0   # factor beta is multiplied or divided by


@dataclass
class Result:
    z: np.ndarray              # (N,) complex, the global image (average scale)
    X: np.ndarray              # (Q, N) complex, per-sensor images
    u: np.ndarray              # (N,) complex, scaled dual
    active: np.ndarray         # (Q, N) bool, final selector masks
    iters: int
    converged: bool
    prune_events: int
    reinstated: int
    history: dict = field(default_factory=dict)
    kkt_violations: int = 0    # violations left when the reinstatement round cap ended it

    def active_indices(self, q: int) -> np.ndarray:
        return np.flatnonzero(self.active[q])


def nonneg_threshold(v: np.ndarray, tau: float) -> np.ndarray:
    """Proximal map of tau*|.| plus the indicator of the non-negative reals:
    argmin_{z >= 0} tau z + 1/2 |z - v|^2 = max(Re v - tau, 0) (the image as
    a magnitude, Sec. II; the imaginary part of v only adds a constant)."""
    return np.maximum(np.real(v) - tau, 0.0).astype(np.complex128)


def stack_real(A, y):
    """The real form of the model for a real unknown x (Sec. II, x_q the
    magnitude): |y - A x|^2 = |[Re y; Im y] - [Re A; Im A] x|^2, returned as
    complex128 arrays with zero imaginary parts (2 KM rows)."""
    As = [np.vstack([np.real(a), np.imag(a)]).astype(np.complex128) for a in A]
    ys = np.stack([np.concatenate([np.real(v), np.imag(v)]) for v in np.asarray(y)]).astype(np.complex128)
    return As, ys


def soft_threshold(v: np.ndarray, tau: float) -> np.ndarray:
    """Proximal map of tau*|.| on complex entries (eq. (3), row 2)."""
    mag = np.abs(v)
    scale = np.zeros(mag.shape)
    keep = mag > tau
    scale[keep] = 1.0 - tau / mag[keep]
    return v * scale


def _adjoint(A: np.ndarray, w: np.ndarray) -> np.ndarray:
    """A^H w without materialising conj(A)."""
    return (w.conj() @ A).conj()


class _SensorSolve:
    """Exact solve of (mu Ahat^H Ahat + c I) x = b for one sensor."""

    def __init__(self, Ahat: np.ndarray, mu: float, c: float):
        self.Ahat = Ahat
        self.c = c
        km, nq = Ahat.shape
        self.direct = nq <= km
        if nq == 0:
            self.cho = None
        elif self.direct:
            G = mu * (Ahat.conj().T @ Ahat) + c * np.eye(nq)
            self.cho = sla.cho_factor(G, lower=True)
        else:
            G = (c / mu) * np.eye(km) + Ahat @ Ahat.conj().T
            self.cho = sla.cho_factor(G, lower=True)

    def solve(self, b: np.ndarray) -> np.ndarray:
        if self.cho is None:
            return b.copy()
        if self.direct:
            return sla.cho_solve(self.cho, b)
        t = self.Ahat @ b
        w = sla.cho_solve(self.cho, t)
        return (b - _adjoint(self.Ahat, w)) / self.c


def residual_norms(Xn, zn, un, xbn, X, z, xb, beta):
    """r, s, ||X||_F, ||Z||_F, ||u|| for one iteration (replicated-form
    residuals; Z[q] = x_q + z - xbar is sensor q's copy of the shared variable)."""
    Q = Xn.shape[0]
    r = np.sqrt(Q) * np.linalg.norm(xbn - zn)
    Zn = Xn + (zn - xbn)[None, :]
    dZ = Zn - (X + (z - xb)[None, :])
    s = beta * np.linalg.norm(dZ)
    return r, s, np.linalg.norm(Xn), np.linalg.norm(Zn), np.linalg.norm(un)


def kkt_gradient(A: List[np.ndarray], y: np.ndarray, X: np.ndarray, u: np.ndarray,
                 p: Params) -> np.ndarray:
    """g_q = mu A_q^H (A_q x_q - y_q) + gamma x_q + beta u, shape (Q, N)."""
    Q = len(A)
    g = np.empty_like(X)
    for q in range(Q):
        e = A[q] @ X[q] - y[q]
        g[q] = p.mu * _adjoint(A[q], e) + p.gamma * X[q] + p.beta * u
    return g


def solve(A: List[np.ndarray], y: np.ndarray, p: Params,
          mask0: Optional[np.ndarray] = None,
          x_ref: Optional[np.ndarray] = None,
          record_iterates: bool = False) -> Result:
    """Run SADMM (p.prune False) or ASADMM (p.prune True) in FP64.

    A: list of Q complex arrays (KM, N); y: (Q, KM) complex.
    mask0: optional (Q, N) bool initial selector (False = eliminated from the
    start, frozen at x = 0); None means P_q = I.
    x_ref: optional reference image; its NMSE ||z - x_ref||^2/||x_ref||^2 is
    recorded per iteration.
    """
    Q = len(A)
    KM, N = A[0].shape
    A = [np.ascontiguousarray(a, dtype=np.complex128) for a in A]
    y = np.asarray(y, dtype=np.complex128).reshape(Q, KM)
    mu, beta, gamma = float(p.mu), float(p.beta), float(p.gamma)
    c = beta + gamma
    tau = p.lam / beta

    X = np.zeros((Q, N), dtype=np.complex128)
    z = np.zeros(N, dtype=np.complex128)
    u = np.zeros(N, dtype=np.complex128)
    xb = np.zeros(N, dtype=np.complex128)
    active = np.ones((Q, N), dtype=bool) if mask0 is None else np.array(mask0, dtype=bool)
    start_restricted = not active.all()
    yp = y.copy()                                   # y'_q: measurement minus frozen pixels
    D = np.zeros((max(p.Kp, 1), Q, N))              # ring of |x^(i) - x^(i-1)|

    solvers: list = [None] * Q
    b0: list = [None] * Q

    def setup(q):
        J = np.flatnonzero(active[q])
        Ahat = A[q] if J.size == N else np.ascontiguousarray(A[q][:, J])
        solvers[q] = (J, _SensorSolve(Ahat, mu, c))
        b0[q] = mu * _adjoint(Ahat, yp[q])

    for q in range(Q):
        setup(q)

    hist = {k: [] for k in ("r", "s", "eps_pri", "eps_dual", "max_active_frac",
                            "active", "nmse", "pruned", "beta")}
    if record_iterates:
        hist["X"], hist["z"], hist["u"], hist["masks"] = [], [], [], []
    prune_events = 0
    reinstated = 0
    kkt_rounds = 0
    violations = 0
    converged = False
    k = 0
    sqQN = np.sqrt(Q * N)
    while k < p.max_iter:
        k += 1
        # x-updates (eq. (3), row 1), all sensors from iteration-k values
        Xn = X.copy()
        for q in range(Q):
            J, sv = solvers[q]
            if J.size == 0:
                continue
            v = (X[q] - xb + z - u)[J]
            Xn[q, J] = sv.solve(b0[q] + beta * v)
        xbn = Xn.mean(axis=0)
        zn = (nonneg_threshold if p.nonneg else soft_threshold)(xbn + u, tau)   # eq. (3), row 2
        un = u + xbn - zn                                 # eq. (3), row 3
        r, s, nX, nZ, nu = residual_norms(Xn, zn, un, xbn, X, z, xb, beta)
        eps_pri = sqQN * p.eps_abs + p.eps_rel * max(nX, nZ)
        eps_dual = sqQN * p.eps_abs + p.eps_rel * beta * np.sqrt(Q) * nu
        # history of per-pixel changes over the active set (Alg. 1, step 1)
        slot = (k - 1) % D.shape[0]
        for q in range(Q):
            J = solvers[q][0]
            D[slot, q, J] = np.abs(Xn[q, J] - X[q, J])
        hist["r"].append(r)
        hist["s"].append(s)
        hist["eps_pri"].append(eps_pri)
        hist["eps_dual"].append(eps_dual)
        if x_ref is not None:
            hist["nmse"].append(float(np.linalg.norm(zn - x_ref) ** 2
                                      / max(np.linalg.norm(x_ref) ** 2, 1e-300)))
        X, z, u, xb = Xn, zn, un, xbn
        done = p.stop and r <= eps_pri and s <= eps_dual
        pruned_now = 0
        if (not done) and p.prune and k >= p.Kp and r <= eps_pri:
            # Alg. 1: keep pixels whose mean recent change is >= eps_p
            zeta = D.sum(axis=0) / p.Kp
            for q in range(Q):
                J = solvers[q][0]
                if J.size == 0:
                    continue
                keep = zeta[q, J] >= p.eps_p
                if keep.all():
                    continue
                gone = J[~keep]
                if p.mode == "freeze":
                    yp[q] = yp[q] - A[q][:, gone] @ X[q, gone]
                else:
                    X[q, gone] = 0.0
                active[q, gone] = False
                pruned_now += gone.size
                setup(q)
            if pruned_now:
                prune_events += 1
        hist["pruned"].append(pruned_now)
        # residual balancing (Boyd et al. 2011, Sec. 3.4.1): beta up when the
        # primal residual dominates, down when the dual one does; the scaled
        # dual is rescaled so that the unscaled one (beta u) is unchanged, and
        # every x-update is refactored for the new c = beta + gamma
        if (not done) and p.balance_every > 0 and k % p.balance_every == 0 and k < p.max_iter:
            f = 1.0
            if r > p.balance_mu * s:
                f = p.balance_tau
            elif s > p.balance_mu * r:
                f = 1.0 / p.balance_tau
            if f != 1.0:
                u = u / f
                beta *= f
                c = beta + gamma
                tau = p.lam / beta
                for q in range(Q):
                    setup(q)
        hist["beta"].append(beta)
        counts = active.sum(axis=1)
        hist["active"].append(counts.copy())
        hist["max_active_frac"].append(float(counts.max()) / N)
        if record_iterates:
            hist["X"].append(X.copy())
            hist["z"].append(z.copy())
            hist["u"].append(u.copy())
            hist["masks"].append(active.copy())
        if done:
            if p.kkt and start_restricted and (~active).any():
                if kkt_rounds >= p.kkt_rounds:
                    left = _reinstate(A, y, X, u, replace(p, beta=beta), active, yp, D, check_only=True)
                    if left:
                        violations = left
                        break
                else:
                    kkt_rounds += 1
                    back = _reinstate(A, y, X, u, replace(p, beta=beta), active, yp, D)
                    if back:
                        reinstated += back
                        for q in range(Q):
                            setup(q)
                        continue
            converged = True
            break
    return Result(z=z, X=X, u=u, active=active, iters=k, converged=converged,
                  prune_events=prune_events, reinstated=reinstated, history=hist,
                  kkt_violations=violations)


def _reinstate(A, y, X, u, p, active, yp, D, check_only=False) -> int:
    """Put eliminated pixels that violate the optimality condition,
    |g_qj| > kkt_tol * lambda, back (only count them when check_only)."""
    g = kkt_gradient(A, y, X, u, p)
    thr = p.kkt_tol * (p.lam if p.lam > 0 else 1.0)
    back = 0
    for q in range(len(A)):
        bad = np.flatnonzero((~active[q]) & (np.abs(g[q]) > thr))
        if bad.size == 0:
            continue
        if check_only:
            back += bad.size
            continue
        if p.mode == "freeze":
            yp[q] = yp[q] + A[q][:, bad] @ X[q, bad]
        active[q, bad] = True
        D[:, q, bad] = np.inf
        back += bad.size
    return back


def matched_filter(A: List[np.ndarray], y: np.ndarray) -> np.ndarray:
    """|A_q^H y_q| per sensor and pixel, shape (Q, N): the back-projection image
    of each sensor (the data term's gradient at x = 0, up to mu)."""
    return np.stack([np.abs(_adjoint(np.asarray(a), np.asarray(yy))) for a, yy in zip(A, y)])
