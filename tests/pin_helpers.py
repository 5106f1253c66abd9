"""Independent textbook routines the oracle is pinned against.

None of these reuse the oracle's code; each is a different algorithm (or the
brute-force definition) for a quantity the oracle also produces.
"""

import numpy as np


def tiny_problem(Q=3, KM=8, N=12, seed=0, scale=1.0):
    """Random complex operators/measurements small enough for brute force."""
    rng = np.random.default_rng(seed)
    A = [(rng.standard_normal((KM, N)) + 1j * rng.standard_normal((KM, N))) / np.sqrt(2)
         for _ in range(Q)]
    xt = np.zeros((Q, N))
    sup = rng.choice(N, size=max(1, N // 4), replace=False)
    for q in range(Q):
        xt[q, sup] = rng.uniform(0.5, 1.0, size=sup.size)
    y = np.stack([A[q] @ xt[q] for q in range(Q)])
    y = y + 0.05 * (rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape))
    return A, scale * y


def prox_bruteforce(v, lam, beta, half_width=None, n=801):
    """argmin_z lam|z| + beta/2 |z - v|^2 by exhaustive search on a 2-D grid,
    refined twice around the best point."""
    if half_width is None:
        half_width = abs(v) + 1.0
    cx, cy, hw = 0.0, 0.0, half_width
    best = 0j
    for _ in range(3):
        xs = np.linspace(cx - hw, cx + hw, n)
        ys = np.linspace(cy - hw, cy + hw, n)
        Z = xs[None, :] + 1j * ys[:, None]
        F = lam * np.abs(Z) + 0.5 * beta * np.abs(Z - v) ** 2
        i = np.unravel_index(np.argmin(F), F.shape)
        best = Z[i]
        cx, cy, hw = best.real, best.imag, 4 * hw / (n - 1)
    return best


def cd_quadratic_l1(H, b, lam, tol=1e-15, maxit=200000):
    """Complex coordinate descent for  min 1/2 s^H H s - Re(b^H s) + lam ||s||_1
    (H Hermitian positive definite).  Each coordinate step is exact:
    s_j = S_lam(b_j - sum_{i != j} H_ji s_i) / H_jj."""
    n = b.size
    s = np.zeros(n, dtype=np.complex128)
    Hs = np.zeros(n, dtype=np.complex128)
    for _ in range(maxit):
        delta = 0.0
        for j in range(n):
            hjj = H[j, j].real
            rho = b[j] - (Hs[j] - hjj * s[j])
            m = abs(rho)
            new = 0j if m <= lam else rho * (1 - lam / m) / hjj
            d = new - s[j]
            if d != 0:
                Hs += H[:, j] * d
                s[j] = new
                delta = max(delta, abs(d))
        if delta <= tol * max(1.0, np.abs(s).max()):
            break
    return s


def sharing_reduction(A, y, mu, gamma):
    """H, btilde of the single-variable problem in s = sum_q x_q that the
    Q-sensor problem reduces to (inf-convolution of the per-sensor quadratics):
    H = (sum_q G_q^-1)^-1, btilde = H sum_q G_q^-1 mu A_q^H y_q,
    G_q = mu A_q^H A_q + gamma I."""
    N = A[0].shape[1]
    Sinv = np.zeros((N, N), dtype=np.complex128)
    rhs = np.zeros(N, dtype=np.complex128)
    for a, yy in zip(A, y):
        G = mu * a.conj().T @ a + gamma * np.eye(N)
        Gi = np.linalg.inv(G)
        Sinv += Gi
        rhs += Gi @ (mu * a.conj().T @ yy)
    H = np.linalg.inv(Sinv)
    H = 0.5 * (H + H.conj().T)
    return H, H @ rhs


def lasso_admm_boyd(A, y, mu, beta, gamma, lam, iters, eps_abs, eps_rel):
    """Boyd et al. 2011 Sec. 6.4 LASSO ADMM (one block x, one block z) for
    min mu/2||y-Ax||^2 + gamma/2||x||^2 + lam||z||_1, x = z, scaled form,
    with the Sec. 3.3.1 residuals and tolerances.  Returns per-iteration
    (z, r, s, eps_pri, eps_dual)."""
    N = A.shape[1]
    M = mu * A.conj().T @ A + (gamma + beta) * np.eye(N)
    Minv = np.linalg.inv(M)
    Aty = mu * A.conj().T @ y
    x = np.zeros(N, complex)
    z = np.zeros(N, complex)
    u = np.zeros(N, complex)
    out = []
    for _ in range(iters):
        x = Minv @ (Aty + beta * (z - u))
        v = x + u
        m = np.abs(v)
        zn = np.where(m > lam / beta, v * (1 - (lam / beta) / np.maximum(m, 1e-300)), 0)
        u = u + x - zn
        r = np.linalg.norm(x - zn)
        s = beta * np.linalg.norm(zn - z)
        z = zn
        ep = np.sqrt(N) * eps_abs + eps_rel * max(np.linalg.norm(x), np.linalg.norm(z))
        ed = np.sqrt(N) * eps_abs + eps_rel * np.linalg.norm(beta * u)
        out.append((z.copy(), r, s, ep, ed))
    return out


def sharing_admm_replicated(A, y, mu, beta, gamma, lam, iters, eps_abs, eps_rel):
    """Boyd et al. 2011 Sec. 7.3 sharing problem written in the general
    two-block form of Sec. 3 with the shared variable replicated per sensor:

        min sum_i f_i(x_i) + g(sum_i z_i)   s.t.  x_i - z_i = 0,
        f_i(x) = mu/2||y_i - A_i x||^2 + gamma/2||x||^2,  g(s) = lam ||s||_1

    (the l1 term on the sum of sub-images).  Every block keeps its own z_i and
    u_i (Q copies, no averaging shortcut).  The x-step is a dense solve per
    sensor; the z-step is the joint prox of lam||sum z_i||_1 over the stacked
    z, solved per pixel in closed form (for a fixed sum s the stacked
    minimiser is z_i = v_i + (s - V)/Q with V = sum_i v_i, and s itself is the
    prox of lam Q/beta |.| at V).  Residuals and tolerances are Sec. 3.3.1's,
    eq. (3.12), on the stacked vectors with A = I, B = -I, c = 0:
    r = ||x - z||, s = beta ||z^k - z^{k-1}||, eps_pri = sqrt(p) eps_abs +
    eps_rel max(||x||, ||z||), eps_dual = sqrt(n) eps_abs + eps_rel ||beta u||,
    with p = n = Q N (complex entries).

    Returns per iteration (x, zbar, r, s, eps_pri, eps_dual), zbar = mean_i z_i.
    """
    Q = len(A)
    N = A[0].shape[1]
    Ms = [mu * a.conj().T @ a + (gamma + beta) * np.eye(N) for a in A]
    rhs0 = [mu * a.conj().T @ yy for a, yy in zip(A, y)]
    x = np.zeros((Q, N), complex)
    z = np.zeros((Q, N), complex)
    u = np.zeros((Q, N), complex)
    out = []
    for _ in range(iters):
        x = np.stack([np.linalg.solve(Ms[i], rhs0[i] + beta * (z[i] - u[i])) for i in range(Q)])
        v = x + u
        V = v.sum(axis=0)
        t = lam * Q / beta
        m = np.abs(V)
        S = np.where(m > t, V * (1.0 - t / np.maximum(m, 1e-300)), 0.0)
        zn = v + (S - V)[None, :] / Q
        u = u + x - zn
        r = np.linalg.norm((x - zn).ravel())
        s = beta * np.linalg.norm((zn - z).ravel())
        z = zn
        dim = Q * N
        ep = np.sqrt(dim) * eps_abs + eps_rel * max(np.linalg.norm(x.ravel()), np.linalg.norm(z.ravel()))
        ed = np.sqrt(dim) * eps_abs + eps_rel * np.linalg.norm((beta * u).ravel())
        out.append((x.copy(), z.mean(axis=0), r, s, ep, ed))
    return out


def misfit_gradient_fd(A, y, h=1e-3):
    """Gradient of the data misfit f(x) = 1/2 ||y - A x||^2 at x = 0 by central
    differences along the real and imaginary unit directions of each pixel
    (exact up to rounding for a quadratic).  Returns the complex gradient
    df/dRe(x_n) + i df/dIm(x_n), whose modulus is |a_n^H y|."""
    N = A.shape[1]
    g = np.zeros(N, complex)
    f = lambda x: 0.5 * np.linalg.norm(y - A @ x) ** 2
    for n in range(N):
        e = np.zeros(N, complex)
        e[n] = h
        gr = (f(e) - f(-e)) / (2 * h)
        e[n] = 1j * h
        gi = (f(e) - f(-e)) / (2 * h)
        g[n] = gr + 1j * gi
    return g


def lasso_admm_boyd_balanced(A, y, mu, beta, gamma, lam, iters, eps_abs, eps_rel, every,
                             mu_b=10.0, tau_b=2.0):
    """lasso_admm_boyd with Boyd et al. 2011 Sec. 3.4.1 residual balancing:
    after iteration k (k a multiple of `every`), rho <- tau rho if r > mu_b s,
    rho <- rho / tau if s > mu_b r, the scaled dual divided by the same factor
    (the unscaled dual rho u is unchanged).  Returns per-iteration
    (z, r, s, eps_pri, eps_dual, rho after the iteration)."""
    N = A.shape[1]
    AhA = mu * A.conj().T @ A
    Aty = mu * A.conj().T @ y
    rho = beta
    Minv = np.linalg.inv(AhA + (gamma + rho) * np.eye(N))
    x = np.zeros(N, complex)
    z = np.zeros(N, complex)
    u = np.zeros(N, complex)
    out = []
    for k in range(1, iters + 1):
        x = Minv @ (Aty + rho * (z - u))
        v = x + u
        m = np.abs(v)
        zn = np.where(m > lam / rho, v * (1 - (lam / rho) / np.maximum(m, 1e-300)), 0)
        u = u + x - zn
        r = np.linalg.norm(x - zn)
        s = rho * np.linalg.norm(zn - z)
        z = zn
        ep = np.sqrt(N) * eps_abs + eps_rel * max(np.linalg.norm(x), np.linalg.norm(z))
        ed = np.sqrt(N) * eps_abs + eps_rel * np.linalg.norm(rho * u)
        if k % every == 0 and k < iters:
            f = tau_b if r > mu_b * s else (1.0 / tau_b if s > mu_b * r else 1.0)
            if f != 1.0:
                rho *= f
                u = u / f
                Minv = np.linalg.inv(AhA + (gamma + rho) * np.eye(N))
        out.append((z.copy(), r, s, ep, ed, rho))
    return out
