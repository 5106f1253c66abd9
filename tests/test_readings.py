"""CPU checks of two engine readings that the oracle does not model (it works
on the exact FP64 operator): the direct x-update form used for small active
sets, and the correction of a rounded (16-bit) operator.

Both are identities of linear algebra, checked here with NumPy on small
random problems so that a mistake in the formulas (a dropped term, a sign, the
wrong operator in one place) fails.
"""

import numpy as np


def _problem(seed=0, KM=24, N=40):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((KM, N)) + 1j * rng.standard_normal((KM, N))) / np.sqrt(2)
    y = rng.standard_normal(KM) + 1j * rng.standard_normal(KM)
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return A, y, v


def _xupd(A, y, v, mu, beta, c):
    """Minimiser of (mu/2)|A x - y|^2 + (beta/2)|x - v|^2 + ((c - beta)/2)|x|^2."""
    N = A.shape[1]
    return np.linalg.solve(mu * A.conj().T @ A + c * np.eye(N), mu * A.conj().T @ y + beta * v)


def test_direct_and_woodbury_forms_agree():
    """x = (mu A^H A + cI)^{-1}(mu A^H y + beta v) (direct, order N) equals
    A^H W y + (beta/c)(v - A^H W A v) with W = ((c/mu) I + A A^H)^{-1} (order KM)."""
    mu, beta, gamma = 1.3, 0.7, 0.9
    c = beta + gamma
    for seed, (KM, N) in enumerate([(24, 40), (40, 24), (16, 16)]):
        A, y, v = _problem(seed, KM, N)
        direct = _xupd(A, y, v, mu, beta, c)
        W = np.linalg.inv((c / mu) * np.eye(KM) + A @ A.conj().T)
        wood = A.conj().T @ W @ y + (beta / c) * (v - A.conj().T @ W @ A @ v)
        np.testing.assert_allclose(wood, direct, rtol=1e-11, atol=1e-12)


def _round16(A, bits):
    """Real and imaginary parts rounded to `bits` significant bits."""
    def r(x):
        m, e = np.frexp(x)
        return np.ldexp(np.round(m * 2.0 ** bits) / 2.0 ** bits, e)
    return r(A.real) + 1j * r(A.imag)


def test_correction_fixed_point_is_the_accurate_update():
    """With the stored operator Ahat (rounded) and the accurate A, iterating
    x <- (mu Ahat^H Ahat + cI)^{-1}(mu Ahat^H y + beta v + g(x)),
    g(x) = mu (A^H (y - A x) - Ahat^H (y - Ahat x)),
    converges to the x-update of A itself; without g it stops at Ahat's."""
    mu, beta, gamma = 1.0, 1.0, 1.0
    c = beta + gamma
    A, y, v = _problem(3, 32, 48)
    for bits in (8, 11):                     # BF16 and FP16 significands
        Ah = _round16(A, bits)
        exact = _xupd(A, y, v, mu, beta, c)
        plain = _xupd(Ah, y, v, mu, beta, c)
        assert np.linalg.norm(plain - exact) > 1e-4 * np.linalg.norm(exact)
        N = A.shape[1]
        F = np.linalg.inv(mu * Ah.conj().T @ Ah + c * np.eye(N))
        x = plain.copy()
        for _ in range(40):
            g = mu * (A.conj().T @ (y - A @ x) - Ah.conj().T @ (y - Ah @ x))
            x = F @ (mu * Ah.conj().T @ y + beta * v + g)
        assert np.linalg.norm(x - exact) <= 1e-12 * np.linalg.norm(exact)
        # the Woodbury application of F to g used for these sensors
        W = np.linalg.inv((c / mu) * np.eye(A.shape[0]) + Ah @ Ah.conj().T)
        g = mu * (A.conj().T @ (y - A @ x) - Ah.conj().T @ (y - Ah @ x))
        np.testing.assert_allclose((g - Ah.conj().T @ W @ Ah @ g) / c, F @ g, rtol=1e-10, atol=1e-14)
