"""Pins of the back-projection image and the 30 dB rendering (Sec. IV, Fig. 1)
against closed forms and a scalar loop."""

import numpy as np
import pytest

import oracle
from scenegen import make_geometry, steering


def test_render_levels_closed_form():
    """Magnitudes placed strictly between consecutive thresholds get exactly
    floor(255 (1 + 20 log10 r / D)); the maximum is 255; below -D dB and 0 give 0."""
    D = 30.0
    L = np.arange(1, 255)
    lo = np.power(10.0, (L / 255.0 - 1.0) * D / 20.0)
    hi = np.power(10.0, ((L + 1) / 255.0 - 1.0) * D / 20.0)
    r = np.sqrt(lo * hi)                       # geometric middle of level L
    img = np.concatenate([[1.0], r, [10 ** (-D / 20) * 0.999, 0.0]])
    got = oracle.render_db(img * 3.7, D)       # scale-free
    want = np.concatenate([[255], np.floor(255 * (1 + 20 * np.log10(r) / D)), [0, 0]])
    assert np.array_equal(got, want.astype(np.uint8))
    assert np.array_equal(got[1:-2], L.astype(np.uint8))


def test_render_other_range_and_complex_input():
    rng = np.random.default_rng(3)
    z = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    for D in (20.0, 40.0):
        got = oracle.render_db(z, D).astype(int)
        r = np.abs(z) / np.abs(z).max()
        v = 255 * (1 + 20 * np.log10(r) / D)
        want = np.where(r < 10 ** (-D / 20), 0, np.clip(np.floor(v), 0, 255)).astype(int)
        near = np.abs(v - np.round(v)) < 1e-9          # exact level boundaries
        assert np.array_equal(got[~near], want[~near])
    assert not oracle.render_db(np.zeros(7), 30.0).any()


def test_back_projection_scalar_loop_and_point_target():
    """|sum_q A_q^H y_q| equals a scalar double loop; for one sensor and a
    noise-free unit point target at pixel j the peak is |a_j|^2 = KM at j."""
    g = make_geometry(Q=2, M=2, K=8, n_side=6)
    A = [steering(g, q) for q in range(g.Q)]
    rng = np.random.default_rng(0)
    y = rng.standard_normal((g.Q, g.K * g.M)) + 1j * rng.standard_normal((g.Q, g.K * g.M))
    loop = np.zeros(g.N)
    for n in range(g.N):
        acc = 0j
        for q in range(g.Q):
            for i in range(g.K * g.M):
                acc += np.conj(A[q][i, n]) * y[q, i]
        loop[n] = abs(acc)
    assert np.allclose(oracle.back_projection(A, y), loop, rtol=1e-12, atol=0)
    j = 17
    bp = oracle.back_projection(A[:1], A[0][:, j][None, :])
    assert int(np.argmax(bp)) == j
    assert bp[j] == pytest.approx(g.K * g.M, rel=1e-12)
