"""Seeded target scenes and noisy measurements y_q = A_q x_q + w_q (eq. (1)).

Recipe (all draws from one `numpy.random.default_rng(seed)`, in this order):

1. Targets.  For each of `n_targets` targets: a centre pixel (uniform over
   the grid, distinct centres), an amplitude U(0.5, 1), and a shape.  With
   `extended=False` every target is a single pixel.  With `extended=True` a
   target is a single pixel with probability 1/2, otherwise a straight run of
   L ~ U{2..6} pixels from the centre along one of the four grid directions
   (horizontal, vertical, two diagonals), clipped to the grid.
2. Visibility (aspect-dependent scattering, Sec. IV).  Each target is seen by
   a uniform number of sensors in {2..Q} ({1} when Q = 1), chosen without
   replacement, each
   with its own gain U(0.3, 1).  x_q[j] = amplitude * gain_q; a pixel covered
   by two targets keeps the larger value, so every entry stays in [0, 1].
3. Noise.  Per sensor, sigma_w^2 = mean |A_q x_q|^2 / 10^(SNR/10); w_q is
   circular complex Gaussian with sigma_w^2/2 per real and imaginary part
   (real parts drawn first, then imaginary, sensor by sensor).

The composite ground truth of Sec. IV is sum_q x_q.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .geometry import Geometry, steering

_DIRS = ((1, 0), (0, 1), (1, 1), (1, -1))


@dataclass
class Scene:
    geom: Geometry
    seed: int
    x_true: np.ndarray          # (Q, N) float64, per-sensor reflectivity magnitude
    y: np.ndarray               # (Q, KM) complex128
    noise_var: np.ndarray       # (Q,) float64, sigma_w^2 per sensor
    snr_db: float
    target_pixels: list = field(default_factory=list)   # pixel lists per target

    @property
    def composite(self) -> np.ndarray:
        return self.x_true.sum(axis=0)

    @property
    def support(self) -> np.ndarray:
        return np.flatnonzero(self.composite > 0)


def _target_pixels(rng, n_side: int, centre: int, extended: bool):
    if not extended or rng.random() < 0.5:
        return [centre]
    length = int(rng.integers(2, 7))
    dx, dy = _DIRS[int(rng.integers(0, 4))]
    cx, cy = centre % n_side, centre // n_side
    pts = []
    for s in range(length):
        x, y = cx + s * dx, cy + s * dy
        if 0 <= x < n_side and 0 <= y < n_side:
            pts.append(y * n_side + x)
    return pts


def make_scene(g: Geometry, seed: int, n_targets: int, snr_db: float,
               extended: bool = False) -> Scene:
    rng = np.random.default_rng(seed)
    Q, N = g.Q, g.N
    centres = rng.choice(N, size=n_targets, replace=False)
    amps = rng.uniform(0.5, 1.0, size=n_targets)
    shapes = [_target_pixels(rng, g.n_side, int(c), extended) for c in centres]
    x_true = np.zeros((Q, N))
    for t in range(n_targets):
        count = int(rng.integers(min(2, Q), Q + 1))
        seen = rng.choice(Q, size=count, replace=False)
        gains = rng.uniform(0.3, 1.0, size=count)
        for q, gq in zip(seen, gains):
            idx = np.asarray(shapes[t])
            x_true[q, idx] = np.maximum(x_true[q, idx], amps[t] * gq)
    y = np.zeros((Q, g.KM), dtype=np.complex128)
    noise_var = np.zeros(Q)
    for q in range(Q):
        cols = np.flatnonzero(x_true[q])
        if cols.size:
            sig = steering(g, q, cols) @ x_true[q, cols]
        else:
            sig = np.zeros(g.KM, dtype=np.complex128)
        p = float(np.mean(np.abs(sig) ** 2))
        var = p / 10.0 ** (snr_db / 10.0)
        re = rng.standard_normal(g.KM)
        im = rng.standard_normal(g.KM)
        y[q] = sig + np.sqrt(var / 2.0) * (re + 1j * im)
        noise_var[q] = var
    return Scene(g, seed, x_true, y, noise_var, float(snr_db), shapes)
