"""Sensor geometry and the dense measurement operator of Sec. II, eq. (1).

Layout conventions (used by every consumer of these arrays):

* Q sensors sit at angles 2*pi*q/Q on a circle of radius R around the scene
  centre.  Each sensor carries one Tx at its centre and an M-element
  half-wavelength uniform linear array of Rx antennas whose axis is tangent to
  the circle; Rx m sits at offset (m - (M-1)/2) * lambda0/2 along that axis,
  with lambda0 = c/f0.
* The scene is an n_side x n_side grid of pixel centres covering a square of
  side `side` metres centred at the origin; pixel n = iy*n_side + ix, with
  coordinates ((ix+0.5)/n_side - 0.5)*side, ((iy+0.5)/n_side - 0.5)*side.
* The LFM chirp is sampled at K fast-time samples, frequency
  f_k = f0 + BW*k/K, k = 0..K-1.
* Row (m, k) of A_q is row index m*K + k (antenna-major stacking of the Rx
  measurements into y_q, as eq. (1) stacks them).
* A_q[m*K+k, n] = exp(-j*2*pi*f_k*tau_{q,m,n}), with tau the two-way delay
  Tx_q -> pixel n -> Rx_{q,m}, |tx - p|/c + |rx - p|/c.  Every entry has unit
  modulus.  The reflectivity phase is folded into the real magnitude x_q
  (Sec. II), so A_q carries only the propagation phase.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SPEED_OF_LIGHT = 299_792_458.0


@dataclass(frozen=True)
class Geometry:
    Q: int
    M: int
    K: int
    n_side: int
    side: float
    radius: float
    f0: float
    bw: float
    tx: np.ndarray      # (Q, 2) float64, Tx position of each sensor
    rx: np.ndarray      # (Q, M, 2) float64, Rx positions
    pix: np.ndarray     # (N, 2) float64, pixel centres
    freqs: np.ndarray   # (K,) float64, f_k

    @property
    def N(self) -> int:
        return self.n_side * self.n_side

    @property
    def KM(self) -> int:
        return self.K * self.M


def make_geometry(Q: int, M: int, K: int, n_side: int, side: float = 4.0,
                  radius: float = 10.0, f0: float = 77e9, bw: float = 1e9) -> Geometry:
    lam0 = SPEED_OF_LIGHT / f0
    spacing = lam0 / 2.0
    tx = np.empty((Q, 2))
    rx = np.empty((Q, M, 2))
    offs = (np.arange(M) - (M - 1) / 2.0) * spacing
    for q in range(Q):
        ang = 2.0 * np.pi * q / Q
        centre = radius * np.array([np.cos(ang), np.sin(ang)])
        axis = np.array([-np.sin(ang), np.cos(ang)])     # tangent to the circle
        tx[q] = centre
        rx[q] = centre[None, :] + offs[:, None] * axis[None, :]
    c1 = ((np.arange(n_side) + 0.5) / n_side - 0.5) * side
    gx, gy = np.meshgrid(c1, c1, indexing="xy")          # gx varies along ix
    pix = np.stack([gx.ravel(), gy.ravel()], axis=1)
    freqs = f0 + bw * np.arange(K) / K
    return Geometry(Q, M, K, n_side, float(side), float(radius), float(f0),
                    float(bw), tx, rx, pix, freqs)


def delays(g: Geometry, q: int, cols=None) -> np.ndarray:
    """Two-way delays tau[m, j] (seconds) for pixels `cols` (all if None)."""
    p = g.pix if cols is None else g.pix[np.asarray(cols)]
    d_tx = np.hypot(p[:, 0] - g.tx[q, 0], p[:, 1] - g.tx[q, 1])
    d_rx = np.hypot(p[None, :, 0] - g.rx[q, :, None, 0],
                    p[None, :, 1] - g.rx[q, :, None, 1])
    return (d_tx[None, :] + d_rx) / SPEED_OF_LIGHT


def steering(g: Geometry, q: int, cols=None) -> np.ndarray:
    """Columns `cols` (all if None) of A_q as complex128, shape (K*M, ncols).

    Column-major consumers should take `np.asfortranarray` of the result.
    """
    tau = delays(g, q, cols)                               # (M, ncols)
    # cycles = f_k * tau; reduce modulo 1 in FP64 before the exponential so
    # the phase keeps full FP64 accuracy for f0*tau of several thousand
    # cycles.
    cyc = g.freqs[None, :, None] * tau[:, None, :]         # (M, K, ncols)
    cyc = cyc - np.floor(cyc)
    a = np.exp(-2j * np.pi * cyc)
    return a.reshape(g.M * g.K, -1)
