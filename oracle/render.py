"""Back-projection image and dynamic-range rendering -- test infrastructure.

Only tests, the smoke check and the benchmark's CPU-baseline leg may use this
module (see the package docstring).

Sec. IV compares the sparse reconstructions with the back-projection (BP)
image and shows every image on a 30 dB dynamic range (Fig. 1).  The paper
states neither in formulas; the readings taken here:

* BP image: |sum_q A_q^H y_q|, the coherent sum over the Q sensors of each
  sensor's adjoint applied to its measurements (the data term of eq. (3) at
  x = 0 summed over sensors), as a magnitude per pixel.
* Rendering on a D dB range: with r = |x_n| / max_m |x_m|, the pixel's level
  is floor(255 (1 + 20 log10(r) / D)) clipped to [0, 255], and 0 where
  r < 10^(-D/20) or the image is all zero.  Equivalently the level is the
  number of thresholds t_L = 10^((L/255 - 1) D / 20), L = 1..255, with
  |x_n| >= t_L * max_m |x_m|; that comparison form is what decides here.
"""

from __future__ import annotations

import numpy as np


def back_projection(A, y) -> np.ndarray:
    """|sum_q A_q^H y_q| per pixel (N,), float64."""
    acc = None
    for a, yy in zip(A, y):
        b = np.conj(np.asarray(a, np.complex128)).T @ np.asarray(yy, np.complex128)
        acc = b if acc is None else acc + b
    return np.abs(acc)


def db_thresholds(range_db: float = 30.0) -> np.ndarray:
    """t_L = 10^((L/255 - 1) range_db / 20) for L = 1..255 (t_255 = 1)."""
    L = np.arange(1, 256, dtype=np.float64)
    return np.power(10.0, (L / 255.0 - 1.0) * range_db / 20.0)


def render_db(img, range_db: float = 30.0) -> np.ndarray:
    """8-bit levels of |img| on a range_db dynamic range (see module doc)."""
    mag = np.abs(np.asarray(img)).astype(np.float64).ravel()
    mx = mag.max() if mag.size else 0.0
    out = np.zeros(mag.shape, np.uint8)
    if mx <= 0.0:
        return out
    thr = db_thresholds(range_db) * mx
    # level = number of thresholds at or below |x_n|
    out[:] = np.searchsorted(thr, mag, side="right").astype(np.uint8)
    return out
