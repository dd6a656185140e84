"""Azimuthal DFT in real "planes" and the exact discrete eigenvalue (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (azimuthal_dft): ``f^_m = (1/N) sum_j f_j exp(-2 pi i m j / N)``, with the
unnormalised inverse ``f_j = sum_m f^_m exp(2 pi i m j / N)`` (Sec. 3.1).  For
real f only ``m = 0 .. floor(N/2)`` are unique (the R2C modes, Sec. 3.1) and
``f^_{N-m}`` is the conjugate of ``f^_m``.  The N real degrees of freedom of
those modes are stored as N real planes:

* plane ``p = m`` for ``m = 0 .. floor(N/2)``  holds ``Re f^_m``  (cos planes),
* plane ``p = floor(N/2) + m`` for ``m = 1 .. ceil(N/2) - 1`` holds ``Im f^_m``
  (sin planes).

The operator of every plane is the real 2-D operator of mode m, so the real
and imaginary parts of a mode solve independently with the same shift.
"""
from __future__ import annotations

import numpy as np


def plane_modes(ntheta: int) -> np.ndarray:
    """Fourier index m carried by each plane (length ntheta)."""
    nc = ntheta // 2 + 1
    ms = list(range(nc)) + list(range(1, ntheta - nc + 1))
    return np.array(ms, dtype=np.int64)


def plane_is_sine(ntheta: int) -> np.ndarray:
    nc = ntheta // 2 + 1
    return np.arange(ntheta) >= nc


def discrete_eigenvalue(m, ntheta: int, dtheta, dtype=np.float64):
    """``lambda_m = (4/dtheta^2) sin^2(pi m / N)``, Eq. (discrete_azimuthal_eigenvalue),
    evaluated in ``dtype`` (``numpy.longdouble`` for extended precision)."""
    t = dtype
    m = np.asarray(m, dtype=t)
    pi = t(2) * np.arccos(t(0))
    dtheta = t(dtheta)
    return t(4) / (dtheta * dtheta) * np.sin(pi * m / t(ntheta)) ** 2


def plane_eigenvalues(ntheta: int, dtheta: float) -> np.ndarray:
    return discrete_eigenvalue(plane_modes(ntheta), ntheta, dtheta)


def forward(x: np.ndarray) -> np.ndarray:
    """Real planes of the DFT of ``x`` along axis 0, written out as sums (Eq. (azimuthal_dft))."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    j = np.arange(n)
    out = np.empty_like(x)
    modes = plane_modes(n)
    sine = plane_is_sine(n)
    for p in range(n):
        ang = 2.0 * np.pi * ((modes[p] * j) % n) / n
        w = -np.sin(ang) if sine[p] else np.cos(ang)
        out[p] = np.tensordot(w, x, axes=(0, 0)) / n
    return out


def inverse(planes: np.ndarray) -> np.ndarray:
    """Inverse of :func:`forward`: ``f_j = sum_m f^_m e^{i theta_m j}`` over all N modes.

    Using conjugate symmetry, mode m and N-m together contribute
    ``2 (Re f^_m cos - Im f^_m sin)``; m = 0 and (even N) m = N/2 appear once.
    """
    planes = np.asarray(planes, dtype=np.float64)
    n = planes.shape[0]
    j = np.arange(n)
    modes = plane_modes(n)
    sine = plane_is_sine(n)
    out = np.zeros_like(planes)
    for p in range(n):
        m = modes[p]
        ang = 2.0 * np.pi * ((m * j) % n) / n
        single = (m == 0) or (2 * m == n)
        mult = 1.0 if single else 2.0
        w = -mult * np.sin(ang) if sine[p] else mult * np.cos(ang)
        out += w.reshape((n,) + (1,) * (planes.ndim - 1)) * planes[p]
    return out


def parseval_weights(ntheta: int) -> np.ndarray:
    """``sum_j x_j^2 = N sum_p w_p P_p^2``: w = 1 for m = 0 and m = N/2, else 2."""
    modes = plane_modes(ntheta)
    return np.where((modes == 0) | (2 * modes == ntheta), 1.0, 2.0)
