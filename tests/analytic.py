"""Closed-form solutions used to pin the oracle (test helpers only)."""
from __future__ import annotations

import math

import numpy as np


def capillary_wave_height(t: np.ndarray, sigma: float, nu: float, k: float, rho0: float = 1.0) -> np.ndarray:
    """Scaled interface displacement of a small-amplitude capillary wave between
    two fluids of equal density and viscosity (Eq. 3.5 of the paper; Prosperetti's
    initial-value solution).  Returns h~(t) = (h_eq - h_0(t))/A_p, h~(0) = 1.

    exp(z^2 t) erfc(z sqrt t) is evaluated as the scaled erfcx(z sqrt t) so that
    no intermediate overflows."""
    from scipy.special import erfcx
    w0 = math.sqrt(sigma * k ** 3 / (2.0 * rho0))
    eps = nu * k * k / w0
    ew = eps * w0
    coeffs = [1.0, -math.sqrt(ew), -ew, ew ** 1.5, w0 * w0]
    z = np.roots(coeffs).astype(complex)
    t = np.asarray(t, dtype=float)
    out = np.zeros_like(t, dtype=complex)
    for i in range(4):
        Zi = 1.0 + 0j
        for j in range(4):
            if j != i:
                Zi *= (z[j] - z[i])
        coef = z[i] * w0 * w0 / (Zi * (z[i] ** 2 - ew))
        out += coef * np.exp(-ew * t) * erfcx(z[i] * np.sqrt(t))
    return out.real


def first_maximum_time(t: np.ndarray, h: np.ndarray) -> float:
    """Time of the first local maximum after the first minimum (parabolic fit)."""
    i_min = int(np.argmin(h[: len(h) // 2 + 1])) if len(h) > 2 else 0
    seg = h[i_min:]
    i = i_min + int(np.argmax(seg))
    if 0 < i < len(h) - 1:
        y0, y1, y2 = h[i - 1], h[i], h[i + 1]
        den = y0 - 2 * y1 + y2
        off = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        return float(t[i] + off * (t[1] - t[0]))
    return float(t[i])


def crossing_height(phi_col: np.ndarray, y: np.ndarray) -> float:
    """Position where a monotone column of phi crosses zero (linear interpolation)."""
    s = np.sign(phi_col)
    idx = np.where(s[:-1] * s[1:] <= 0)[0]
    j = int(idx[0])
    f0, f1 = phi_col[j], phi_col[j + 1]
    return float(y[j] + (y[j + 1] - y[j]) * (0.0 - f0) / (f1 - f0))
