"""Gradient waveforms, b-values and direction sets (inputs only).

The Bloch-Torrey model takes a separable gradient G(t) = G0 f(t) (Sec. 2.1).
The lattice scheme samples f at the left end of every time step and holds it
constant over the step (reaction split, Sec. 2.3), so a waveform here is the
array f_k, k = 0..K-1, with f_k acting on [k dt, (k+1) dt).
"""
from __future__ import annotations

import math

import numpy as np

# Gyromagnetic ratio of 1H in rad/(s*T).  The paper never states a value; it
# is only used to convert mT/m to the gamma*G0 the library takes.
GAMMA_H1 = 2.6752218744e8


def gamma_g_from_mT_per_m(g_mT_per_m: float) -> float:
    """gamma*G in rad/(um*ms) for a gradient in mT/m."""
    # rad/(s*T) * T/m = rad/(s*m) = 1e-6 rad/(um) * 1e-3 per ms
    return GAMMA_H1 * g_mT_per_m * 1e-3 * 1e-6 * 1e-3


def pgse_waveform(delta: float, Delta: float, dt: float) -> np.ndarray:
    """Effective (post-refocusing) PGSE waveform, one sample per step.

    Rectangular bipolar pulses (Sec. 2.1, Fig. 2): f = +1 on [0, delta),
    0 on [delta, Delta), -1 on [Delta, Delta + delta); echo at
    TE = Delta + delta.  Durations are rounded to whole steps.
    """
    nd = int(round(delta / dt))
    nD = int(round(Delta / dt))
    if nd <= 0 or nD < nd:
        raise ValueError("need 0 < delta <= Delta (in whole steps)")
    f = np.zeros(nD + nd, dtype=np.float64)
    f[:nd] = 1.0
    f[nD:nD + nd] = -1.0
    return f


def ogse_cosine_waveform(period: float, n_periods: int, Delta: float,
                         dt: float) -> np.ndarray:
    """Effective cosine OGSE waveform: lobe cos(2 pi t / period) for
    n_periods periods, a gap until Delta, then the negated lobe."""
    nl = int(round(period * n_periods / dt))
    nD = int(round(Delta / dt))
    if nD < nl:
        raise ValueError("Delta shorter than the first lobe")
    t = (np.arange(nl) * dt)
    lobe = np.cos(2.0 * math.pi * t / period)
    f = np.zeros(nD + nl, dtype=np.float64)
    f[:nl] = lobe
    f[nD:nD + nl] = -lobe
    return f


def gamma_g_for_b_pgse(b: float, delta: float, Delta: float) -> float:
    """|gamma G0| giving b = (gamma G0)^2 delta^2 (Delta - delta/3) (Sec. 2.1)."""
    return math.sqrt(b / (delta * delta * (Delta - delta / 3.0)))


def b_of_waveform(f: np.ndarray, dt: float, gG: float = 1.0) -> float:
    """b = int_0^TE (gamma G0 F(t))^2 dt for the piecewise-constant samples f,
    with F(t) = int_0^t f; exact for the piecewise-linear F."""
    f = np.asarray(f, dtype=np.float64)
    F0 = np.concatenate([[0.0], np.cumsum(f * dt)])
    a, c = F0[:-1], F0[1:]
    # integral of a linear segment squared from a to c over dt
    return float(gG * gG * np.sum((a * a + a * c + c * c) / 3.0 * dt))


def golden_spiral(n: int, hemisphere: bool = True) -> np.ndarray:
    """n nearly uniform unit vectors (golden-angle spiral), shape (n, 3)."""
    i = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - i / n if hemisphere else 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def axon_directions() -> np.ndarray:
    """Six non-collinear directions (1,+-1,0), (1,0,+-1), (0,1,+-1) / sqrt 2."""
    s = 1.0 / math.sqrt(2.0)
    return np.array([[s, s, 0], [s, -s, 0], [s, 0, s], [s, 0, -s],
                     [0, s, s], [0, s, -s]], dtype=np.float64)
