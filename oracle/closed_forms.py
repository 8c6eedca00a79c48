"""Textbook closed forms used to pin the oracle (FP64).

Test infrastructure only.

One-band chain: m = 1, H00 = 0, H01 = -t, S = 1, so E(k) = -2t cos k and the
group velocity is 2t sin k.  A rectangular barrier of height V over n sites
has (transfer-matrix result; U_k is the Chebyshev polynomial of the second
kind, U_{k}(cos q) = sin((k+1) q) / sin q)

    T(E) = 1 / (1 + (V / (2 t sin k))^2 U_{n-1}((V - E) / (2t))^2),

valid for E inside the band, for tunnelling (|V - E| > 2t) and above-barrier
energies alike.  n = 1 reduces to the single-impurity result
1 / (1 + V^2 / (4 t^2 sin^2 k)).
"""
from __future__ import annotations

import numpy as np


def chebyshev_u(k: int, x: float) -> float:
    """U_k(x) by the three-term recurrence U_{j+1} = 2x U_j - U_{j-1}."""
    if k < 0:
        return 0.0
    u_prev, u = 1.0, 2.0 * x
    if k == 0:
        return 1.0
    for _ in range(k - 1):
        u_prev, u = u, 2.0 * x * u - u_prev
    return u


def barrier_1band(E: float, t: float, V: float, n: int) -> float:
    ck = -E / (2.0 * t)
    if abs(ck) >= 1.0:
        return 0.0
    sk = np.sqrt(1.0 - ck * ck)
    u = chebyshev_u(n - 1, (V - E) / (2.0 * t))
    return 1.0 / (1.0 + (V / (2.0 * t * sk)) ** 2 * u * u)


def open_channels_1band(E: float, t: float) -> int:
    return 1 if abs(E) < 2.0 * abs(t) else 0
