"""Closed forms used to pin the oracle (independent of it).

Exit probability of Brownian motion sigma W from (0, L) by time T, started at x
(paper Section 4.1, Eq. (e45)).  The printed series runs over every n >= 1 with
coefficient 4/(n pi); the sine coefficients of the constant 1 on (0, L) vanish
for even n, so only odd n belong in it (with the even terms it returns about
0.5 at tiny T).  ``p_exit_series`` uses odd n; ``p_exit_images`` is the
method-of-images form of the same probability, which converges fast for small
T and serves as the cross-check.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtr


def p_exit_series(T, x, L, sigma=1.0, n_terms=4001):
    x = np.asarray(x, dtype=np.float64)
    s = np.zeros_like(x)
    for n in range(1, n_terms + 1, 2):
        k = n * math.pi / L
        term = 4.0 / (n * math.pi) * np.sin(k * x) * math.exp(-0.5 * (k * sigma) ** 2 * T)
        s += term
        if math.exp(-0.5 * (k * sigma) ** 2 * T) < 1e-18:
            break
    return 1.0 - s


def p_exit_images(T, x, L, sigma=1.0, n_images=50):
    """1 - survival, survival = int_0^L sum_k [phi(y-x+2kL) - phi(y+x+2kL)] dy."""
    x = np.asarray(x, dtype=np.float64)
    s = sigma * math.sqrt(T)
    surv = np.zeros_like(x)
    for k in range(-n_images, n_images + 1):
        o = 2.0 * k * L
        surv += (ndtr((L - x + o) / s) - ndtr((-x + o) / s)
                 - ndtr((L + x + o) / s) + ndtr((x + o) / s))
    return 1.0 - surv
