"""Imaginary-time and Matsubara grids (oracle; test infrastructure only).

Matsubara frequencies follow the Implementation section: omega_n =
(2n+1) pi / beta.  Only n >= 0 is stored; negative frequencies follow
from X(-i omega) = conj(X(i omega)) for the real-symmetric matrices of a
real AO basis.

The paper uses a non-equidistant tau grid (Implementation section); the
reading taken here is a uniform grid tau_k = k beta / M, k = 0..M, with
M = ntau - 1 intervals, so ``ntau`` counts both endpoints.  tau_0 and
tau_M stand for the one-sided limits 0+ and beta-.
"""
import numpy as np


def tau_grid(beta: float, ntau: int) -> np.ndarray:
    """tau_k = k*beta/M, k = 0..M (M = ntau-1)."""
    if ntau < 4:
        raise ValueError("ntau must be >= 4 (not-a-knot cubic spline needs M >= 3)")
    return beta * np.arange(ntau, dtype=np.float64) / (ntau - 1)


def matsubara(beta: float, niw: int) -> np.ndarray:
    """Fermionic Matsubara frequencies omega_n = (2n+1) pi / beta, n = 0..niw-1."""
    return (2.0 * np.arange(niw, dtype=np.float64) + 1.0) * np.pi / beta
