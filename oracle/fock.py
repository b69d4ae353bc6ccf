"""Fock matrix from the density, Eq. (FockMatrix) (oracle).

    F_ij = h_ij + sum_kl P_kl ( v_ijlk - 1/2 v_iklj )

with P the spin-summed density (tr(P S) = N_e) and v_ijkl = (ij|kl) in
chemist notation, i.e. F = h + J - K/2.
"""
import numpy as np


def fock(h: np.ndarray, v: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Eq. (FockMatrix), written out as two contractions over (k, l)."""
    J = np.einsum("ijlk,kl->ij", v, P)
    K = np.einsum("iklj,kl->ij", v, P)
    return h + J - 0.5 * K
