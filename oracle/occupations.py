"""Natural occupation numbers of the correlated density (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper reports the natural occupation numbers (NONs) of the correlated
one-particle density at self-consistency (Introduction; Results, H32
lattice and its figure of NONs against the lattice parameter; Supplementary
Material, plots of natural occupation numbers) without writing out a
formula.  Reading taken here: the NONs are the eigenvalues of the
spin-summed AO density P expressed in the symmetrically orthonormalised
(Loewdin) basis, S^{1/2} P S^{1/2}.  With tr(P S) = N_e they lie in
[0, 2] and sum to N_e; "all NONs approach unity" at dissociation is the
half-filled limit of this convention.  They are the eigenvalues of P S
(similar matrices), so any factor X with X X^T = S gives the same values.
"""
import numpy as np


def natural_occupations(P: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Eigenvalues of S^{1/2} P S^{1/2}, largest first.

    S^{1/2} from the eigen-decomposition of S (a library eigensolver as a
    step); the symmetric part of the product is taken before the second
    eigensolve so rounding cannot leave a complex spectrum.
    """
    w, U = np.linalg.eigh(np.asarray(S, dtype=np.float64))
    Sh = (U * np.sqrt(w)) @ U.T
    A = Sh @ np.asarray(P, dtype=np.float64) @ Sh
    occ = np.linalg.eigvalsh(0.5 * (A + A.T))
    return occ[::-1].copy()
