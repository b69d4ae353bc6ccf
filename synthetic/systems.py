"""Seeded synthetic GF2 inputs (overlap S, core Hamiltonian h, AO integrals v).

This module is shared by the FP64 oracle and the GPU path as a source of
*inputs only*.  It holds none of the method's arithmetic: no Fock build,
no Green's function, no self-energy, no transform.  Every array is drawn
from ``numpy.random.default_rng(seed)`` in a fixed order, so a system is a
pure function of its seed and sizes.

The paper's own workloads (Li2/6-31G, H6/TZ, H12/STO-3G and the H32
4x4x2 lattice, Results section) need Gaussian basis sets and real AO
integrals, which are not available; these generators stand in for them
with the same shapes and the same structure that matters to the method:

* a non-orthogonal, unit-diagonal, positive definite overlap S;
* a real symmetric core Hamiltonian h (optionally banded);
* real two-electron integrals v_ijkl = (ij|kl) in chemist notation with
  the 8-fold permutational symmetry of real AO integrals, built as a sum
  of products of symmetric factors, v_ijkl = sum_P B^P_ij B^P_kl, which
  also makes the pair matrix v_(ij),(kl) positive semidefinite.

Workload recipes (sizes, temperatures and grids are the ones the
benchmark suite uses):

* ``generic``   small/medium "molecule-shaped" systems;
* ``lattice``   the 4x4x2 hydrogen-lattice-shaped system (32 sites, one
  basis function per site, half filling, hopping t scanned).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class System:
    """One closed-shell system: S, h, v plus its grid parameters."""
    name: str
    S: np.ndarray          # [n][n] overlap, SPD, unit diagonal
    h: np.ndarray          # [n][n] core Hamiltonian, symmetric (Eh)
    v: np.ndarray          # [n][n][n][n] (ij|kl), 8-fold symmetric (Eh)
    B: np.ndarray          # [naux][n][n] symmetric factors, v = sum_P B^P (x) B^P
    nelec: int             # electrons (spin-summed), even
    beta: float            # inverse temperature (1/Eh)
    niw: int               # Matsubara frequencies, n = 0..niw-1
    ntau: int              # imaginary-time points incl. both endpoints
    seed: int = 0
    meta: dict = field(default_factory=dict)
    tau: Optional[np.ndarray] = None   # non-uniform tau grid (ntau points), None = uniform

    @property
    def n(self) -> int:
        return self.S.shape[0]


def _unit_diag_overlap(rng: np.random.Generator, n: int, amp: float = 0.05) -> np.ndarray:
    R = np.eye(n) + amp * rng.standard_normal((n, n))
    S = R.T @ R
    d = 1.0 / np.sqrt(np.diag(S))
    S = S * d[:, None] * d[None, :]
    return 0.5 * (S + S.T)


def _core_hamiltonian(rng: np.random.Generator, n: int, diag_lo: float, diag_hi: float,
                      half_band: Optional[int]) -> np.ndarray:
    h = np.zeros((n, n))
    h[np.diag_indices(n)] = rng.uniform(diag_lo, diag_hi, n)
    iu, ju = np.triu_indices(n, k=1)            # row-major upper triangle
    z = rng.standard_normal(iu.size)
    vals = 0.3 * z * np.exp(-np.abs(iu - ju) / 2.0)
    if half_band is not None:
        vals = np.where(np.abs(iu - ju) <= half_band, vals, 0.0)
    h[iu, ju] = vals
    h[ju, iu] = vals
    return h


def _factors_to_v(B: np.ndarray) -> np.ndarray:
    naux, n, _ = B.shape
    Bm = B.reshape(naux, n * n)
    return (Bm.T @ Bm).reshape(n, n, n, n)


def generic_system(n: int, seed: int, *, naux: Optional[int] = None,
                   diag=(-2.0, -0.5), half_band: Optional[int] = None,
                   vdiag: float = 0.7, nelec: Optional[int] = None,
                   beta: float = 50.0, niw: int = 2048, ntau: int = 257,
                   name: str = "generic") -> System:
    """Generic seeded system.

    Draw order: R (overlap), h diagonal, h upper triangle, the naux
    factor matrices A_P; B^P = (A_P + A_P^T)/2; v scaled so that the mean
    over i of v_iiii equals ``vdiag``.
    """
    rng = np.random.default_rng(seed)
    naux = 3 * n if naux is None else naux
    S = _unit_diag_overlap(rng, n)
    h = _core_hamiltonian(rng, n, diag[0], diag[1], half_band)
    A = rng.standard_normal((naux, n, n))
    B = 0.5 * (A + A.transpose(0, 2, 1))
    ii = np.arange(n)
    mean_diag = float(np.mean(np.einsum("pi,pi->i", B[:, ii, ii], B[:, ii, ii])))
    B *= np.sqrt(vdiag / mean_diag)
    v = _factors_to_v(B)
    ne = n if nelec is None else nelec
    return System(name=name, S=S, h=h, v=v, B=B, nelec=ne, beta=beta, niw=niw,
                  ntau=ntau, seed=seed, meta={"naux": naux, "half_band": half_band})


def lattice_sites(nx: int = 4, ny: int = 4, nz: int = 2) -> np.ndarray:
    """Site coordinates of an nx*ny*nz simple-cubic block, x fastest."""
    return np.array([(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)],
                    dtype=float)


def lattice_system(t: float, seed: int, *, onsite: float = -1.0, s_nn: float = 0.1,
                   v0: float = 0.6, n_bond_factors: int = 64, bond_scale: float = 0.05,
                   beta: float = 100.0, niw: int = 8192, ntau: int = 1025,
                   name: str = "lattice") -> System:
    """4x4x2 lattice-shaped system (32 sites, 32 electrons).

    h = onsite*I + t*A, S = I + s_nn*A (A = nearest-neighbour adjacency,
    unit spacing).  Integrals: a density part with (ii|jj) = v0*exp(-d_ij)
    from diagonal factors built from the Cholesky factor of that kernel,
    plus ``n_bond_factors`` random symmetric factors supported on bonded
    pairs, scaled by ``bond_scale``.
    """
    rng = np.random.default_rng(seed)
    X = lattice_sites()
    n = X.shape[0]
    d = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
    A = (np.abs(d - 1.0) < 1e-12).astype(float)
    h = onsite * np.eye(n) + t * A
    S = np.eye(n) + s_nn * A
    C = v0 * np.exp(-d)
    L = np.linalg.cholesky(C)
    Bd = np.zeros((n, n, n))
    for P in range(n):
        Bd[P][np.diag_indices(n)] = L[:, P]
    iu, ju = np.nonzero(np.triu(A, k=1))
    Bb = np.zeros((n_bond_factors, n, n))
    for P in range(n_bond_factors):
        z = bond_scale * rng.standard_normal(iu.size)
        Bb[P, iu, ju] = z
        Bb[P, ju, iu] = z
    B = np.concatenate([Bd, Bb], axis=0)
    v = _factors_to_v(B)
    return System(name=name, S=S, h=h, v=v, B=B, nelec=n, beta=beta, niw=niw, ntau=ntau,
                  seed=seed, meta={"t": t, "naux": B.shape[0]})


# ---------------------------------------------------------------------------
# The benchmark workloads
# ---------------------------------------------------------------------------

def small_molecule(seed: int = 0) -> System:
    """N=10, 10 electrons, beta=50, 2048 frequencies, 257 tau points."""
    return generic_system(10, seed, naux=30, diag=(-2.0, -0.5), beta=50.0, niw=2048,
                          ntau=257, name="generic-n10")


LATTICE_T = tuple(float(x) for x in np.linspace(-0.5, -0.05, 8))


def lattice_sweep(index: int) -> System:
    """One of the 8 lattice systems of the hopping scan (seeds 100..107)."""
    return lattice_system(LATTICE_T[index], 100 + index, name=f"lattice-n32-t{index}")


def batched_sizes(count: int = 64, seed: int = 199) -> np.ndarray:
    """Basis sizes of the batched sweep: even N drawn uniformly from [8, 48]."""
    rng = np.random.default_rng(seed)
    return rng.choice(np.arange(8, 49, 2), size=count)


def batched_member(index: int) -> System:
    """Member ``index`` of the 64-system batched sweep (seeds 200..263)."""
    n = int(batched_sizes()[index])
    return generic_system(n, 200 + index, naux=3 * n, diag=(-2.0, -0.5), beta=100.0,
                          niw=4096, ntau=513, name=f"batch-{index}-n{n}")


def molecule_n100(seed: int = 300) -> System:
    """N=100, 100 electrons, banded h (half-bandwidth 12), naux=400, beta=200,
    16384 frequencies, 512 tau points."""
    return generic_system(100, seed, naux=400, diag=(-3.0, -0.3), half_band=12,
                          beta=200.0, niw=16384, ntau=512, name="generic-n100")


def molecule_n160(seed: int = 400) -> System:
    """N=160, 160 electrons, half-bandwidth 16, naux=640, beta=200,
    16384 frequencies, 512 tau points."""
    return generic_system(160, seed, naux=640, diag=(-3.0, -0.3), half_band=16,
                          beta=200.0, niw=16384, ntau=512, name="generic-n160")


# ---------------------------------------------------------------------------
# Generic random helpers for unit tests (inputs only)
# ---------------------------------------------------------------------------

def random_symmetric(rng: np.random.Generator, n: int, scale: float = 1.0) -> np.ndarray:
    A = rng.standard_normal((n, n)) * scale
    return 0.5 * (A + A.T)


def random_integrals(rng: np.random.Generator, n: int, naux: Optional[int] = None,
                     scale: float = 0.3) -> np.ndarray:
    """Random 8-fold symmetric v = sum_P B^P (x) B^P."""
    naux = 2 * n if naux is None else naux
    A = rng.standard_normal((naux, n, n)) * scale
    B = 0.5 * (A + A.transpose(0, 2, 1))
    return _factors_to_v(B)


def random_tau_stack(rng: np.random.Generator, ntau: int, n: int, scale: float = 0.5) -> np.ndarray:
    """[ntau][n][n] stack of random symmetric matrices."""
    X = rng.standard_normal((ntau, n, n)) * scale
    return 0.5 * (X + X.transpose(0, 2, 1))


def power_tau_grid(beta: float, levels: int, per_level: int) -> np.ndarray:
    """Non-equidistant tau grid, dense at both ends and symmetric about beta/2.

    On [0, beta/2] the nodes x_l = (beta/2) 2^-l (l = 0..levels-1) and 0 cut
    the half interval into `levels` pieces, each split into `per_level`
    equal steps; the other half is the mirror image tau -> beta - tau.
    2 levels per_level + 1 points, tau_0 = 0, tau_M = beta, and
    tau_{M-k} = beta - tau_k (so G(-tau_k) = -G(tau_{M-k}) stays on the grid).
    """
    if levels < 1 or per_level < 1 or 2 * levels * per_level < 3:
        raise ValueError("power_tau_grid: needs levels, per_level >= 1 and at least 4 points")
    half = 0.5 * beta
    edges = [0.0] + [half * 2.0 ** (-l) for l in range(levels - 1, -1, -1)]
    pts = []
    for a, b in zip(edges[:-1], edges[1:]):
        pts.extend(a + (b - a) * np.arange(per_level) / per_level)
    left = np.array(pts + [half])
    right = beta - left[-2::-1]
    tau = np.concatenate([left, right])
    tau[0], tau[-1] = 0.0, beta
    return tau
