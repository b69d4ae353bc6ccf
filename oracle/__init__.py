"""FP64 CPU oracle for self-consistent second-order Green's function theory (GF2).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously
correct NumPy/SciPy implementation of the method of Phillips & Zgid,
"The description of strong correlation within self-consistent Green's
function second-order perturbation theory" (arXiv:1405.3273).  It exists
to check the HIP library.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.
It shares no code with the HIP library (no kernels, headers, tables or
helpers); the only thing both sides use is the seeded input generator in
``synthetic``.

Every function cites the passage of the paper it follows:

* Eq. (FockMatrix)  -- Fock matrix from the density (Implementation).
* Eq. (Sigma)       -- second-order self-energy in imaginary time.
* Eq. (GF)          -- Dyson equation on the Matsubara axis.
* natural occupation numbers of the correlated density (Results).
* Supplementary Material, "Implementation of GF2 algorithm", steps 1-3.

Where the paper is silent (energy formula, transform quadrature, grid
conventions, mu search, convergence tests) the oracle takes one stated
reading; each is listed in the module that implements it.

Parity status of every function is "pinned" (checked by the CPU tests
in ``tests/test_oracle_*.py`` against closed forms, textbook limits,
invariants or brute force) unless its docstring says "parity unpinned".
"""
from .grids import tau_grid, matsubara
from .sigma import (gbar_from_gtau, sigma_bruteforce, sigma_literal, sigma_factored,
                    sigma_tau, bracket_W, sigma_df, sigma_tau_df)
from .fourier import sigma_tau_to_iw, g_iw_to_tau, spline_coefficients, moments_unit, tail_tau
from .dyson import (tail_moments, green_iw, density_from_giw, particle_number, find_mu,
                    BracketError, NoConvergence)
from .fock import fock
from .energy import e_one_body, e_two_body, trigamma
from .loop import Params, State, OuterReport, inner_loop, outer_iteration, run, pulay_mix
from .occupations import natural_occupations

__all__ = [
    "tau_grid", "matsubara",
    "gbar_from_gtau", "sigma_bruteforce", "sigma_literal", "sigma_factored", "sigma_tau",
    "bracket_W", "sigma_df", "sigma_tau_df",
    "sigma_tau_to_iw", "g_iw_to_tau", "spline_coefficients", "moments_unit", "tail_tau",
    "tail_moments", "green_iw", "density_from_giw", "particle_number", "find_mu",
    "BracketError", "NoConvergence",
    "fock", "e_one_body", "e_two_body", "trigamma",
    "Params", "State", "OuterReport", "inner_loop", "outer_iteration", "run", "pulay_mix",
    "natural_occupations",
]
