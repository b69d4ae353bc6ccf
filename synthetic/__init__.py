"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark."""
from .systems import (System, generic_system, lattice_system, small_molecule, lattice_sweep,
                      batched_sizes, batched_member, molecule_n100, molecule_n160,
                      random_symmetric, random_integrals, random_tau_stack, LATTICE_T,
                      power_tau_grid)

__all__ = ["System", "generic_system", "lattice_system", "small_molecule", "lattice_sweep",
           "batched_sizes", "batched_member", "molecule_n100", "molecule_n160",
           "random_symmetric", "random_integrals", "random_tau_stack", "LATTICE_T",
           "power_tau_grid"]
