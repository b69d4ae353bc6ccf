"""Pins for the oracle's density-fitted Eq. (Sigma): it equals the dense
factored form (itself pinned against the brute-force sum) when the integrals
are built from the same factors, and a one-orbital, one-factor case in closed
form."""
import numpy as np

import oracle as O
from synthetic import generic_system, random_tau_stack


def test_df_equals_dense_for_factorised_integrals():
    for n, naux in [(1, 1), (3, 2), (5, 15), (8, 24)]:
        s = generic_system(n, 60 + n, naux=naux, ntau=7)
        rng = np.random.default_rng(n)
        Gt = random_tau_stack(rng, 7, n)
        ref = O.sigma_tau(Gt, s.v)
        got = O.sigma_tau_df(Gt, s.B)
        assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_one_orbital_one_factor_closed_form():
    # v = b^4: Sigma = -(2 - 1) g^2 gb b^4 (direct 2 g^2 gb b^4, exchange g^2 gb b^4)
    b, g, gb = 0.7, -0.3, 0.45
    got = O.sigma_df(np.array([[g]]), np.array([[gb]]), np.array([[[b]]]))
    assert abs(got[0, 0] - (-(g * g * gb * b ** 4))) < 1e-15
