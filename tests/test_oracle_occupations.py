"""Pins for the oracle's natural occupation numbers: a 2x2 closed form with a
non-unit overlap, the idempotent (zero-temperature) density, the Fermi
occupations of a finite-beta Hartree-Fock density, and invariance under a
change of AO basis."""
import numpy as np

import oracle as O
from oracle import reference as R
from synthetic import generic_system


def test_two_by_two_closed_form_with_diagonal_overlap():
    # S = diag(s1, s2): S^{1/2} P S^{1/2} = [[s1 p11, sqrt(s1 s2) p12], [., s2 p22]]
    s1, s2 = 1.7, 0.6
    p11, p22, p12 = 1.3, 0.4, -0.35
    P = np.array([[p11, p12], [p12, p22]])
    S = np.diag([s1, s2])
    a, d, b = s1 * p11, s2 * p22, np.sqrt(s1 * s2) * p12
    m, r = 0.5 * (a + d), np.sqrt(0.25 * (a - d) ** 2 + b * b)
    got = O.natural_occupations(P, S)
    np.testing.assert_allclose(got, [m + r, m - r], rtol=0, atol=1e-14)


def test_idempotent_density_gives_two_and_zero():
    """P = 2 C_occ C_occ^T with C^T S C = 1 (C from a Cholesky factor of S,
    not from the oracle's eigen-decomposition): NONs are 2 (occupied) and 0."""
    n, nocc = 9, 4
    s = generic_system(n, 11)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    L = np.linalg.cholesky(s.S)
    C = np.linalg.solve(L.T, Q)
    np.testing.assert_allclose(C.T @ s.S @ C, np.eye(n), atol=1e-12)
    P = 2.0 * C[:, :nocc] @ C[:, :nocc].T
    got = O.natural_occupations(P, s.S)
    np.testing.assert_allclose(got, [2.0] * nocc + [0.0] * (n - nocc), atol=1e-12)


def test_finite_beta_hf_density_gives_fermi_occupations():
    """The Hartree-Fock density at finite beta (closed form, and the oracle's
    Matsubara sum with its tail) has NONs 2 f(eps_k - mu), eps_k the
    generalized eigenvalues of (F, S)."""
    n, beta = 8, 20.0
    s = generic_system(n, 5, beta=beta)
    F = s.h
    eps, _ = R.generalized_eig(F, s.S)
    mu = R.mu_closed_form(eps, s.nelec, beta)
    want = np.sort(2.0 * R.fermi(eps - mu, beta))[::-1]
    P = R.hf_density(s.S, F, mu, beta)
    np.testing.assert_allclose(O.natural_occupations(P, s.S), want, atol=1e-12)
    niw = 4096
    G = O.green_iw(mu, s.S, F, None, beta, niw)
    Pm = O.density_from_giw(G, *O.tail_moments(s.S, F, mu), beta)
    occ = O.natural_occupations(Pm, s.S)
    np.testing.assert_allclose(occ, want, atol=1e-6)
    assert abs(occ.sum() - np.trace(Pm @ s.S)) < 1e-10
    assert occ.max() <= 2.0 + 1e-6 and occ.min() >= -1e-6


def test_invariant_under_change_of_ao_basis():
    """Basis functions chi' = chi X: S' = X^T S X, P' = X^{-1} P X^{-T}."""
    n = 7
    s = generic_system(n, 21)
    rng = np.random.default_rng(8)
    A = rng.standard_normal((n, n))
    P = A @ np.diag(rng.uniform(0.0, 2.0, n)) @ A.T / n
    X = np.eye(n) + 0.3 * rng.standard_normal((n, n))
    Xi = np.linalg.inv(X)
    got = O.natural_occupations(Xi @ P @ Xi.T, X.T @ s.S @ X)
    np.testing.assert_allclose(got, O.natural_occupations(P, s.S), atol=1e-11)
