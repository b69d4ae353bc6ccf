"""Pins for the oracle's Dyson solve, density, mu search, Fock build and mixing."""
import numpy as np
import pytest

import oracle as O
from oracle import reference as R
from oracle.loop import pulay_mix
from synthetic import generic_system, random_symmetric


def _sys(n=5, seed=31, beta=20.0, niw=2048, ntau=65):
    return generic_system(n, seed, beta=beta, niw=niw, ntau=ntau)


def test_green_function_without_sigma_is_free_resolvent():
    s = _sys()
    eps, C = R.generalized_eig(s.h, s.S)
    mu = float(np.mean(eps))
    G = O.green_iw(mu, s.S, s.h, None, s.beta, 64)
    ref = R.hf_green_iw(s.S, s.h, mu, s.beta, 64)
    assert np.max(np.abs(G - ref)) < 1e-13


def test_green_function_complex_symmetric_and_conjugate_symmetric():
    s = _sys()
    rng = np.random.default_rng(5)
    Sig = 0.1 * (random_symmetric(rng, s.n) + 1j * random_symmetric(rng, s.n))
    G = O.green_iw(-1.0, s.S, s.h, np.broadcast_to(Sig, (8, s.n, s.n)), s.beta, 8)
    assert np.max(np.abs(G - G.transpose(0, 2, 1))) < 1e-13
    # G(-i w) = [(-i w + mu) S - F - conj(Sigma)]^-1 = conj(G(i w))
    iw = 1j * O.matsubara(s.beta, 8)
    Gm = np.linalg.inv((-iw[:, None, None] - 1.0) * s.S - s.h - np.conj(Sig))
    assert np.max(np.abs(Gm - np.conj(G))) < 1e-13


def test_density_and_mu_match_fermi_dirac_closed_form():
    s = _sys()
    eps, C = R.generalized_eig(s.h, s.S)
    mu_ref = R.mu_closed_form(eps, s.nelec, s.beta)
    for method in ("bisect", "illinois", "secant"):
        mu, _ = O.find_mu(s.nelec, s.S, s.h, None, None, s.beta, s.niw, mu0=0.0,
                          method=method, tol_N=1e-12)
        assert mu == pytest.approx(mu_ref, abs=1e-7)
    # a good slope hint and a nearby start need very few evaluations
    mu1, ev1, sl = O.find_mu(s.nelec, s.S, s.h, None, None, s.beta, s.niw, mu0=mu_ref + 0.01,
                             method="secant", tol_N=1e-12, return_slope=True)
    mu2, ev2, _ = O.find_mu(s.nelec, s.S, s.h, None, None, s.beta, s.niw, mu0=mu_ref + 1e-4,
                            method="secant", tol_N=1e-12, slope=sl, return_slope=True)
    assert sl > 0 and mu2 == pytest.approx(mu_ref, abs=1e-7) and ev2 <= 4
    G = O.green_iw(mu_ref, s.S, s.h, None, s.beta, s.niw)
    P = O.density_from_giw(G, *O.tail_moments(s.S, s.h, mu_ref), s.beta)
    assert np.max(np.abs(P - R.hf_density(s.S, s.h, mu_ref, s.beta))) < 1e-9
    assert np.trace(P @ s.S) == pytest.approx(s.nelec, abs=1e-9)


def test_mu_search_rejects_impossible_electron_counts():
    s = _sys()
    with pytest.raises(O.BracketError):
        O.find_mu(2 * s.n + 1, s.S, s.h, None, None, s.beta, 64)
    with pytest.raises(O.BracketError):
        O.find_mu(-1, s.S, s.h, None, None, s.beta, 64)


def test_density_tail_terms_matter():
    """Dropping the G2 tail in the density visibly breaks tr(PS) = N_e."""
    s = _sys()
    eps, _ = R.generalized_eig(s.h, s.S)
    mu = R.mu_closed_form(eps, s.nelec, s.beta)
    G = O.green_iw(mu, s.S, s.h, None, s.beta, s.niw)
    G1, G2, G3 = O.tail_moments(s.S, s.h, mu)
    good = O.density_from_giw(G, G1, G2, G3, s.beta)
    bad = O.density_from_giw(G, G1, 0 * G2, G3, s.beta)
    err_good = abs(np.trace(good @ s.S) - s.nelec)
    err_bad = abs(np.trace(bad @ s.S) - s.nelec)
    assert err_bad > 1e-5 and err_bad > 1e4 * err_good


def test_fock_matches_density_fitted_form():
    """With v = sum_P B^P (x) B^P: J = sum_P B^P tr(B^P P), K = sum_P B^P P B^P."""
    s = _sys(n=6)
    rng = np.random.default_rng(8)
    P = random_symmetric(rng, s.n)
    J = np.einsum("pij,p->ij", s.B, np.einsum("pkl,lk->p", s.B, P))
    K = np.einsum("pik,kl,plj->ij", s.B, P, s.B)
    assert np.max(np.abs(O.fock(s.h, s.v, P) - (s.h + J - 0.5 * K))) < 1e-12


def test_fock_hubbard_atom():
    U, h0 = 1.1, -0.4
    F = O.fock(np.array([[h0]]), np.full((1, 1, 1, 1), U), np.array([[1.0]]))
    assert F[0, 0] == pytest.approx(h0 + 0.5 * U, rel=1e-15)


def test_pulay_with_one_pair_is_plain_damping():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 4))
    r = rng.standard_normal((4, 4))
    a = 0.3
    got, _ = pulay_mix([(x, r)], a)
    assert np.allclose(got, (1 - a) * (x + r) + a * x, atol=1e-15)


def test_pulay_solves_linear_fixed_point_in_few_steps():
    """Anderson mixing on x = A x + b (contractive A) converges fast."""
    rng = np.random.default_rng(3)
    n = 6
    A = rng.standard_normal((n, n))
    A *= 0.9 / np.max(np.abs(np.linalg.eigvals(A)))
    b = rng.standard_normal(n)
    xstar = np.linalg.solve(np.eye(n) - A, b)
    x = np.zeros(n)
    hist = []
    for _ in range(n + 3):
        r = A @ x + b - x
        hist.append((x, r))
        hist = hist[-(n + 1):]
        x, hist = pulay_mix(hist, 0.0)
    assert np.max(np.abs(x - xstar)) < 1e-8


def test_hartree_fock_inner_loop_reaches_closed_form_fixed_point():
    s = generic_system(6, 41, beta=30.0, niw=2048, ntau=33)
    params = O.Params(tol_P=1e-11)
    mu, P, F, G, mom, n_in, n_ev = O.inner_loop(s, params, s.h.copy(), None, 0.0, None,
                                                np.zeros((s.n, s.n)))
    eps, C = R.generalized_eig(F, s.S)
    mu_ref = R.mu_closed_form(eps, s.nelec, s.beta)
    P_ref = R.hf_density(s.S, F, mu_ref, s.beta)
    assert mu == pytest.approx(mu_ref, abs=1e-8)
    assert np.max(np.abs(P - P_ref)) < 1e-8
    assert np.max(np.abs(F - O.fock(s.h, s.v, P))) < 1e-14
    assert np.trace(P @ s.S) == pytest.approx(s.nelec, abs=1e-9)


def test_pulay_restart_factor_zero_is_plain_damping(monkeypatch):
    """With the restart factor at 0 every pass empties the history, so the
    inner loop takes exactly the steps of plain damping (mix_depth 1); Pulay
    mixing reaches the same fixed point in fewer passes.  (A weakly coupled
    system, v_iiii ~ 0.1 Eh, on which plain damping converges.)"""
    import oracle.loop as LP
    s = generic_system(6, 41, beta=30.0, niw=512, ntau=33, vdiag=0.1)
    zero = np.zeros((s.n, s.n))
    kw = dict(tol_P=1e-10, max_inner=300)
    damped = O.inner_loop(s, O.Params(mix_depth=1, **kw), s.h.copy(), None, 0.0, None, zero)
    mixed = O.inner_loop(s, O.Params(**kw), s.h.copy(), None, 0.0, None, zero)
    monkeypatch.setattr(LP, "PULAY_RESTART", 0.0)
    restarted = O.inner_loop(s, O.Params(**kw), s.h.copy(), None, 0.0, None, zero)
    assert restarted[5] == damped[5] and restarted[6] == damped[6]     # passes, evaluations
    np.testing.assert_array_equal(restarted[1], damped[1])
    assert mixed[5] < damped[5]
    assert np.max(np.abs(mixed[1] - damped[1])) < 1e-9


def test_pulay_caps_large_coefficients():
    """Nearly parallel residuals make the minimising coefficients huge; above
    the cap the history is cut to the newest pair (a damped step)."""
    rng = np.random.default_rng(4)
    x1, x2 = rng.standard_normal((2, 4, 4))
    r = rng.standard_normal((4, 4))
    hist = [(x1, r), (x2, 1.001 * r + 1e-9 * rng.standard_normal((4, 4)))]
    got, h = pulay_mix(hist, 0.3)
    assert len(h) == 1
    assert np.allclose(got, x2 + 0.7 * hist[1][1], atol=1e-14)
    # well-separated residuals keep both pairs
    hist = [(x1, r), (x2, rng.standard_normal((4, 4)))]
    _, h = pulay_mix(hist, 0.3)
    assert len(h) == 2
