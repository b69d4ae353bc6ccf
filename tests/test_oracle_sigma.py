"""Pins for the oracle's Eq. (Sigma): brute force, symmetry, special cases."""
import numpy as np
import pytest

import oracle as O
from synthetic import random_integrals, random_symmetric


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_factored_equals_literal_six_index_sum(n):
    rng = np.random.default_rng(100 + n)
    v = random_integrals(rng, n)
    G = random_symmetric(rng, n)
    Gb = random_symmetric(rng, n)
    ref = O.sigma_bruteforce(G, Gb, v)
    fac = O.sigma_factored(G, Gb, v)
    lit = O.sigma_literal(G, Gb, v)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(fac - ref)) <= 1e-13 * scale
    assert np.max(np.abs(lit - ref)) <= 1e-13 * scale


def test_bruteforce_catches_planted_index_mistake():
    """Bra/ket indices mixed up (v_iqmk for v_imqk) must change the result,
    so the brute-force pin has teeth."""
    rng = np.random.default_rng(7)
    n = 3
    v = random_integrals(rng, n)
    G = rng.standard_normal((n, n))
    Gb = rng.standard_normal((n, n))
    good = O.sigma_bruteforce(G, Gb, v)
    W = O.bracket_W(v)
    bad = -np.einsum("kl,mn,pq,iqmk,lpnj->ij", G, G, Gb, v, W)
    assert np.max(np.abs(good - bad)) > 1e-3 * np.max(np.abs(good))
    # exchange sign flipped
    W_bad = 2.0 * v + np.transpose(v, (2, 1, 0, 3))
    bad2 = -np.einsum("kl,mn,pq,imqk,lpnj->ij", G, G, Gb, v, W_bad)
    assert np.max(np.abs(good - bad2)) > 1e-3 * np.max(np.abs(good))


def test_sigma_symmetric_for_symmetric_inputs():
    rng = np.random.default_rng(11)
    n = 6
    v = random_integrals(rng, n)
    G = random_symmetric(rng, n)
    Gb = random_symmetric(rng, n)
    S = O.sigma_factored(G, Gb, v)
    assert np.max(np.abs(S - S.T)) <= 1e-14 * np.max(np.abs(S))


def test_sigma_vanishes_without_interaction():
    rng = np.random.default_rng(12)
    n = 5
    G = random_symmetric(rng, n)
    assert np.all(O.sigma_factored(G, G, np.zeros((n,) * 4)) == 0.0)


def test_hubbard_atom_second_order_sigma():
    """N=1, half filling: G(tau) = -1/2, Sigma(tau) = -U^2/8 (textbook)."""
    U = 1.7
    v = np.full((1, 1, 1, 1), U)
    G = np.array([[-0.5]])
    Gb = np.array([[0.5]])          # G(-tau) = -G(beta - tau) = +1/2
    assert O.sigma_factored(G, Gb, v)[0, 0] == pytest.approx(-U * U / 8.0, rel=1e-15)


def test_sigma_tau_uses_antiperiodic_gbar():
    rng = np.random.default_rng(13)
    n, ntau = 3, 6
    v = random_integrals(rng, n)
    Gt = np.stack([random_symmetric(rng, n) for _ in range(ntau)])
    St = O.sigma_tau(Gt, v)
    for k in range(ntau):
        ref = O.sigma_bruteforce(Gt[k], -Gt[ntau - 1 - k], v)
        assert np.allclose(St[k], ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))


def test_sigma_linear_in_each_green_function_argument():
    """Eq. (Sigma) is trilinear in (G, G, Gbar) -> homogeneous of degree 2 in G."""
    rng = np.random.default_rng(14)
    n = 4
    v = random_integrals(rng, n)
    G = random_symmetric(rng, n)
    Gb = random_symmetric(rng, n)
    a = 1.7
    base = O.sigma_factored(G, Gb, v)
    assert np.allclose(O.sigma_factored(a * G, Gb, v), a * a * base, rtol=1e-13, atol=0)
    assert np.allclose(O.sigma_factored(G, a * Gb, v), a * base, rtol=1e-13, atol=0)
