"""Pins for the oracle's imaginary-time <-> Matsubara transforms."""
import numpy as np
import pytest

import oracle as O
from oracle import reference as R
from synthetic import generic_system


def _poly_transform(coef, beta, w):
    """int_0^beta exp(i w tau) sum_k coef[k] tau^k dtau via the recursion
    I_k = -beta^k / x - (k/x) I_{k-1},  I_0 = -2/x  (x = i w, exp(x beta) = -1)."""
    x = 1j * w
    out = np.zeros(w.shape + coef.shape[1:], dtype=complex)
    Ik = -2.0 / x
    for k in range(coef.shape[0]):
        if k > 0:
            Ik = -beta ** k / x - (k / x) * Ik
        out += Ik[(...,) + (None,) * (coef.ndim - 1)] * coef[k][None]
    return out


@pytest.mark.parametrize("method", ["direct", "fft"])
def test_tau_to_iw_exact_for_cubic_polynomials(method):
    rng = np.random.default_rng(3)
    beta, ntau, niw, n = 7.5, 33, 300, 3
    coef = rng.standard_normal((4, n, n))
    tau = O.tau_grid(beta, ntau)
    Y = sum(coef[k][None] * tau[:, None, None] ** k for k in range(4))
    got, s1 = O.sigma_tau_to_iw(Y, beta, niw, method=method)
    ref = _poly_transform(coef, beta, O.matsubara(beta, niw))
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.allclose(s1, -(Y[0] + Y[-1]), rtol=0, atol=1e-15)


def test_tau_to_iw_direct_equals_fft_for_generic_data():
    rng = np.random.default_rng(4)
    beta, ntau, niw = 10.0, 41, 500
    Y = rng.standard_normal((ntau, 2, 2))
    a, _ = O.sigma_tau_to_iw(Y, beta, niw, method="direct")
    b, _ = O.sigma_tau_to_iw(Y, beta, niw, method="fft")
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_hubbard_atom_constant_sigma_transforms_to_u2_over_4iw():
    U, beta, ntau, niw = 1.3, 20.0, 17, 64
    Y = np.full((ntau, 1, 1), -U * U / 8.0)
    S_iw, s1 = O.sigma_tau_to_iw(Y, beta, niw)
    iw = 1j * O.matsubara(beta, niw)
    assert np.max(np.abs(S_iw[:, 0, 0] - U * U / (4.0 * iw))) < 1e-15
    assert s1[0, 0] == pytest.approx(U * U / 4.0, rel=1e-15)


def _hf_case(beta=10.0):
    s = generic_system(4, 21, beta=beta)
    eps, C = R.generalized_eig(s.h, s.S)
    mu = 0.5 * (eps[1] + eps[2])
    return s, mu


def test_iw_to_tau_reproduces_closed_form_free_green_function():
    s, mu = _hf_case()
    beta, niw, ntau = s.beta, 4096, 65
    Giw = R.hf_green_iw(s.S, s.h, mu, beta, niw)
    G1, G2, G3 = O.tail_moments(s.S, s.h, mu)
    for method in ("direct", "fft"):
        Gt = O.g_iw_to_tau(Giw, G1, G2, G3, beta, ntau, method=method)
        ref = R.hf_green_tau(s.S, s.h, mu, beta, O.tau_grid(beta, ntau))
        assert np.max(np.abs(Gt - ref)) < 1e-8


def test_tau_to_iw_of_closed_form_g_matches_exact_matsubara_values():
    s, mu = _hf_case()
    beta, niw, ntau = s.beta, 200, 2049
    Gt = R.hf_green_tau(s.S, s.h, mu, beta, O.tau_grid(beta, ntau))
    got, s1 = O.sigma_tau_to_iw(Gt, beta, niw)
    ref = R.hf_green_iw(s.S, s.h, mu, beta, niw)
    assert np.max(np.abs(got - ref)) < 1e-8
    # first moment of G is S^-1 (G(0+) + G(beta-) = -S^-1)
    assert np.max(np.abs(s1 - np.linalg.inv(s.S))) < 1e-12


def test_endpoints_sum_to_minus_inverse_overlap():
    """G(0+) + G(beta-) = -S^-1 holds for the tail-corrected transform."""
    s, mu = _hf_case()
    rng = np.random.default_rng(9)
    beta, niw, ntau, n = s.beta, 256, 33, s.n
    Giw = R.hf_green_iw(s.S, s.h, mu, beta, niw)
    Giw = Giw + 1e-3 * (rng.standard_normal(Giw.shape) + 1j * rng.standard_normal(Giw.shape))
    Giw = 0.5 * (Giw + Giw.transpose(0, 2, 1))
    G1, G2, G3 = O.tail_moments(s.S, s.h, mu)
    Gt = O.g_iw_to_tau(Giw, G1, G2, G3, beta, ntau)
    assert np.max(np.abs(Gt[0] + Gt[-1] + np.linalg.inv(s.S))) < 1e-13 * n


def test_tail_moments_match_large_frequency_expansion():
    rng = np.random.default_rng(10)
    s, mu = _hf_case()
    n = s.n
    Sig1 = rng.standard_normal((n, n)); Sig1 = Sig1 + Sig1.T
    w = 1e3
    iw = 1j * w
    Sig = Sig1 / iw
    G = np.linalg.inv((iw + mu) * s.S - s.h - Sig)
    G1, G2, G3 = O.tail_moments(s.S, s.h, mu, Sig1)
    resid = G - (G1 / iw + G2 / iw ** 2 + G3 / iw ** 3)
    assert np.max(np.abs(resid)) < 50.0 / w ** 4
    # dropping the Sigma_1 term is visible at this order
    G3_bad = O.tail_moments(s.S, s.h, mu)[2]
    bad = G - (G1 / iw + G2 / iw ** 2 + G3_bad / iw ** 3)
    assert np.max(np.abs(bad)) > 10.0 * np.max(np.abs(resid))
