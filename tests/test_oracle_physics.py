"""Physics pins for the oracle: MP2 limit, Hubbard atom, size-extensivity,
AO-basis invariance, the paper's beta criterion and the energy functional."""
import numpy as np
import pytest

import oracle as O
from oracle import reference as R
from oracle.energy import e_two_body_tau
from synthetic import System, generic_system


def _rhf_case(seed=7, n=4):
    """A gapped one-particle reference: orbitals of F0 = h.  The identities
    between Eq. (Sigma) and the MO-basis sums hold for any reference F0."""
    s = generic_system(n, seed, naux=2 * n, beta=50.0, niw=4096, ntau=2001)
    F0 = s.h.copy()
    eps, C = R.generalized_eig(F0, s.S)
    nocc = s.nelec // 2
    mu = 0.5 * (eps[nocc - 1] + eps[nocc])
    return s, None, eps, C, F0, mu


def test_closed_form_second_order_sum_tends_to_twice_mp2():
    """(1/beta) sum_n tr[G0 Sigma[G0]] -> 2 E_MP2 as beta -> infinity."""
    s, E0, eps, C, F0, mu = _rhf_case()
    emp2 = R.mp2_energy(C, eps, s.v, s.nelec // 2)
    assert emp2 < 0
    t2 = R.e2b_hf_closed_form(s.S, F0, mu, 100.0, s.v)
    assert 0.5 * t2 == pytest.approx(emp2, rel=1e-10)
    # and it is a genuine finite-temperature quantity below that
    assert abs(0.5 * R.e2b_hf_closed_form(s.S, F0, mu, 5.0, s.v) - emp2) > 1e-4


def test_numerical_first_iteration_energy_matches_closed_form():
    """Eq. (Sigma) on the closed-form G0(tau), spline transform, Galitskii-Migdal
    Matsubara sum with tail: equals the closed form at finite beta."""
    s, E0, eps, C, F0, mu = _rhf_case()
    beta, ntau, niw = 20.0, 2001, 4000
    tau = O.tau_grid(beta, ntau)
    Gt = R.hf_green_tau(s.S, F0, mu, beta, tau)
    St = O.sigma_tau(Gt, s.v)
    Siw, S1 = O.sigma_tau_to_iw(St, beta, niw)
    Giw = R.hf_green_iw(s.S, F0, mu, beta, niw)
    e_iw = O.e_two_body(Giw, Siw, np.linalg.inv(s.S), S1, beta)
    ref = R.e2b_hf_closed_form(s.S, F0, mu, beta, s.v)
    assert e_iw == pytest.approx(ref, rel=2e-8)
    assert e_two_body_tau(St, Gt, beta) == pytest.approx(ref, rel=1e-6)


def test_energy_tail_correction_matters():
    s, E0, eps, C, F0, mu = _rhf_case()
    beta, ntau, niw = 20.0, 513, 200
    Gt = R.hf_green_tau(s.S, F0, mu, beta, O.tau_grid(beta, ntau))
    Siw, S1 = O.sigma_tau_to_iw(O.sigma_tau(Gt, s.v), beta, niw)
    Giw = R.hf_green_iw(s.S, F0, mu, beta, niw)
    ref = R.e2b_hf_closed_form(s.S, F0, mu, beta, s.v)
    with_tail = O.e_two_body(Giw, Siw, np.linalg.inv(s.S), S1, beta)
    head_only = O.e_two_body(Giw, Siw, np.linalg.inv(s.S), 0 * S1, beta)
    assert abs(with_tail - ref) < 0.1 * abs(head_only - ref)


def test_hubbard_atom_reference_and_first_sigma():
    """N=1, S=1, v=U, one electron: mu = h + U/2, G(tau) = -1/2,
    Sigma(i w) = U^2/(4 i w)."""
    U, h0 = 1.0, -0.7
    s = System(name="atom", S=np.eye(1), h=np.array([[h0]]),
               v=np.full((1, 1, 1, 1), U), B=np.full((1, 1, 1), np.sqrt(U)),
               nelec=1, beta=10.0, niw=1024, ntau=33)
    st = O.State(mu=0.0, F=s.h.copy())
    O.outer_iteration(s, O.Params(tol_P=1e-12, tol_N=1e-13), st)
    assert st.mu == pytest.approx(h0 + 0.5 * U, abs=1e-9)
    assert np.max(np.abs(st.G_tau + 0.5)) < 1e-9
    St = O.sigma_tau(st.G_tau, s.v)
    assert np.max(np.abs(St + U * U / 8.0)) < 1e-9
    Siw, _ = O.sigma_tau_to_iw(St, s.beta, s.niw)
    iw = 1j * O.matsubara(s.beta, s.niw)
    assert np.max(np.abs(Siw[:, 0, 0] - U * U / (4 * iw))) < 1e-9


def _block_diag_system(a: System) -> System:
    n = a.n
    S = np.zeros((2 * n, 2 * n)); h = np.zeros_like(S)
    S[:n, :n] = S[n:, n:] = a.S
    h[:n, :n] = h[n:, n:] = a.h
    v = np.zeros((2 * n,) * 4)
    v[:n, :n, :n, :n] = a.v
    v[n:, n:, n:, n:] = a.v
    return System(name="dimer", S=S, h=h, v=v, B=np.zeros((0, 2 * n, 2 * n)),
                  nelec=2 * a.nelec, beta=a.beta, niw=a.niw, ntau=a.ntau)


def test_size_extensivity_two_decoupled_copies():
    a = generic_system(3, 51, naux=6, beta=10.0, niw=512, ntau=65, nelec=2)
    b = _block_diag_system(a)
    p = O.Params(tol_P=1e-12, tol_N=1e-12)
    sa, sb = O.State(mu=0.0, F=a.h.copy()), O.State(mu=0.0, F=b.h.copy())
    for _ in range(2):
        ra = O.outer_iteration(a, p, sa)
        rb = O.outer_iteration(b, p, sb)
        assert rb.energy == pytest.approx(2 * ra.energy, rel=1e-9)
    n = a.n
    St = O.sigma_tau(sb.G_tau, b.v)
    assert np.max(np.abs(St[:, :n, n:])) < 1e-14


def test_ao_basis_invariance():
    """S -> X^T S X, h -> X^T h X, v transformed on all four indices: the
    energy is invariant and Sigma transforms covariantly."""
    a = generic_system(4, 61, naux=8, beta=10.0, niw=512, ntau=65)
    rng = np.random.default_rng(0)
    X = np.eye(a.n) + 0.2 * rng.standard_normal((a.n, a.n))
    v2 = np.einsum("pi,qj,rk,sl,pqrs->ijkl", X, X, X, X, a.v)
    b = System(name="rot", S=X.T @ a.S @ X, h=X.T @ a.h @ X, v=v2, B=np.zeros((0, a.n, a.n)),
               nelec=a.nelec, beta=a.beta, niw=a.niw, ntau=a.ntau)
    p = O.Params(tol_P=1e-12, tol_N=1e-12)
    sa, sb = O.State(mu=0.0, F=a.h.copy()), O.State(mu=0.0, F=b.h.copy())
    for _ in range(2):
        ra = O.outer_iteration(a, p, sa)
        rb = O.outer_iteration(b, p, sb)
        assert rb.energy == pytest.approx(ra.energy, rel=1e-9)
    Sa = O.sigma_tau(sa.G_tau, a.v)
    Sb = O.sigma_tau(sb.G_tau, b.v)
    assert np.max(np.abs(Sb - np.einsum("ki,tkl,lj->tij", X, Sa, X))) < 1e-9


def test_finite_beta_hf_approaches_zero_temperature_rhf():
    """The paper picks beta so that the HF Green's function reproduces the HF
    energy and particle number; the finite-beta HF energy tends to the
    zero-temperature RHF energy as beta grows."""
    kw = dict(naux=8, vdiag=0.2)
    base = generic_system(4, 7, **kw)
    E0, *_ = R.rhf_zero_T(base.S, base.h, base.v, base.nelec)
    gaps = []
    for beta in (5.0, 20.0, 100.0, 400.0):
        s = generic_system(4, 7, beta=beta, niw=8192, ntau=33, **kw)
        st = O.State(mu=0.0, F=s.h.copy())
        r = O.outer_iteration(s, O.Params(tol_P=1e-11), st)
        assert np.trace(st.P @ s.S) == pytest.approx(s.nelec, abs=1e-8)
        gaps.append(abs(r.energy - E0))
    assert gaps[0] > gaps[1] > gaps[2] > gaps[3]
    assert gaps[3] < 1e-6


@pytest.mark.slow
def test_n10_workload_converges_with_sigma_damping():
    """The N=10 workload runs to self-consistency with Sigma damping 0.5."""
    from synthetic import small_molecule
    s = small_molecule()
    s.niw, s.ntau = 1024, 129
    p = O.Params(damp_Sigma=0.5, tol_E=1e-8, tol_P=1e-7)
    st, reps, conv = O.run(s, p, mu0=-1.0, max_outer=60)
    assert conv
    assert reps[-1].e2b < 0.0
    assert np.trace(st.P @ s.S) == pytest.approx(s.nelec, abs=1e-8)


# ---- composition of the outer loop (Supplementary Material, steps 2-3) ----------
#
# Each outer iteration must hand on the right objects: Sigma(tau) of Eq. (Sigma)
# from the G(tau) the previous iteration produced, the inner loop at that fixed
# Sigma, the Galitskii-Migdal energy from the Green's function / self-energy pair
# of the last Dyson solve, and G(tau) from that same solve.  The checks below use
# routes that do not go through the loop: the Hartree-Fock Green's function in
# closed form (eigenvectors of the generalized problem), the literal six-index sum
# of Eq. (Sigma), the imaginary-time form of the two-body energy,
# E_2b = -int_0^beta tr[Sigma(tau) G(beta - tau)] dtau, and the density as
# -2 G(beta-) of the handed-on G(tau).

def _loop_case(ntau=1025):
    return generic_system(4, 11, naux=8, beta=10.0, niw=1024, ntau=ntau)


def _fock_direct(h, v, P):
    """Eq. (FockMatrix) written out: F_ij = h_ij + sum_kl P_kl (v_ijlk - v_iklj / 2)."""
    n = h.shape[0]
    F = h.copy()
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for l in range(n):
                    F[i, j] += P[k, l] * (v[i, j, l, k] - 0.5 * v[i, k, l, j])
    return F


def test_loop_hands_on_sigma_and_green_function_iteration_by_iteration():
    s = _loop_case()
    p = O.Params(tol_P=1e-12, tol_N=1e-12, damp_Sigma=0.0)
    st = O.State(mu=-1.0, F=s.h.copy())
    O.outer_iteration(s, p, st)
    # iteration 0 is the finite-beta Hartree-Fock solution: its G(tau) is the
    # closed form at the final F and mu
    tau = O.tau_grid(s.beta, s.ntau)
    G_hf = R.hf_green_tau(s.S, st.F, st.mu, s.beta, tau)
    assert np.max(np.abs(st.G_tau - G_hf)) < 1e-9
    ks = [0, 1, 300, 512, 1023, 1024]
    G_prev = G_hf
    for it in (1, 2, 3):
        rep = O.outer_iteration(s, p, st)
        # Sigma(tau) of this iteration = Eq. (Sigma) (six-index sum) of the previous G(tau)
        Gb = O.gbar_from_gtau(G_prev)
        ref = np.stack([O.sigma_bruteforce(G_prev[k], Gb[k], s.v) for k in ks])
        tol = 1e-9 if it == 1 else 1e-12      # iteration 1: closed form vs transformed G_HF
        assert np.max(np.abs(st.Sigma_tau[ks] - ref)) < tol * np.max(np.abs(ref))
        # the density and the handed-on G(tau) come from the same (last) Dyson solve
        assert np.max(np.abs(st.P + 2.0 * st.G_tau[-1])) < 1e-12
        assert np.trace(st.P @ s.S) == pytest.approx(s.nelec, abs=1e-10)
        # F = F(P) and the one-body energy of that pair
        assert np.max(np.abs(st.F - _fock_direct(s.h, s.v, st.P))) < 1e-12
        assert rep.e1b == pytest.approx(0.5 * np.sum(st.P * (s.h + st.F)), abs=1e-12)
        # E_2b of the Sigma used in the inner loop and the G of its last solve
        # (imaginary-time form; Simpson on 1025 points is good to ~1e-8 Eh here)
        assert rep.e2b == pytest.approx(e_two_body_tau(st.Sigma_tau, st.G_tau, s.beta), abs=1e-7)
        assert rep.energy == pytest.approx(rep.e1b + rep.e2b, abs=1e-14)
        G_prev = st.G_tau.copy()


@pytest.mark.slow
def test_converged_loop_is_a_fixed_point_of_the_equations():
    """Run to |dE| < 1e-12: the final state satisfies Eq. (Sigma), Eq. (GF) with
    the density as -2 G(beta-), Eq. (FockMatrix), tr(PS) = N_e and the energy
    functional at once, and the fixed point does not depend on the Sigma damping
    or on the depth of the density mixing."""
    s = _loop_case(ntau=513)
    energies, dens = [], []
    # plain damping (mix_depth 1) needs a heavier density damping on this system
    for damp, depth, damp_P in ((0.3, 8, 0.3), (0.5, 8, 0.3), (0.3, 1, 0.7), (0.5, 1, 0.7)):
        p = O.Params(tol_P=1e-12, tol_N=1e-12, tol_E=1e-12, damp_Sigma=damp, mix_depth=depth,
                     damp_P=damp_P, max_inner=1000, max_outer=300)
        st, reps, conv = O.run(s, p, mu0=-1.0)
        assert conv, (damp, depth)
        energies.append(st.energy)
        dens.append(st.P)
        if (damp, depth) != (0.3, 8):
            continue
        # Eq. (Sigma): the stored (damped) Sigma(tau) is Sigma[G(tau)] of the final G
        ks = [0, 5, 256, 400, 512]
        Gb = O.gbar_from_gtau(st.G_tau)
        ref = np.stack([O.sigma_bruteforce(st.G_tau[k], Gb[k], s.v) for k in ks])
        assert np.max(np.abs(st.Sigma_tau[ks] - ref)) < 1e-10 * np.max(np.abs(ref))
        # density = -2 G(beta-), particle number, Eq. (FockMatrix)
        assert np.max(np.abs(st.P + 2.0 * st.G_tau[-1])) < 1e-12
        assert np.trace(st.P @ s.S) == pytest.approx(s.nelec, abs=1e-10)
        assert np.max(np.abs(st.F - _fock_direct(s.h, s.v, st.P))) < 1e-11
        # energy functional of the final pair (imaginary-time E_2b, Simpson on 513 points)
        e1 = 0.5 * np.sum(st.P * (s.h + st.F))
        assert st.energy == pytest.approx(e1 + e_two_body_tau(st.Sigma_tau, st.G_tau, s.beta),
                                          abs=1e-6)
        assert reps[-1].e2b < 0.0
    assert max(energies) - min(energies) < 1e-10
    assert max(float(np.max(np.abs(d - dens[0]))) for d in dens) < 1e-9
