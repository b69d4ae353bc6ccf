"""The GF2 self-consistency loop (oracle).

Follows the steps of the Supplementary Material ("Implementation of GF2
algorithm"):

1. Reference.  The paper starts from a zero-temperature RHF computed by
   another program.  Reading: the reference is the finite-temperature
   Hartree-Fock solution obtained by running step 2 with Sigma = 0 from
   the core guess F = h ("iteration 0").
2. Build G(i w) from Eq. (GF).
   2.a find mu such that P(G) has the right particle number;
   2.b rebuild F(P) from Eq. (FockMatrix) and update G; repeat 2.a-2.b to
   self-consistency (the "inner loop"), optionally damping P; then
   transform G(i w) -> G(tau).
3. Build Sigma(tau) from Eq. (Sigma) (optionally damped against the
   previous Sigma(tau)), transform Sigma(tau) -> Sigma(i w), go to 2.

Readings for what the paper leaves open (tolerances and order):

* the mu search of each pass starts from the previous pass's mu and slope
  dN/dmu (the first pass of an outer iteration has no slope);
* one inner pass: F = F(P_in) -> mu search at that F -> Dyson solve at
  that mu -> P_out; the residual is r = P_out - P_in and the inner loop
  stops when max|r| < tol_P.  The next input density is the damped
  Pulay/Anderson mix of the last ``mix_depth`` pairs (P_in, r):
  c = argmin |sum_i c_i r_i| subject to sum_i c_i = 1 (Frobenius norm),
  P_in <- sum_i c_i (P_in,i + (1 - a_P) r_i).  With ``mix_depth = 1`` this
  is exactly the paper's damping P_in <- (1 - a_P) P_out + a_P P_in.  The
  mixing history starts empty in every outer iteration.  If the small
  bordered system is singular the history is cut to the newest pair; a
  pass whose max|r| exceeds ``PULAY_RESTART`` (10) times the smallest
  max|r| of the inner loop so far empties the history before its pair is
  added (a damped step; extrapolation over a diverging history is what
  makes Pulay mixing unstable).
  The very first pass of the run (core guess F = h) has no P_in: its
  P_out simply becomes the next P_in;
* on convergence the inner loop returns mu, P = P_out and F = F(P_out);
* the energy of an outer iteration uses the G(i w) of the last Dyson solve
  (with the F and mu of that solve), Sigma(i w), P and F = F(P); G(tau)
  for the next Sigma is the transform of that same G(i w);
* Sigma damping: Sigma(tau) <- (1-a_S) Sigma_new + a_S Sigma_old from the
  second correlated iteration on;
* outer convergence: |dE| < tol_E and max|dP| < tol_P between outer
  iterations.

Pinned (tests/test_oracle_physics.py): iteration by iteration, the Sigma(tau)
an iteration uses is the six-index sum of Eq. (Sigma) over the G(tau) the
previous iteration handed on (the closed-form Hartree-Fock G(tau) after
iteration 0), P = -2 G(beta-) of the handed-on G(tau), F = F(P), and E_2b
equals the imaginary-time form of the two-body energy of the same pair; the
converged state satisfies all of them at once, independently of the Sigma
damping and the mixing depth.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .dyson import find_mu, green_iw, tail_moments, density_from_giw, NoConvergence
from .energy import e_one_body, e_two_body
from .fock import fock
from .fourier import g_iw_to_tau, sigma_tau_to_iw
from .sigma import sigma_tau


@dataclass
class Params:
    tol_mu: float = 1e-12
    tol_N: float = 1e-10
    tol_P: float = 1e-10
    tol_E: float = 1e-11
    max_inner: int = 100
    max_outer: int = 50
    max_bisect: int = 200
    mu_halfwidth: float = 0.5
    damp_P: float = 0.3
    mix_depth: int = 8
    damp_Sigma: float = 0.0
    mu_method: str = "secant"


@dataclass
class State:
    """Outer-loop state; ``iteration`` counts completed outer iterations."""
    mu: float
    F: np.ndarray
    P: Optional[np.ndarray] = None
    G_tau: Optional[np.ndarray] = None
    Sigma_tau: Optional[np.ndarray] = None
    iteration: int = 0
    energy: float = float("nan")


@dataclass
class OuterReport:
    energy: float
    e1b: float
    e2b: float
    dE: float
    dP: float
    mu: float
    n_inner: int
    n_eval: int
    extras: dict = field(default_factory=dict)


# A pass whose max|P_out - P_in| exceeds this factor times the smallest one of
# the inner loop so far drops the Pulay history (restart with a damped step).
PULAY_RESTART = 10.0
# Mixing coefficients larger than this in magnitude cut the history to the
# newest pair, as a singular bordered system does.
PULAY_CMAX = 20.0


def pulay_mix(hist, damp):
    """Damped Pulay/Anderson mix of the history [(x_i, r_i)] (oldest first).

    Solves the bordered system [[B, 1], [1^T, 0]] [c; lam] = [0; 1] with
    B_ij = <r_i, r_j> / max_i <r_i, r_i> (the scaling leaves c unchanged);
    returns sum_i c_i (x_i + (1 - damp) r_i) and the (possibly shortened)
    history.
    """
    while True:
        k = len(hist)
        A = np.zeros((k + 1, k + 1))
        for a in range(k):
            for b in range(k):
                A[a, b] = float(np.sum(hist[a][1] * hist[b][1]))
        A[:k, :k] /= max(float(np.max(np.diag(A)[:k])), 1e-300)
        A[k, :k] = 1.0
        A[:k, k] = 1.0
        rhs = np.zeros(k + 1)
        rhs[k] = 1.0
        c = _solve_pivoted(A, rhs)
        if c is not None and k > 1 and float(np.max(np.abs(c[:k]))) > PULAY_CMAX:
            c = None                # extrapolation too far: treated like a singular system
        if c is not None or k == 1:
            break
        hist = hist[-1:]
    if c is None:
        c = np.array([1.0, 0.0])
    x = sum(c[a] * (hist[a][0] + (1.0 - damp) * hist[a][1]) for a in range(len(hist)))
    return x, hist


def _solve_pivoted(A, b, rel_tol=1e-14):
    """Gaussian elimination with partial pivoting; None if a pivot is negligible."""
    A = A.astype(np.float64).copy()
    b = b.astype(np.float64).copy()
    n = A.shape[0]
    scale = np.max(np.abs(A))
    for k in range(n):
        r = k + int(np.argmax(np.abs(A[k:, k])))
        if abs(A[r, k]) <= rel_tol * scale:
            return None
        if r != k:
            A[[k, r]] = A[[r, k]]
            b[[k, r]] = b[[r, k]]
        for i in range(k + 1, n):
            f = A[i, k] / A[k, k]
            A[i, k:] -= f * A[k, k:]
            b[i] -= f * b[k]
    x = np.zeros(n)
    for k in range(n - 1, -1, -1):
        x[k] = (b[k] - A[k, k + 1:] @ x[k + 1:]) / A[k, k]
    return x


def inner_loop(sysm, params: Params, F, P_in, mu0, Sigma_iw, Sigma1):
    """Steps 2.a-2.b to self-consistency at fixed Sigma.

    ``F`` must equal F(P_in) (or h with P_in None at the start of a run).
    Returns mu, P_out, F(P_out), the last G(i w), its moments,
    #passes, #mu evaluations.
    """
    S, h, v = sysm.S, sysm.h, sysm.v
    beta, niw = sysm.beta, sysm.niw
    mu = mu0
    n_eval = 0
    hist = []
    slope = None
    rbest = float("inf")
    for it in range(1, params.max_inner + 1):
        mu, ne, slope = find_mu(sysm.nelec, S, F, Sigma_iw, Sigma1, beta, niw, mu,
                                halfwidth=params.mu_halfwidth, tol_mu=params.tol_mu,
                                tol_N=params.tol_N, max_steps=params.max_bisect,
                                method=params.mu_method, slope=slope, return_slope=True)
        n_eval += ne
        G = green_iw(mu, S, F, Sigma_iw, beta, niw)
        mom = tail_moments(S, F, mu, Sigma1)
        P_out = density_from_giw(G, *mom, beta)
        if P_in is None:
            P_next = P_out
        else:
            r = P_out - P_in
            rn = float(np.max(np.abs(r)))
            if rn < params.tol_P:
                return mu, P_out, fock(h, v, P_out), G, mom, it, n_eval
            if rn > PULAY_RESTART * rbest:
                hist = []           # restart: the mix below is a damped step
            rbest = min(rbest, rn)
            hist.append((P_in, r))
            hist = hist[-max(1, params.mix_depth):]
            P_next, hist = pulay_mix(hist, params.damp_P)
        P_in = P_next
        F = fock(h, v, P_in)
    raise NoConvergence("inner loop did not converge")


def _method(sysm) -> str:
    """The FFT form for a uniform grid, the defining sum for a given grid."""
    return "direct" if getattr(sysm, "tau", None) is not None else "fft"


def outer_iteration(sysm, params: Params, st: State) -> OuterReport:
    """One outer iteration.  Iteration 0 is the finite-beta HF reference."""
    n = sysm.n
    beta, niw, ntau = sysm.beta, sysm.niw, sysm.ntau
    if st.iteration == 0:
        Sigma_iw = None
        Sigma1 = np.zeros((n, n))
        Sig_tau = np.zeros((ntau, n, n))
    else:
        Sig_tau = sigma_tau(st.G_tau, sysm.v)
        if st.iteration >= 2 and params.damp_Sigma > 0.0:
            Sig_tau = (1.0 - params.damp_Sigma) * Sig_tau + params.damp_Sigma * st.Sigma_tau
        Sigma_iw, Sigma1 = sigma_tau_to_iw(Sig_tau, beta, niw, method=_method(sysm),
                                           tau=getattr(sysm, "tau", None))
    P_prev = st.P
    mu, P, F, G, mom, n_inner, n_eval = inner_loop(
        sysm, params, st.F, st.P, st.mu, Sigma_iw, Sigma1)
    e1 = e_one_body(P, sysm.h, F)
    e2 = 0.0 if Sigma_iw is None else e_two_body(G, Sigma_iw, mom[0], Sigma1, beta)
    E = e1 + e2
    G_tau = g_iw_to_tau(G, *mom, beta, ntau, tau=getattr(sysm, "tau", None))
    dE = E - st.energy if np.isfinite(st.energy) else float("inf")
    dP = float(np.max(np.abs(P - P_prev))) if P_prev is not None else float("inf")
    st.mu, st.F, st.P, st.G_tau, st.Sigma_tau = mu, F, P, G_tau, Sig_tau
    st.energy = E
    st.iteration += 1
    return OuterReport(E, e1, e2, dE, dP, mu, n_inner, n_eval)


def run(sysm, params: Params = None, mu0: float = 0.0, max_outer: int = None, callback=None):
    """Iterate from the core guess F = h until |dE| < tol_E and max|dP| < tol_P."""
    params = params or Params()
    st = State(mu=mu0, F=sysm.h.copy())
    reports = []
    limit = params.max_outer if max_outer is None else max_outer
    for _ in range(limit):
        r = outer_iteration(sysm, params, st)
        reports.append(r)
        if callback:
            callback(st, r)
        if st.iteration > 1 and abs(r.dE) < params.tol_E and r.dP < params.tol_P:
            return st, reports, True
    return st, reports, False
