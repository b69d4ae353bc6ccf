"""Dyson equation, high-frequency tail, density and chemical potential (oracle).

Eq. (GF) (Implementation section and Supplementary Material):

    G(i w_n) = [ (mu + i w_n) S - F - Sigma(i w_n) ]^{-1}.

Tail moments (the analytic high-frequency tail of the Implementation
section).  Expanding Eq. (GF) in 1/(i w) with H = F - mu S and
Sigma(i w) = Sigma_1/(i w) + O(w^-2):

    G1 = S^-1,  G2 = S^-1 H S^-1,  G3 = S^-1 H S^-1 H S^-1 + S^-1 Sigma_1 S^-1.

Density.  The paper writes P = (1/2 pi i) closed-contour integral of G.
At finite temperature the reading is P = -2 G(beta-) (spin-summed), which
with the tail summed analytically is

    P = (4/beta) sum_{n<niw} Re[G - G1/(iw) - G2/(iw)^2 - G3/(iw)^3]
        + G1 - (beta/2) G2.

Chemical potential (step 2.a: "find mu such that P(G) has good particle
number"; the method is not given).  Reading: a bracketing root search on
N(mu) = tr(P(mu) S), which increases monotonically with mu.  The initial
bracket is [mu0 - hw, mu0 + hw] around the previous mu; while N(lo) > N_e
the bracket moves down by its own width ([lo - w, lo]), while N(hi) < N_e
it moves up ([hi, hi + w]).  Each step evaluates one interior point; it is
accepted when |N - N_e| < tol_N, otherwise it replaces the end of the
bracket with the same sign; the search stops when the bracket is
narrower than tol_mu and returns its midpoint.  The interior point is
either the midpoint (``method='bisect'``) or the Illinois modified
regula-falsi point (``method='illinois'``: the secant through the two
ends, with the function value kept at an end that survives two steps in
a row halved; the midpoint is used whenever the secant point is not
strictly inside the bracket).
"""
import numpy as np

from .grids import matsubara


class BracketError(RuntimeError):
    """N_e cannot be bracketed (N_e outside [0, 2n] or a non-monotone N)."""


class NoConvergence(RuntimeError):
    """An iteration did not reach its tolerance within its step limit."""


def tail_moments(S, F, mu, Sigma1=None):
    """(G1, G2, G3) of Eq. (GF) for chemical potential mu."""
    Sinv = np.linalg.inv(S)
    H = F - mu * S
    G1 = Sinv
    G2 = Sinv @ H @ Sinv
    G3 = Sinv @ H @ Sinv @ H @ Sinv
    if Sigma1 is not None:
        G3 = G3 + Sinv @ Sigma1 @ Sinv
    return G1, G2, G3


def green_iw(mu, S, F, Sigma_iw, beta, niw, n_idx=None):
    """Eq. (GF) for each requested Matsubara frequency (LU with partial pivoting)."""
    ns = np.arange(niw) if n_idx is None else np.asarray(n_idx)
    iw = 1j * matsubara(beta, niw)[ns]
    A = (iw[:, None, None] + mu) * S[None] - F[None]
    if Sigma_iw is not None:
        A = A - (Sigma_iw if n_idx is None else Sigma_iw[ns])
    return np.linalg.inv(A)


def density_from_giw(G_iw, G1, G2, G3, beta):
    """P = -2 G(beta-) with the tail summed in closed form."""
    niw = G_iw.shape[0]
    iw = 1j * matsubara(beta, niw)[:, None, None]
    R = G_iw - G1 / iw - G2 / iw ** 2 - G3 / iw ** 3
    return (4.0 / beta) * R.real.sum(axis=0) + G1 - 0.5 * beta * G2


def particle_number(mu, S, F, Sigma_iw, Sigma1, beta, niw):
    """N(mu) = tr(P(mu) S) at fixed F and Sigma."""
    G = green_iw(mu, S, F, Sigma_iw, beta, niw)
    G1, G2, G3 = tail_moments(S, F, mu, Sigma1)
    P = density_from_giw(G, G1, G2, G3, beta)
    return float(np.trace(P @ S))


def find_mu(nelec, S, F, Sigma_iw, Sigma1, beta, niw, mu0=0.0, *, halfwidth=0.5,
            tol_mu=1e-12, tol_N=1e-10, max_steps=200, method="illinois"):
    """Bracketing search for mu with tr(P(mu) S) = nelec.  Returns (mu, evaluations)."""
    n = S.shape[0]
    if nelec < 0 or nelec > 2 * n:
        raise BracketError(f"nelec={nelec} outside [0, {2 * n}]")
    if method not in ("bisect", "illinois"):
        raise ValueError(method)

    def f(mu):
        return particle_number(mu, S, F, Sigma_iw, Sigma1, beta, niw) - nelec

    evals = 0
    lo, hi = mu0 - halfwidth, mu0 + halfwidth
    f_lo = f(lo); evals += 1
    while f_lo > 0.0:
        if evals > max_steps:
            raise BracketError("lower end of the mu bracket not found")
        lo, hi = lo - (hi - lo), lo
        f_lo = f(lo); evals += 1
    f_hi = f(hi); evals += 1
    while f_hi < 0.0:
        if evals > max_steps:
            raise BracketError("upper end of the mu bracket not found")
        lo, hi = hi, hi + (hi - lo)
        f_hi = f(hi); evals += 1
    side = 0
    for _ in range(max_steps):
        mid = 0.5 * (lo + hi)
        if method == "illinois" and f_hi > f_lo:
            x = (lo * f_hi - hi * f_lo) / (f_hi - f_lo)
            if lo < x < hi:
                mid = x
        fm = f(mid); evals += 1
        if abs(fm) < tol_N:
            return mid, evals
        if fm < 0.0:
            lo, f_lo = mid, fm
            if side == -1:
                f_hi *= 0.5
            side = -1
        else:
            hi, f_hi = mid, fm
            if side == 1:
                f_lo *= 0.5
            side = 1
        if hi - lo < tol_mu:
            return 0.5 * (lo + hi), evals
    raise NoConvergence("mu search did not converge")
