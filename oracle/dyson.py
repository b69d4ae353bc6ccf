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

``method='secant'`` builds the bracket from the previous mu instead: it
evaluates N at mu0 first (accepting it when |N - N_e| < tol_N), then steps
by -f(mu0)/slope, where slope is dN/dmu from the previous search (or
1/hw without one), clamped to [4 tol_mu, hw] in size, and doubles the step
while the sign does not change; the bracket found is then closed by the
Illinois iteration above.  It returns the secant slope of the final
bracket for the next search.
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
            tol_mu=1e-12, tol_N=1e-10, max_steps=200, method="illinois", slope=None,
            return_slope=False):
    """Bracketing search for mu with tr(P(mu) S) = nelec.

    Returns (mu, evaluations), or (mu, evaluations, slope) with return_slope.
    """
    n = S.shape[0]
    if nelec < 0 or nelec > 2 * n:
        raise BracketError(f"nelec={nelec} outside [0, {2 * n}]")
    if method not in ("bisect", "illinois", "secant"):
        raise ValueError(method)

    def f(mu):
        return particle_number(mu, S, F, Sigma_iw, Sigma1, beta, niw) - nelec

    def done(mu, ev, lo=None, f_lo=None, hi=None, f_hi=None):
        sl = slope
        if lo is not None and hi is not None and hi > lo and f_hi > f_lo:
            sl = (f_hi - f_lo) / (hi - lo)
        return (mu, ev, sl) if return_slope else (mu, ev)

    evals = 0
    if method == "secant":
        a = mu0
        fa = f(a); evals += 1
        if abs(fa) < tol_N:
            return done(a, evals)
        s_ = slope if (slope is not None and slope > 0.0) else 1.0 / halfwidth
        step = -fa / s_
        mag = min(max(abs(step), 4.0 * tol_mu), halfwidth)
        step = mag if step > 0.0 else -mag
        b = a + step
        while True:
            if evals > max_steps:
                raise BracketError("mu bracket not found")
            fb = f(b); evals += 1
            if abs(fb) < tol_N:
                lo, flo, hi, fhi = (a, fa, b, fb) if a < b else (b, fb, a, fa)
                return done(b, evals, lo, flo, hi, fhi)
            if (fb > 0.0) != (fa > 0.0):
                break
            a, fa, b = b, fb, b + 2.0 * (b - a)
        lo, f_lo, hi, f_hi = (a, fa, b, fb) if a < b else (b, fb, a, fa)
    else:
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
    t_lo, t_hi = f_lo, f_hi          # true values at the bracket ends
    side = 0
    for _ in range(max_steps):
        mid = 0.5 * (lo + hi)
        if method != "bisect" and f_hi > f_lo:
            x = (lo * f_hi - hi * f_lo) / (f_hi - f_lo)
            if lo < x < hi:
                mid = x
        fm = f(mid); evals += 1
        if abs(fm) < tol_N:
            if fm < 0.0:
                return done(mid, evals, mid, fm, hi, t_hi)
            return done(mid, evals, lo, t_lo, mid, fm)
        if fm < 0.0:
            lo, f_lo, t_lo = mid, fm, fm
            if side == -1:
                f_hi *= 0.5
            side = -1
        else:
            hi, f_hi, t_hi = mid, fm, fm
            if side == 1:
                f_lo *= 0.5
            side = 1
        if hi - lo < tol_mu:
            return done(0.5 * (lo + hi), evals, lo, t_lo, hi, t_hi)
    raise NoConvergence("mu search did not converge")
