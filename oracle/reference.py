"""Closed forms used to pin the oracle (test infrastructure only).

Nothing here is part of the GF2 iteration; these are independent
textbook results the iteration must reproduce in special cases:

* non-interacting / Hartree-Fock Green's function at finite temperature
  from the generalized eigenproblem F C = S C eps (C^T S C = 1):
  G(tau) = -C (1-f) exp(-(eps-mu) tau) C^T,  G(i w) = C (i w + mu - eps)^-1 C^T,
  P = 2 C f C^T, with f the Fermi function;
* zero-temperature restricted Hartree-Fock (Roothaan iterations with
  Aufbau filling), the reference of step 1 of the Supplementary Material;
* closed-shell MP2 in spatial orbitals,
  E_MP2 = sum_{ijab} (ia|jb)[2(ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b);
* the Matsubara sum of tr[G0 Sigma[G0]] for a Hartree-Fock G0 at finite
  beta in closed form (derived by inserting G0(tau) into Eq. (Sigma) and
  integrating exp(-Delta tau) over [0, beta]).
"""
import numpy as np
from scipy.linalg import eigh
from scipy.optimize import brentq
from scipy.special import expit

from .fock import fock


def generalized_eig(F, S):
    eps, C = eigh(F, S)
    return eps, C


def fermi(x, beta):
    return expit(-beta * np.asarray(x))


def hf_green_tau(S, F, mu, beta, tau):
    """G0(tau) for 0 <= tau <= beta (one-sided limits at the ends)."""
    eps, C = generalized_eig(F, S)
    xi = eps - mu
    tau = np.atleast_1d(tau)
    # (1-f) exp(-xi tau) = exp(-xi tau - log(1 + exp(-beta xi)))
    w = np.exp(-np.outer(tau, xi) - np.logaddexp(0.0, -beta * xi)[None, :])
    return -np.einsum("ik,tk,jk->tij", C, w, C)


def hf_green_iw(S, F, mu, beta, niw):
    eps, C = generalized_eig(F, S)
    w = (2.0 * np.arange(niw) + 1.0) * np.pi / beta
    d = 1.0 / (1j * w[:, None] + mu - eps[None, :])
    return np.einsum("ik,nk,jk->nij", C, d, C)


def hf_density(S, F, mu, beta):
    eps, C = generalized_eig(F, S)
    return 2.0 * (C * fermi(eps - mu, beta)) @ C.T


def mu_closed_form(eps, nelec, beta):
    """Root of 2 sum_k f(eps_k - mu) = nelec (non-interacting electrons)."""
    g = lambda mu: 2.0 * fermi(eps - mu, beta).sum() - nelec
    return brentq(g, eps.min() - 50.0, eps.max() + 50.0, xtol=1e-15, rtol=1e-15, maxiter=500)


def rhf_zero_T(S, h, v, nelec, *, damping=0.3, depth=8, tol=1e-11, max_iter=500):
    """Zero-temperature RHF by Roothaan iterations (Aufbau), core guess,
    accelerated by the same damped Pulay mixing of the density as the GF2
    inner loop.  Raises if it does not converge."""
    from .loop import pulay_mix
    nocc = nelec // 2

    def density(F):
        eps, C = generalized_eig(F, S)
        Co = C[:, :nocc]
        return 2.0 * Co @ Co.T

    P_in = density(h)
    hist = []
    for _ in range(max_iter):
        F = fock(h, v, P_in)
        P_out = density(F)
        r = P_out - P_in
        if np.max(np.abs(r)) < tol:
            P = P_out
            F = fock(h, v, P)
            eps, C = generalized_eig(F, S)
            E = 0.5 * float(np.sum(P * (h + F)))
            return E, eps, C, P, F
        hist.append((P_in, r))
        hist = hist[-depth:]
        P_in, hist = pulay_mix(hist, damping)
    raise RuntimeError("zero-temperature RHF did not converge")


def mo_integrals(C, v):
    return np.einsum("pi,qj,rk,sl,pqrs->ijkl", C, C, C, C, v, optimize=True)


def mp2_energy(C, eps, v, nocc):
    """Closed-shell MP2 correlation energy from MO integrals."""
    g = mo_integrals(C, v)
    o = slice(0, nocc)
    vv = slice(nocc, C.shape[1])
    iajb = g[o, vv, o, vv]                       # (ia|jb)
    ibja = iajb.transpose(0, 3, 2, 1)            # (ib|ja) indexed [i,a,j,b]
    eo, ev = eps[o], eps[vv]
    den = eo[:, None, None, None] - ev[None, :, None, None] + eo[None, None, :, None] \
        - ev[None, None, None, :]
    return float(np.sum(iajb * (2.0 * iajb - ibja) / den))


def e2b_hf_closed_form(S, F, mu, beta, v):
    """(1/beta) sum_n tr[G0 Sigma[G0]] for a Hartree-Fock G0, in closed form.

    With G0 diagonal in the MO basis, Eq. (Sigma) gives
    E = -sum_{akmp} I_akmp [X - Y]/Delta,  Delta = e_k + e_m - e_p - e_a,
    I_akmp = (am|pk)[2(kp|ma) - (mp|ka)],
    X = (1-f_k)(1-f_m) f_p f_a,  Y = f_k f_m (1-f_p)(1-f_a),
    and beta*X in the limit Delta -> 0.
    """
    eps, C = generalized_eig(F, S)
    f = fermi(eps - mu, beta)
    g = mo_integrals(C, v)
    I = np.einsum("amPk,kPma->akmP", g, 2.0 * g) - np.einsum("amPk,mPka->akmP", g, g)
    # I[a,k,m,p] = (am|pk)[2(kp|ma) - (mp|ka)]
    fa = f[:, None, None, None]
    fk = f[None, :, None, None]
    fm = f[None, None, :, None]
    fp = f[None, None, None, :]
    X = (1 - fk) * (1 - fm) * fp * fa
    Y = fk * fm * (1 - fp) * (1 - fa)
    ea = eps[:, None, None, None]
    ek = eps[None, :, None, None]
    em = eps[None, None, :, None]
    ep = eps[None, None, None, :]
    D = ek + em - ep - ea
    small = np.abs(beta * D) < 1e-7
    Dsafe = np.where(small, 1.0, D)
    ratio = np.where(small, beta * X * (1.0 - 0.5 * beta * D), (X - Y) / Dsafe)
    return -float(np.sum(I * ratio))
