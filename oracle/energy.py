"""Total energy (oracle).

The paper plots total energies (Results section) but prints no formula.
Reading: the Galitskii-Migdal energy for a spin-restricted Green's
function,

    E = 1/2 tr[P (h + F)] + E_2b,
    E_2b = (1/beta) sum_{n in Z} tr[G(i w_n) Sigma(i w_n)]
         = (2/beta) sum_{n<niw} Re tr[G Sigma]
           - (2/beta) tr[G1 Sigma_1] (beta/(2 pi))^2 psi'(niw + 1/2),

where the last term is the exact sum over the truncated frequencies of
the leading tail tr[G1 Sigma_1]/(i w)^2 (Re 1/(i w)^2 = -1/w^2 and
sum_{n>=niw} 1/(2n+1)^2 = psi'(niw + 1/2)/4), and psi' is the trigamma
function.  G is per spin, P spin-summed; the factor 1/2 of the
Galitskii-Migdal formula and the spin sum cancel in E_2b.
"""
import numpy as np
from scipy.special import polygamma



def trigamma(x: float) -> float:
    return float(polygamma(1, x))


def e_one_body(P, h, F) -> float:
    """1/2 tr[P (h + F)]."""
    return 0.5 * float(np.einsum("ij,ji->", P, h + F))


def e_two_body(G_iw, Sigma_iw, G1, Sigma1, beta) -> float:
    """(1/beta) sum over all n of tr[G Sigma], truncated sum plus exact 1/w^2 tail."""
    niw = G_iw.shape[0]
    tr = np.einsum("nij,nji->n", G_iw, Sigma_iw)
    head = (2.0 / beta) * float(tr.real.sum())
    tail = -(2.0 / beta) * float(np.einsum("ij,ji->", G1, Sigma1)) \
        * (beta / (2.0 * np.pi)) ** 2 * trigamma(niw + 0.5)
    return head + tail


def e_two_body_tau(Sig_tau, G_tau, beta) -> float:
    """Cross-check: E_2b = -int_0^beta tr[Sigma(tau) G(beta - tau)] dtau (Simpson)."""
    from scipy.integrate import simpson
    ntau = Sig_tau.shape[0]
    tau = beta * np.arange(ntau) / (ntau - 1)
    f = np.einsum("kij,kji->k", Sig_tau, G_tau[::-1])
    return -float(simpson(f, x=tau))

