"""Second-order self-energy in imaginary time, Eq. (Sigma) (oracle).

Eq. (Sigma) of the Implementation section (repeated in the
Supplementary Material) gives, for each imaginary time tau,

    Sigma_ij(tau) = - sum_{klmnpq} G_kl(tau) G_mn(tau) G_pq(-tau)
                      * v_imqk * (2 v_lpnj - v_nplj)

with v_ijkl = (ij|kl) the AO two-electron integrals in chemist notation
(real, 8-fold symmetric), G the spin-restricted (per-spin) Green's
function and Sigma the per-spin self-energy.  The two terms are the
second-order direct and exchange diagrams (Figure 1); the factor 2 is
the spin sum of the closed loop.

Reading for G(-tau): antiperiodicity G(-tau) = -G(beta - tau) for
0 < tau < beta, so on the uniform grid G(-tau_k) = -G(tau_{M-k}); the
endpoint samples are the one-sided limits (G(tau_0) = G(0+),
G(tau_M) = G(beta-)).

Three evaluations are provided: the literal six-index sum (pure Python
loops, tiny N only), the literal sum as one ``einsum`` (small N), and
the factored chain of four contractions that the method's O(N_tau n^5)
cost statement refers to (Implementation section).  The factored chain
is the one used for real sizes:

    T1_{inqk} = sum_m v_imqk G_mn(tau)
    T2_{inpk} = sum_q T1_{inqk} G_pq(-tau)
    T3_{inpl} = sum_k T2_{inpk} G_kl(tau)
    Sigma_ij  = - sum_{npl} T3_{inpl} W_{lpnj},   W_lpnj = 2 v_lpnj - v_nplj
"""
import numpy as np


def bracket_W(v: np.ndarray) -> np.ndarray:
    """W_lpnj = 2 v_lpnj - v_nplj, the bracket of Eq. (Sigma)."""
    # v_nplj re-indexed to (l,p,n,j): swap the first and third index.
    return 2.0 * v - np.transpose(v, (2, 1, 0, 3))


def gbar_from_gtau(G_tau: np.ndarray) -> np.ndarray:
    """G(-tau_k) = -G(tau_{M-k}) (antiperiodicity), on any grid symmetric
    about beta/2 (tau_{M-k} = beta - tau_k): the uniform grid and the
    power grid of the inputs."""
    return -G_tau[::-1]


def sigma_bruteforce(G: np.ndarray, Gb: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Eq. (Sigma) as the literal six-index sum, pure Python loops (N <= 4)."""
    n = G.shape[0]
    out = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for k in range(n):
                for l in range(n):
                    for m in range(n):
                        for nn in range(n):
                            for p in range(n):
                                for q in range(n):
                                    acc += (G[k, l] * G[m, nn] * Gb[p, q] * v[i, m, q, k]
                                            * (2.0 * v[l, p, nn, j] - v[nn, p, l, j]))
            out[i, j] = -acc
    return out


def sigma_literal(G: np.ndarray, Gb: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Eq. (Sigma) as one einsum over all six summation indices (small N)."""
    W = bracket_W(v)
    return -np.einsum("kl,mn,pq,imqk,lpnj->ij", G, G, Gb, v, W, optimize=False)


def sigma_factored(G: np.ndarray, Gb: np.ndarray, v: np.ndarray,
                   W: np.ndarray = None) -> np.ndarray:
    """Eq. (Sigma) as the chain of four contractions (8 N^5 flops)."""
    if W is None:
        W = bracket_W(v)
    n = G.shape[0]
    # T1_{i q k n} = sum_m v_{i m q k} G_{m n}
    T1 = np.tensordot(v, G, axes=([1], [0]))                 # (i, q, k, n)
    # T2_{i k n p} = sum_q T1_{i q k n} Gb_{p q}
    T2 = np.tensordot(T1, Gb, axes=([1], [1]))               # (i, k, n, p)
    # T3_{i n p l} = sum_k T2_{i k n p} G_{k l}
    T3 = np.tensordot(T2, G, axes=([1], [0]))                # (i, n, p, l)
    # Sigma_ij = - sum_{n p l} T3_{i n p l} W_{l p n j}
    Wt = np.transpose(W, (2, 1, 0, 3)).reshape(n * n * n, n)  # rows (n, p, l), cols j
    return -(T3.reshape(n, n * n * n) @ Wt)


def sigma_tau(G_tau: np.ndarray, v: np.ndarray, taus=None) -> np.ndarray:
    """Sigma(tau_k) for every grid point (or the listed indices ``taus``).

    G_tau: [ntau][n][n].  Returns [len(taus)][n][n].
    """
    ntau = G_tau.shape[0]
    W = bracket_W(v)
    Gb = gbar_from_gtau(G_tau)
    ks = range(ntau) if taus is None else taus
    return np.stack([sigma_factored(G_tau[k], Gb[k], v, W) for k in ks])


def sigma_df(G: np.ndarray, Gb: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Eq. (Sigma) with density-fitted integrals v_ijkl = sum_P B^P_ij B^P_kl
    (the cheaper route the Implementation section proposes, recalled in the
    Conclusions; its O(n^3 m) estimate holds for the direct term, the exchange
    term below costs O(n^3 m^2)).

    Substituting the factors into both integrals of Eq. (Sigma) and grouping
    the sums gives, with X^{PQ} = B^P G B^Q (N x N, P, Q over the auxiliary
    index) and Gb = G(-tau),

        direct:   2 sum_{PQ} X^{PQ}_ij tr(X^{PQ} Gb)
        exchange:   sum_{PQ} (X^{PQ} Gb X^{PQ})_ij
        Sigma_ij = -(direct - exchange).

    Written with matrix products as steps, P and Q looped in order.
    """
    m, n = B.shape[0], B.shape[1]
    out = np.zeros((n, n))
    for P in range(m):
        Y = B[P] @ G
        for Q in range(m):
            X = Y @ B[Q]
            t = float(np.sum(X * Gb.T))          # tr(X Gb)
            out += 2.0 * t * X - X @ Gb @ X
    return -out


def sigma_tau_df(G_tau: np.ndarray, B: np.ndarray, taus=None) -> np.ndarray:
    """sigma_df at every grid point (or the listed indices ``taus``)."""
    Gb = gbar_from_gtau(G_tau)
    ks = range(G_tau.shape[0]) if taus is None else taus
    return np.stack([sigma_df(G_tau[k], Gb[k], B) for k in ks])
