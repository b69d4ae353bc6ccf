"""Transforms between imaginary time and Matsubara frequency (oracle).

Conventions (the paper fixes none of them; these are the readings):

* G(i omega_n) = int_0^beta exp(i omega_n tau) G(tau) dtau,
  G(tau) = (1/beta) sum_{n in Z} exp(-i omega_n tau) G(i omega_n).
* Uniform grid tau_k = k beta/M (see ``grids``), or any strictly increasing
  grid tau_0 = 0 < ... < tau_M = beta passed as ``tau`` (the paper uses a
  non-equidistant grid, Implementation section).  Only the 'direct' sums
  apply to a non-uniform grid.

Sigma(tau) -> Sigma(i omega) (step 3 of the Supplementary Material).  The
paper says only that an FFT is used.  Reading: interpolate every matrix
element by a not-a-knot cubic spline on the grid and take the Fourier
integral of the spline exactly, interval by interval.  On [tau_j,
tau_{j+1}] (width h) the spline is sum_k c_kj t^k, t = tau - tau_j, so

  Sigma(i w_n) = sum_j exp(i w_n tau_j) sum_{k=0..3} c_kj h^{k+1} mu_k(w_n h),
  mu_k(theta) = int_0^1 s^k exp(i theta s) ds.

exp(i w_n tau_j) = exp(i pi (2n+1) j / M) is M-periodic in n, so the four
sums over j are length-M DFTs evaluated once and reused for every n.
mu_k is summed as its Taylor series for theta < 1 and by the recursion
mu_0 = (e^{i theta} - 1)/(i theta), mu_k = (e^{i theta} - k mu_{k-1})/(i theta)
otherwise.  (The same integral written by parts over the whole interval
[0, beta] has terms growing like (i w)^-4 that cancel at low frequency;
the interval-by-interval form avoids that loss.)  The first moment is
Sigma_1 = -(Sigma(0+) + Sigma(beta-)) exactly.

G(i omega) -> G(tau) (step 2.b).  The paper uses the analytic high
frequency tail G ~ G1/(i w) + G2/(i w)^2 + G3/(i w)^3 (Implementation
section).  The tail is subtracted, the remainder summed over the stored
frequencies (both signs of n through complex conjugation) and the tail
added back in closed form.  For 0 <= tau <= beta (one-sided limits at
the ends):

  1/(i w)   -> -1/2
  1/(i w)^2 -> (2 tau - beta)/4
  1/(i w)^3 -> (beta tau - tau^2)/4.
"""
import numpy as np
from scipy.interpolate import CubicSpline

from .grids import tau_grid, matsubara


def _phase(num: np.ndarray, M: int) -> np.ndarray:
    """exp(i pi num / M) with the integer numerator reduced mod 2M first."""
    r = np.mod(num, 2 * M).astype(np.float64)
    return np.exp(1j * np.pi * r / M)


def spline_coefficients(Y: np.ndarray, beta: float, tau=None) -> np.ndarray:
    """Not-a-knot cubic spline of Y[k] over the tau grid (axis 0; uniform
    when ``tau`` is None).

    Returns c[k][j] (k = 0..3): the spline on [tau_j, tau_{j+1}] is
    sum_k c[k][j] (tau - tau_j)^k.
    """
    ntau = Y.shape[0]
    tau = tau_grid(beta, ntau) if tau is None else np.asarray(tau, dtype=np.float64)
    spl = CubicSpline(tau, Y, axis=0, bc_type="not-a-knot")
    return spl.c[::-1]            # scipy stores the highest power first


def moments_unit(theta: np.ndarray, kmax: int = 3) -> np.ndarray:
    """mu_k(theta) = int_0^1 s^k exp(i theta s) ds for k = 0..kmax, theta >= 0."""
    theta = np.asarray(theta, dtype=np.float64)
    out = np.zeros((kmax + 1,) + theta.shape, dtype=np.complex128)
    small = theta < 1.0
    # Taylor series: sum_p (i theta)^p / (p! (p + k + 1))
    ts = theta[small]
    term = np.ones_like(ts, dtype=np.complex128)
    for p in range(0, 30):
        if p > 0:
            term = term * (1j * ts) / p
        for k in range(kmax + 1):
            out[k][small] += term / (p + k + 1)
    # recursion
    tl = theta[~small]
    e = np.exp(1j * tl)
    it = 1j * tl
    m = (e - 1.0) / it
    out[0][~small] = m
    for k in range(1, kmax + 1):
        m = (e - k * m) / it
        out[k][~small] = m
    return out


def _phase_grid(n_odd: np.ndarray, tau: np.ndarray, beta: float) -> np.ndarray:
    """exp(i pi n_odd tau / beta) for a general grid, the argument reduced mod 2."""
    x = np.mod(np.multiply.outer(n_odd.astype(np.float64), tau / beta), 2.0)
    return np.exp(1j * np.pi * x)


def sigma_tau_to_iw(Sig_tau: np.ndarray, beta: float, niw: int, n_idx=None,
                    method: str = "fft", tau=None):
    """Sigma(tau) [ntau][n][n] -> (Sigma(i omega_n) [len][n][n] complex, Sigma_1).

    ``method='direct'`` sums over the intervals term by term for the
    requested frequencies (the definition); ``'fft'`` evaluates the four
    M-periodic sums over intervals with length-M FFTs (uniform grid only).
    With a grid ``tau`` the interval widths h_j = tau_{j+1} - tau_j enter
    each term: Sigma(i w_n) = sum_j exp(i w_n tau_j) sum_k c_kj h_j^{k+1}
    mu_k(w_n h_j).
    """
    ntau = Sig_tau.shape[0]
    M = ntau - 1
    ns = np.arange(niw) if n_idx is None else np.asarray(n_idx)
    if tau is not None:
        tau = np.asarray(tau, dtype=np.float64)
        if tau.shape != (ntau,):
            raise ValueError("tau grid length differs from Sig_tau")
        c = spline_coefficients(Sig_tau, beta, tau)        # [4][M][n][n]
        hj = np.diff(tau)
        w = np.pi * (2 * ns + 1) / beta
        mom = moments_unit(np.multiply.outer(w, hj))       # [4][len][M]
        ph = _phase_grid(2 * ns + 1, tau[:-1], beta)       # [len][M]
        Sig_iw = sum(np.tensordot(ph * mom[k] * hj[None, :] ** (k + 1), c[k], axes=([1], [0]))
                     for k in range(4))
        return Sig_iw, -(Sig_tau[0] + Sig_tau[-1])
    h = beta / M
    c = spline_coefficients(Sig_tau, beta)                 # [4][M][n][n]
    mom = moments_unit(np.pi * (2 * ns + 1) / M)           # mu_k(w_n h), [4][len]
    j = np.arange(M)
    if method == "direct":
        ph = _phase(np.outer(2 * ns + 1, j), M)            # exp(i w_n tau_j)
        C = np.stack([np.tensordot(ph, c[k], axes=([1], [0])) for k in range(4)])
    elif method == "fft":
        a = _phase(j, M)[:, None, None]                    # exp(i pi j / M)
        Ck = [M * np.fft.ifft(c[k] * a, axis=0) for k in range(4)]   # sum_j (.) exp(2 pi i r j / M)
        C = np.stack([Ck[k][np.mod(ns, M)] for k in range(4)])
    else:
        raise ValueError(method)
    Sig_iw = sum((h ** (k + 1)) * mom[k][:, None, None] * C[k] for k in range(4))
    return Sig_iw, -(Sig_tau[0] + Sig_tau[-1])


def tail_tau(tau, G1, G2, G3, beta):
    """Closed-form transform of G1/(iw) + G2/(iw)^2 + G3/(iw)^3 at tau in [0, beta]."""
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    t = tau[:, None, None]
    return -0.5 * G1 + G2 * (2.0 * t - beta) / 4.0 + G3 * (beta * t - t * t) / 4.0


def g_iw_to_tau(G_iw: np.ndarray, G1, G2, G3, beta: float, ntau: int, k_idx=None,
                method: str = "fft", tau=None) -> np.ndarray:
    """G(i omega_n), n = 0..niw-1 -> G(tau_k) on the tau grid (uniform when
    ``tau`` is None; a grid ``tau`` takes the direct sum).

    G(tau) = (2/beta) Re sum_{n<niw} exp(-i w_n tau) [G - tail](i w_n) + tail(tau).
    """
    niw = G_iw.shape[0]
    M = ntau - 1
    ks = np.arange(ntau) if k_idx is None else np.asarray(k_idx)
    iw = 1j * matsubara(beta, niw)[:, None, None]
    R = G_iw - G1 / iw - G2 / iw ** 2 - G3 / iw ** 3
    if tau is not None:
        tk = np.asarray(tau, dtype=np.float64)[ks]
        ph = np.conj(_phase_grid(2 * np.arange(niw) + 1, tk, beta)).T   # [k][n]
        S = np.tensordot(ph, R, axes=([1], [0]))
        return (2.0 / beta) * S.real + tail_tau(tk, G1, G2, G3, beta)
    if method == "direct":
        ph = _phase(-np.outer(ks, 2 * np.arange(niw) + 1), M)   # exp(-i w_n tau_k)
        S = np.tensordot(ph, R, axes=([1], [0]))
    elif method == "fft":
        Fr = np.zeros((M,) + R.shape[1:], dtype=np.complex128)
        np.add.at(Fr, np.mod(np.arange(niw), M), R)            # fold n mod M
        Y = np.fft.fft(Fr, axis=0)                             # sum_r exp(-2 pi i r k/M) F_r
        S = _phase(-ks, M)[:, None, None] * Y[np.mod(ks, M)]
    else:
        raise ValueError(method)
    tau = tau_grid(beta, ntau)[ks]
    return (2.0 / beta) * S.real + tail_tau(tau, G1, G2, G3, beta)
