"""Python front end of libgf2: owns a context, the system and the loop state
as torch device tensors and calls the C ABI.  Argument marshalling only.
"""
from __future__ import annotations

import math

from . import _lib as L


class Gf2:
    """One GF2 problem on one GPU.

    ``S``, ``h``: [n][n] float64; ``v``: [n][n][n][n] float64 (ij|kl); any
    device or host tensor/array (copied to ``device``).
    """

    def __init__(self, S, h, v, nelec, beta, niw, ntau, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        t = lambda x: torch.as_tensor(x, dtype=torch.float64).to(self.device).contiguous()
        self.S, self.h, self.v = t(S), t(h), t(v)
        self.n = int(self.S.shape[0])
        self.dims = L.make_dims(self.n, nelec, ntau, niw, beta)
        self.ctx = L.gf2_ctx_create(device)
        L.gf2_set_system(self.ctx, self.S, self.h, self.v)
        self.state = None
        self._keep = None

    # -- context -------------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None) is not None:
            L.gf2_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, *shape, complex_=False):
        dt = self.torch.complex128 if complex_ else self.torch.float64
        return self.torch.empty(*shape, dtype=dt, device=self.device)

    def dims_with(self, **kw):
        d = self.dims
        args = dict(n=d.n, nelec=d.nelec, ntau=d.ntau, niw=d.niw, beta=d.beta)
        args.update(kw)
        return L.make_dims(**args)

    # -- single stages ---------------------------------------------------------
    def sigma_tau(self, G_tau, prec="fp32", out=None):
        ntau = int(G_tau.shape[0])
        out = self._empty(ntau, self.n, self.n) if out is None else out
        L.gf2_sigma_tau(self.ctx, self.dims_with(ntau=ntau), prec, G_tau, out)
        return out

    def set_df_factors(self, B):
        """Density-fitting factors [naux][n][n] (v = sum_P B^P (x) B^P) for
        sigma_tau_df and for iterations with params.sigma_df = 1."""
        self.B = self.torch.as_tensor(B, dtype=self.torch.float64).to(self.device).contiguous()
        L.gf2_set_df_factors(self.ctx, self.B)

    def sigma_tau_df(self, G_tau, prec="fp64", out=None):
        ntau = int(G_tau.shape[0])
        out = self._empty(ntau, self.n, self.n) if out is None else out
        L.gf2_sigma_tau_df(self.ctx, self.dims_with(ntau=ntau), prec, G_tau, out)
        return out

    def tau_to_iw(self, Sig_tau, niw=None, beta=None):
        ntau = int(Sig_tau.shape[0])
        d = self.dims_with(ntau=ntau, niw=niw or self.dims.niw, beta=beta or self.dims.beta)
        out = self._empty(d.niw, self.n, self.n, complex_=True)
        s1 = self._empty(self.n, self.n)
        L.gf2_fourier(self.ctx, d, L.GF2_TAU2IW, Sig_tau, None, out, s1)
        return out, s1

    def iw_to_tau(self, G_iw, moments, ntau=None, beta=None):
        d = self.dims_with(niw=int(G_iw.shape[0]), ntau=ntau or self.dims.ntau,
                           beta=beta or self.dims.beta)
        out = self._empty(d.ntau, self.n, self.n)
        L.gf2_fourier(self.ctx, d, L.GF2_IW2TAU, G_iw, moments, out)
        return out

    def dyson(self, mode, mu, F, Sigma_iw=None, Sigma1=None, want_G=False):
        P = self._empty(self.n, self.n) if mode != L.GF2_DYSON_TRACE else None
        G = self._empty(self.dims.niw, self.n, self.n, complex_=True) if want_G else None
        r = L.gf2_dyson(self.ctx, self.dims, mode, mu, F, Sigma_iw, Sigma1, G, P)
        return r, P, G

    def fock(self, P):
        F = self._empty(self.n, self.n)
        L.gf2_fock(self.ctx, P, F)
        return F

    def set_tau_grid(self, tau):
        """Sample G(tau), Sigma(tau) on the grid tau (ntau points; None: uniform)."""
        if tau is None:
            L.gf2_set_tau_grid(self.ctx, None)
            self._grid = None
            return
        t = self.torch.as_tensor(tau, dtype=self.torch.float64).to(self.device).contiguous()
        L.gf2_set_tau_grid(self.ctx, t)
        self._grid = t
        self.dims = self.dims_with(ntau=int(t.numel()))

    def natural_occupations(self, P):
        """Natural occupation numbers of the density P, largest first."""
        occ = self._empty(self.n)
        L.gf2_natural_occupations(self.ctx, P, occ)
        return occ

    def density_fock(self, params, F_in, mu, Sigma_iw=None, Sigma1=None, want_G=False):
        P = self._empty(self.n, self.n)
        F = self._empty(self.n, self.n)
        G = self._empty(self.dims.niw, self.n, self.n, complex_=True) if want_G else None
        mu, info = L.gf2_density_fock(self.ctx, self.dims, params, F_in, Sigma_iw, Sigma1, mu,
                                      P, F, G)
        return mu, P, F, G, info

    # -- the loop ----------------------------------------------------------------
    def reset(self, mu0=0.0):
        """Core guess F = h, no density yet, iteration 0 next."""
        n, ntau = self.n, self.dims.ntau
        self.F = self.h.clone()
        self.P = self.torch.zeros(n, n, dtype=self.torch.float64, device=self.device)
        self.G_tau = self.torch.zeros(ntau, n, n, dtype=self.torch.float64, device=self.device)
        self.Sigma_tau = self.torch.zeros_like(self.G_tau)
        self.state = L.gf2_state(float(mu0), self.F.data_ptr(), self.P.data_ptr(),
                                 self.G_tau.data_ptr(), self.Sigma_tau.data_ptr(), 0, 0,
                                 float("nan"))

    def iterate(self, params) -> L.gf2_report:
        if self.state is None:
            self.reset()
        return L.gf2_iterate(self.ctx, self.dims, params, self.state)

    def run(self, params, max_outer=50, tol_E=None, callback=None):
        tol_E = params.tol_E if tol_E is None else tol_E
        reps = []
        for _ in range(max_outer):
            r = self.iterate(params)
            reps.append(r)
            if callback:
                callback(self, r)
            if self.state.iteration > 1 and abs(r.dE) < tol_E and r.dP < params.tol_P:
                return reps, True
        return reps, False

    @property
    def mu(self):
        return self.state.mu if self.state is not None else math.nan


class Gf2Batch:
    """Several independent GF2 problems (e.g. a geometry sweep) on one GPU,
    iterated together with gf2_iterate_batched.  ``systems``: Gf2 objects on
    the same device (each keeps its own state)."""

    def __init__(self, systems):
        self.systems = list(systems)
        if not self.systems:
            raise ValueError("Gf2Batch needs at least one system")

    def reset(self, mu0=None):
        for g in self.systems:
            g.reset(mu0=float(g.torch.diagonal(g.h).mean()) if mu0 is None else mu0)

    def iterate(self, params):
        for g in self.systems:
            if g.state is None:
                g.reset()
        return L.gf2_iterate_batched([g.ctx for g in self.systems], [g.dims for g in self.systems],
                                     params, [g.state for g in self.systems])

    def close(self):
        for g in self.systems:
            g.close()
