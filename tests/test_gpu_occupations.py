"""GPU parity of gf2_natural_occupations against the oracle.

Densities with known natural occupation numbers are built on the host:
P = C diag(occ) C^T with C^T S C = 1 (C from a Cholesky factor of S and a
random orthogonal matrix), so the NONs are exactly the chosen occ (up to the
rounding of building P).  Sizes span odd and even n, the LDS/global-memory
switch of the eigensolver (n = 136 / 137) and n = 160; degenerate clusters
(many exact 2s and 0s) are included."""
import numpy as np
import pytest

import oracle as O
from oracle import reference as R
from synthetic import generic_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _overlap(rng, n):
    """S = R^T R rescaled to unit diagonal, R = 1 + 0.05 Gaussian."""
    Rm = np.eye(n) + 0.05 * rng.standard_normal((n, n))
    S = Rm.T @ Rm
    d = 1.0 / np.sqrt(np.diag(S))
    return S * d[:, None] * d[None, :]


def _density_with_occupations(rng, S, occ):
    n = S.shape[0]
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    C = np.linalg.solve(np.linalg.cholesky(S).T, Q)
    P = (C * occ) @ C.T
    return 0.5 * (P + P.T)


def _ctx_for_overlap(torch, S):
    """A context whose system has this overlap (h and v zero, on the device)."""
    from paper_1405_3273_amd.runtime import Gf2
    n = S.shape[0]
    zeros4 = torch.zeros((n, n, n, n), dtype=torch.float64, device="cuda")
    return Gf2(S, np.zeros((n, n)), zeros4, nelec=n, beta=10.0, niw=8, ntau=5)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 100, 136, 137, 160])
def test_natural_occupations_match_oracle(torch, n):
    print(f"natural occupations n={n}", flush=True)
    rng = np.random.default_rng(1000 + n)
    S = _overlap(rng, n)
    occ = rng.uniform(0.0, 2.0, n)
    occ[: n // 3] = 2.0                       # a degenerate cluster
    occ[n // 3: n // 2] = 0.0                 # and another
    P = _density_with_occupations(rng, S, occ)
    ref = O.natural_occupations(P, S)
    g = _ctx_for_overlap(torch, S)
    got = g.natural_occupations(torch.as_tensor(P).cuda()).cpu().numpy()
    err = np.max(np.abs(got - ref))
    print(f"  max|gpu - oracle| {err:.2e}, max|gpu - chosen| "
          f"{np.max(np.abs(got - np.sort(occ)[::-1])):.2e}")
    assert np.all(np.diff(got) <= 0.0)
    assert err <= 1e-11
    np.testing.assert_allclose(got, np.sort(occ)[::-1], rtol=0, atol=1e-10)
    g.close()


def test_natural_occupations_of_hartree_fock_density(torch):
    """The finite-beta HF density from gf2_density_fock (Sigma = 0) has NONs
    2 f(eps_k - mu); GPU and oracle agree on the same P."""
    from paper_1405_3273_amd import make_params
    from paper_1405_3273_amd.runtime import Gf2
    s = generic_system(10, 0, naux=30, beta=50.0, niw=2048, ntau=257)
    g = Gf2(s.S, s.h, s.v, nelec=s.nelec, beta=s.beta, niw=s.niw, ntau=s.ntau)
    F = torch.as_tensor(s.h).cuda()
    mu, P, _, _, info = g.density_fock(make_params(), F, 0.0)
    got = g.natural_occupations(P).cpu().numpy()
    Ph = P.cpu().numpy()
    np.testing.assert_allclose(got, O.natural_occupations(Ph, s.S), rtol=0, atol=1e-12)
    eps, _ = R.generalized_eig(s.h, s.S)
    want = np.sort(2.0 * R.fermi(eps - mu, s.beta))[::-1]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-6)
    assert got.sum() == pytest.approx(s.nelec, abs=1e-8)
    g.close()


def test_natural_occupations_errors(torch):
    from paper_1405_3273_amd import _lib as L
    rng = np.random.default_rng(5)
    S = _overlap(rng, 6)
    g = _ctx_for_overlap(torch, S)
    P = torch.as_tensor(_density_with_occupations(rng, S, rng.uniform(0, 2, 6))).cuda()
    occ = torch.empty(6, dtype=torch.float64, device="cuda")
    with pytest.raises(L.Gf2Error) as e:
        L.gf2_natural_occupations(g.ctx, None, occ)
    assert e.value.code == L.GF2_EINVAL
    P[2, 3] = float("nan")
    with pytest.raises(L.Gf2Error) as e:
        L.gf2_natural_occupations(g.ctx, P, occ)
    assert e.value.code == L.GF2_ENONFINITE
    g.close()
    ctx = L.gf2_ctx_create(0)
    with pytest.raises(L.Gf2Error) as e:
        L.gf2_natural_occupations(ctx, P, occ)
    assert e.value.code == L.GF2_ESTATE
    L.gf2_ctx_destroy(ctx)


def test_natural_occupations_reject_an_indefinite_overlap(torch):
    """An overlap that is invertible but not positive definite has no Cholesky
    factor: GF2_EINVAL, and the library stays usable."""
    from paper_1405_3273_amd import _lib as L
    S = np.diag([1.0, 1.0, -0.5, 1.0])
    g = _ctx_for_overlap(torch, S)
    P = torch.eye(4, dtype=torch.float64, device="cuda")
    occ = torch.empty(4, dtype=torch.float64, device="cuda")
    with pytest.raises(L.Gf2Error) as e:
        L.gf2_natural_occupations(g.ctx, P, occ)
    assert e.value.code == L.GF2_EINVAL
    g.close()
    rng = np.random.default_rng(9)
    S2 = _overlap(rng, 5)
    g2 = _ctx_for_overlap(torch, S2)
    occ2 = g2.natural_occupations(torch.as_tensor(_density_with_occupations(rng, S2, np.full(5, 1.5))).cuda())
    np.testing.assert_allclose(occ2.cpu().numpy(), 1.5, atol=1e-12)
    g2.close()
