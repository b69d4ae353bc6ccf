"""gf2_dyson_noalloc (the Dyson solve on the library's fixed per-GPU workspace)
against gf2_dyson: same kernels on the same workgroups, so the results must
agree bit for bit.  Two calls in a row, the second on a smaller input, both
through the C ABI; then a solve too large for the fixed workspace is refused."""
import numpy as np
import pytest

from synthetic import generic_system

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _setup(torch, n, niw, seed):
    from paper_1405_3273_amd.runtime import Gf2
    s = generic_system(n, seed, naux=2 * n, beta=50.0, niw=niw, ntau=9)
    g = Gf2(s.S, s.h, s.v, nelec=s.nelec, beta=s.beta, niw=s.niw, ntau=s.ntau)
    rng = np.random.default_rng(seed)
    A = 0.05 * (rng.standard_normal((niw, n, n)) + 1j * rng.standard_normal((niw, n, n)))
    sig = torch.as_tensor(0.5 * (A + A.transpose(0, 2, 1))).cuda()   # complex symmetric
    B = 0.05 * rng.standard_normal((n, n))
    s1 = torch.as_tensor(0.5 * (B + B.T)).cuda()
    F = torch.as_tensor(s.h).cuda()
    return s, g, sig, s1, F


def _both(torch, g, mode, mu, F, sig, s1):
    from paper_1405_3273_amd import _lib as L
    n, niw = g.n, g.dims.niw
    res = []
    for fn in (L.gf2_dyson, L.gf2_dyson_noalloc):
        P = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
        G = torch.full((niw, n, n), complex("nan"), dtype=torch.complex128, device="cuda")
        if mode == L.GF2_DYSON_TRACE:
            out = fn(g.ctx, g.dims, mode, mu, F, sig, s1, None, None)
        else:
            out = fn(g.ctx, g.dims, mode, mu, F, sig, s1, G, P)
        torch.cuda.synchronize()
        res.append((out, P.cpu().numpy(), G.cpu().numpy()))
    return res


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_noalloc_dyson_equals_dyson_two_calls(torch, mode):
    from paper_1405_3273_amd import _lib as L
    for n, niw, seed in ((100, 2048, 1), (40, 512, 2)):    # second call: smaller input
        print(f"noalloc: mode={mode} n={n} niw={niw}", flush=True)
        s, g, sig, s1, F = _setup(torch, n, niw, seed)
        mu = float(np.mean(np.diag(s.h)))
        (o_ref, P_ref, G_ref), (o_na, P_na, G_na) = _both(torch, g, mode, mu, F, sig, s1)
        assert o_na == o_ref
        assert np.isfinite(o_ref[0])
        if mode != L.GF2_DYSON_TRACE:
            assert np.all(np.isfinite(P_ref))
            assert np.array_equal(P_na, P_ref)
            assert np.array_equal(G_na, G_ref)
        g.close()


def test_noalloc_dyson_refuses_a_solve_larger_than_its_workspace(torch):
    from paper_1405_3273_amd import _lib as L
    from paper_1405_3273_amd.runtime import Gf2
    n, niw = 128, 1024           # FULL: 512 partials of n^2 doubles > 64 MiB
    print(f"noalloc: oversize n={n}", flush=True)
    S = np.eye(n)
    h = np.diag(np.linspace(-2.0, -0.5, n))
    v = torch.zeros((n, n, n, n), dtype=torch.float64, device="cuda")
    g = Gf2(S, h, v, nelec=n, beta=20.0, niw=niw, ntau=9)
    F = torch.as_tensor(h).cuda()
    P = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(L.Gf2Error) as e:
        L.gf2_dyson_noalloc(g.ctx, g.dims, L.GF2_DYSON_FULL, -1.0, F, None, None, None, P)
    assert e.value.code == L.GF2_EINVAL
    assert "workspace" in L.gf2_last_error()
    # TRACE of the same system fits, and equals gf2_dyson
    a = L.gf2_dyson_noalloc(g.ctx, g.dims, L.GF2_DYSON_TRACE, -1.0, F)
    b = L.gf2_dyson(g.ctx, g.dims, L.GF2_DYSON_TRACE, -1.0, F)
    assert a == b
    g.close()
