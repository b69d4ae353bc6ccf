"""GPU parity of the density-fitted Eq. (Sigma) (gf2_sigma_tau_df) against the
oracle: the oracle's factored form (oracle.sigma_tau_df) at small sizes, the
dense form (oracle.sigma_tau, equal for integrals built from the factors) at
the benchmark sizes on sampled tau points, and whole outer iterations with
sigma_df = 1 against the oracle loop."""
import numpy as np
import pytest

import oracle as O
from synthetic import generic_system, random_tau_stack, small_molecule

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 3e-5}     # max|err| / max|ref|


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _gf2(sysm, **kw):
    from paper_1405_3273_amd.runtime import Gf2
    args = dict(nelec=sysm.nelec, beta=sysm.beta, niw=sysm.niw, ntau=sysm.ntau)
    args.update(kw)
    g = Gf2(sysm.S, sysm.h, sysm.v, **args)
    g.set_df_factors(sysm.B)
    return g


def _dev(torch, x):
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def _relerr(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


# n, naux, ntau: one and several 16-wide tiles, ragged tails, one factor,
# naux below and above n, naux above n^2 (the tensor route's transposed exchange
# GEMM with more columns than rows), naux giving a 400-column Pi (split-K over N^2)
CASES = [(1, 1, 4), (2, 3, 5), (2, 5, 4), (3, 11, 4), (5, 15, 6), (16, 16, 4), (17, 40, 5),
         (33, 7, 4), (40, 120, 4), (20, 400, 4)]


@pytest.mark.parametrize("n,naux,ntau", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sigma_df_matches_oracle(torch, n, naux, ntau, prec):
    print(f"sigma_df n={n} naux={naux} ntau={ntau} prec={prec}", flush=True)
    s = generic_system(n, 700 + n, naux=naux, beta=20.0, ntau=ntau)
    rng = np.random.default_rng(n + naux)
    Gt = random_tau_stack(rng, ntau, n)
    ref = O.sigma_tau_df(Gt, s.B)
    g = _gf2(s)
    got = g.sigma_tau_df(_dev(torch, Gt), prec).cpu().numpy()
    err = _relerr(got, ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert err <= TOL[prec]
    assert np.array_equal(got, got.transpose(0, 2, 1))    # exactly symmetric
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sigma_df_equals_dense_path(torch, prec):
    """The factored and the dense contraction on the same integrals agree."""
    n, naux, ntau = 24, 72, 6
    print(f"sigma_df vs dense n={n} prec={prec}", flush=True)
    s = generic_system(n, 91, naux=naux, beta=20.0, ntau=ntau)
    Gt = _dev(torch, random_tau_stack(np.random.default_rng(3), ntau, n))
    g = _gf2(s)
    a = g.sigma_tau_df(Gt, prec).cpu().numpy()
    b = g.sigma_tau(Gt, prec).cpu().numpy()
    err = _relerr(a, b)
    print(f"  rel diff {err:.3e}", flush=True)
    assert err <= TOL[prec]
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sigma_df_n100_sampled(torch, prec):
    """N=100 with 400 factors (the benchmark system's shape): tau points 0, 2
    and 5 of six, every element, against the dense oracle contraction."""
    n, ntau = 100, 6
    print(f"sigma_df n=100 naux=400 prec={prec}", flush=True)
    s = generic_system(n, 300, naux=400, half_band=12, diag=(-3.0, -0.3), beta=200.0, ntau=ntau)
    Gt = random_tau_stack(np.random.default_rng(7), ntau, n, scale=0.05)
    ref = O.sigma_tau(Gt, s.v, taus=[0, 2, 5])
    g = _gf2(s)
    got = g.sigma_tau_df(_dev(torch, Gt), prec).cpu().numpy()[[0, 2, 5]]
    err = _relerr(got, ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert err <= TOL[prec]
    g.close()


@pytest.mark.parametrize("route", ["pair", "tensor"])
def test_sigma_df_n160(torch, route):
    """N=160 with 640 factors, both routes of the exchange term (pair route: the
    products of one tau point exceed the 1 GiB chunk, so P runs in chunks;
    tensor route: one 5.2 GB n^4 array); one tau point against the dense
    oracle contraction."""
    import os
    n, ntau = 160, 4
    print(f"sigma_df n=160 naux=640 fp64 {route}", flush=True)
    s = generic_system(n, 400, naux=640, half_band=16, diag=(-3.0, -0.3), beta=200.0, ntau=ntau)
    Gt = random_tau_stack(np.random.default_rng(9), ntau, n, scale=0.05)
    ref = O.sigma_tau(Gt, s.v, taus=[1])
    g = _gf2(s)
    os.environ["GF2_DF_ROUTE"] = route
    try:
        got = g.sigma_tau_df(_dev(torch, Gt), "fp64").cpu().numpy()[[1]]
    finally:
        os.environ.pop("GF2_DF_ROUTE", None)
    err = _relerr(got, ref)
    print(f"  rel err {err:.3e}", flush=True)
    assert err <= TOL["fp64"]
    g.close()


@pytest.mark.parametrize("n,naux", [(17, 40), (33, 7), (24, 72)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sigma_df_routes_agree(torch, n, naux, prec):
    """The pair and the tensor route of the exchange term, each forced, against
    the oracle's factored form (the automatic choice takes the tensor route
    when naux > n)."""
    import os
    print(f"sigma_df routes n={n} naux={naux} {prec}", flush=True)
    s = generic_system(n, 800 + n, naux=naux, beta=20.0, ntau=5)
    Gt = random_tau_stack(np.random.default_rng(n), 5, n)
    ref = O.sigma_tau_df(Gt, s.B)
    g = _gf2(s)
    try:
        for route in ("pair", "tensor"):
            os.environ["GF2_DF_ROUTE"] = route
            got = g.sigma_tau_df(_dev(torch, Gt), prec).cpu().numpy()
            err = _relerr(got, ref)
            print(f"  {route}: rel err {err:.3e}", flush=True)
            assert err <= TOL[prec]
    finally:
        os.environ.pop("GF2_DF_ROUTE", None)
    g.close()


def test_sigma_df_errors(torch):
    from paper_1405_3273_amd import _lib as L
    from paper_1405_3273_amd.runtime import Gf2
    s = generic_system(4, 5, naux=6, beta=10.0, ntau=5)
    g = Gf2(s.S, s.h, s.v, nelec=s.nelec, beta=s.beta, niw=s.niw, ntau=s.ntau)
    Gt = _dev(torch, random_tau_stack(np.random.default_rng(1), 5, 4))
    with pytest.raises(L.Gf2Error) as e:          # no factors yet
        g.sigma_tau_df(Gt, "fp64")
    assert e.value.code == L.GF2_ESTATE
    g.set_df_factors(s.B)
    for prec in ("bf16x3", "bf16mix"):
        with pytest.raises(L.Gf2Error) as e:
            g.sigma_tau_df(Gt, prec)
        assert e.value.code == L.GF2_EINVAL
    with pytest.raises(L.Gf2Error) as e:          # no factors
        L.gf2_set_df_factors(g.ctx, torch.empty(0, 4, 4, dtype=torch.float64, device="cuda"))
    assert e.value.code == L.GF2_EINVAL
    g.sigma_tau_df(Gt, "fp64")                    # the context stays usable
    L.gf2_set_system(g.ctx, g.S, g.h, g.v)        # a new system drops the factors
    with pytest.raises(L.Gf2Error) as e:
        g.sigma_tau_df(Gt, "fp64")
    assert e.value.code == L.GF2_ESTATE
    g.close()


@pytest.fixture(scope="module")
def oracle_run():
    """Iteration 0 and two correlated iterations of the N=10 workload (dense
    oracle loop; its integrals are the product of the 30 factors)."""
    s = small_molecule()
    p = O.Params(damp_Sigma=0.5)
    st = O.State(mu=-1.0, F=s.h.copy())
    reps = [O.outer_iteration(s, p, st) for _ in range(3)]
    return s, p, reps, st


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_loop_with_df_sigma_matches_oracle(torch, oracle_run, prec):
    from paper_1405_3273_amd import make_params
    s, p, reps, st = oracle_run
    g = _gf2(s)
    g.reset(mu0=-1.0)
    prm = make_params(tol_mu=p.tol_mu, tol_N=p.tol_N, tol_P=p.tol_P, tol_E=p.tol_E,
                      max_inner=p.max_inner, max_bisect=p.max_bisect, mu_halfwidth=p.mu_halfwidth,
                      damp_P=p.damp_P, mix_depth=p.mix_depth, damp_Sigma=p.damp_Sigma,
                      mu_method=p.mu_method, prec=prec, sigma_df=True)
    for it, ref in enumerate(reps):
        r = g.iterate(prm)
        print(f"df {prec} it {it}: E {r.energy:.12f} / {ref.energy:.12f}", flush=True)
        if prec == "fp64" or it == 0:
            assert r.energy == pytest.approx(ref.energy, rel=1e-10)
        else:
            assert abs(r.energy - ref.energy) <= 1e-6
    if prec == "fp64":
        assert np.max(np.abs(g.Sigma_tau.cpu().numpy() - st.Sigma_tau)) < 1e-9 * max(
            1.0, np.max(np.abs(st.Sigma_tau)))
    g.close()


def test_loop_sigma_df_needs_factors(torch):
    from paper_1405_3273_amd import _lib as L, make_params
    from paper_1405_3273_amd.runtime import Gf2
    s = small_molecule()
    g = Gf2(s.S, s.h, s.v, nelec=s.nelec, beta=s.beta, niw=s.niw, ntau=s.ntau)
    g.reset(mu0=-1.0)
    with pytest.raises(L.Gf2Error) as e:
        g.iterate(make_params(prec="fp64", sigma_df=True))
    assert e.value.code == L.GF2_ESTATE
    with pytest.raises(L.Gf2Error) as e:
        g.iterate(make_params(prec="bf16x3", sigma_df=True))
    assert e.value.code == L.GF2_EINVAL
    g.close()
