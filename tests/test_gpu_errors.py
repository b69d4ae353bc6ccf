"""Failure paths of the C ABI, forced from the host: a NaN in the input Green's
function, an inner-loop step limit of one pass, an electron count outside
[0, 2n].  Every kernel still runs to its normal end; the status code is what is
checked, and the context stays usable afterwards."""
import numpy as np
import pytest

from synthetic import generic_system, random_tau_stack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _gf2(sysm, **kw):
    from paper_1405_3273_amd.runtime import Gf2
    args = dict(nelec=sysm.nelec, beta=sysm.beta, niw=sysm.niw, ntau=sysm.ntau)
    args.update(kw)
    return Gf2(sysm.S, sysm.h, sysm.v, **args)


def _system():
    return generic_system(6, 31, naux=12, beta=20.0, niw=256, ntau=33)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6", "bf16mix"])
def test_sigma_tau_nonfinite_input_reports_enonfinite(torch, prec):
    from paper_1405_3273_amd import _lib as L
    print(f"errors: sigma_tau NaN prec={prec}", flush=True)
    s = _system()
    g = _gf2(s)
    Gt = random_tau_stack(np.random.default_rng(3), s.ntau, s.n)
    bad = Gt.copy()
    bad[5, 2, 3] = bad[5, 3, 2] = np.nan
    with pytest.raises(L.Gf2Error) as e:
        g.sigma_tau(torch.as_tensor(bad).cuda(), prec)
    assert e.value.code == L.GF2_ENONFINITE
    assert "non-finite" in L.gf2_last_error()
    # the context is still usable
    out = g.sigma_tau(torch.as_tensor(Gt).cuda(), prec).cpu().numpy()
    assert np.all(np.isfinite(out))
    g.close()


def test_iterate_nonfinite_sigma_reports_enonfinite(torch):
    from paper_1405_3273_amd import _lib as L
    print("errors: iterate with NaN in G(tau)", flush=True)
    s = _system()
    g = _gf2(s)
    g.reset(mu0=-1.0)
    prm = L.make_params(prec="fp64")
    g.iterate(prm)                            # Hartree-Fock reference
    g.G_tau[7, 1, 1] = float("nan")
    with pytest.raises(L.Gf2Error) as e:
        g.iterate(prm)
    assert e.value.code == L.GF2_ENONFINITE
    # a fresh start on the same context works
    g.reset(mu0=-1.0)
    r = g.iterate(prm)
    assert np.isfinite(r.energy)
    g.close()


def test_iterate_inner_step_limit_reports_enoconv(torch):
    from paper_1405_3273_amd import _lib as L
    print("errors: iterate with max_inner = 1", flush=True)
    s = _system()
    g = _gf2(s)
    g.reset(mu0=-1.0)
    # the first pass of a run has no input density to compare with, so one pass
    # cannot end the inner loop
    with pytest.raises(L.Gf2Error) as e:
        g.iterate(L.make_params(prec="fp64", max_inner=1))
    assert e.value.code == L.GF2_ENOCONV
    g.reset(mu0=-1.0)
    r = g.iterate(L.make_params(prec="fp64"))
    assert np.isfinite(r.energy)
    g.close()


def test_mu_search_step_limit_reports_enoconv_or_ebracket(torch):
    from paper_1405_3273_amd import _lib as L
    print("errors: density_fock with max_bisect = 1", flush=True)
    s = _system()
    g = _gf2(s)
    F = torch.as_tensor(s.h).cuda()
    with pytest.raises(L.Gf2Error) as e:
        g.density_fock(L.make_params(prec="fp64", max_bisect=1), F, mu=5.0)
    assert e.value.code in (L.GF2_ENOCONV, L.GF2_EBRACKET)
    g.close()


@pytest.mark.parametrize("nelec", [-2, 13])
def test_iterate_electron_count_outside_range_reports_ebracket(torch, nelec):
    from paper_1405_3273_amd import _lib as L
    print(f"errors: iterate with nelec={nelec}", flush=True)
    s = _system()
    g = _gf2(s, nelec=nelec)
    g.reset(mu0=-1.0)
    with pytest.raises(L.Gf2Error) as e:
        g.iterate(L.make_params(prec="fp64"))
    assert e.value.code == L.GF2_EBRACKET
    g.close()
