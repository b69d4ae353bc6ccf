"""The batched sweep at its full configuration: 64 generic systems with even N
drawn from [8, 48], beta = 100, 4096 Matsubara frequencies, 513 tau points,
FP32 Sigma(tau) and FP64 everything else, iterated together by
gf2_iterate_batched (the Hartree-Fock reference and one correlated iteration).
The density mixing keeps 12 pairs with damping 0.5 (SWEEP_MIX): with the
default 8 pairs and 0.3, member 34 (n = 22, a Hartree-Fock gap of 0.01 Eh,
beta x gap = 1) stalls near max|dP| = 1e-6; with 16 pairs members 5 and 53 do.
Every system must come out bitwise equal to gf2_iterate on that system alone,
and the smallest member (FP64 Sigma) must match the oracle loop."""
import numpy as np
import pytest

import oracle as O
from synthetic import batched_member, batched_sizes

pytestmark = pytest.mark.gpu

SWEEP_MIX = dict(damp_P=0.5, mix_depth=12, max_inner=200)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _make(sysm):
    from paper_1405_3273_amd.runtime import Gf2
    g = Gf2(sysm.S, sysm.h, sysm.v, nelec=sysm.nelec, beta=sysm.beta, niw=sysm.niw,
            ntau=sysm.ntau)
    g.reset(mu0=float(np.mean(np.diag(sysm.h))))
    return g


def test_sweep_64_systems_batched_equals_single(torch):
    from paper_1405_3273_amd import make_params
    from paper_1405_3273_amd.runtime import Gf2Batch
    members = [batched_member(k) for k in range(64)]
    assert len(members) == 64 and min(m.n for m in members) >= 8 and max(m.n for m in members) <= 48
    assert all(m.niw == 4096 and m.ntau == 513 and m.beta == 100.0 for m in members)
    prm = make_params(damp_Sigma=0.5, prec="fp32", tol_N_rel=1e-2, **SWEEP_MIX)
    batch = Gf2Batch([_make(m) for m in members])
    rb = [batch.iterate(prm) for _ in range(2)]
    print(f"batched: {rb[1][0].ms_total:.0f} ms for the correlated iteration of 64 systems "
          f"(sigma {rb[1][0].ms_sigma:.0f}, inner {rb[1][0].ms_inner:.0f})", flush=True)
    for k, m in enumerate(members):
        g = _make(m)
        for it in range(2):
            r = g.iterate(prm)
            a = rb[it][k]
            assert a.energy == r.energy and a.mu == r.mu, (k, it)
            assert a.n_inner == r.n_inner and a.n_eval == r.n_eval, (k, it)
        print(f"  member {k} (n = {m.n}): E {r.energy:.10f} equal", flush=True)
        gb = batch.systems[k]
        for name in ("P", "F", "G_tau", "Sigma_tau"):
            assert torch.equal(getattr(gb, name), getattr(g, name)), (k, name)
        g.close()
    batch.close()


def test_sweep_smallest_member_matches_oracle(torch):
    from paper_1405_3273_amd import make_params
    from paper_1405_3273_amd.runtime import Gf2Batch
    sizes = batched_sizes()
    k = int(np.argmin(sizes))
    members = [batched_member(j) for j in range(64)]
    s = members[k]
    print(f"oracle check on member {k} (n = {s.n})", flush=True)
    p = O.Params(damp_Sigma=0.5, **SWEEP_MIX)
    st = O.State(mu=float(np.mean(np.diag(s.h))), F=s.h.copy())
    refs = [O.outer_iteration(s, p, st) for _ in range(2)]
    batch = Gf2Batch([_make(m) for m in members])
    prm = make_params(damp_Sigma=0.5, prec="fp64", **SWEEP_MIX)
    for it, ref in enumerate(refs):
        r = batch.iterate(prm)[k]
        print(f"it {it}: E {r.energy:.12f} / {ref.energy:.12f}", flush=True)
        assert r.energy == pytest.approx(ref.energy, rel=1e-10)
        assert r.mu == pytest.approx(ref.mu, abs=1e-9)
    assert np.max(np.abs(batch.systems[k].P.cpu().numpy() - st.P)) < 1e-9
    assert np.max(np.abs(batch.systems[k].G_tau.cpu().numpy() - st.G_tau)) < 1e-9
    batch.close()
