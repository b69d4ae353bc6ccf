"""Batched sweep (gf2_iterate_batched): several uneven systems iterated
together give, system by system, exactly what gf2_iterate gives alone, and
agree with the oracle loop."""
import numpy as np
import pytest

import oracle as O
from synthetic import generic_system

pytestmark = pytest.mark.gpu

# uneven sizes spanning the inversion size classes 1-3 and the Sigma tile counts 1-3
SIZES = (6, 10, 17, 24, 33, 40)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _members():
    return [generic_system(n, 700 + n, naux=3 * n, beta=40.0, niw=256, ntau=33) for n in SIZES]


def _make(sysm):
    from paper_1405_3273_amd.runtime import Gf2
    g = Gf2(sysm.S, sysm.h, sysm.v, nelec=sysm.nelec, beta=sysm.beta, niw=sysm.niw, ntau=sysm.ntau)
    g.reset(mu0=float(np.mean(np.diag(sysm.h))))
    return g


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6", "bf16mix"])
def test_batched_equals_single(torch, prec):
    from paper_1405_3273_amd import make_params
    from paper_1405_3273_amd.runtime import Gf2Batch
    members = _members()
    prm = make_params(damp_Sigma=0.5, prec=prec)
    singles = [_make(s) for s in members]
    batch = Gf2Batch([_make(s) for s in members])
    for it in range(3):
        print(f"{prec} iteration {it}", flush=True)
        rb = batch.iterate(prm)
        rs = [g.iterate(prm) for g in singles]
        for k, (a, b) in enumerate(zip(rb, rs)):
            print(f"  n={SIZES[k]}: E {a.energy:.12f} / {b.energy:.12f} inner {a.n_inner}/{b.n_inner} "
                  f"evals {a.n_eval}/{b.n_eval}", flush=True)
            assert a.energy == b.energy and a.mu == b.mu
            assert a.n_inner == b.n_inner and a.n_eval == b.n_eval
    for gb, gs in zip(batch.systems, singles):
        for name in ("P", "F", "G_tau", "Sigma_tau"):
            assert torch.equal(getattr(gb, name), getattr(gs, name)), name
    batch.close()
    for g in singles:
        g.close()


def test_batched_member_matches_oracle(torch):
    """The n=17 member through the batch against the oracle loop (FP64 Sigma)."""
    from paper_1405_3273_amd import make_params
    from paper_1405_3273_amd.runtime import Gf2Batch
    members = _members()
    k = SIZES.index(17)
    s = members[k]
    p = O.Params(damp_Sigma=0.5)
    st = O.State(mu=float(np.mean(np.diag(s.h))), F=s.h.copy())
    refs = [O.outer_iteration(s, p, st) for _ in range(2)]
    batch = Gf2Batch([_make(m) for m in members])
    prm = make_params(damp_Sigma=0.5, prec="fp64")
    for it, ref in enumerate(refs):
        r = batch.iterate(prm)[k]
        print(f"it {it}: E {r.energy:.12f} / {ref.energy:.12f}", flush=True)
        assert r.energy == pytest.approx(ref.energy, rel=1e-10)
        assert r.mu == pytest.approx(ref.mu, abs=1e-9)
    assert np.max(np.abs(batch.systems[k].P.cpu().numpy() - st.P)) < 1e-9
    batch.close()


def test_batched_rejects_repeated_context(torch):
    from paper_1405_3273_amd import Gf2Error, make_params
    from paper_1405_3273_amd.runtime import Gf2Batch
    g = _make(_members()[0])
    with pytest.raises(Gf2Error):
        Gf2Batch([g, g]).iterate(make_params())
    g.close()
