"""GPU runs of the remaining workload configurations at their full sizes:
the lattice hopping scan (N = 32, FP64 against FP32 Sigma, one member against
the oracle's stored iterations), the N = 160 molecule-shaped system (one
correlated FP32 iteration, Sigma(tau) sampled against the oracle) and the
N = 100 workload (the Sigma arithmetics' energies against FP64; the inexact mu
search against the exact one)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from synthetic import lattice_sweep, molecule_n160

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _make(s):
    from paper_1405_3273_amd.runtime import Gf2
    g = Gf2(s.S, s.h, s.v, nelec=s.nelec, beta=s.beta, niw=s.niw, ntau=s.ntau)
    g.reset(mu0=float(np.mean(np.diag(s.h))))
    return g


def test_lattice_scan_fp32_against_fp64(torch):
    """The 8 lattice systems (N = 32, beta = 100, 8192 frequencies, 1025 tau
    points) as one batch: the Hartree-Fock reference and one correlated
    iteration with FP64 and with FP32 Sigma.  Member 3 (FP64) equals the
    oracle's stored iterations; FP32 stays within 1e-6 Eh of FP64."""
    from paper_1405_3273_amd import make_params
    from paper_1405_3273_amd.runtime import Gf2Batch
    members = [lattice_sweep(k) for k in range(8)]
    with open(os.path.join(HERE, "golden", "lattice_n32_t3.json")) as f:
        gold = json.load(f)
    energies = {}
    for prec in ("fp64", "fp32"):
        batch = Gf2Batch([_make(m) for m in members])
        prm = make_params(damp_Sigma=0.5, prec=prec)
        for it in range(2):
            reps = batch.iterate(prm)
            print(f"{prec} it {it}: " + " ".join(f"{r.energy:.9f}" for r in reps), flush=True)
            if prec == "fp64":
                ref = gold["iterations"][it]
                r = reps[gold["index"]]
                assert r.energy == pytest.approx(ref["energy"], rel=1e-10)
                assert r.mu == pytest.approx(ref["mu"], abs=1e-9)
        energies[prec] = np.array([r.energy for r in reps])
        batch.close()
    diff = np.abs(energies["fp32"] - energies["fp64"])
    print("fp32 - fp64:", diff, flush=True)
    assert np.all(diff <= 1e-6)


def test_n160_correlated_iteration(torch):
    """N = 160 (naux 640, 16384 frequencies, 512 tau points), FP32 Sigma in
    the configuration bench.py times: after the Hartree-Fock iteration, the
    first correlated iteration's Sigma(tau) equals the oracle's at sampled tau
    points of the same G(tau); tr(P S) = N_elec; Sigma(tau) is symmetric."""
    from paper_1405_3273_amd import make_params
    s = molecule_n160()
    g = _make(s)
    prm = make_params(damp_Sigma=0.5, prec="fp32")
    r0 = g.iterate(prm)
    print(f"HF: E {r0.energy:.9f} inner {r0.n_inner} evals {r0.n_eval} {r0.ms_total:.0f} ms", flush=True)
    Ghf = g.G_tau.cpu().numpy()
    r1 = g.iterate(prm)
    print(f"it 1: E {r1.energy:.9f} inner {r1.n_inner} evals {r1.n_eval} {r1.ms_total:.0f} ms "
          f"(sigma {r1.ms_sigma:.0f})", flush=True)
    taus = [0, 1, s.ntau // 2, s.ntau - 1]
    Sig = g.Sigma_tau.cpu().numpy()[taus]
    ref = O.sigma_tau(Ghf, s.v, taus=taus)
    err = float(np.max(np.abs(Sig - ref)) / np.max(np.abs(ref)))
    print(f"Sigma rel err {err:.2e}", flush=True)
    assert err <= 3e-5
    asym = float(np.max(np.abs(Sig - Sig.transpose(0, 2, 1))) / np.max(np.abs(Sig)))
    assert asym <= 3e-6
    P = g.P.cpu().numpy()
    # the mu search stops at |N(mu) - N_elec| < 1e-10 (trace formula); <P, S> of the
    # assembled P agrees to rounding of the sums over 16384 frequencies
    assert abs(float(np.trace(P @ s.S)) - s.nelec) < 1e-9 * s.nelec
    assert np.isfinite(r1.energy)
    g.close()


def test_n100_split_forms_energy_against_fp64(torch):
    """The N = 100 workload (beta = 200, 16384 frequencies, 512 tau points): five
    outer iterations from the same start with each Sigma arithmetic.  The
    energies after every iteration stay within the bars against the FP64 form:
    FP32 1e-6 Eh; the mixed split form (three-term split in the second and third
    transforms) 1e-5 Eh.  The two-term split (BF16x3) does not meet 1e-5 Eh at
    this size (its operands carry 2^-16 relative error; measured 4e-5 to 8e-5 Eh):
    its bound here is 2e-4 Eh."""
    from paper_1405_3273_amd import make_params
    from synthetic import molecule_n100
    s = molecule_n100()
    bars = {"fp32": 1e-6, "bf16mix": 1e-5, "bf16x3": 2e-4}
    energies = {}
    for prec in ("fp64", "fp32", "bf16mix", "bf16x3"):
        g = _make(s)
        prm = make_params(damp_Sigma=0.5, prec=prec, tol_N_rel=1e-2)
        energies[prec] = [g.iterate(prm).energy for _ in range(5)]
        print(prec, " ".join(f"{e:.10f}" for e in energies[prec]), flush=True)
        g.close()
    for prec, bar in bars.items():
        d = np.abs(np.array(energies[prec]) - np.array(energies["fp64"]))
        print(f"{prec} - fp64: {d}", flush=True)
        assert np.all(d <= bar), prec


def test_n100_inexact_mu_search_reaches_the_same_iterations(torch):
    """The benchmark's inexact mu search (tol_N_rel = 1e-2: early inner passes
    locate mu loosely, every inner loop still ends on a pass that used tol_N)
    against the loop as the oracle runs it (tol_N_rel = 0) on the N = 100
    workload with FP32 Sigma: the Hartree-Fock iteration and four correlated
    iterations agree to 1e-10 relative in the energy and 1e-9 in mu, with fewer
    Dyson evaluations."""
    from paper_1405_3273_amd import make_params
    from synthetic import molecule_n100
    s = molecule_n100()
    runs = {}
    for rel in (0.0, 1e-2):
        g = _make(s)
        prm = make_params(damp_Sigma=0.5, prec="fp32", tol_N_rel=rel)
        runs[rel] = [g.iterate(prm) for _ in range(5)]
        print(f"tol_N_rel {rel}: " + " ".join(f"{r.energy:.12f}/{r.n_eval}" for r in runs[rel]),
              flush=True)
        g.close()
    for a, b in zip(runs[0.0], runs[1e-2]):
        assert b.energy == pytest.approx(a.energy, rel=1e-10)
        assert b.mu == pytest.approx(a.mu, abs=1e-9)
    assert sum(r.n_eval for r in runs[1e-2]) < sum(r.n_eval for r in runs[0.0])
