"""GPU parity on a non-equidistant tau grid (gf2_set_tau_grid) against the
oracle's grid transforms and loop, plus the grid path against the uniform
path on a uniform grid."""
import time

import numpy as np
import pytest

import oracle as O
from oracle.grids import tau_grid
from synthetic import generic_system, power_tau_grid, random_tau_stack, small_molecule

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _gf2(s, **kw):
    from paper_1405_3273_amd.runtime import Gf2
    args = dict(nelec=s.nelec, beta=s.beta, niw=s.niw, ntau=s.ntau)
    args.update(kw)
    return Gf2(s.S, s.h, s.v, **args)


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _random_giw(rng, niw, n, beta):
    """A smooth G(i w)-like stack: sum of poles 1/(i w - e) with random weights."""
    w = (2 * np.arange(niw) + 1) * np.pi / beta
    G = np.zeros((niw, n, n), dtype=np.complex128)
    for _ in range(4):
        A = rng.standard_normal((n, n))
        G += (A + A.T)[None] / (1j * w[:, None, None] - rng.uniform(-2, 2))
    return G


@pytest.mark.parametrize("levels,per_level,n", [(2, 2, 3), (4, 6, 5), (6, 16, 7)])
def test_tau_to_iw_on_power_grid_matches_oracle(torch, levels, per_level, n):
    beta, niw = 20.0, 700
    tau = power_tau_grid(beta, levels, per_level)
    print(f"tau->iw grid {levels}x{per_level} ({len(tau)} points) n={n}", flush=True)
    rng = np.random.default_rng(levels * 10 + n)
    Y = random_tau_stack(rng, len(tau), n)
    ref, ref1 = O.sigma_tau_to_iw(Y, beta, niw, tau=tau)
    s = generic_system(n, 1, beta=beta, niw=niw, ntau=len(tau))
    g = _gf2(s)
    g.set_tau_grid(tau)
    got, got1 = g.tau_to_iw(torch.as_tensor(Y).cuda())
    err = _rel(got.cpu().numpy(), ref)
    print(f"  rel err {err:.2e}")
    assert err < 1e-11
    assert np.max(np.abs(got1.cpu().numpy() - ref1)) < 1e-14
    g.close()


@pytest.mark.parametrize("levels,per_level,n", [(3, 4, 4), (6, 16, 6)])
def test_iw_to_tau_on_power_grid_matches_oracle(torch, levels, per_level, n):
    beta, niw = 20.0, 900
    tau = power_tau_grid(beta, levels, per_level)
    print(f"iw->tau grid {levels}x{per_level} ({len(tau)} points) n={n}", flush=True)
    rng = np.random.default_rng(7 + n)
    G = _random_giw(rng, niw, n, beta)
    mom = [rng.standard_normal((n, n)) for _ in range(3)]
    mom = [0.5 * (m + m.T) for m in mom]
    ref = O.g_iw_to_tau(G, *mom, beta, len(tau), tau=tau)
    s = generic_system(n, 1, beta=beta, niw=niw, ntau=len(tau))
    g = _gf2(s)
    g.set_tau_grid(tau)
    got = g.iw_to_tau(torch.as_tensor(G).cuda(), torch.as_tensor(np.stack(mom)).cuda())
    err = _rel(got.cpu().numpy(), ref)
    print(f"  rel err {err:.2e}")
    assert err < 1e-11
    g.close()


def test_grid_path_equals_uniform_path_on_a_uniform_grid(torch):
    beta, niw, ntau, n = 15.0, 500, 65, 5
    rng = np.random.default_rng(3)
    Y = random_tau_stack(rng, ntau, n)
    G = _random_giw(rng, niw, n, beta)
    mom = np.stack([np.eye(n), 0.1 * np.eye(n), 0.01 * np.eye(n)])
    s = generic_system(n, 1, beta=beta, niw=niw, ntau=ntau)
    g = _gf2(s)
    Yd, Gd, md = (torch.as_tensor(x).cuda() for x in (Y, G, mom))
    u_iw, _ = g.tau_to_iw(Yd)
    u_tau = g.iw_to_tau(Gd, md)
    g.set_tau_grid(tau_grid(beta, ntau))
    q_iw, _ = g.tau_to_iw(Yd)
    q_tau = g.iw_to_tau(Gd, md)
    assert _rel(q_iw.cpu().numpy(), u_iw.cpu().numpy()) < 1e-12
    assert _rel(q_tau.cpu().numpy(), u_tau.cpu().numpy()) < 1e-12
    g.set_tau_grid(None)
    r_iw, _ = g.tau_to_iw(Yd)
    assert torch.equal(r_iw, u_iw)
    g.close()


@pytest.mark.parametrize("levels,per_level", [(8, 32), (12, 160)])
def test_workload_size_transforms_sampled(torch, levels, per_level):
    """N = 100, 16384 frequencies, a 513-point power grid and one of 3841 points
    (the paper's "3000-4000 points"): every element is transformed on the GPU;
    a 3x3 block is checked against the oracle (the transforms act element by
    element).  Prints the transform times."""
    n, beta, niw = 100, 200.0, 16384
    tau = power_tau_grid(beta, levels, per_level)
    print(f"grid {levels}x{per_level}: {len(tau)} points", flush=True)
    rng = np.random.default_rng(11)
    Y = random_tau_stack(rng, len(tau), n)
    G = _random_giw(rng, niw, 3, beta)
    from paper_1405_3273_amd.runtime import Gf2
    S = np.eye(n)
    v = torch.zeros((n, n, n, n), dtype=torch.float64, device="cuda")
    g = Gf2(S, np.zeros((n, n)), v, nelec=n, beta=beta, niw=niw, ntau=len(tau))
    g.set_tau_grid(tau)
    Yd = torch.as_tensor(Y).cuda()
    Gfull = torch.zeros((niw, n, n), dtype=torch.complex128, device="cuda")
    Gfull[:, :3, :3] = torch.as_tensor(G).cuda()
    mom = torch.zeros((3, n, n), dtype=torch.float64, device="cuda")
    mom[0] = torch.eye(n, dtype=torch.float64)
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        got_iw, _ = g.tau_to_iw(Yd)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        got_tau = g.iw_to_tau(Gfull, mom)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    print(f"power grid {len(tau)} points, n={n}, niw={niw}: tau->iw {1e3 * (t1 - t0):.1f} ms, "
          f"iw->tau {1e3 * (t2 - t1):.1f} ms", flush=True)
    ref_iw, _ = O.sigma_tau_to_iw(Y[:, :3, :3], beta, niw, tau=tau)
    assert _rel(got_iw[:, :3, :3].cpu().numpy(), ref_iw) < 1e-11
    m3 = mom[:, :3, :3].cpu().numpy()
    ref_tau = O.g_iw_to_tau(G, *m3, beta, len(tau), tau=tau)
    assert _rel(got_tau[:, :3, :3].cpu().numpy(), ref_tau) < 1e-11
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x6"])
def test_loop_on_power_grid_matches_oracle(torch, prec):
    """HF reference plus two correlated iterations of the N=10 workload on a
    129-point power grid: energies against the oracle's loop on the same grid
    (FP64 to 1e-10 relative, FP32 and BF16x6 Sigma to 1e-6 Eh)."""
    from paper_1405_3273_amd import make_params
    s = small_molecule()
    s.ntau = 129
    s.tau = power_tau_grid(s.beta, 4, 16)
    p = O.Params(damp_Sigma=0.5)
    st = O.State(mu=-1.0, F=s.h.copy())
    ref = [O.outer_iteration(s, p, st).energy for _ in range(3)]
    g = _gf2(s)
    g.set_tau_grid(s.tau)
    g.reset(mu0=-1.0)
    prm = make_params(tol_mu=p.tol_mu, tol_N=p.tol_N, tol_P=p.tol_P, tol_E=p.tol_E,
                      max_inner=p.max_inner, max_bisect=p.max_bisect,
                      mu_halfwidth=p.mu_halfwidth, damp_P=p.damp_P, mix_depth=p.mix_depth,
                      damp_Sigma=p.damp_Sigma, mu_method=p.mu_method, prec=prec)
    got = [g.iterate(prm).energy for _ in range(3)]
    print(f"{prec}: E gpu {got} oracle {ref}", flush=True)
    assert got[0] == pytest.approx(ref[0], rel=1e-10)
    for a, b in zip(got[1:], ref[1:]):
        if prec == "fp64":
            assert a == pytest.approx(b, rel=1e-10)
        else:
            assert abs(a - b) <= 1e-6
    if prec == "fp64":
        assert np.max(np.abs(g.G_tau.cpu().numpy() - st.G_tau)) < 1e-9
    g.close()


def test_set_tau_grid_rejects_bad_grids(torch):
    from paper_1405_3273_amd import _lib as L
    s = generic_system(3, 1, beta=10.0, ntau=9)
    g = _gf2(s)
    bad = [np.array([0.0, 1.0, 2.0, 10.0]),          # not symmetric
           np.array([0.0, 5.0, 5.0, 10.0]),          # not increasing
           np.array([0.5, 4.0, 6.0, 9.5]),           # does not start at 0
           np.array([0.0, 10.0])]                    # too short
    for tau in bad:
        with pytest.raises(L.Gf2Error) as e:
            L.gf2_set_tau_grid(g.ctx, torch.as_tensor(tau).cuda())
        assert e.value.code == L.GF2_EINVAL
    g.set_tau_grid(power_tau_grid(10.0, 2, 2))       # 9 points
    d = g.dims_with(ntau=17)
    Y = torch.zeros((17, 3, 3), dtype=torch.float64, device="cuda")
    out = torch.empty((d.niw, 3, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(L.Gf2Error) as e:
        L.gf2_fourier(g.ctx, d, L.GF2_TAU2IW, Y, None, out, None)
    assert e.value.code == L.GF2_EINVAL
    g.close()


def test_batched_sweep_on_power_grids_equals_single(torch):
    """gf2_iterate_batched over systems with different power grids gives, system
    by system, exactly what gf2_iterate gives alone on the same grid."""
    from paper_1405_3273_amd import make_params
    from paper_1405_3273_amd.runtime import Gf2, Gf2Batch
    grids = {6: (3, 4), 17: (4, 4), 33: (2, 8)}
    members = []
    for n, (lv, u) in grids.items():
        s = generic_system(n, 900 + n, naux=3 * n, beta=40.0, niw=256, ntau=2 * lv * u + 1)
        s.tau = power_tau_grid(s.beta, lv, u)
        members.append(s)

    def make(s):
        g = Gf2(s.S, s.h, s.v, nelec=s.nelec, beta=s.beta, niw=s.niw, ntau=s.ntau)
        g.set_tau_grid(s.tau)
        g.reset(mu0=float(np.mean(np.diag(s.h))))
        return g

    prm = make_params(damp_Sigma=0.5, prec="fp32")
    singles = [make(s) for s in members]
    batch = Gf2Batch([make(s) for s in members])
    for it in range(3):
        rb = batch.iterate(prm)
        rs = [g.iterate(prm) for g in singles]
        for s, a, b in zip(members, rb, rs):
            print(f"it {it} n={s.n}: E {a.energy:.12f} / {b.energy:.12f}", flush=True)
            assert a.energy == b.energy and a.mu == b.mu
    for gb, gs in zip(batch.systems, singles):
        for name in ("P", "G_tau", "Sigma_tau"):
            assert torch.equal(getattr(gb, name), getattr(gs, name)), name
    batch.close()
    for g in singles:
        g.close()
