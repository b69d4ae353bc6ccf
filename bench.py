#!/usr/bin/env python3
"""GF2 benchmark on one MI355X.

A step is one outer GF2 iteration of the Supplementary Material's loop on
the N=100 molecule-shaped workload (100 electrons, banded h, naux=400,
beta=200, 16384 Matsubara frequencies, 512 tau points, seed 300):
Eq. (Sigma) at every tau point, Sigma(tau) -> Sigma(i w), the inner loop
(mu search + Dyson + Fock, Pulay-mixed density) to max|dP| < 1e-10, the
Galitskii-Migdal energy and G(i w) -> G(tau).  By default the mu search of
early inner passes is inexact (--mu-tol-rel); every inner loop still ends on a
pass that located mu to tol_N = 1e-10 electrons.  Warm-up iterations include
the Hartree-Fock reference (iteration 0).  Inputs are resident in HBM before
the timed region.

Prints one JSON line (see --help for the knobs).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GF2 iterations/s + Σ(τ) TFLOP/s at N=100,nτ=512; FP32/BF16-split vs FP64"

PEAK = {  # MI355X published dense peaks
    "fp64": 78.6e12, "fp32": 157.3e12, "bf16x3": 2.5e15, "bf16x6": 2.5e15, "bf16mix": 2.5e15, "hbm": 8.0e12, "fp64_vector": 78.6e12,
}

WORKLOADS = {
    "n100": ("molecule_n100", "generic-n100: N=100, 100 electrons, half-band 12, naux=400, "
             "beta=200, niw=16384, ntau=512, seed 300"),
    "n10": ("small_molecule", "generic-n10: N=10, 10 electrons, naux=30, beta=50, niw=2048, "
            "ntau=257, seed 0"),
    "n160": ("molecule_n160", "generic-n160: N=160, 160 electrons, half-band 16, naux=640, "
             "beta=200, niw=16384, ntau=512, seed 400"),
    "c2": ("batched_member", "batched-sweep-64: 64 generic systems, even N drawn from [8, 48] "
           "(seed 199), N electrons, naux=3N, beta=100, niw=4096, ntau=513, seeds 200..263"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sigma_flops(n, ntau):
    return 8.0 * n ** 5 * ntau


KERNEL_SOURCES = {"dyson": "dyson.hip", "sigma_gemm": "sigma.hip", "sigma_s23": "sigma.hip",
                  "sigma_splitk": "sigma.hip", "t2i_expand": "fourier.hip", "i2t_fold": "fourier.hip",
                  "fock": "fock.hip", "sigma_df": "sigma_df.hip"}


def source_hash(kernel_class):
    import hashlib
    f = os.path.join(ROOT, "paper_1405_3273_amd", "csrc", KERNEL_SOURCES[kernel_class])
    with open(f, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kernel_class, workload, prec):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (profiles/pmc_traffic.md), or None when there is none for this
    kernel class and workload or the kernel's source changed since."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    i = text.find("```json")
    if i < 0:
        return None
    j = text.find("```", i + 7)
    try:
        data = json.loads(text[i + 7:j])
    except ValueError:
        return None
    for e in data.get("entries", []):
        if (e.get("kernel_class") == kernel_class and e.get("workload") == workload
                and e.get("prec") in (prec, None) and e.get("source_sha") == source_hash(kernel_class)):
            return e.get("bytes_per_launch")
    return None


def cpu_baseline(sysm, counts, sample_tau=3, sample_freq=512):
    """The oracle, as it stands, on a bounded sample of one outer iteration:
    Eq. (Sigma) at `sample_tau` tau points and Eq. (GF) (+ density trace) at
    `sample_freq` frequencies; scaled to a whole iteration with the numbers
    of Dyson solves the GPU iteration performed."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    n, ntau, niw = sysm.n, sysm.ntau, sysm.niw
    rng = np.random.default_rng(0)
    Gt = 0.05 * rng.standard_normal((ntau, n, n))
    Gt = 0.5 * (Gt + Gt.transpose(0, 2, 1))
    t0 = time.perf_counter()
    O.sigma_tau(Gt, sysm.v, taus=list(range(sample_tau)))
    t_sig = (time.perf_counter() - t0) / sample_tau * ntau
    ns = np.arange(sample_freq) * (niw // sample_freq)
    F = sysm.h
    t0 = time.perf_counter()
    G = O.green_iw(-1.0, sysm.S, F, None, sysm.beta, niw, n_idx=ns)
    _ = float(np.einsum("nij,ji->", G.real, sysm.S))
    t_dys = (time.perf_counter() - t0) / sample_freq * niw
    solves = counts["solves"]
    t_iter = t_sig + t_dys * solves
    return {
        "value": 1.0 / t_iter, "unit": "iterations/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"Eq. (Sigma) at {sample_tau} of {ntau} tau points ({t_sig:.1f} s scaled) and "
                   f"Eq. (GF) at {sample_freq} of {niw} frequencies ({t_dys:.2f} s per full solve) "
                   f"x {solves} solves per iteration (the GPU iteration's count)"),
        "seconds_per_iteration": t_iter,
    }


def cpu_baseline_sweep(members, solves_per_system, sample_freq=64):
    """The oracle on a bounded sample of one batched outer iteration: Eq. (Sigma)
    at one tau point of every member and Eq. (GF) at `sample_freq` frequencies of
    every member, scaled to all tau points, all frequencies and the GPU
    iteration's Dyson solves per system."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t_sig = t_dys = 0.0
    for m in members:
        rng = np.random.default_rng(0)
        Gt = 0.05 * rng.standard_normal((m.ntau, m.n, m.n))
        Gt = 0.5 * (Gt + Gt.transpose(0, 2, 1))
        t0 = time.perf_counter()
        O.sigma_tau(Gt, m.v, taus=[1])
        t_sig += (time.perf_counter() - t0) * m.ntau
        ns = np.arange(sample_freq) * (m.niw // sample_freq)
        t0 = time.perf_counter()
        G = O.green_iw(-1.0, m.S, m.h, None, m.beta, m.niw, n_idx=ns)
        _ = float(np.einsum("nij,ji->", G.real, m.S))
        t_dys += (time.perf_counter() - t0) / sample_freq * m.niw * solves_per_system
    t_iter = t_sig + t_dys
    return {"value": 1.0 / t_iter, "unit": "iterations/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"Eq. (Sigma) at 1 tau point of each of the {len(members)} systems "
                       f"({t_sig:.1f} s scaled to every tau point) and Eq. (GF) at {sample_freq} "
                       f"frequencies of each ({t_dys:.1f} s scaled to all frequencies x "
                       f"{solves_per_system:.1f} solves per system)"),
            "seconds_per_iteration": t_iter}


def run_sweep(args, desc):
    """The batched sweep: one step is one outer iteration of all 64 systems
    through gf2_iterate_batched (Sigma(tau) of every system in one captured
    graph, the inner loops in lockstep, one captured graph per Dyson round)."""
    import numpy as np
    import torch
    import synthetic
    from paper_1405_3273_amd import _lib as L
    from paper_1405_3273_amd.runtime import Gf2, Gf2Batch

    t0 = time.perf_counter()
    members = [synthetic.batched_member(k) for k in range(64)]
    log(f"workload {desc} generated in {time.perf_counter() - t0:.1f} s")
    batch = Gf2Batch([Gf2(m.S, m.h, m.v, nelec=m.nelec, beta=m.beta, niw=m.niw, ntau=m.ntau)
                      for m in members])
    batch.reset()
    # 12 mixing pairs, damping 0.5: with the default 8 and 0.3 one member (n = 22,
    # Hartree-Fock gap 0.01 Eh at beta = 100) stalls near max|dP| = 1e-6
    prm = L.make_params(prec=args.prec, damp_Sigma=0.5, tol_N_rel=args.mu_tol_rel, damp_P=0.5,
                        mix_depth=12, max_inner=200)
    for w in range(args.warmup):
        reps = batch.iterate(prm)
        log(f"warmup {w}: {reps[0].ms_total:.0f} ms (sigma {reps[0].ms_sigma:.0f}, "
            f"inner {reps[0].ms_inner:.0f}); max inner passes {max(r.n_inner for r in reps)}")
    lead = batch.systems[0].ctx
    torch.cuda.synchronize()
    L.gf2_profile_enable(lead, True)
    steps = args.steps
    all_reps = []
    t_start = time.perf_counter()
    for k in range(steps):
        reps = batch.iterate(prm)
        all_reps.append(reps)
        log(f"step {k}: {reps[0].ms_total:.0f} ms (sigma {reps[0].ms_sigma:.0f}, fourier "
            f"{reps[0].ms_fourier:.0f}, inner {reps[0].ms_inner:.0f}); max |dE| "
            f"{max(abs(r.dE) for r in reps):.2e}; max inner passes {max(r.n_inner for r in reps)}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = L.gf2_profile_read(lead)
    L.gf2_profile_enable(lead, False)
    sig_flops = sum(sigma_flops(m.n, m.ntau) for m in members)
    ms_sigma = float(np.mean([r[0].ms_sigma for r in all_reps]))
    achieved = sig_flops / (ms_sigma / 1e3)
    pk = PEAK[args.prec]
    dy_ms, dy_n, dy_work = prof["dyson"]
    line = {
        "metric": METRIC, "value": steps / elapsed, "unit": "iterations/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16",
                  "bf16mix": "bf16+f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": desc, "systems": len(members),
                   "sizes": [int(m.n) for m in members], "sigma_arithmetic": args.prec,
                   "other_stages": "f64", "damp_Sigma": prm.damp_Sigma,
                   "mu_tol_N_rel": prm.tol_N_rel, "mix_depth": prm.mix_depth,
                   "damp_P": prm.damp_P,
                   "step": "one outer iteration of all systems"},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": pk / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / pk, "traffic": None,
                     "kernel": "sigma_graph (all Sigma(tau) launches of the 64 systems, one "
                               "captured graph; host clock around the synchronised replay)",
                     "launches": steps, "avg_launch_ms": ms_sigma, "work_per_launch": sig_flops},
        "dyson_rounds": {"launches": dy_n, "ms": dy_ms,
                         "tflops": (dy_work / (dy_ms / 1e3) / 1e12) if dy_ms > 0 else None},
        "per_step": {"ms_sigma": ms_sigma,
                     "ms_fourier": float(np.mean([r[0].ms_fourier for r in all_reps])),
                     "ms_inner": float(np.mean([r[0].ms_inner for r in all_reps])),
                     "max_inner_passes": float(np.mean([max(x.n_inner for x in r) for r in all_reps])),
                     "energies": [r.energy for r in all_reps[-1]]},
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        solves = dy_n / steps     # Dyson rounds per step: each round solves every pending system
        line["cpu_baseline"] = cpu_baseline_sweep(members, solves)
    batch.close()
    print(json.dumps(line), flush=True)


def run_converge(args, sysm, desc):
    """Run the loop from the core guess to |dE| < tol_E on two consecutive outer
    iterations.  The reduced-precision Sigma(tau) forms reach a noise floor
    between iterations (FP32 at N = 160: about 5e-7 Eh); once |dE| falls below
    --switch-dE, Sigma(tau) runs in --prec-final (the loop state carries over:
    the iteration simply continues with the other arithmetic)."""
    import numpy as np
    import torch
    from paper_1405_3273_amd import _lib as L
    from paper_1405_3273_amd.runtime import Gf2

    g = Gf2(sysm.S, sysm.h, sysm.v, nelec=sysm.nelec, beta=sysm.beta, niw=sysm.niw,
            ntau=sysm.ntau)
    if sysm.tau is not None:
        g.set_tau_grid(sysm.tau)
    g.reset(mu0=float(np.mean(np.diag(sysm.h))))
    prec = args.prec
    tol_P, tol_N = 1e-10, 1e-10
    hist = []
    below = 0
    switched_at = None
    t_start = time.perf_counter()
    for it in range(args.max_outer):
        prm = L.make_params(prec=prec, damp_Sigma=0.5, tol_N_rel=args.mu_tol_rel, tol_P=tol_P,
                            tol_N=tol_N)
        r = g.iterate(prm)
        hist.append({"iteration": it, "prec": prec, "energy": r.energy, "dE": r.dE, "dP": r.dP,
                     "n_inner": r.n_inner, "n_eval": r.n_eval, "ms": r.ms_total,
                     "ms_sigma": r.ms_sigma})
        log(f"iteration {it} [{prec}]: E {r.energy:.10f} dE {r.dE:+.2e} dP {r.dP:.1e} inner "
            f"{r.n_inner} evals {r.n_eval} {r.ms_total:.0f} ms (sigma {r.ms_sigma:.0f})")
        if it >= 2 and switched_at is None and abs(r.dE) < args.switch_dE:
            prec = args.prec_final
            tol_P, tol_N = args.tol_P_final, min(1e-10, args.tol_P_final)
            switched_at = it + 1
            below = 0
            log(f"|dE| < {args.switch_dE:g}: Sigma(tau) in {prec}, inner tol_P {tol_P:g} from "
                f"iteration {switched_at}")
            continue
        below = below + 1 if (it >= 2 and abs(r.dE) < args.tol_E) else 0
        if below >= 2:
            break
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    g.close()
    line = {
        "metric": METRIC, "value": len(hist) / elapsed, "unit": "iterations/s", "n_gpus": 1,
        "steps": len(hist), "warmup": 0, "ms_per_step": elapsed / len(hist) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16",
                  "bf16mix": "bf16+f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": desc, "mode": "converge", "sigma_arithmetic": args.prec,
                   "sigma_arithmetic_final": args.prec_final, "switch_dE": args.switch_dE,
                   "inner_tol_P": 1e-10, "inner_tol_P_final": args.tol_P_final,
                   "tol_E": args.tol_E, "damp_Sigma": 0.5, "mu_tol_N_rel": args.mu_tol_rel},
        "convergence": {"converged": below >= 2, "iterations": len(hist),
                        "switched_at": switched_at, "seconds": elapsed,
                        "energy": hist[-1]["energy"], "last_dE": [h["dE"] for h in hist[-3:]],
                        "history": hist},
    }
    print(json.dumps(line), flush=True)


def run_beta_scan(args, desc):
    """Temperature dependence of the converged GF2 state of the N=10 system: the loop
    run to |dE| < 1e-9 Eh and max|dP| < 1e-8 (FP64 Sigma) at each inverse temperature,
    with the Matsubara cutoff (2 n_w + 1) pi / beta and the tau step beta / (n_tau - 1) of
    the beta = 50 workload kept fixed.  Reports E(T), mu(T), the natural occupations
    and the heat capacity C = dE/dT by central differences in T."""
    import numpy as np
    import torch
    import synthetic
    from paper_1405_3273_amd import _lib as L
    from paper_1405_3273_amd.runtime import Gf2

    rows = []
    t_start = time.perf_counter()
    total_it = 0
    for beta in [float(b) for b in args.betas.split(",")]:
        s = synthetic.small_molecule()
        scale = beta / 50.0
        s.beta, s.niw, s.ntau = beta, int(round(2048 * scale)), int(round(256 * scale)) + 1
        g = Gf2(s.S, s.h, s.v, nelec=s.nelec, beta=s.beta, niw=s.niw, ntau=s.ntau)
        g.reset(mu0=-1.0)
        prm = L.make_params(prec="fp64", damp_Sigma=0.5)
        conv = False
        for it in range(200):
            r = g.iterate(prm)
            total_it += 1
            if it > 1 and abs(r.dE) < 1e-9 and r.dP < 1e-8:
                conv = True
                break
        occ = g.natural_occupations(g.P).cpu().numpy()
        rows.append({"beta": beta, "T": 1.0 / beta, "niw": s.niw, "ntau": s.ntau, "converged": conv,
                     "iterations": it + 1, "energy": r.energy, "e1b": r.e1b, "e2b": r.e2b, "mu": r.mu,
                     "occupations": [float(x) for x in occ]})
        log(f"beta {beta:g}: {it + 1} iterations, E {r.energy:.10f} (E_2b {r.e2b:.8f}), mu {r.mu:.8f}, "
            f"NONs {occ[0]:.6f} .. {occ[-1]:.6f}")
        g.close()
    elapsed = time.perf_counter() - t_start
    T = np.array([r["T"] for r in rows])
    E = np.array([r["energy"] for r in rows])
    order = np.argsort(T)
    for a in range(1, len(order) - 1):
        i0, i1, i2 = order[a - 1], order[a], order[a + 1]
        rows[i1]["heat_capacity"] = float((E[i2] - E[i0]) / (T[i2] - T[i0]))
    line = {
        "metric": METRIC, "value": total_it / elapsed, "unit": "iterations/s", "n_gpus": 1,
        "steps": total_it, "warmup": 0, "ms_per_step": elapsed / total_it * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "mode": "beta scan (converged at each temperature)",
                   "betas": args.betas, "sigma_arithmetic": "fp64", "damp_Sigma": 0.5},
        "temperature_dependence": rows,
    }
    print(json.dumps(line), flush=True)


def df_flops(n, naux, route):
    """Flops of the density-fitted Eq. (Sigma) per tau point (gf2_sigma_tau_df), by the
    route its exchange term takes."""
    if route == "tensor":
        return 4.0 * naux * n ** 4 + 4.0 * naux ** 2 * n ** 2 + 10.0 * naux * n ** 3
    return 4.0 * naux ** 2 * n ** 3 + 4.0 * naux ** 2 * n ** 2 + 8.0 * naux * n ** 3


def run_sigma_df(args, sysm, desc):
    """Density-fitted Eq. (Sigma) at every tau point of the workload, FP64 and FP32,
    timed beside the dense contraction on the same G(tau) (the Hartree-Fock G(tau)
    of iteration 0); one JSON line."""
    import numpy as np
    import torch
    from paper_1405_3273_amd import _lib as L
    from paper_1405_3273_amd.runtime import Gf2

    g = Gf2(sysm.S, sysm.h, sysm.v, nelec=sysm.nelec, beta=sysm.beta, niw=sysm.niw,
            ntau=sysm.ntau)
    g.set_df_factors(sysm.B)
    g.reset(mu0=float(np.mean(np.diag(sysm.h))))
    g.iterate(L.make_params(prec="fp64"))
    Gt = g.G_tau
    naux, n, ntau = int(sysm.B.shape[0]), g.n, sysm.ntau
    res = {}
    for pr in [p for p in args.df_prec.split(",") if p]:
        out = torch.empty_like(Gt)
        g.sigma_tau_df(Gt[:4].contiguous(), pr)          # workspaces
        torch.cuda.synchronize()
        L.gf2_profile_enable(g.ctx, True)
        t1 = time.perf_counter()
        g.sigma_tau_df(Gt, pr, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        prof = L.gf2_profile_read(g.ctx)["sigma_df"]
        L.gf2_profile_enable(g.ctx, False)
        fl = prof[2] / prof[1]                               # flops per tau point, route taken
        route = "tensor" if abs(fl - df_flops(n, naux, "tensor")) < 1e-6 * fl else "pair"
        dense = torch.empty_like(Gt)
        g.sigma_tau(Gt, pr, out=dense)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g.sigma_tau(Gt, pr, out=dense)
        torch.cuda.synchronize()
        dt_dense = time.perf_counter() - t2
        diff = float((out - dense).abs().max() / dense.abs().max())
        per_tau = prof[0] / prof[1] / 1e3
        res[pr] = {"seconds": dt, "ms_per_tau": dt / ntau * 1e3, "exchange_route": route,
                   "flops_per_tau": fl, "pair_route_flops_per_tau": df_flops(n, naux, "pair"),
                   "tflops_algorithmic": fl * ntau / dt / 1e12,
                   "event_ms_per_tau": per_tau * 1e3, "event_tflops": fl / per_tau / 1e12,
                   "frac_of_peak": fl / per_tau / PEAK[pr],
                   "dense_seconds": dt_dense, "dense_over_df_time": dt_dense / dt,
                   "max_rel_diff_vs_dense": diff}
        log(f"sigma_df {pr} ({route} route): {dt:.2f} s ({dt / ntau * 1e3:.2f} ms per tau, "
            f"{res[pr]['tflops_algorithmic']:.1f} TFLOP/s); dense {dt_dense * 1e3:.0f} ms; "
            f"max rel diff {diff:.2e}")
    g.close()
    main_pr = [p for p in args.df_prec.split(",") if p][0]
    r = res[main_pr]
    line = {
        "metric": "density-fitted Σ(τ) TFLOP/s (flops of the exchange route taken per τ point)",
        "value": r["tflops_algorithmic"], "unit": "TFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": r["seconds"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32"}[main_pr], "data": "synthetic",
        "config": {"workload": desc, "mode": "density-fitted Sigma(tau), all tau points",
                   "naux": naux, "n": n, "ntau": ntau, "G_tau": "Hartree-Fock G(tau) of iteration 0"},
        "roofline": {"bound": "mfma", "achieved": r["event_tflops"], "peak": PEAK[main_pr] / 1e12,
                     "unit": "TFLOP/s", "frac": r["frac_of_peak"],
                     "traffic": measured_traffic("sigma_df", args.workload, main_pr),
                     "kernel": "sigma_df (one tau point: the whole GEMM chain)"},
        "sigma_df": res,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32", "bf16x3", "bf16x6", "bf16mix"])
    ap.add_argument("--workload", default="n100", choices=sorted(WORKLOADS))
    ap.add_argument("--sigma-prec", default="fp64,fp32,bf16x3,bf16x6,bf16mix",
                    help="precisions for the stand-alone Sigma(tau) timing ('' to skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mu-tol-rel", type=float, default=1e-2,
                    help="inexact mu search in early inner passes: tolerance\n"
                         "max(tol_N, rel * max|dP| of the previous pass); each inner loop still\n"
                         "ends on a pass that used tol_N (0 = tol_N throughout)")
    ap.add_argument("--forms", default="fp64,bf16x3,bf16x6,bf16mix",
                    help="other Sigma precisions run through the same iterations from the same\n"
                         "start, for the whole-iteration speedup and energy difference against\n"
                         "the FP64 form ('' to skip)")
    ap.add_argument("--beta-scan", action="store_true",
                    help="N=10 system converged at each of --betas (temperature dependence)")
    ap.add_argument("--betas", default="25,37.5,50,75,100,150,200")
    ap.add_argument("--tau-grid", default="",
                    help="'L,U': run on the non-equidistant power grid of L halvings with U\n"
                         "steps each (2 L U + 1 points) instead of the uniform grid")
    ap.add_argument("--converge", action="store_true",
                    help="run from the core guess until |dE| < --tol-E twice in a row (no timing\n"
                         "legs); Sigma(tau) switches to --prec-final once |dE| < --switch-dE")
    ap.add_argument("--tol-E", type=float, default=1e-7)
    ap.add_argument("--switch-dE", type=float, default=2e-6)
    ap.add_argument("--prec-final", default="fp64", choices=["fp64", "fp32", "bf16x6", "bf16mix"])
    ap.add_argument("--tol-P-final", type=float, default=1e-10,
                    help="inner-loop max|dP| tolerance from the switch on (1e-10 before)")
    ap.add_argument("--max-outer", type=int, default=150)
    ap.add_argument("--sigma-df", action="store_true",
                    help="time the density-fitted Sigma(tau) (gf2_sigma_tau_df) at every tau\n"
                         "point of the workload against the dense contraction; one JSON line")
    ap.add_argument("--df-prec", default="fp64,fp32")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="copy 1 GiB device-to-device before the workload (a kernel of known\n"
                         "traffic, for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures one GPU: this build has no multi-GPU path (the tau axis of "
            "Eq. (Sigma) would shard across GPUs; see DESIGN.md). Run with --gpus 1.")
        sys.exit(2)

    import numpy as np
    import torch
    import synthetic
    from paper_1405_3273_amd import _lib as L
    from paper_1405_3273_amd.runtime import Gf2

    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del a, b

    gen, desc = WORKLOADS[args.workload]
    if args.beta_scan:
        return run_beta_scan(args, WORKLOADS["n10"][1].split(",")[0] + " system (N=10, seed 0)")
    if args.workload == "c2":
        return run_sweep(args, desc)
    t0 = time.perf_counter()
    sysm = getattr(synthetic, gen)()
    log(f"workload {desc} generated in {time.perf_counter() - t0:.1f} s")
    if args.tau_grid:
        lv, per = (int(x) for x in args.tau_grid.split(","))
        sysm.tau = synthetic.power_tau_grid(sysm.beta, lv, per)
        sysm.ntau = len(sysm.tau)
        desc += f"; power tau grid {lv} x {per} ({sysm.ntau} points)"
    if args.converge:
        return run_converge(args, sysm, desc)
    if args.sigma_df:
        return run_sigma_df(args, sysm, desc)
    g = Gf2(sysm.S, sysm.h, sysm.v, nelec=sysm.nelec, beta=sysm.beta, niw=sysm.niw,
            ntau=sysm.ntau)
    if sysm.tau is not None:
        g.set_tau_grid(sysm.tau)
    g.reset(mu0=float(np.mean(np.diag(sysm.h))))
    prm = L.make_params(prec=args.prec, damp_Sigma=0.5, tol_N_rel=args.mu_tol_rel)

    for w in range(args.warmup):
        r = g.iterate(prm)
        log(f"warmup {w}: E {r.energy:.10f} inner {r.n_inner} evals {r.n_eval} "
            f"{r.ms_total:.0f} ms (sigma {r.ms_sigma:.0f})")

    torch.cuda.synchronize()
    L.gf2_profile_enable(g.ctx, True)
    reps = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        r = g.iterate(prm)
        reps.append(r)
        log(f"step {k}: E {r.energy:.10f} dE {r.dE:.2e} inner {r.n_inner} evals {r.n_eval} "
            f"{r.ms_total:.0f} ms (sigma {r.ms_sigma:.0f}, fourier {r.ms_fourier:.0f}, "
            f"inner {r.ms_inner:.0f})")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = L.gf2_profile_read(g.ctx)
    L.gf2_profile_enable(g.ctx, False)
    steps = args.steps
    value = steps / elapsed

    # dominant kernel class over the timed region
    kind = {"sigma_gemm": ("mfma", args.prec), "sigma_splitk": ("mfma", args.prec),
            "sigma_s23": ("mfma", args.prec),
            "dyson": ("alu", "fp64_vector"), "t2i_expand": ("hbm", "hbm"),
            "i2t_fold": ("hbm", "hbm"), "fock": ("hbm", "hbm"),
            "occupations": ("latency", None), "sigma_df": ("mfma", args.prec)}
    dom = max((k for k in prof if kind[k][0] != "latency"), key=lambda k: prof[k][0])
    ms, cnt, work = prof[dom]
    bound, pk = kind[dom]
    avg_s = ms / cnt / 1e3
    per_launch = work / cnt
    achieved = per_launch / avg_s
    unit = "GB/s" if bound == "hbm" else "TFLOP/s"
    scale = 1e9 if bound == "hbm" else 1e12
    roofline = {"bound": bound, "achieved": achieved / scale, "peak": PEAK[pk] / scale,
                "unit": unit, "frac": achieved / PEAK[pk],
                "traffic": measured_traffic(dom, args.workload, args.prec),
                "kernel": dom, "launches": cnt, "avg_launch_ms": avg_s * 1e3,
                "work_per_launch": per_launch}
    if bound == "mfma" and args.prec in ("bf16x3", "bf16x6"):
        k = 3 if args.prec == "bf16x3" else 6
        roofline["note"] = (f"{args.prec} issues {k} bf16 MFMA products per algorithmic FP32 MAC: "
                            f"frac is at most 1/{k} against the bf16 peak")
    classes = {k: {"ms": v[0], "launches": v[1],
                   "rate": (v[2] / (v[0] / 1e3) / (1e9 if kind[k][0] == "hbm" else 1e12))
                   if v[0] > 0 else None,
                   "rate_unit": "GB/s" if kind[k][0] == "hbm" else "TFLOP/s"}
               for k, v in prof.items() if kind[k][0] != "latency"}

    # natural occupation numbers of the last density (not part of an iteration)
    occ = g.natural_occupations(g.P)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nrep = 5
    for _ in range(nrep):
        occ = g.natural_occupations(g.P)
    torch.cuda.synchronize()
    occ_ms = (time.perf_counter() - t1) / nrep * 1e3
    occ_h = occ.cpu().numpy()
    nons = {"ms": occ_ms, "n": int(g.n), "largest": float(occ_h[0]), "smallest": float(occ_h[-1]),
            "sum": float(occ_h.sum()),
            "fractional": int(np.sum((occ_h > 0.02) & (occ_h < 1.98)))}
    log(f"natural occupations: {occ_ms:.2f} ms, sum {nons['sum']:.10f}, "
        f"{nons['fractional']} in (0.02, 1.98)")

    # stand-alone Sigma(tau) per precision on the current G(tau)
    sig_rates = {}
    for pr in [p for p in args.sigma_prec.split(",") if p]:
        out = torch.empty_like(g.G_tau)
        g.sigma_tau(g.G_tau, pr, out=out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.sigma_tau(g.G_tau, pr, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        sig_rates[pr] = {"seconds": dt, "tflops_algorithmic": sigma_flops(g.n, sysm.ntau) / dt / 1e12}
        log(f"sigma {pr}: {dt * 1e3:.1f} ms, {sig_rates[pr]['tflops_algorithmic']:.1f} TFLOP/s")

    counts = {"n_inner": float(np.mean([r.n_inner for r in reps])),
              "n_eval": float(np.mean([r.n_eval for r in reps])),
              "solves": prof["dyson"][1] / steps}   # Dyson launches per iteration
    energy_main = reps[-1].energy
    g.close()

    # the other precision forms: same start, same number of iterations
    forms = {}
    for pr in [p for p in args.forms.split(",") if p and p != args.prec]:
        gf = Gf2(sysm.S, sysm.h, sysm.v, nelec=sysm.nelec, beta=sysm.beta, niw=sysm.niw,
                 ntau=sysm.ntau)
        if sysm.tau is not None:
            gf.set_tau_grid(sysm.tau)
        gf.reset(mu0=float(np.mean(np.diag(sysm.h))))
        pf = L.make_params(prec=pr, damp_Sigma=0.5, tol_N_rel=args.mu_tol_rel)
        for w in range(args.warmup):
            gf.iterate(pf)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(steps):
            rf = gf.iterate(pf)
        torch.cuda.synchronize()
        forms[pr] = {"ms_per_step": (time.perf_counter() - t1) / steps * 1e3, "energy": rf.energy}
        log(f"form {pr}: {forms[pr]['ms_per_step']:.0f} ms/iteration, E {rf.energy:.10f}")
        gf.close()
    forms[args.prec] = {"ms_per_step": elapsed / steps * 1e3, "energy": energy_main}
    if "fp64" in forms:
        ref = forms["fp64"]
        for pr, f in forms.items():
            f["speedup_vs_fp64"] = ref["ms_per_step"] / f["ms_per_step"]
            f["energy_minus_fp64"] = f["energy"] - ref["energy"]
    line = {
        "metric": METRIC, "value": value, "unit": "iterations/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16", "bf16x6": "bf16", "bf16mix": "bf16+f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": desc, "sigma_arithmetic": args.prec,
                   "other_stages": "f64", "inner_tol_P": prm.tol_P, "damp_Sigma": prm.damp_Sigma,
                   "mu_search": "secant", "mu_tol_N": prm.tol_N, "mu_tol_N_rel": prm.tol_N_rel,
                   "mix_depth": prm.mix_depth},
        "roofline": roofline,
        "kernel_classes": classes,
        "sigma_tflops": sig_rates,
        "natural_occupations": nons,
        "precision_forms": {"iterations": args.warmup + steps, "timed": steps, "forms": forms,
                            "note": "energy after the same iterations from the same start; "
                                    "not a converged energy"},
        "per_step": {"n_inner": counts["n_inner"], "n_eval": counts["n_eval"],
                     "ms_sigma": float(np.mean([r.ms_sigma for r in reps])),
                     "ms_fourier": float(np.mean([r.ms_fourier for r in reps])),
                     "ms_inner": float(np.mean([r.ms_inner for r in reps])),
                     "energy": reps[-1].energy, "dE": reps[-1].dE},
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        line["cpu_baseline"] = cpu_baseline(sysm, counts)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
