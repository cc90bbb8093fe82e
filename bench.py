"""Throughput benchmark: population annealing at L = 16 on one MI355X.

Workload (the throughput configuration): 3D +-J spin glass, L = 16 (4096 spins),
R0 = 1e6 replicas bit-packed (0.5 GB per population buffer), beta linear 0 -> 5 in 301
temperatures, 10 Metropolis sweeps per temperature.  Couplings and initial spins are drawn
from seeds on the device (synthetic data).

A step is one temperature of the schedule through the whole hot path: resample
(histogram, FP64 normalisation, Poisson copy numbers, scan, gather), 10 fused sweeps,
measurement (energy moments) and the free-energy estimate.  W warm-up steps run first
(untimed), then K steps are timed between device synchronisations; the population is
resident in HBM throughout.  value = spin-flip attempts (replicas x spins x sweeps) per
second over the K timed steps.

Printed: one JSON line with the metric, the roofline of the dominant kernel (the sweep,
timed live with HIP events on its stream) and the CPU oracle's throughput on a bounded
sample of the same sweep (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/s at L=16; wall time to var(βF)≤1e-3, learned vs fixed Δβ"
# algorithmic VALU work per Metropolis attempt, int32 lane-ops: 1/8 of a Philox4x32-10 call
# (10 rounds x (2 wide multiplies + 2 three-input xors) = 40 ops per call, 8 attempts per call)
# plus the threshold select, compare and flip (3 ops)
OPS_PER_ATTEMPT = 40 / 8 + 3
# MI355X vector ALU from its unit counts and clock: the published FP32 vector peak, 157.3 TFLOP/s,
# is 256 CUs x 2.4 GHz x 128 lanes x 2 flops (one FMA); the same 128 32-bit lanes per clock per CU
# give 78.6 T int32 lane-ops/s.  (The probe in libpa_calib.so reaches ~100 lanes per clock per CU
# with two-operand adds and xors at the clock the chip sustains under load; 64-bit multiplies and
# three-operand ops issue at about half that.)
PEAK_LANE_OPS = 256 * 128 * 2.4e9
COUNTERS = os.path.join(ROOT, "profiles", "sweep_L16_R1e6_counters.json")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=295)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--L", type=int, default=16)
    p.add_argument("--R0", type=int, default=1_000_000)
    p.add_argument("--n-temps", type=int, default=301)
    p.add_argument("--n-sweeps", type=int, default=10)
    p.add_argument("--layout", default="bits64")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU work of the oracle baseline")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "sweep_L16_R1e6_traffic.json"))
    p.add_argument("--workload", default="L16", choices=["L16", "batched", "learned", "bias", "bias_gauss", "stepped", "gauss", "gauss_survey",
                            "gauss_stepped"],
                   help="L16: the throughput configuration (default); batched: 256 runs in one graph; "
                        "learned: learned vs fixed schedules, wall time to Var(beta F~) <= 1e-3 at L=12; "
                        "bias: weighted vs plain averages against the exact ring (18 realizations x 200 runs); "
                        "bias_gauss: the same on the paper's Gaussian chain (N=256, R=1000, 100 temperatures, 50 sweeps); "
                        "stepped: Var(beta F~(beta)) for constant, stepped and learned schedules at equal work; "
                        "gauss: the Gaussian 3D ensemble, L=8, R=2000, 100 temperatures, 100 sweeps, 126 runs; "
                        "gauss_survey: 25 Gaussian L=8 realizations (Var(beta F~) vs Gamma) and the worst at R=2000 and 10000; "
                        "gauss_stepped: constant R=2000 vs R_beta 1000/3000 (beta_c=0.9) on the worst Gaussian realization")
    p.add_argument("--ensemble", type=int, default=100, help="runs per schedule (learned vs fixed)")
    p.add_argument("--no-learned", action="store_true", help="skip the learned-vs-fixed leg of the default run")
    p.add_argument("--no-probe", action="store_true", help="skip the live vector-ALU probe of the default run")
    p.add_argument("--oracle-runs", action="store_true",
                   help="time whole oracle runs of the ring and of the L=8 cube on the host, then exit")
    return p.parse_args()


BATCH_COUNTERS = os.path.join(ROOT, "profiles", "batched_256runs_L6-10_counters.json")


def batched_by_size(specs):
    """Per lattice size of the batched configuration: one batched sweep launch (10 sweeps of every
    run of that size, at its initial size) per first-look regime (beta = 0.5, 2, 4), timed live
    with HIP events on the batch's stream; with the counted VALU instructions per attempt of the
    committed counter summary while the colour-string kernel's sources still match it."""
    import torch

    from paper_1006_0252_amd import pa, workloads
    from paper_1006_0252_amd.profile_summary import STRING_SOURCES, sweep_source_digest

    counted = None
    try:
        with open(BATCH_COUNTERS) as f:
            c = json.load(f)
        if c.get("source_digest") == sweep_source_digest(STRING_SOURCES):
            counted = c["by_size"]
    except (ValueError, OSError, KeyError):
        pass
    out = {}
    for L in sorted({sp["L"] for sp in specs}):
        sub = [sp for sp in specs if sp["L"] == L]
        batch = pa.Batch(sub, 4, layout="bits64", device="cuda:0").init()
        sched = pa.Schedule([0.0, 0.5, 2.0, 4.0], workloads.C3_SWEEPS, batch.runs[0].n_bins, device="cuda:0")
        att = float(sum(sp["R0"] for sp in sub)) * L ** 3 * workloads.C3_SWEEPS
        for k in (1, 2, 3):
            step = sched.step(k)
            batch.sweep(step)  # warm-up launch
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(batch.stream)
            batch.sweep(step)
            b.record(batch.stream)
            b.synchronize()
            ms = a.elapsed_time(b)
            v = {"ms": ms, "attempts_per_s": att / (ms * 1e-3)}
            reg = str(k - 1)
            if counted and str(L) in counted and reg in counted[str(L)]:
                v["valu_per_attempt"] = counted[str(L)][reg].get("SQ_INSTS_VALU")
            out.setdefault(str(L), {})[reg] = v
        del batch
        torch.cuda.empty_cache()
    return out


def bench_batched(args):
    """256 runs (64 realisations x 4 seeds, L in {6,8,10}, R0 in [1e4,1e5]) annealed together:
    one sweep launch per lattice size per step, the whole schedule one HIP graph; value =
    attempts/s of the graph replay (steps = the 100 temperature steps).  by_size_and_regime: each
    size's sweep timed alone in each first-look regime (batched_by_size)."""
    from paper_1006_0252_amd import ensemble, workloads

    specs = workloads.batched_specs()
    r = ensemble.run_batched(specs, workloads.C3_TEMPS, workloads.C3_SWEEPS, tune=True, graph=True)
    w = r["weighted"]
    rec = r["records"]
    groups = {}
    for i, sp in enumerate(specs):  # sweep attempts of the schedule per lattice size
        g = groups.setdefault(str(sp["L"]), {"runs": 0, "attempts": 0.0})
        g["runs"] += 1
        g["attempts"] += float(np.sum(rec[i, 1:, 4])) * sp["L"] ** 3 * workloads.C3_SWEEPS
    out = {
        "metric": METRIC, "value": r["attempts_per_s"], "unit": "attempts/s", "n_gpus": 1,
        "steps": workloads.C3_TEMPS - 1, "warmup": 0,
        "ms_per_step": r["seconds"] / (workloads.C3_TEMPS - 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batched_64x4_L6-10_R1e4-1e5", "runs": len(specs), "n_temps": workloads.C3_TEMPS,
                   "n_sweeps": workloads.C3_SWEEPS, "layout": "bits64", "graph": True,
                   "tuned_blocks_per_cu_order": r["tuned"]},
        "batched": {"attempts": r["attempts"], "seconds": r["seconds"],
                    "mean_var_betaF": float(np.mean(w["var_betaF"])),
                    "max_var_betaF": float(np.max(w["var_betaF"])),
                    "mean_gamma": float(np.mean(w["gamma"])), "mean_binder": float(np.mean(w["binder"])),
                    "groups": groups},
    }
    del r
    out["by_size_and_regime"] = batched_by_size(specs)
    print(json.dumps(out), flush=True)


def bench_learned(args):
    """The learned-vs-fixed protocol (learned_vs_fixed) as the benchmark line: value = best fixed
    time to target / best learned time to target."""
    out = learned_vs_fixed(args.ensemble)
    print(json.dumps(out), flush=True)


def learned_vs_fixed(M):
    """Learned vs fixed temperature steps on the 3D +-J cube L = 12, R0 = 2e5, 10 sweeps per
    temperature, beta 0 -> 5, one coupling realization (disorder seed 1).

    Networks (one per target resampled fraction rho* in {0.1, 0.2, 0.3, 0.5}) are trained on
    the GPU from fixed-schedule traces of the ring (N = 64, R0 = 1000, 51 temperatures) and the
    L = 8 cube (R0 = 5e4, 101 temperatures).  For each rho* a pilot run picks the schedule,
    which M production runs then follow; fixed linear schedules use N_T in {51, 101, 201, 401}.
    Per schedule: Var(beta F~) over the M runs at beta = 5 and the wall time per run T_run;
    time to target = T_run ceil(Var / 1e-3) (+ the pilot's time for a learned schedule).
    value = best fixed time to target / best learned time to target."""
    import torch

    from paper_1006_0252_amd import learned, pa

    dev = "cuda:0"
    L, R0, ns = 12, 200_000, 10
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    Xt, Dt, Xv, Dv = learned.training_set(device=dev)
    torch.cuda.synchronize()
    t_traces = time.perf_counter() - t0
    log(f"traces: {Xt.shape[0]} training and {Xv.shape[0]} validation samples in {t_traces:.1f} s")
    t0 = time.perf_counter()
    nets, logs = learned.train_networks(Xt, Dt, Xv, Dv, steps=3000, log_every=2999, device=dev)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"training: 4 networks in {t_train:.1f} s; final train/validation loss " +
        ", ".join(f"{rs}: {h[-1][1]:.4g}/{h[-1][2]:.4g}" for rs, h in logs.items()))
    out_l, out_f = {}, {}
    prod_steps, prod_seconds = 0, 0.0
    for rs in learned.RHO_TARGETS:
        betas, info = learned.pilot_schedule(nets[rs], L, R0, seed=10 ** 6, disorder_seed=1, n_sweeps=ns,
                                             dmin=1e-4, dmax=0.25, device=dev)
        e = learned.ensemble(betas, M, L, R0, ns, disorder_seed=1, device=dev)
        ttt = learned.time_to_target(e["var"], e["seconds_per_run"], overhead=info["seconds"])
        out_l[str(rs)] = dict(n_temps=len(betas), pilot_ok=info["ok"], pilot_s=info["seconds"], var=e["var"],
                             minus_betaF_bar=e["minus_betaF_bar"], T_run_s=e["seconds_per_run"], time_to_target_s=ttt,
                             attempts_per_s=e["attempts"] / e["seconds"])
        prod_steps += len(betas) - 1
        prod_seconds += e["seconds"]
        log(f"learned rho*={rs}: {len(betas)} temperatures, Var {e['var']:.4g}, T_run {e['seconds_per_run']:.4f} s, "
            f"time to target {ttt:.2f} s")
    for nT in (51, 101, 201, 401):
        e = learned.ensemble(pa.linear_schedule(nT), M, L, R0, ns, disorder_seed=1, device=dev)
        ttt = learned.time_to_target(e["var"], e["seconds_per_run"])
        out_f[str(nT)] = dict(n_temps=nT, var=e["var"], minus_betaF_bar=e["minus_betaF_bar"],
                              T_run_s=e["seconds_per_run"], time_to_target_s=ttt,
                              attempts_per_s=e["attempts"] / e["seconds"])
        prod_steps += nT - 1
        prod_seconds += e["seconds"]
        log(f"fixed N_T={nT}: Var {e['var']:.4g}, T_run {e['seconds_per_run']:.4f} s, time to target {ttt:.2f} s")
    bl = min(out_l, key=lambda k: out_l[k]["time_to_target_s"])
    bf = min(out_f, key=lambda k: out_f[k]["time_to_target_s"])
    ref = out_f["401"]
    dev_sigma = {k: (v["minus_betaF_bar"] - ref["minus_betaF_bar"]) / np.sqrt(v["var"] / M + ref["var"] / M)
                 for k, v in out_l.items()}
    out = {
        "metric": METRIC, "value": out_f[bf]["time_to_target_s"] / out_l[bl]["time_to_target_s"],
        "unit": "x (fixed / learned wall time to Var(beta F)<=1e-3)", "n_gpus": 1, "steps": prod_steps,
        "warmup": 0, "ms_per_step": prod_seconds / prod_steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32+bf16", "data": "synthetic",
        "config": {"workload": "learned_vs_fixed_cube_L12_R200000", "L": L, "R0": R0, "n_sweeps": ns,
                   "runs_per_schedule": M, "disorder_seed": 1, "rho_targets": list(learned.RHO_TARGETS),
                   "fixed_n_temps": [51, 101, 201, 401], "dbeta_clamp": [1e-4, 0.25]},
        "best_learned": {"rho_target": float(bl), **out_l[bl]}, "best_fixed": {"n_temps": int(bf), **out_f[bf]},
        "learned": out_l, "fixed": out_f,
        "learned_minus_reference_sigma": dev_sigma,
        "training": {"trace_seconds": t_traces, "train_seconds": t_train, "samples": int(Xt.shape[0]),
                     "validation_samples": int(Xv.shape[0]),
                     "final_loss": {str(rs): [h[-1][1], h[-1][2]] for rs, h in logs.items()}},
    }
    return out



def sweep_source_digest():
    """sha256 over the sources the sweep kernel is compiled from."""
    from paper_1006_0252_amd.profile_summary import sweep_source_digest as digest

    return digest()


def sweep_traffic(path):
    """HBM bytes per sweep launch from the committed counter summary (FETCH_SIZE and WRITE_SIZE,
    scaled by a plain copy's readings), or None when the sweep sources changed since."""
    try:
        with open(path) as f:
            tr = json.load(f)
    except (ValueError, OSError):
        return None
    if tr.get("source_digest") != sweep_source_digest():
        return None
    return tr.get("bytes_per_launch")


def bench_bias(args, chain="pm1"):
    """Sec. IV's 1D bias measurement: 18 realizations x 200 runs of a periodic chain; weighted and
    plain energy and free energy at beta = 1, 2, 5 (nearest schedule points) against the exact chain,
    bootstrap errors, and the block bias mu_k.  chain "pm1": the ±J ring N = 64, R0 = 1000, 51
    temperatures, 5 sweeps; chain "gauss": the paper's Gaussian chain N = 256, R = 1000, 100
    temperatures (19 steps evenly in beta to 0.5, 80 evenly in T to 0.2), 50 sweeps.
    value = mean weighted -beta F_bar minus exact at beta = 5."""
    from paper_1006_0252_amd import bias

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    cfg = bias.CHAINS[chain]
    r = bias.run(n_real=18, M=200, n_boot=100, betas=(1.0, 2.0, 5.0), log=log, chain=chain)
    res = r["by_beta"]
    fb = res[5.0]["free_energy_bias_weighted"]
    n_temps = len(cfg["betas"]())
    steps = 18 * (n_temps - 1)
    name = "ring_N64_bias_18x200" if chain == "pm1" else "gauss_chain_N256_bias_18x200"
    out = {
        "metric": METRIC, "value": fb[0], "unit": "weighted -beta F_bar minus exact at beta=5, mean over realizations",
        "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": r["anneal_seconds"] / steps * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u8+f64", "data": "synthetic",
        "config": {"workload": name, "N": cfg["N"], "couplings": cfg["couplings"], "R0": cfg["R0"], "n_temps": n_temps,
                   "n_sweeps": cfg["n_sweeps"], "realizations": 18, "runs_per_realization": 200,
                   "bootstrap_replicates": 100},
        "by_beta": {str(b): {"beta_grid": v["beta_grid"],
                             "energy_bias": {"weighted": list(v["energy_bias_weighted"]),
                                             "plain": list(v["energy_bias_plain"])},
                             "free_energy_bias": {"weighted": list(v["free_energy_bias_weighted"]),
                                                  "plain": list(v["free_energy_bias_plain"])},
                             "mean_var_betaF": v["mean_var"], "mu_k": {str(k): m for k, m in v["mu_k"].items()}}
                    for b, v in res.items()},
        "anneal_attempts_per_s": r["attempts"] / r["anneal_seconds"],
    }
    print(json.dumps(out), flush=True)


def bench_stepped(args):
    """Sec. IV's stepped population size on the L = 8 cube: the worst of 25 realizations at R = 2000
    (101 temperatures, 10 sweeps), then 200 runs each with constant R, with R_beta stepped x3 at
    beta = 0.9 at equal work, and with learned schedules (rho* = 0.1, 0.2) at constant R.
    value = Var(beta F~) at beta = 5, constant over stepped."""
    from paper_1006_0252_amd import learned, stepped

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    Xt, Dt, Xv, Dv = learned.training_set(device="cuda:0")
    nets, _ = learned.train_networks(Xt, Dt, targets=learned.RHO_TARGETS, steps=3000, device="cuda:0")
    r = stepped.run(learned_nets={0.1: nets[0.1], 0.2: nets[0.2]}, log=log)

    def summ(v):
        b = np.array(v["betas"])
        return {"var_beta5": v["var"][-1], "attempts": v["attempts"], "var_x_work": v["var"][-1] * v["attempts"],
                "n_temps": len(b), "seconds": v["seconds"], "minus_betaF_bar": v["minus_betaF_bar"][-1],
                "var_at": {f"{x:.2f}": v["var"][int(np.argmin(np.abs(b - x)))] for x in (0.5, 0.9, 1.5, 2.5, 3.5, 5.0)}}

    summary = {w: {k: summ(v) for k, v in P.items()} for w, P in r["profiles"].items()}
    W = summary["worst"]
    best_step = min((k for k in W if k.startswith("stepped")), key=lambda k: W[k]["var_beta5"])
    n_steps = sum(v["n_temps"] - 1 for P in summary.values() for v in P.values())
    out = {
        "metric": METRIC, "value": W["constant"]["var_beta5"] / W[best_step]["var_beta5"],
        "unit": "Var(beta F~) at beta=5 on the worst realization, constant R / best stepped R (equal work)",
        "n_gpus": 1, "steps": n_steps, "warmup": 0,
        "ms_per_step": sum(v["seconds"] for P in summary.values() for v in P.values()) / n_steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32+f64", "data": "synthetic",
        "config": {"workload": "stepped_R_cube_L8_R2000", "L": 8, "R": 2000, "n_temps": 101, "n_sweeps": 10,
                   "runs": 200, "beta_c": [0.9, 2.0], "ratio": 3, "realizations": r["picks"]},
        "schedules": summary, "var_by_realization": r["var_by_realization"],
    }
    print(json.dumps(out), flush=True)


# algorithmic VALU work per tabled Gaussian attempt, lane-ops: 1/8 of a Philox call (5), the
# 6-bit neighbour pattern (one op per neighbour) and the table compare and flip (3)
OPS_PER_ATTEMPT_GAUSS = 40 / 8 + 6 + 3


def cpu_baseline_gauss(L, n_sweeps, target_s):
    """The oracle's Gaussian sweep on the first replicas of the L = 8 ensemble's first run, beta = 1."""
    from oracle import oracle as o

    J = o.couplings_gauss(3, L, 1)
    threads = o.num_threads()
    n = max(threads, 16)
    s, E = o.init_replicas_gauss(3, L, J, 1, 0, n)
    t = time.perf_counter()
    o.sweep_replicas_gauss(3, L, J, 1, 1.0, 0, s, E, 0, n_sweeps)
    per_rep = (time.perf_counter() - t) / n
    m = int(max(threads, target_s / max(per_rep, 1e-9)))
    s, E = o.init_replicas_gauss(3, L, J, 1, 0, m)
    t = time.perf_counter()
    o.sweep_replicas_gauss(3, L, J, 1, 1.0, 0, s, E, 0, n_sweeps)
    dt = time.perf_counter() - t
    attempts = m * L ** 3 * n_sweeps
    return {"value": attempts / dt, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle Gaussian sweep of {m} replicas of the L={L} cube, {n_sweeps} sweeps at beta=1 "
                      f"({attempts:.3e} attempts in {dt:.1f} s)"}


def bench_gauss(args):
    """Sec. IV's 3D Gaussian ensemble: L = 8, R = 2000, 100 temperatures evenly spaced in T from 2
    to 0.2 (the random start equilibrated at T = 2), 100 sweeps per temperature, 126 runs of one realization (the
    paper's 125-run ensemble of its worst realization, rounded up to whole pairs for the overlap),
    all runs one batch.  value = attempts/s of
    the whole hot path (resample, sweep, measure with pair overlaps) over the 99 steps and the 100
    sweep blocks; the free energies are relative to T = 2."""
    from paper_1006_0252_amd import gauss3d

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    gauss3d.run(M=4, R=200, n_temps=3, n_sweeps=2)            # warm-up: module load, first launches
    r = gauss3d.run(log=log)
    n_steps = r["n_steps"]
    sweep_s = float(r["sweep_ms"].sum()) / 1e3
    rate = r["attempts"] / sweep_s
    achieved = rate * OPS_PER_ATTEMPT_GAUSS
    out = {
        "metric": METRIC, "value": r["attempts"] / r["wall_seconds"], "unit": "attempts/s", "n_gpus": 1,
        "steps": n_steps, "warmup": 0, "ms_per_step": r["wall_seconds"] / n_steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32+f64", "data": "synthetic",
        "config": {"workload": "gauss3d_L8_R2000_126runs", "L": 8, "R": 2000, "n_temps": 100, "T": [2.0, 0.2],
                   "n_sweeps": 100, "runs": 126, "disorder_seed": 1, "layout": "u8"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "T lane-ops/s", "frac": achieved / PEAK_LANE_OPS, "traffic": None,
                     "kernel": "k_gauss_table + k_sweep_gauss_tab (HIP events around pa_sweep)",
                     "ops_per_attempt": OPS_PER_ATTEMPT_GAUSS, "sweep_attempts_per_s": rate},
        "physics": {"free_energy_reference": "T=2", "minus_betaF_bar": r["minus_betaF_bar"], "var_betaF": r["var_betaF"],
                    "mean_minus_betaF": r["mean_minus_betaF"], "E_bar": r["E_bar"], "gamma_bar": r["gamma_bar"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_gauss(8, 100, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_gauss_survey(args):
    """Sec. IV's 3D study on the Gaussian L = 8 cube: 25 realizations x 100 runs (50 pairs) at
    R = 2000 give Var(beta F~) and the pair-weighted Gamma = P(|q| < 0.2) at T = 0.2; the realization
    with the largest Var is rerun with 126 runs at R = 2000 and at R = 10000.
    value = Var(beta F~) at R = 2000 over Var at R = 10000 on that realization (the paper: 4.7)."""
    from paper_1006_0252_amd import gauss3d

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    gauss3d.run(M=4, R=200, n_temps=3, n_sweeps=2)            # warm-up
    r = gauss3d.survey(log=log)
    rows, w = r["rows"], r["worst_runs"]
    v = np.array([x["var_betaF"] for x in rows])
    g = np.array([x["gamma_bar"] for x in rows])
    secs = sum(x["seconds"] for x in rows) + sum(x["seconds"] for x in w.values())
    att = sum(x["attempts"] for x in rows) + sum(x["attempts"] for x in w.values())
    n_steps = 99 * (len(rows) + 2)
    out = {
        "metric": METRIC, "value": w[2000]["var_betaF"] / w[10000]["var_betaF"],
        "unit": "Var(beta F~) at R=2000 / at R=10000, worst of 25 realizations", "n_gpus": 1, "steps": n_steps,
        "warmup": 0, "ms_per_step": secs / n_steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32+f64", "data": "synthetic",
        "config": {"workload": "gauss3d_L8_survey_25x100", "L": 8, "R": 2000, "R_big": 10000, "n_temps": 100,
                   "T": [2.0, 0.2], "n_sweeps": 100, "realizations": 25, "runs_per_realization": 100,
                   "runs_worst": 126},
        "realizations": rows, "worst": r["worst"], "worst_runs": {str(k): x for k, x in w.items()},
        "var_max": float(v.max()), "var_median": float(np.median(v)),
        "corr_var_gamma": float(np.corrcoef(v, g)[0, 1]) if g.std() > 0 else None,
        "attempts_per_s": att / secs,
    }
    print(json.dumps(out), flush=True)


def bench_gauss_stepped(args):
    """Sec. IV's population size stepped with temperature, on the Gaussian L = 8 cube: the realization
    with the largest Var(beta F~) of the 25 of gauss_survey (disorder seed 10), 250 runs each with
    R_beta = 2000 throughout and with R_beta = 1000 for beta < 0.9, 3000 from beta = 0.9 on (nearly
    equal work); 100 temperatures from T = 2 to 0.2, 100 sweeps.  value = Var(beta F~) at T = 0.2,
    constant over stepped (the paper: 0.57 / 0.36)."""
    from paper_1006_0252_amd import gauss3d

    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    gauss3d.run(M=4, R=200, n_temps=3, n_sweeps=2)            # warm-up
    betas = gauss3d.schedule()
    out_s = {}
    for name, Rt in (("constant", np.full(len(betas), 2000.0)), ("stepped", np.where(betas < 0.9, 1000.0, 3000.0))):
        r = gauss3d.run(M=250, disorder_seed=10, seed0=20_000 + (0 if name == "constant" else 1000), R_targets=Rt)
        vp = r["var_profile"]
        out_s[name] = {"R_targets": {"beta<0.9": float(Rt[0]), "beta>=0.9": float(Rt[-1])}, "attempts": r["attempts"],
                       "seconds": r["wall_seconds"], "var_beta5": float(vp[-1]), "E_bar": r["E_bar"],
                       "minus_betaF_bar": r["minus_betaF_bar"],
                       "var_at": {f"{b:.3f}": float(vp[int(np.argmin(np.abs(betas[1:] - b)))]) for b in (0.9, 1.5, 2.0, 3.0, 4.0, 5.0)}}
        log(f"{name}: Var(beta=5) {vp[-1]:.4f}, attempts {r['attempts']:.3e}, E {r['E_bar']:.3f}")
    c, st = out_s["constant"], out_s["stepped"]
    n_steps = 2 * (len(betas) - 1)
    out = {
        "metric": METRIC, "value": c["var_beta5"] / st["var_beta5"],
        "unit": "Var(beta F~) at T=0.2, constant R / stepped R_beta (equal work)", "n_gpus": 1, "steps": n_steps,
        "warmup": 0, "ms_per_step": (c["seconds"] + st["seconds"]) / n_steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32+f64", "data": "synthetic",
        "config": {"workload": "gauss3d_L8_stepped_R_worst", "L": 8, "disorder_seed": 10, "runs": 250, "n_temps": 100,
                   "T": [2.0, 0.2], "n_sweeps": 100, "beta_c": 0.9},
        "schedules": out_s, "work_ratio": st["attempts"] / c["attempts"],
    }
    print(json.dumps(out), flush=True)


def first_look_regime(beta):
    """Regime of the sweep's 16-bit first look at beta (3D, dE = 4, 8, 12): 0 while the top 16 bits
    of the dE = 8 threshold are non-zero, 1 while only dE = 4 has a non-zero top, 2 beyond."""
    top = lambda dE: int(np.floor(np.ldexp(np.exp(-beta * dE), 16)))  # noqa: E731
    return 0 if top(8) > 0 else (1 if top(4) > 0 else 2)


def sweep_by_regime(betas, sweep_ms, attempts):
    """Mean sweep launch time and attempts/s per first-look regime over the timed steps."""
    reg = np.array([first_look_regime(b) for b in betas])
    out = {}
    for r in (0, 1, 2):
        sel = reg == r
        if sel.any():
            out[str(r)] = {"steps": int(sel.sum()), "avg_launch_ms": float(np.mean(sweep_ms[sel])),
                           "attempts_per_s": float(np.sum(attempts[sel]) / (np.sum(sweep_ms[sel]) * 1e-3))}
    return out


def cpu_info():
    """Model name and logical CPUs available to this process."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def oracle_sweep_rate(o, L, n_sweeps, beta, target_s, max_replicas):
    """The oracle's sweep of the first replicas of the L-cube's initial population (disorder seed 1,
    run seed 1): attempts/s on the oracle's current threads, on about target_s seconds of work."""
    dim = 3
    J = o.couplings(dim, L, 1)
    threads = o.num_threads()
    n = max(threads, 16)
    s, E = o.init_replicas(dim, L, J, 1, 0, n)
    t = time.perf_counter()
    o.sweep_replicas(dim, L, J, 1, beta, 0, s, E, 0, n_sweeps)
    per_rep = (time.perf_counter() - t) / n
    m = int(min(max_replicas, max(threads, target_s / max(per_rep, 1e-9))))
    s, E = o.init_replicas(dim, L, J, 1, 0, m)
    t = time.perf_counter()
    o.sweep_replicas(dim, L, J, 1, beta, 0, s, E, 0, n_sweeps)
    dt = time.perf_counter() - t
    return m * L ** 3 * n_sweeps / dt, m, dt


def cpu_baseline(L, R0, n_sweeps, target_s):
    """The oracle on this host: its pa_sweep (10 sweeps) on the first replicas of the benchmark's
    own population at beta = 1 (the value, all threads) and beta = 5, and at beta = 1 on one
    thread; plus one whole run of the ring configuration (N = 64, R0 = 1000, 51 temperatures, 5
    sweeps)."""
    from oracle import oracle as o

    model, nproc = cpu_info()
    threads = o.num_threads()
    v1, m1, dt1 = oracle_sweep_rate(o, L, n_sweeps, 1.0, target_s, R0)
    v5, m5, dt5 = oracle_sweep_rate(o, L, n_sweeps, 5.0, target_s / 2, R0)
    o.set_num_threads(1)
    try:
        vs, ms, dts = oracle_sweep_rate(o, L, n_sweeps, 1.0, target_s / 4, R0)
    finally:
        o.set_num_threads(threads)
    c1 = oracle_ring_run(o)
    return {"value": v1, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle sweep of the first {m1} replicas of the L={L} population, {n_sweeps} sweeps at "
                      f"beta=1 ({m1 * L ** 3 * n_sweeps:.3e} attempts in {dt1:.1f} s)",
            "beta5": {"value": v5, "cores": threads, "replicas": m5, "seconds": dt5},
            "one_core": {"value": vs, "cores": 1, "replicas": ms, "seconds": dts, "beta": 1.0},
            "ring_full_run": c1, "cpu_model": model, "logical_cpus": nproc}


def oracle_ring_run(o):
    """One whole oracle run of the ring configuration: N = 64, R0 = 1000, 51 temperatures, 5 sweeps."""
    J = o.couplings(1, 64, 1)
    betas = [5.0 * k / 50 for k in range(51)]
    t = time.perf_counter()
    st, rec, _, _ = o.run(1, 64, J, 1, 1000, betas, 5)
    dt = time.perf_counter() - t
    attempts = float(rec[1:, 1].sum()) * 64 * 5
    return {"seconds": dt, "attempts": attempts, "attempts_per_s": attempts / dt, "status": int(st),
            "cores": o.num_threads()}


def oracle_full_runs(args):
    """--oracle-runs: whole oracle runs of the ring (N = 64, R0 = 1000, 51 temperatures, 5 sweeps)
    and of the L = 8 cube (R0 = 5e4, 101 temperatures, 10 sweeps) on all threads; minutes of CPU."""
    from oracle import oracle as o

    model, nproc = cpu_info()
    out = {"cpu_model": model, "logical_cpus": nproc, "threads": o.num_threads(), "ring": oracle_ring_run(o)}
    print(f"ring run: {out['ring']['seconds']:.3f} s; cube L=8 next (about two minutes)", file=sys.stderr, flush=True)
    J = o.couplings(3, 8, 1)
    betas = [5.0 * k / 100 for k in range(101)]
    t = time.perf_counter()
    st, rec, _, _ = o.run(3, 8, J, 1, 50_000, betas, 10)
    dt = time.perf_counter() - t
    attempts = float(rec[1:, 1].sum()) * 512 * 10
    out["cube_L8"] = {"seconds": dt, "attempts": attempts, "attempts_per_s": attempts / dt, "status": int(st)}
    print(json.dumps(out), flush=True)


def issue_ceilings():
    """Live probe of the vector ALU (libpa_calib.so): lane-instructions/s of a few instruction kinds
    and the engine clock the probe ran at."""
    from paper_1006_0252_amd import valu_calibration as vc

    res = vc.measure(kinds=[0, 1, 2, 5], iters=8000, repeats=2)
    return {"clock_ghz": float(np.median([v["clock_hz"] for v in res.values()])) / 1e9,
            "lane_instr_per_s": {k: v["rate"] for k, v in res.items()},
            "lanes_per_clock_per_cu": {k: v["per_cu_per_clock"] for k, v in res.items()}}


def counted_valu(path):
    """VALU instructions per attempt of the sweep per first-look regime, from the committed
    counter summary, or None when the sweep sources changed since it was taken."""
    try:
        with open(path) as f:
            c = json.load(f)
    except (ValueError, OSError):
        return None
    if c.get("source_digest") != sweep_source_digest():
        return None
    return c.get("valu_per_attempt")


def main():
    args = parse()
    if args.oracle_runs:
        oracle_full_runs(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); nothing to do", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1006_0252_amd import pa

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "learned":
        bench_learned(args)
        return
    if args.workload == "bias":
        bench_bias(args)
        return
    if args.workload == "bias_gauss":
        bench_bias(args, chain="gauss")
        return
    if args.workload == "stepped":
        bench_stepped(args)
        return
    if args.workload == "gauss":
        bench_gauss(args)
        return
    if args.workload == "gauss_survey":
        bench_gauss_survey(args)
        return
    if args.workload == "gauss_stepped":
        bench_gauss_stepped(args)
        return
    dev = "cuda:0"
    n_steps = args.n_temps - 1
    if args.warmup + args.steps > n_steps:
        print(f"warmup + steps must not exceed the {n_steps} steps of the schedule", file=sys.stderr)
        sys.exit(2)
    betas = pa.linear_schedule(args.n_temps, 5.0)
    cap = int(np.ceil(args.R0 * 1.25 / 64)) * 64
    run = pa.Run(3, args.L, args.R0, seed=1, disorder_seed=1, n_records=args.n_temps, capacity=cap,
                 layout=args.layout, device=dev)
    run.init()
    sched = pa.Schedule(betas, args.n_sweeps, run.n_bins, device=dev)
    fe = torch.zeros(1, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    N = run.N

    def step(k, ev=None):
        st = sched.step(k)
        run.resample(st)
        if ev is not None:
            ev[0].record(stream)
        run.sweep(st)
        if ev is not None:
            ev[1].record(stream)
        pa.measure([run])
        run.free_energy(fe)

    for k in range(1, args.warmup + 1):
        step(k)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    ks = list(range(args.warmup + 1, args.warmup + args.steps + 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, k in enumerate(ks):
        step(k, events[i])
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    code, flags = run.status()
    if code != pa.PA_OK:
        raise RuntimeError(f"run failed: status {code} flags {flags}")
    rec = run.records()
    R_steps = rec[ks, 4]
    attempts = float(np.sum(R_steps) * N * args.n_sweeps)
    value = attempts / T
    sweep_ms = np.array([a.elapsed_time(b) for a, b in events])
    sweep_s = float(np.mean(sweep_ms)) * 1e-3
    per_launch_attempts = float(np.mean(R_steps)) * N * args.n_sweeps
    achieved = per_launch_attempts * OPS_PER_ATTEMPT / sweep_s
    traffic = sweep_traffic(args.traffic)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"cube_L{args.L}_R{args.R0}_{args.layout}", "L": args.L, "R0": args.R0,
                   "n_temps": args.n_temps, "n_sweeps": args.n_sweeps, "layout": args.layout,
                   "steps_timed": f"k={ks[0]}..{ks[-1]}", "parallelism": "1 GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved / PEAK_LANE_OPS, "traffic": traffic,
                     "kernel": "k_sweep16c (pa_sweep, 10 fused sweeps)", "avg_launch_ms": sweep_s * 1e3,
                     "ops_per_attempt": OPS_PER_ATTEMPT,
                     "peak_basis": "256 CUs x 128 lanes x 2.4 GHz (FP32 vector 157.3 TFLOP/s / 2)",
                     "hbm_frac": (traffic / sweep_s / 8e12) if traffic else None},
        "sweep_attempts_per_s": per_launch_attempts / sweep_s,
        "sweep_by_regime": sweep_by_regime(betas[ks], sweep_ms, R_steps * N * args.n_sweeps),
        "final_minus_betaF": float(rec[ks[-1], 2]),
    }
    valu = counted_valu(COUNTERS)
    for r, v in out["sweep_by_regime"].items():
        v["frac"] = v["attempts_per_s"] * OPS_PER_ATTEMPT / PEAK_LANE_OPS
        if valu and r in valu:
            v["valu_per_attempt"] = valu[r]
            v["valu_lane_instr_per_s"] = v["attempts_per_s"] * valu[r]
    if not args.no_probe:
        probe = issue_ceilings()
        mix = probe["lane_instr_per_s"]["mad_u64+bitop3"]
        for v in out["sweep_by_regime"].values():
            if "valu_lane_instr_per_s" in v:
                v["issue_frac_of_philox_mix"] = v["valu_lane_instr_per_s"] / mix
        out["roofline"]["probe"] = probe
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.L, args.R0, args.n_sweeps, args.cpu_seconds)
    if not args.no_learned:
        del run, sched
        torch.cuda.empty_cache()
        lf = learned_vs_fixed(args.ensemble)
        out["learned_vs_fixed"] = {
            "workload": lf["config"]["workload"], "runs_per_schedule": args.ensemble,
            "fixed_over_learned_time_to_target": lf["value"],
            "best_learned": lf["best_learned"], "best_fixed": lf["best_fixed"],
            "time_to_target_s": {**{f"learned_rho{k}": v["time_to_target_s"] for k, v in lf["learned"].items()},
                                 **{f"fixed_nT{k}": v["time_to_target_s"] for k, v in lf["fixed"].items()}},
            "learned_minus_reference_sigma": lf["learned_minus_reference_sigma"],
            "training_seconds": lf["training"]["train_seconds"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
