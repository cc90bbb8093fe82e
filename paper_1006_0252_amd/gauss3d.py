"""The 3D Gaussian spin glass ensemble of Sec. IV on one GPU.

L = 8 (512 spins), Gaussian couplings of one realization, target population R = 2000, 100
temperatures evenly spaced in T from T = 2 down to T = 0.2 (beta 0.5 -> 5), theta = 100
Metropolis sweeps at every temperature (the random start is equilibrated by the sweeps at T = 2,
which is far above the transition), M (even) independent runs in pairs (0,1), (2,3), ... for the
overlap.  The highest temperature is finite, so the free energy is known relative to T = 2 only:
the runs' sum of ln Q over the 99 steps, -beta_0 F~ + beta_K F(T = 2), carries all of Var(beta F~)
and gives the same weights.  All M runs are one batch: each step is one launch per kernel
over all runs (the sweep: one table kernel and one tabled sweep kernel).

At the lowest temperature the runs give -beta F~_r, the energy E_r and, per pair, Gamma = P(|q| < 0.2);
the weighted averages are eqs. weight, omega and bestf over runs and eq. omegaprime over pairs,
with Var(beta F~) as the convergence diagnostic.
"""
from __future__ import annotations

import time

import numpy as np

from . import pa

REC = {n: i for i, n in enumerate(pa.RECORD_FIELDS)}


def schedule(n_temps=100, T_hi=2.0, T_lo=0.2):
    """n_temps inverse temperatures evenly spaced in T from T_hi to T_lo."""
    return 1.0 / np.linspace(T_hi, T_lo, n_temps)


def run(M=126, R=2000, L=8, n_temps=100, n_sweeps=100, disorder_seed=1, seed0=1, device="cuda:0", log=None,
        R_targets=None):
    """M runs of one realization; R_targets (per temperature, optional) makes the population size
    follow the temperature (Sec. IV: R_beta), the random start then has R_targets[0] replicas."""
    import torch

    betas = schedule(n_temps)
    nT = len(betas)
    Rt = None if R_targets is None else np.asarray(R_targets, np.float64)
    R0 = R if Rt is None else int(Rt[0])
    cf = 1.25 if Rt is None else 1.25 * float(Rt.max()) / R0
    specs = [dict(dim=3, L=L, R0=R0, seed=seed0 + i, disorder_seed=disorder_seed, couplings="gauss") for i in range(M)]
    batch = pa.Batch(specs, nT, layout="u8", device=device, capacity_factor=cf)
    batch.init()
    sched = pa.Schedule(betas, n_sweeps, batch.runs[0].n_bins, device=device, R_targets=Rt)
    s = batch.stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(1, nT)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    ev0[0].record(s)
    batch.sweep(sched.start_sweeps())
    ev0[1].record(s)
    for k in range(1, nT):
        st = sched.step(k)
        batch.resample(st)
        ev[k - 1][0].record(s)
        batch.sweep(st)
        ev[k - 1][1].record(s)
        batch.measure(pairs=True)
        if log and k % 20 == 0:
            log(f"step {k}/{nT - 1} queued")
    s.synchronize()
    wall = time.perf_counter() - t0
    code, flags = batch.status()
    if code != pa.PA_OK:
        raise RuntimeError(f"gaussian ensemble failed: status {code}, runs {np.nonzero(flags)[0].tolist()}")
    sweep_ms = np.array([ev0[0].elapsed_time(ev0[1])] + [a.elapsed_time(b) for a, b in ev])
    rec = batch.records()                                        # [M][nT][13]
    R_per_step = np.concatenate([[float(R0 * M)], rec[:, 1:, REC["R"]].sum(axis=0)])  # replicas swept per block
    attempts = float(R_per_step.sum()) * L ** 3 * n_sweeps
    x = rec[:, 1:, REC["lnQ"]].sum(axis=1)                      # -beta_0 F~ relative to T = 2
    E = rec[:, -1, REC["E_mean"]]
    w = pa.weighted_average(x, E[:, None])
    xp = x[0::2] + x[1::2]
    gam = rec[0::2, -1, REC["gamma"]]
    wp = pa.weighted_average(xp, gam[:, None])
    # Var(beta F~(beta_k)) over the runs at every temperature (relative to T = 2, as above)
    xk = np.cumsum(rec[:, 1:, REC["lnQ"]], axis=1)
    var_profile = np.array([pa.weighted_average(xk[:, k])["var"] for k in range(nT - 1)])
    return dict(betas=betas, n_steps=nT - 1, wall_seconds=wall, var_profile=var_profile, sweep_ms=sweep_ms, attempts=attempts,
                attempts_per_sweep_step=R_per_step * L ** 3 * n_sweeps,
                minus_betaF_bar=w["minus_betaF_bar"], var_betaF=w["var"], mean_minus_betaF=w["mean"],
                E_bar=float(w["A_bar"][0]), gamma_bar=float(wp["A_bar"][0]), R_final=rec[:, -1, REC["R"]])


def survey(n_real=25, M=100, R=2000, R_big=10000, M_worst=126, device="cuda:0", log=None):
    """Sec. IV's 3D study: per realization (disorder seeds 1..n_real), M runs at R give Var(beta F~),
    the weighted energy and the pair-weighted Gamma; the realization with the largest Var is rerun
    with M_worst runs at R and at R_big (the paper: R = 2000 and 10000)."""
    rows = []
    for d in range(1, n_real + 1):
        r = run(M=M, R=R, disorder_seed=d, seed0=1000 * d + 1, device=device)
        rows.append(dict(disorder_seed=d, var_betaF=r["var_betaF"], gamma_bar=r["gamma_bar"], E_bar=r["E_bar"],
                         gap=r["minus_betaF_bar"] - r["mean_minus_betaF"], seconds=r["wall_seconds"],
                         attempts=r["attempts"]))
        if log:
            log(f"realization {d}: Var {r['var_betaF']:.4f} Gamma {r['gamma_bar']:.4f} E {r['E_bar']:.3f}")
    worst = max(rows, key=lambda x: x["var_betaF"])["disorder_seed"]
    rw = {}
    for RR in (R, R_big):
        r = run(M=M_worst, R=RR, disorder_seed=worst, seed0=10 ** 6 + RR, device=device)
        rw[RR] = dict(var_betaF=r["var_betaF"], gamma_bar=r["gamma_bar"], E_bar=r["E_bar"],
                      gap=r["minus_betaF_bar"] - r["mean_minus_betaF"], seconds=r["wall_seconds"], attempts=r["attempts"])
        if log:
            log(f"worst realization {worst}, R={RR}: Var {r['var_betaF']:.4f} Gamma {r['gamma_bar']:.4f} E {r['E_bar']:.3f}")
    return dict(rows=rows, worst=worst, worst_runs=rw)
