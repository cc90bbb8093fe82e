"""Temperature-dependent population size R_beta and the profile Var(beta F~(beta)) (Sec. IV).

-beta F~(beta) is a sum of one ln Q per step (eq. sumQ), so its variance over independent runs
grows towards low temperature; where it grows fast, more replicas pay off.  The harness:
1. ranks disorder seeds 1..n by Var(beta F~) at beta = 5 (L = 8 cube, constant R, a short
   ensemble per realization) and takes the worst and the median;
2. on each, measures the whole profile Var(beta F~(beta_k)) for
   a. constant R_beta = R;
   b. R_beta = R_lo for beta < beta_c and 3 R_lo beyond, with R_lo chosen so that the total
      work sum_k R_beta_k N N_S equals that of (a), for each beta_c given;
   c. (optionally) learned schedules at constant R (learned.py), compared by Var x work.
The per-step target sizes enter through pa_step.R_target (the resampling of Sec. II with
R_beta' / R~_beta in the Poisson means); every ensemble is one batch, the schedule one graph.
"""
from __future__ import annotations

import time

import numpy as np

from . import pa

REC = {n: i for i, n in enumerate(pa.RECORD_FIELDS)}


def ensemble(betas, R_targets, M, L, disorder_seed, n_sweeps, seed0=1, R_init=None, device="cuda"):
    """M runs on one schedule with per-temperature target sizes (R_targets[k], k >= 1).  Returns the
    records [M][n_temps][13], wall time and spin-flip attempts."""
    import torch

    R_targets = np.asarray(R_targets, np.float64)
    R0 = int(R_init if R_init is not None else R_targets[1])
    cap_factor = 1.25 * float(np.max(R_targets[1:])) / R0
    specs = [dict(dim=3, L=L, R0=R0, seed=seed0 + i, disorder_seed=disorder_seed) for i in range(M)]
    nT = len(betas)
    batch = pa.Batch(specs, nT, layout="bits64", device=device, capacity_factor=cap_factor)
    batch.init()
    sched = pa.Schedule(betas, n_sweeps, batch.runs[0].n_bins, device=device, R_targets=R_targets)
    g = batch.capture(sched, range(1, nT))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.launch()
    batch.stream.synchronize()
    T = time.perf_counter() - t0
    code, flags = batch.status()
    if code != pa.PA_OK:
        raise RuntimeError(f"ensemble failed: status {code}, runs {np.nonzero(flags)[0].tolist()}")
    rec = batch.records()
    attempts = float(rec[:, 1:, REC["R"]].sum()) * L ** 3 * n_sweeps
    return rec, T, attempts


def var_profile(rec, device="cuda"):
    """Var(beta F~) over runs at every temperature (pa_weighted_average_dev, one set per
    temperature) and the weighted -beta F_bar."""
    import torch

    x = np.ascontiguousarray(rec[:, :, REC["minus_betaF"]].T)      # [n_temps][M]
    nT, M = x.shape
    xd = torch.tensor(x, dtype=torch.float64, device=device)
    out = torch.zeros((nT, 3), dtype=torch.float64, device=device)
    pa.check(pa.lib().pa_weighted_average_dev(nT, M, xd.data_ptr(), None, None, 0, out.data_ptr(),
                                              torch.cuda.current_stream(device).cuda_stream), "pa_weighted_average_dev")
    o = out.cpu().numpy()
    return o[:, 1], o[:, 0]      # Var, -beta F_bar


def worst_realization(n_real=25, M=50, R=2000, L=8, n_temps=101, n_sweeps=10, device="cuda"):
    betas = pa.linear_schedule(n_temps)
    Rt = np.full(n_temps, float(R))
    v = []
    for d in range(1, n_real + 1):
        rec, _, _ = ensemble(betas, Rt, M, L, d, n_sweeps, seed0=10_000, device=device)
        v.append(var_profile(rec, device)[0][-1])
    order = np.argsort(v)[::-1]
    return int(order[0]) + 1, v


def equal_work_step(betas, R, beta_c, ratio=3.0):
    """R_lo for beta < beta_c and ratio R_lo beyond, with sum over steps k >= 1 equal to R per step."""
    b = np.asarray(betas)[1:]
    f = float(np.mean(b < beta_c))
    R_lo = R / (f + ratio * (1.0 - f))
    Rt = np.where(np.asarray(betas) < beta_c, R_lo, ratio * R_lo)
    return np.round(Rt), R_lo


def run(M=200, R=2000, L=8, n_temps=101, n_sweeps=10, beta_cs=(0.9, 2.0), n_real=25, learned_nets=None,
        device="cuda", log=None):
    """Profiles on the worst and the median realization (by Var at beta = 5): constant R, R_beta
    stepped x3 at each beta_c (equal work), and learned schedules at constant R."""
    t0 = time.perf_counter()
    _, v_all = worst_realization(n_real=n_real, R=R, L=L, n_temps=n_temps, n_sweeps=n_sweeps, device=device)
    order = np.argsort(v_all)
    picks = {"worst": int(order[-1]) + 1, "median": int(order[len(order) // 2]) + 1}
    if log:
        log(f"realizations by Var at beta=5 (M=50): worst seed {picks['worst']} ({max(v_all):.3f}), "
            f"median seed {picks['median']} ({np.median(v_all):.3f})")
    betas = pa.linear_schedule(n_temps)
    out = dict(picks=picks, var_by_realization=v_all, select_seconds=time.perf_counter() - t0, profiles={})
    for which, seed in picks.items():
        scheds = [("constant", betas, np.full(n_temps, float(R)))]
        for bc in beta_cs:
            scheds.append((f"stepped_x3_at_{bc}", betas, equal_work_step(betas, R, bc)[0]))
        if learned_nets:
            from . import learned

            for rs, net in learned_nets.items():
                bl, _ = learned.pilot_schedule(net, L, R, seed=10 ** 6, disorder_seed=seed, n_sweeps=n_sweeps,
                                               device=device)
                scheds.append((f"learned_rho{rs}", bl, np.full(len(bl), float(R))))
        prof = {}
        for name, bs, Rt in scheds:
            rec, T, att = ensemble(bs, Rt, M, L, seed, n_sweeps, seed0=1, R_init=Rt[1], device=device)
            var, fbar = var_profile(rec, device)
            prof[name] = dict(betas=list(map(float, bs)), R_targets=list(map(float, Rt)), var=var.tolist(),
                              minus_betaF_bar=fbar.tolist(), seconds=T, attempts=att)
            if log:
                log(f"{which} seed {seed} {name}: {len(bs)} temperatures, Var(beta=5) {var[-1]:.4f}, "
                    f"-bF_bar {fbar[-1]:.3f}, attempts {att:.3g}")
        out["profiles"][which] = prof
    return out
