"""Bias of weighted and unweighted averages on the periodic chain (Sec. IV, the 1D measurements).

For each disorder realization, M independent runs anneal the ring (one batch per realization):
* the ±J ring N = 64, R0 = 1000, 51 temperatures, 5 sweeps (the default); or
* the paper's own chain: Gaussian couplings, N = 256, R = 1000, 100 temperatures (19 steps evenly
  spaced in beta up to 0.5, then 80 evenly spaced in T down to T = 0.2), 50 sweeps
  (`paper_schedule_1d`, `run(..., chain="gauss")`).  At β = 5 the run free energies -βF̃_r and
energies E_r feed:
* the weighted energy Ē and free energy -βF̄ of the whole ensemble (eqs. weight, omega, bestf), and
  the plain means, each with a bootstrap error (Sec. III; pa_bootstrap_dev);
* the block bias μ_k: the M runs are cut into B = M/k blocks of k, each block gives a weighted
  Ē^b, and μ_k is the mean over realizations of (mean over blocks of Ē^b) - E_exact (Sec. IV).
  The plain mean is k = 1.

The exact values come from the closed form of the periodic chain (exact.py) with the couplings the
library drew.  All averaging over runs runs on the device (pa_weighted_average_dev,
pa_bootstrap_dev); the host only forms the final means over realizations.
"""
from __future__ import annotations

import time

import numpy as np

from . import exact, pa

REC = {n: i for i, n in enumerate(pa.RECORD_FIELDS)}


def paper_schedule_1d():
    """beta = 0, 19 steps evenly spaced in beta up to 0.5, then 80 evenly spaced in T from T = 2
    to T = 0.2: 100 temperatures (Sec. IV)."""
    b1 = np.linspace(0.0, 0.5, 20)
    T2 = np.linspace(2.0, 0.2, 81)[1:]
    return np.concatenate([b1, 1.0 / T2])


CHAINS = {
    "pm1": dict(N=64, R0=1000, n_sweeps=5, couplings="pm1", betas=lambda: pa.linear_schedule(51)),
    "gauss": dict(N=256, R0=1000, n_sweeps=50, couplings="gauss", betas=paper_schedule_1d),
}


def ring_ensemble(disorder_seed, M, R0=1000, n_temps=51, n_sweeps=5, device="cuda", N=64, couplings="pm1",
                  betas=None, graph=True):
    """M runs of one ring realization; returns (-beta F~ [M][n_temps], E mean [M][n_temps], betas,
    couplings, seconds, attempts).  graph: the schedule is captured once as one HIP graph and the
    seconds are those of its replay (the same kernels, hence the same sample, as stepping eagerly)."""
    import torch

    betas = pa.linear_schedule(n_temps) if betas is None else np.asarray(betas, np.float64)
    n_temps = len(betas)
    specs = [dict(dim=1, L=N, R0=R0, seed=100_000 * disorder_seed + r + 1, disorder_seed=disorder_seed,
                  couplings=couplings) for r in range(M)]
    batch = pa.Batch(specs, n_temps, layout="u8", device=device)
    batch.init()
    sched = pa.Schedule(betas, n_sweeps, batch.runs[0].n_bins, device=device)
    g = batch.capture(sched, range(1, n_temps)) if graph else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if graph:
        g.launch()
    else:
        for k in range(1, n_temps):
            batch.step(sched, k)
    batch.stream.synchronize()
    T = time.perf_counter() - t0
    code, flags = batch.status()
    if code != pa.PA_OK:
        raise RuntimeError(f"ring ensemble failed: status {code}")
    rec = batch.records()
    attempts = float(rec[:, 1:, REC["R"]].sum()) * N * n_sweeps
    return rec[:, :, REC["minus_betaF"]].copy(), rec[:, :, REC["E_mean"]].copy(), sched.betas, \
        batch.runs[0].couplings(), T, attempts


def device_weighted(x, A, n_sets, M, device="cuda"):
    """pa_weighted_average_dev over n_sets consecutive sets of M runs: [n_sets][n_obs + 3]."""
    import torch

    n_obs = A.shape[1]
    xd = torch.tensor(np.ascontiguousarray(x, np.float64), device=device)
    Ad = torch.tensor(np.ascontiguousarray(A, np.float64), device=device)
    out = torch.zeros((n_sets, n_obs + 3), dtype=torch.float64, device=device)
    pa.check(pa.lib().pa_weighted_average_dev(n_sets, M, xd.data_ptr(), None, Ad.data_ptr(), n_obs, out.data_ptr(),
                                              torch.cuda.current_stream(device).cuda_stream), "pa_weighted_average_dev")
    return out.cpu().numpy()


def device_bootstrap(x, A, idx, device="cuda"):
    """pa_bootstrap_dev for one set: (replicates [n_boot][n_obs + 3], errors [n_obs + 3])."""
    import torch

    M, n_obs = A.shape
    n_boot = idx.shape[0]
    xd = torch.tensor(np.ascontiguousarray(x, np.float64), device=device)
    Ad = torch.tensor(np.ascontiguousarray(A, np.float64), device=device)
    idd = torch.tensor(np.ascontiguousarray(idx, np.int32), device=device)
    rep = torch.zeros((n_boot, n_obs + 3), dtype=torch.float64, device=device)
    err = torch.zeros(n_obs + 3, dtype=torch.float64, device=device)
    pa.check(pa.lib().pa_bootstrap_dev(1, M, xd.data_ptr(), None, Ad.data_ptr(), n_obs, n_boot, idd.data_ptr(),
                                       rep.data_ptr(), err.data_ptr(), torch.cuda.current_stream(device).cuda_stream),
             "pa_bootstrap_dev")
    return rep.cpu().numpy(), err.cpu().numpy()


def run(n_real=18, M=200, n_boot=100, betas=(1.0, 2.0, 5.0), boot_seed=11, device="cuda", log=None, chain="pm1"):
    """Per temperature in betas (the nearest of the schedule): per-realization weighted and plain
    estimates with bootstrap errors, their means over realizations against the exact chain, and mu_k
    for every divisor k of M."""
    cfg = CHAINS[chain]
    ks = [k for k in range(1, M + 1) if M % k == 0]
    g = np.random.default_rng(boot_seed)
    idx = g.integers(0, M, (n_boot, M))
    per = {b: [] for b in betas}
    block = {b: {k: [] for k in ks} for b in betas}
    seconds, attempts = 0.0, 0.0
    zero = np.zeros(M)
    for d in range(1, n_real + 1):
        X, EE, sb, J, T, att = ring_ensemble(d, M, R0=cfg["R0"], n_sweeps=cfg["n_sweeps"], device=device, N=cfg["N"],
                                             couplings=cfg["couplings"], betas=cfg["betas"]())
        seconds += T
        attempts += att
        for beta in betas:
            kk = int(np.argmin(np.abs(sb - beta)))
            x, E = X[:, kk], EE[:, kk]
            E_ex, F_ex = exact.ring_energy(J, sb[kk]), exact.ring_lnZ(J, sb[kk])
            w = device_weighted(x, E[:, None], 1, M, device)[0]
            _, err = device_bootstrap(x, E[:, None], idx, device)
            # plain averages: the same device averages with equal free energies
            u = device_weighted(zero, E[:, None], 1, M, device)[0]
            _, err_u = device_bootstrap(zero, E[:, None], idx, device)
            per[beta].append(dict(beta_grid=float(sb[kk]), E_exact=E_ex, F_exact=F_ex, E_w=w[0], E_w_err=err[0], F_w=w[1], F_w_err=err[1],
                                  var=w[2], E_u=u[0], E_u_err=err_u[0], F_u=w[3], F_u_err=err[3]))
            for k in ks:
                bl = device_weighted(x, E[:, None], M // k, k, device)[:, 0]
                block[beta][k].append((bl.mean() - E_ex, bl.std(ddof=1) / np.sqrt(len(bl)) if len(bl) > 1 else err[0]))
            if log:
                p = per[beta][-1]
                log(f"realization {d} beta {sb[kk]:.1f}: Var {p['var']:.3f}  E weighted {p['E_w'] - E_ex:+.5f}"
                    f"+-{p['E_w_err']:.5f} plain {p['E_u'] - E_ex:+.5f}  -bF weighted {p['F_w'] - F_ex:+.4f}"
                    f"+-{p['F_w_err']:.4f} plain {p['F_u'] - F_ex:+.4f}")

    def agg(rows, key, ref, errkey):
        dev = np.array([p[key] - p[ref] for p in rows])
        e = np.array([p[errkey] for p in rows])
        return float(dev.mean()), float(np.sqrt((e ** 2).sum()) / len(rows))

    res = {}
    for beta in betas:
        rows = per[beta]
        mu = {k: (float(np.mean([b[0] for b in block[beta][k]])),
                  float(np.sqrt(sum(b[1] ** 2 for b in block[beta][k])) / n_real)) for k in ks}
        res[beta] = dict(beta_grid=rows[0]["beta_grid"], per_realization=rows, energy_bias_weighted=agg(rows, "E_w", "E_exact", "E_w_err"),
                         energy_bias_plain=agg(rows, "E_u", "E_exact", "E_u_err"),
                         free_energy_bias_weighted=agg(rows, "F_w", "F_exact", "F_w_err"),
                         free_energy_bias_plain=agg(rows, "F_u", "F_exact", "F_u_err"),
                         mean_var=float(np.mean([p["var"] for p in rows])), mu_k=mu)
    return dict(by_beta=res, anneal_seconds=seconds, attempts=attempts)
