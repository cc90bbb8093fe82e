"""Ensembles of independent runs and their weighted averages (Sec. III; Sec. IV eq. omegaprime).

run_batched(): all runs of a batch annealed together (one launch per kernel, persistent
sweep, the whole schedule captured as one HIP graph), then per realisation the run weights
R^(r) exp(-beta F~_r) (runs with unequal target sizes, Sec. III) give the weighted energy
and free energy, and the pair weights R^(1) R^(2) exp(-beta (F~^(1) + F~^(2))) of the overlap
pairs give the weighted <q^2>, <q^4>, Gamma and the Binder ratio, computed on the device by
pa_weighted_average_dev and pa_overlap_average_dev.
"""
from __future__ import annotations

import time

import numpy as np

from . import autotune, pa
from .workloads import linear_betas

REC = {n: i for i, n in enumerate(pa.RECORD_FIELDS)}


def weighted_by_realization(records, specs, k, device="cuda"):
    """Weighted averages at temperature index k for every realisation of a batch."""
    import torch

    reals = sorted({sp["realization"] for sp in specs})
    by_real = {d: [i for i, sp in enumerate(specs) if sp["realization"] == d] for d in reals}
    M = len(by_real[reals[0]])
    assert all(len(v) == M for v in by_real.values()) and M % 2 == 0
    idx = np.array([by_real[d] for d in reals])                       # [n_real][M]
    x = records[idx, k, REC["minus_betaF"]]
    R = np.array([[specs[i]["R0"] for i in row] for row in idx], dtype=np.float64)
    E = records[idx, k, REC["E_mean"]][..., None]
    # overlap pairs (0,1), (2,3), ...: the overlap observables sit in the first run of each pair
    Q = np.stack([records[idx[:, 0::2], k, REC["q2"]], records[idx[:, 0::2], k, REC["q4"]],
                  records[idx[:, 0::2], k, REC["gamma"]]], axis=-1)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)  # noqa: E731
    n_real = len(reals)
    out_e = torch.zeros((n_real, 1 + 3), dtype=torch.float64, device=device)
    out_q = torch.zeros((n_real, 4), dtype=torch.float64, device=device)
    s = torch.cuda.current_stream(device).cuda_stream
    xd, Rd, Ed, Qd = dev(x), dev(R), dev(E), dev(Q)
    pa.check(pa.lib().pa_weighted_average_dev(n_real, M, xd.data_ptr(), Rd.data_ptr(), Ed.data_ptr(), 1,
                                              out_e.data_ptr(), s), "pa_weighted_average_dev")
    pa.check(pa.lib().pa_overlap_average_dev(n_real, M // 2, xd.data_ptr(), Rd.data_ptr(), Qd.data_ptr(),
                                             out_q.data_ptr(), s), "pa_overlap_average_dev")
    oe = out_e.cpu().numpy()
    oq = out_q.cpu().numpy()
    return dict(realizations=reals, E_bar=oe[:, 0], minus_betaF_bar=oe[:, 1], var_betaF=oe[:, 2],
                mean_minus_betaF=oe[:, 3], q2=oq[:, 0], q4=oq[:, 1], gamma=oq[:, 2], binder=oq[:, 3],
                L=np.array([specs[i[0]]["L"] for i in idx]))


def run_batched(specs, n_temps, n_sweeps, layout="bits64", device="cuda", tune=True, graph=True, verbose=False):
    import torch

    betas = linear_betas(n_temps)
    batch = pa.Batch(specs, n_temps, layout=layout, device=device)
    batch.init()
    sched = pa.Schedule(betas, n_sweeps, max(r.n_bins for r in batch.runs), device=device)
    torch.cuda.synchronize()
    tuned = None
    if tune:
        # one step in each first-look regime of the schedule (beta near 0, about 2 and about 4)
        ks = sorted({1, min(n_temps - 1, max(1, round(0.4 * (n_temps - 1)))), n_temps - 1 - (n_temps - 1) // 5})
        tuned, timings = autotune.tune_batch(batch, [sched.step(k) for k in ks], verbose=verbose)
    ks = range(1, n_temps)
    if graph:
        g = batch.capture(sched, ks, pairs=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.launch()
        batch.stream.synchronize()
        T = time.perf_counter() - t0
    else:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in ks:
            batch.step(sched, k, pairs=True)
        batch.stream.synchronize()
        T = time.perf_counter() - t0
    code, flags = batch.status()
    if code != pa.PA_OK:
        raise RuntimeError(f"batched run failed: status {code}, runs {np.nonzero(flags)[0].tolist()}")
    rec = batch.records()
    N = np.array([sp["L"] ** 3 for sp in specs], dtype=np.float64)
    attempts = float(np.sum(rec[:, 1:, REC["R"]] * N[:, None]) * n_sweeps)
    res = weighted_by_realization(rec, specs, n_temps - 1, device=device)
    return dict(seconds=T, attempts=attempts, attempts_per_s=attempts / T, tuned=tuned, records=rec,
                weighted=res, graph=graph)
