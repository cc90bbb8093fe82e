"""Fixed, short workloads for hardware-counter passes (rocprofv3 --pmc).

default: one sweep launch (10 sweeps) per first-look regime on the L = 16 cube, R0 = 1e6,
bit-packed: beta = 0.5, 2 and 4.
gauss: the Gaussian ensemble's sweep, 126 runs of L = 8 at R = 2000, one launch of 100 sweeps at
T = 2 and one at T = 0.5 (table kernel and tabled sweep).
batched: the batched configuration's 256 runs (L = 6, 8, 10) at their initial sizes, one batched
sweep of 10 sweeps at beta = 0.5, 2 and 4 (one launch per lattice size each); prints the attempts
of one launch per lattice size."""
from __future__ import annotations

import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def gauss():
    import torch

    from paper_1006_0252_amd import pa

    specs = [dict(dim=3, L=8, R0=2000, seed=1 + i, disorder_seed=1, couplings="gauss") for i in range(126)]
    batch = pa.Batch(specs, 3, layout="u8", device="cuda:0").init()
    sched = pa.Schedule([0.5, 2.0], 100, batch.runs[0].n_bins, device="cuda:0")
    batch.sweep(sched.start_sweeps())
    batch.sweep(sched.step(1))
    batch.stream.synchronize()
    torch.cuda.synchronize()
    print("ok", flush=True)


def batched():
    import torch

    from paper_1006_0252_amd import pa, workloads

    specs = workloads.batched_specs()
    batch = pa.Batch(specs, 4, layout="bits64", device="cuda:0").init()
    sched = pa.Schedule([0.0, 0.5, 2.0, 4.0], workloads.C3_SWEEPS, batch.runs[0].n_bins, device="cuda:0")
    for k in (1, 2, 3):
        batch.sweep(sched.step(k))
    batch.stream.synchronize()
    torch.cuda.synchronize()
    att = {}
    for sp in specs:
        att[sp["L"]] = att.get(sp["L"], 0) + sp["R0"] * sp["L"] ** 3 * workloads.C3_SWEEPS
    print("attempts per launch by L:", {L: att[L] for L in sorted(att)}, flush=True)


def main():
    import numpy as np
    import torch

    from paper_1006_0252_amd import pa

    if len(sys.argv) > 1 and sys.argv[1] == "gauss":
        gauss()
        return
    if len(sys.argv) > 1 and sys.argv[1] == "batched":
        batched()
        return

    L, R0 = 16, 1_000_000
    run = pa.Run(3, L, R0, 1, 1, 4, capacity=int(np.ceil(R0 * 1.25 / 64)) * 64, layout="bits64", device="cuda:0")
    run.init()
    sched = pa.Schedule([0.0, 0.5, 2.0, 4.0], 10, run.n_bins, device="cuda:0")
    for k in (1, 2, 3):
        run.sweep(sched.step(k))
    torch.cuda.synchronize()
    print("ok", flush=True)


if __name__ == "__main__":
    main()
