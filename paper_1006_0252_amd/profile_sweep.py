"""One sweep launch (10 sweeps) per first-look regime on the L = 16 cube, R0 = 1e6, bit-packed:
beta = 0.5, 2 and 4.  A fixed, short workload for hardware-counter passes (rocprofv3 --pmc)."""
from __future__ import annotations

import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    import numpy as np
    import torch

    from paper_1006_0252_amd import pa

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
