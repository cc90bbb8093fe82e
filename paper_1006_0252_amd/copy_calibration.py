"""Plain device-to-device copy of a known size.

Run under rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) to learn how the HBM byte counters
read for a kernel whose traffic is known exactly (each copy reads and writes --mib MiB);
the ratio scales the same counters taken on the library's kernels.  Run alone, it also times
--timed further copies with HIP events: the achieved copy bandwidth is the measured HBM peak
that the library's HBM-bound kernels are compared with.
"""
from __future__ import annotations

import argparse
import json


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--mib", type=int, default=1024)
    p.add_argument("--reps", type=int, default=3)
    p.add_argument("--timed", type=int, default=20)
    a = p.parse_args()
    import torch

    n = a.mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    out = {"copy_bytes_read": n, "copy_bytes_written": n, "reps": a.reps}
    if a.timed > 0:
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(a.timed):
            dst.copy_(src)
        t1.record()
        torch.cuda.synchronize()
        s = t0.elapsed_time(t1) / 1e3 / a.timed
        out.update(timed=a.timed, seconds_per_copy=s, bytes_per_s=2 * n / s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
