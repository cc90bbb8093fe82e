"""Plain device-to-device copy of a known size.

Run under rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) to learn how the HBM byte counters
read for a kernel whose traffic is known exactly (each copy reads and writes --mib MiB);
the ratio scales the same counters taken on the library's kernels.
"""
from __future__ import annotations

import argparse
import json


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--mib", type=int, default=1024)
    p.add_argument("--reps", type=int, default=3)
    a = p.parse_args()
    import torch

    n = a.mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "reps": a.reps}), flush=True)


if __name__ == "__main__":
    main()
