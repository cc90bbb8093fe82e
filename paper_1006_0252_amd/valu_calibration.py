"""Vector-ALU issue rate and engine clock of the GPU, measured live (libpa_calib.so).

For each instruction kind a probe kernel runs a known number of VALU instructions per wave
(16 independent chains, 8 waves per SIMD) and is timed with HIP events on its stream; wave 0 of
every block also reads the shader clock counter and the constant-rate wall clock around its loop.
That gives, per kind:
  rate   = lane-instructions per second (waves x 64 lanes x instructions / event time),
  clock  = shader clock cycles / wall-clock seconds over the loop (median over blocks),
  per_cu = rate / (clock x compute units): lane-instructions per cycle per CU (64 = one wave64
           instruction every 4 cycles on each of the 4 SIMDs).
The ALU roofline of the sweep takes its peak from the measured clock: 64 lanes x CUs x clock.

Run as a module to print the table: python -m paper_1006_0252_amd.valu_calibration
"""
from __future__ import annotations

import ctypes
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpa_calib.so")
KINDS = ["v_xor_b32", "v_bitop3_b32", "v_mad_u64_u32", "v_pk_sub_u16", "v_pk_min_u16", "mad_u64+bitop3"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not built; run python -m paper_1006_0252_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.pa_calib_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        L.pa_calib_valu.restype = ctypes.c_int
        L.pa_calib_instructions_per_iteration.argtypes = [ctypes.c_int]
        L.pa_calib_wall_clock_khz.argtypes = [ctypes.POINTER(ctypes.c_int)]
        _lib = L
    return _lib


def measure(kinds=None, iters=20000, blocks_per_cu=8, repeats=3, device="cuda:0"):
    """Returns a dict per kind: rate (lane-instr/s), clock_hz, per_cu_per_clock, ms."""
    import numpy as np
    import torch

    props = torch.cuda.get_device_properties(device)
    n_cu = props.multi_processor_count
    khz = ctypes.c_int(0)
    if lib().pa_calib_wall_clock_khz(ctypes.byref(khz)) != 0 or khz.value <= 0:
        raise RuntimeError("wall clock rate unavailable")
    n_blocks = n_cu * blocks_per_cu
    clocks = torch.zeros(n_blocks * 4, dtype=torch.int64, device=device)
    sink = torch.zeros(n_blocks * 256, dtype=torch.int32, device=device)
    stream = torch.cuda.current_stream(device)
    out = {}
    for kind in (range(len(KINDS)) if kinds is None else kinds):
        per_iter = lib().pa_calib_instructions_per_iteration(kind)
        best = None
        for rep in range(repeats + 1):  # the first launch warms the code object up
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            rc = lib().pa_calib_valu(kind, n_blocks, iters, clocks.data_ptr(), sink.data_ptr(), stream.cuda_stream)
            b.record(stream)
            if rc != 0:
                raise RuntimeError(f"pa_calib_valu failed ({rc})")
            b.synchronize()
            ms = a.elapsed_time(b)
            if rep > 0 and (best is None or ms < best[0]):
                c = clocks.view(n_blocks, 4).cpu().numpy().astype(np.float64)
                best = (ms, c)
        ms, c = best
        cycles = c[:, 1] - c[:, 0]
        wall = (c[:, 3] - c[:, 2]) / (khz.value * 1e3)
        clock = float(np.median(cycles / wall))
        lane_instr = float(n_blocks) * 256 * per_iter * iters
        rate = lane_instr / (ms * 1e-3)
        out[KINDS[kind]] = dict(rate=rate, clock_hz=clock, per_cu_per_clock=rate / (clock * n_cu), ms=ms,
                                n_cu=n_cu, loop_cycles_median=float(np.median(cycles)))
    return out


def main():
    import torch

    assert torch.cuda.is_available(), "needs the GPU"
    res = measure()
    for k, v in res.items():
        print(f"{k:16s} {v['rate'] / 1e12:7.2f} T lane-instr/s  clock {v['clock_hz'] / 1e9:.3f} GHz  "
              f"{v['per_cu_per_clock']:6.2f} lanes/clk/CU  ({v['ms']:.2f} ms)", flush=True)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
