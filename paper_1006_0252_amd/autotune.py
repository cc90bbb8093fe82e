"""Launch-schedule autotuner: times candidate sweep schedules on the real run mix and keeps
the fastest, after checking that every candidate produces the identical sample.

Candidates for a batch (runs with consecutive device states): persistent blocks per compute
unit and work order (runs as given / larger lattices first).  Candidates for a single run:
lanes per replica and waves per block.  Each candidate sweeps the same saved population
(restored before every trial) so timings and results are comparable; results are compared
bit for bit (spins and energies of every run).
"""
from __future__ import annotations


import numpy as np

from . import pa

# (blocks per CU, group order, launch form) of the batched sweep
BATCH_CANDIDATES = ([(b, o, 0) for b in (8, 16, 24) for o in (0, 1)] + [(b, 1, 1) for b in (8, 16)] +
                    [(16, o, 2) for o in (0, 1)])
# (0, 0): the library's default (for the bit-packed L = 16 cube its colour-packed kernel)
SOLO_CANDIDATES = [(0, 0), (1, 1), (1, 2), (1, 4), (2, 2), (2, 4), (4, 2), (4, 4)]


def _snapshot(runs, stream):
    """copies of the population buffers, taken on the runs' stream (ordered with their kernels)"""
    import torch

    with torch.cuda.stream(stream):
        snap = [(r.spins[0].clone(), r.spins[1].clone(), r.energy[0].clone(), r.energy[1].clone()) for r in runs]
    stream.synchronize()
    return snap


def _restore(runs, snap, stream):
    import torch

    with torch.cuda.stream(stream):
        for r, (s0, s1, e0, e1) in zip(runs, snap):
            r.spins[0].copy_(s0)
            r.spins[1].copy_(s1)
            r.energy[0].copy_(e0)
            r.energy[1].copy_(e1)


def _digest(runs):
    """sha256 of every run's current spins and energies (pa_query synchronises the run's stream)"""
    import hashlib

    h = hashlib.sha256()
    for r in runs:
        info = r.query()
        h.update(r.spins[info.cur].cpu().numpy().tobytes())
        h.update(r.energy[info.cur][: 4 * int(info.R)].cpu().numpy().tobytes())
    return h.hexdigest()


def _time(fn, stream, repeats):
    import torch

    best = float("inf")
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune_batch(batch: "pa.Batch", steps, repeats: int = 2, verbose: bool = False):
    """Pick the persistent-sweep schedule for this batch; returns (best, timings ms).  steps: one
    pa_step or a list of them (e.g. one per first-look regime of the schedule); a candidate's time
    is the sum over the steps of its best sweep time."""
    steps = list(steps) if isinstance(steps, (list, tuple)) else [steps]
    st = batch.stream
    snap = _snapshot(batch.runs, st)
    timings, ref = {}, None
    for cand in BATCH_CANDIDATES:
        pa.set_batch_config(*cand)
        t = 0.0
        for step in steps:
            def one(step=step):
                batch.sweep(step)

            best = float("inf")
            for _ in range(repeats):
                _restore(batch.runs, snap, st)
                best = min(best, _time(one, st, 1))
            t += best
        _restore(batch.runs, snap, st)
        batch.sweep(steps[0])
        d = _digest(batch.runs)
        if ref is None:
            ref = d
        elif d != ref:
            raise RuntimeError(f"batch schedule {cand} changed the sample")
        timings[cand] = t
        if verbose:
            print(f"  blocks/CU={cand[0]:2d} order={cand[1]} launch={cand[2]}: {t:.3f} ms", flush=True)
    _restore(batch.runs, snap, st)
    st.synchronize()
    best = min(timings, key=timings.get)
    pa.set_batch_config(*best)
    return best, timings


def tune_solo(run: "pa.Run", step: "pa.pa_step", repeats: int = 2, verbose: bool = False):
    """Pick lanes per replica and waves per block for one run (or the default kernel, (0, 0));
    returns (best, timings ms)."""
    st = run.stream
    snap = _snapshot([run], st)
    timings, ref = {}, None
    for lpr, wpb in SOLO_CANDIDATES:
        pa.set_sweep_config(lpr, wpb)

        def one():
            run.sweep(step)

        t = float("inf")
        for _ in range(repeats):
            _restore([run], snap, st)
            t = min(t, _time(one, st, 1))
        _restore([run], snap, st)
        run.sweep(step)
        d = _digest([run])
        if ref is None:
            ref = d
        elif d != ref:
            raise RuntimeError(f"sweep shape {lpr}, {wpb} changed the sample")
        timings[(lpr, wpb)] = t
        if verbose:
            print(f"  lanes/replica={lpr} waves/block={wpb}: {t:.3f} ms", flush=True)
    _restore([run], snap, st)
    st.synchronize()
    best = min(timings, key=timings.get)
    pa.set_sweep_config(*best)
    return best, timings
