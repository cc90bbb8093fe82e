"""Summaries of rocprofv3 outputs for the sweep's roofline (the files under profiles/).

counters DIR... OUT: rocprofv3 --pmc passes over profile_sweep.py (one sweep launch per first-look
    regime on the L = 16 cube, R0 = 1e6: beta = 0.5, 2, 4).  Per regime: every counter of the
    sweep kernel's dispatch, and per attempt the lane-weighted counts (counter x 64 / attempts) of
    the instruction counters.  Writes OUT (JSON, with the sha256 of the sweep's sources, which
    bench.py checks before it uses the figures).
traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR OUT: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) of the sweep in the benchmark, scaled by what the same counters read for a plain
    device copy of known size (copy_calibration.py), as bytes per sweep launch.
stats DIR: the kernel_stats table of a --kernel-trace --stats run as markdown.
replay DIR N: the last N sweep dispatches of a --kernel-trace run and every dispatch between the
    first and the last of them (a replayed graph): calls, total and average ms per kernel.
batched TRACE_DIR PMC_DIR... [OUT.json]: profile_sweep.py batched under --kernel-trace and under
    --pmc passes: per lattice size and first-look regime the sweep launch's duration, attempts/s and
    the lane-weighted instruction counts per attempt, as a markdown table (and as JSON).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# the sources each sweep kernel is compiled from (a summary records their sha256; bench.py uses
# its figures only while they are unchanged)
SWEEP_SOURCES = ("paper_1006_0252_amd/csrc/pa_sweep_colour.hip", "paper_1006_0252_amd/csrc/pa_sweep_words.h",
                 "paper_1006_0252_amd/csrc/pa_sweep_util.h", "paper_1006_0252_amd/csrc/pa_common.h")
STRING_SOURCES = ("paper_1006_0252_amd/csrc/pa_sweep_strings.hip", "paper_1006_0252_amd/csrc/pa_sweep_words.h",
                  "paper_1006_0252_amd/csrc/pa_sweep_util.h", "paper_1006_0252_amd/csrc/pa_common.h")
SWEEP_KERNEL = "k_sweep16c"
KERNEL_LABEL = "k_sweep16c (colour-packed words, bit-packed L=16; pa_sweep, 10 sweeps per launch)"
ATTEMPTS_PER_LAUNCH = 1_000_000 * 4096 * 10  # profile_sweep.py: R0 = 1e6 replicas, L = 16, 10 sweeps
# HBM bytes a sweep launch of 1e6 L = 16 replicas must move: each replica's 4096 spin bits read and
# written once (512 + 512 bytes) and its 4-byte energy written
ALGORITHMIC_BYTES_PER_LAUNCH = 1_000_000 * (512 + 512 + 4)
INSTRUCTION_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VALU_INT32",
                        "SQ_INSTS_VALU_INT64", "SQ_INSTS_SMEM", "SQ_INSTS_BRANCH")


def sweep_source_digest(sources=SWEEP_SOURCES):
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _rows(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    out = []
    for fn in files:
        with open(fn) as f:
            out += list(csv.DictReader(f))
    return out


def dispatch_counters(d, kernel):
    """{dispatch id: {counter: value}} of the dispatches of `kernel` (substring of the name), in
    dispatch order."""
    per = {}
    for r in _rows(d, "counter_collection.csv"):
        if kernel not in r.get("Kernel_Name", ""):
            continue
        did = int(r["Dispatch_Id"])
        per.setdefault(did, {})
        name = r["Counter_Name"]
        per[did][name] = per[did].get(name, 0.0) + float(r["Counter_Value"])
    return dict(sorted(per.items()))


def counters(dirs, out):
    regimes = {}
    for d in dirs:
        disp = list(dispatch_counters(d, SWEEP_KERNEL).values())
        if len(disp) != 3:
            raise RuntimeError(f"{d}: expected 3 sweep dispatches (one per regime), found {len(disp)}")
        for reg, c in enumerate(disp):
            regimes.setdefault(str(reg), {}).update(c)
    per_attempt = {r: {k: v * 64 / ATTEMPTS_PER_LAUNCH for k, v in c.items() if k in INSTRUCTION_COUNTERS}
                   for r, c in regimes.items()}
    res = {"kernel": KERNEL_LABEL,
           "workload": "cube L=16, R0=1e6, bit-packed; one launch each at beta = 0.5, 2, 4 (first-look regimes 0, 1, 2)",
           "attempts_per_launch": ATTEMPTS_PER_LAUNCH, "counters": regimes, "per_attempt": per_attempt,
           "valu_per_attempt": {r: v["SQ_INSTS_VALU"] for r, v in per_attempt.items() if "SQ_INSTS_VALU" in v},
           "source_digest": sweep_source_digest()}
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res["valu_per_attempt"]))


def _kib(d, kernel, name):
    disp = dispatch_counters(d, kernel)
    vals = [c[name] for c in disp.values() if name in c]
    if not vals:
        raise RuntimeError(f"{d}: no {name} for {kernel}")
    return sum(vals) / len(vals), len(vals)


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, out, copy_bytes=1 << 30):
    f_kib, nf = _kib(fetch_dir, SWEEP_KERNEL, "FETCH_SIZE")
    w_kib, nw = _kib(write_dir, SWEEP_KERNEL, "WRITE_SIZE")
    # the copy kernel: the one whose dispatches read the most (torch's elementwise copy)
    cf = dispatch_counters(copy_fetch_dir, "")
    cw = dispatch_counters(copy_write_dir, "")
    copy_f = max(c.get("FETCH_SIZE", 0.0) for c in cf.values())
    copy_w = max(c.get("WRITE_SIZE", 0.0) for c in cw.values())
    fs, ws = copy_bytes / (copy_f * 1024), copy_bytes / (copy_w * 1024)
    res = {"kernel": KERNEL_LABEL,
           "workload": "cube L=16, R0=1e6, bit-packed, the first steps of the 301-temperature schedule",
           "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib, "dispatches": [nf, nw],
           "copy_calibration": {"bytes_read": copy_bytes, "bytes_written": copy_bytes, "fetch_kib_read": copy_f,
                                "write_kib_read": copy_w, "fetch_scale": fs, "write_scale": ws},
           "bytes_per_launch": f_kib * 1024 * fs + w_kib * 1024 * ws,
           "algorithmic_bytes_per_launch": ALGORITHMIC_BYTES_PER_LAUNCH,
           "source_digest": sweep_source_digest()}
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({k: res[k] for k in ("fetch_kib_per_dispatch", "write_kib_per_dispatch", "bytes_per_launch")}))


def stats(d):
    rows = _rows(d, "kernel_stats.csv")
    print("| kernel | calls | avg us | min us | max us | % of GPU time |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        name = r["Name"][:72]
        print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
              f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")


# profile_sweep.py batched: attempts of one batched sweep launch (10 sweeps of every run at its
# initial size) per lattice size; its three launches per size are regimes 0, 1, 2 in order
def _batched_attempts():
    sys.path.insert(0, ROOT)
    from paper_1006_0252_amd import workloads

    att = {}
    for sp in workloads.batched_specs():
        att[sp["L"]] = att.get(sp["L"], 0) + sp["R0"] * sp["L"] ** 3 * workloads.C3_SWEEPS
    return att


def _sweep_L(name):
    import re

    m = re.search(r"k_sweep\w*<(\d+),", name)
    return int(m.group(1)) if m else None


def batched(trace_dir, pmc_dirs, out=None):
    """out: also write the per-size, per-regime figures as JSON (with the colour-string kernel's
    source digest), for bench.py's batched line"""
    att = _batched_attempts()
    times = {}
    for r in _rows(trace_dir, "kernel_trace.csv"):
        L = _sweep_L(r["Kernel_Name"])
        if L is None:
            continue
        times.setdefault(L, []).append((int(r["Start_Timestamp"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6))
    counts = {}
    for d in pmc_dirs:
        per = {}
        for r in _rows(d, "counter_collection.csv"):
            L = _sweep_L(r["Kernel_Name"])
            if L is None:
                continue
            key = (L, int(r["Dispatch_Id"]))
            per.setdefault(key, {})
            per[key][r["Counter_Name"]] = per[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        for L in sorted({k[0] for k in per}):
            disp = [per[k] for k in sorted(k for k in per if k[0] == L)]
            for reg, c in enumerate(disp):
                counts.setdefault((L, reg), {}).update(c)
    if out:
        res = {"workload": "profile_sweep.py batched: the 256 runs at their initial sizes, one batched launch of 10 sweeps "
                           "at beta = 0.5, 2, 4",
               "by_size": {}, "source_digest": sweep_source_digest(STRING_SOURCES)}
        for L in sorted(times):
            for reg, (_, ms) in enumerate(sorted(times[L])):
                c = counts.get((L, reg), {})
                res["by_size"].setdefault(str(L), {})[str(reg)] = {
                    "ms": ms, "attempts": att[L], "attempts_per_s": att[L] / (ms * 1e-3),
                    **{k: v * 64 / att[L] for k, v in c.items() if k.startswith("SQ_INSTS")},
                    **({"VALUBusy": c["VALUBusy"]} if "VALUBusy" in c else {})}
        with open(out, "w") as f:
            json.dump(res, f, indent=1)
    print("| L | regime | kernel ms | attempts/s | VALU / attempt | INT64 / attempt | SALU / attempt | LDS / attempt | VALUBusy % |")
    print("|---|---|---|---|---|---|---|---|---|")
    for L in sorted(times):
        for reg, (_, ms) in enumerate(sorted(times[L])):
            c = counts.get((L, reg), {})
            pa = {k: v * 64 / att[L] for k, v in c.items() if k.startswith("SQ_INSTS")}
            f = lambda k: f"{pa[k]:.2f}" if k in pa else "-"
            busy = f"{c['VALUBusy']:.0f}" if "VALUBusy" in c else "-"
            print(f"| {L} | {reg} | {ms:.3f} | {att[L] / (ms * 1e-3):.3g} | {f('SQ_INSTS_VALU')} | {f('SQ_INSTS_VALU_INT64')} | "
                  f"{f('SQ_INSTS_SALU')} | {f('SQ_INSTS_LDS')} | {busy} |")


def replay(d, n):
    rows = sorted(_rows(d, "kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
    sw = [r for r in rows if "k_sweep" in r["Kernel_Name"]][-n:]
    t0, t1 = int(sw[0]["Start_Timestamp"]), int(sw[-1]["End_Timestamp"])
    agg = {}
    for r in rows:
        if t0 <= int(r["Start_Timestamp"]) <= t1:
            a = agg.setdefault(r["Kernel_Name"], [0, 0.0])
            a[0] += 1
            a[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    tot = sum(v[1] for v in agg.values())
    print(f"window {(t1 - t0) / 1e9:.3f} s, {len(sw)} sweep dispatches, kernel time {tot / 1e3:.3f} s")
    print("| kernel | calls | total ms | avg ms | % of kernel time |")
    print("|---|---|---|---|---|")
    for name, (cnt, ms) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:16]:
        print(f"| `{name[:72]}` | {cnt} | {ms:.1f} | {ms / cnt:.3f} | {100 * ms / tot:.2f} |")


def main(argv):
    if not argv:
        print(__doc__)
        return 2
    cmd, rest = argv[0], argv[1:]
    if cmd == "counters":
        counters(rest[:-1], rest[-1])
    elif cmd == "traffic":
        traffic(*rest)
    elif cmd == "stats":
        stats(rest[0])
    elif cmd == "replay":
        replay(rest[0], int(rest[1]))
    elif cmd == "batched":
        js = [a for a in rest if a.endswith(".json")]
        batched(rest[0], [a for a in rest[1:] if not a.endswith(".json")], js[0] if js else None)
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
