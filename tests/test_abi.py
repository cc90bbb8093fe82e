"""The C ABI without a GPU: the library loads, exports every entry point declared in
include/pa.h, rejects bad arguments on the host, and builds host tables identical to the
oracle's (they feed the bit-exact device computation)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as o
from paper_1006_0252_amd import pa

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pa.h")


def no_gpu():
    """The descriptor tests below hand the library fake device addresses that its host checks must
    refuse; they run only where no GPU could be reached if a check let one through."""
    try:
        import torch
    except ImportError:
        return True
    return torch.cuda.device_count() == 0


fake_pointers = pytest.mark.skipif(not no_gpu(), reason="fake device pointers: host checks only, run without a GPU")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    L = pa.lib()
    for n in names:
        assert hasattr(L, n), f"{n} declared in pa.h but not exported"
        assert n in pa.SIGNATURES, f"{n} has no binding signature"


def test_struct_sizes_match_header():
    assert ctypes.sizeof(pa.pa_record) == 128
    assert ctypes.sizeof(pa.pa_run) == 144
    s = pa.buffer_sizes(3, 4, pa.PA_U8, 64, 4)
    assert s.state_bytes == 256 and s.record_bytes == 4 * 128


@pytest.mark.parametrize("dim,L,layout", [(1, 64, 0), (1, 100, 1), (3, 8, 0), (3, 16, 1), (3, 6, 1)])
def test_buffer_sizes(dim, L, layout):
    cap = 1024
    s = pa.buffer_sizes(dim, L, layout, cap, 10)
    N = L if dim == 1 else L ** 3
    B = L if dim == 1 else 3 * N
    assert s.N == N and s.n_bonds == B and s.n_bins == B // 2 + 1
    assert s.row_stride % 16 == 0 and s.row_stride >= N
    if layout == pa.PA_U8:
        assert s.spins_bytes == cap * s.row_stride
    else:
        rows = (N + 31) // 32 if dim == 1 else L * L
        W = 32 if dim == 1 else (8 if L <= 8 else (16 if L <= 16 else 32))
        assert s.spins_bytes == cap * rows * W // 8
    if (dim, L, layout) == (3, 16, 1):
        assert s.spins_bytes == cap * 512  # 0.5 KB per L = 16 replica


@pytest.mark.parametrize("args", [(2, 8, 0, 0, 64), (3, 7, 0, 0, 64), (1, 3, 0, 0, 64), (3, 8, 2, 0, 64),
                                  (3, 8, 0, 0, 100), (3, 8, 0, 0, 0), (3, 34, 0, 0, 64), (3, 8, 0, 2, 64),
                                  (3, 8, 1, 1, 64)])
def test_buffer_sizes_rejects(args):
    s = pa.pa_sizes()
    assert pa.lib().pa_buffer_sizes(*args, 4, ctypes.byref(s)) == pa.PA_ERR_ARG


def test_buffer_sizes_gaussian():
    s = pa.buffer_sizes(3, 8, pa.PA_U8, 128, 5, couplings=pa.PA_GAUSS)
    assert s.J_bytes == 8 * 3 * 512 and s.energy_bytes == 8 * 128
    p = pa.buffer_sizes(3, 8, pa.PA_U8, 128, 5)
    assert p.J_bytes == 3 * 512 and p.energy_bytes == 4 * 128 and p.spins_bytes == s.spins_bytes
    # the Gaussian work buffer also holds the sweep's tables over [2 colours][N / 2][64 patterns]:
    # u16 first-look entries and u64 thresholds
    assert s.work_bytes - p.work_bytes == (2 + 8) * 2 * 256 * 64
    c = pa.buffer_sizes(1, 256, pa.PA_U8, 128, 5, couplings=pa.PA_GAUSS)
    assert c.work_bytes - pa.buffer_sizes(1, 256, pa.PA_U8, 128, 5).work_bytes >= (2 + 8) * 2 * 128 * 4


def test_calls_reject_bad_runs_without_touching_the_device():
    r = pa.pa_run()
    r.dim, r.L, r.layout, r.n_records, r.capacity, r.R0 = 3, 7, 0, 4, 64, 10  # odd L
    step = pa.pa_step()
    step.beta_from, step.beta_to, step.k, step.n_sweeps = 0.0, 0.1, 1, 1
    L = pa.lib()
    assert L.pa_init_couplings(ctypes.byref(r), 1, None) == pa.PA_ERR_ARG
    assert L.pa_sweep(ctypes.byref(r), 1, ctypes.byref(step)) == pa.PA_ERR_ARG
    assert L.pa_resample(ctypes.byref(r), 1, ctypes.byref(step)) == pa.PA_ERR_ARG
    assert L.pa_measure(ctypes.byref(r), 1, None) == pa.PA_ERR_ARG
    assert L.pa_sweep(None, 1, ctypes.byref(step)) == pa.PA_ERR_ARG
    assert L.pa_status(None, 1, None) == pa.PA_ERR_ARG
    assert pa.lib().pa_strerror(pa.PA_ERR_CAPACITY).startswith(b"resampled population")


@fake_pointers
def test_each_bad_descriptor_field_is_rejected_without_touching_the_device():
    # a well-formed descriptor (aligned fake pointers, never dereferenced) with one field at a time
    # set to a value the calls refuse: empty or oversized populations, capacities off the 64-replica
    # grid, no records, unknown layouts and couplings, Gaussian bonds on bit-packed spins, lattices
    # the library has no geometry for, a null buffer
    base = 1 << 40

    def good():
        r = pa.pa_run()
        r.dim, r.L, r.layout, r.n_records, r.capacity, r.R0, r.couplings = 3, 8, pa.PA_BITS64, 4, 128, 100, pa.PA_PM1
        r.J, r.energy[0], r.energy[1], r.counts, r.offsets = base, base + 4096, base + 8192, base + 12288, base + 16384
        r.work, r.record, r.state = base + 20480, base + 24576, base + 28672
        r.spins[0], r.spins[1] = base + 32768, base + 65536
        return r

    bad = [("R0", 0), ("R0", -5), ("R0", 129), ("capacity", 0), ("capacity", 100), ("capacity", -64),
           ("n_records", 0), ("layout", 7), ("couplings", 9), ("couplings", pa.PA_GAUSS), ("L", 7), ("L", 0),
           ("dim", 2), ("dim", 0), ("J", None), ("state", None), ("work", None)]
    step = pa.pa_step()
    step.beta_from, step.beta_to, step.k, step.n_sweeps = 0.0, 0.1, 1, 1
    L = pa.lib()
    for field, value in bad:
        r = good()
        setattr(r, field, value)
        for call in (L.pa_init_couplings, L.pa_measure):
            assert call(ctypes.byref(r), 1, None) == pa.PA_ERR_ARG, (field, value, call)
        for call in (L.pa_sweep, L.pa_resample):
            assert call(ctypes.byref(r), 1, ctypes.byref(step)) == pa.PA_ERR_ARG, (field, value, call)
    # and a bad step with a good descriptor
    for field, value in (("k", 0), ("n_sweeps", -1), ("t0", -1), ("beta_from", -0.1), ("beta_to", float("nan"))):
        st = pa.pa_step()
        st.beta_from, st.beta_to, st.k, st.n_sweeps = 0.0, 0.1, 1, 1
        setattr(st, field, value)
        assert L.pa_sweep(ctypes.byref(good()), 1, ctypes.byref(st)) == pa.PA_ERR_ARG, (field, value)


@fake_pointers
def test_calls_reject_unaligned_buffers_without_touching_the_device():
    # a well-formed descriptor whose spin buffer is 8 bytes off a 256-byte boundary (the pointers
    # are never dereferenced: the check comes first)
    r = pa.pa_run()
    r.dim, r.L, r.layout, r.n_records, r.capacity, r.R0, r.couplings = 3, 8, pa.PA_BITS64, 4, 128, 100, pa.PA_PM1
    base = 1 << 40
    r.J, r.energy[0], r.energy[1], r.counts, r.offsets = base, base + 4096, base + 8192, base + 12288, base + 16384
    r.work, r.record, r.state = base + 20480, base + 24576, base + 28672
    r.spins[0], r.spins[1] = base + 32768 + 8, base + 65536
    step = pa.pa_step()
    step.beta_from, step.beta_to, step.k, step.n_sweeps = 0.0, 0.1, 1, 1
    L = pa.lib()
    assert L.pa_init_couplings(ctypes.byref(r), 1, None) == pa.PA_ERR_ARG
    assert L.pa_sweep(ctypes.byref(r), 1, ctypes.byref(step)) == pa.PA_ERR_ARG
    assert L.pa_resample(ctypes.byref(r), 1, ctypes.byref(step)) == pa.PA_ERR_ARG


def test_weights_equal_oracle_levels():
    # w_d = exp(-dbeta 4d): the same doubles the oracle's C libm exp gives for the level weights
    # (math.exp is the C library's exp; numpy's vectorised exp may round differently)
    import math

    for dbeta in (0.0, 0.05, 0.1, 1 / 60, 5 / 300, 0.7):
        w = pa.fill_weights(dbeta, 400)
        ref = np.array([math.exp(-dbeta * float(4 * d)) for d in range(400)])
        assert np.array_equal(w, ref)


def test_thresholds_equal_oracle():
    for beta in (0.0, 0.05, 0.3, 1.0, 2.5, 5.0):
        for z in (2, 6):
            T, always = pa.thresholds(beta, z)
            for c in range(z + 1):
                To, ao = o.threshold(beta, 4 * c - 2 * z)
                assert bool(always[c]) == ao
                if not ao:
                    assert int(T[c]) == To


@pytest.mark.parametrize("m", list(range(-20, 7)))
def test_ladder_tables_equal_oracle(m):
    assert np.array_equal(pa.ladder_table(m), o.ladder_table(m))


def test_host_weighted_average_matches_oracle():
    rng = np.random.default_rng(0)
    for M, n_obs in ((1, 1), (5, 3), (64, 2)):
        x = rng.normal(size=M) * 3 + 1000
        A = rng.normal(size=(M, n_obs))
        R = rng.uniform(1e4, 1e5, M)
        for RR in (None, R):
            a = pa.weighted_average(x, A, RR)
            b = o.weighted_average(x, A, RR)
            for key in ("A_bar", "omega"):
                assert np.allclose(a[key], b[key], rtol=1e-13, atol=1e-15)
            for key in ("minus_betaF_bar", "var", "mean"):
                assert abs(a[key] - b[key]) <= 1e-12 * max(1.0, abs(b[key]))


def test_unpack_spins_layouts():
    # bit-packed group-major rows decode to the right replica/site (pure host marshalling)
    rng = np.random.default_rng(1)
    for dim, L in ((3, 4), (3, 6), (3, 10), (1, 70)):
        N = L if dim == 1 else L ** 3
        R = 70
        s = rng.integers(0, 2, (R, N)).astype(np.uint8)
        rows = (N + 31) // 32 if dim == 1 else L * L
        rowsites = 32 if dim == 1 else L
        W = 32 if dim == 1 else (8 if L <= 8 else 16)
        dt = {8: np.uint8, 16: np.uint16, 32: np.uint32}[W]
        G = (R + 63) // 64
        words = np.zeros((G, rows, 64), dtype=np.uint64)
        for r in range(R):
            for i in range(N):
                words[r // 64, i // rowsites, r % 64] |= np.uint64(int(s[r, i]) << (i % rowsites))
        raw = words.astype(dt).view(np.uint8).reshape(-1)
        assert np.array_equal(pa.unpack_spins(raw, dim, L, pa.PA_BITS64, R, 0), s)


@pytest.mark.parametrize("n", [2, 8])
def test_bench_refuses_more_than_one_gpu(n):
    # the benchmark is a one-GPU measurement: asked for more it says so and exits before any GPU work
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", str(n)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
