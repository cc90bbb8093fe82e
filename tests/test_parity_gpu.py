"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeds.

Bar: spins, energies, copy numbers, offsets and population sizes bit-exact; FP64 values
(ln Q, -beta F, energy moments, overlap statistics) within 1e-12 relative (they differ only
through the device's log/exp/sqrt last-bit rounding and summation order of variance sums).
Sizes span several waves, blocks and a ragged tail of the last 64-replica group; the
C4-shaped test runs the full 1e6-replica population and checks sampled replicas one by one.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as o

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on a CPU machine only when -m gpu is asked for
    pytest.skip("no GPU", allow_module_level=True)

from paper_1006_0252_amd import pa  # noqa: E402

DEV = "cuda:0"
RTOL = 1e-12


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def close(a, b, rtol=RTOL, atol=0.0):
    return abs(a - b) <= rtol * max(1.0, abs(b)) + atol


def make_run(dim, L, R0, layout, seed=7, dseed=3, n_records=8, capacity=None):
    run = pa.Run(dim, L, R0, seed, dseed, n_records=n_records, capacity=capacity, layout=layout, device=DEV)
    run.init()
    return run


INIT_CASES = [
    (1, 64, "u8", 150), (1, 64, "bits64", 150), (1, 100, "u8", 70), (1, 100, "bits64", 70),
    (3, 2, "u8", 100), (3, 2, "bits64", 100), (3, 4, "bits64", 200), (3, 6, "u8", 130), (3, 6, "bits64", 130),
    (3, 8, "u8", 200), (3, 8, "bits64", 200), (3, 10, "bits64", 90), (3, 12, "bits64", 70),
    (3, 14, "u8", 70), (3, 16, "u8", 70), (3, 16, "bits64", 130),
]


@pytest.mark.parametrize("dim,L,layout,R0", INIT_CASES)
def test_init_parity(dim, L, layout, R0):
    note(f"init dim={dim} L={L} {layout} R0={R0}")
    run = make_run(dim, L, R0, layout)
    J = run.couplings()
    assert np.array_equal(J, o.couplings(dim, L, 3))
    s, E = run.population()
    so, Eo = o.init_population(dim, L, J, 7, R0)
    assert np.array_equal(s, so) and np.array_equal(E, Eo)
    rec = run.records()[0]
    assert rec[2] == o.num_sites(dim, L) * math.log(2.0) or close(rec[2], o.num_sites(dim, L) * math.log(2.0))
    info = run.query()
    assert info.R == R0 and info.status == 0 and info.k == 0


def test_init_with_host_couplings():
    note("init with host couplings")
    dim, L, R0 = 3, 6, 100
    J = np.where(np.random.default_rng(4).random(3 * L ** 3) < 0.3, -1, 1).astype(np.int8)
    run = pa.Run(dim, L, R0, 5, 0, n_records=2, layout="bits64", device=DEV)
    run.init(J)
    assert np.array_equal(run.couplings(), J)
    s, E = run.population()
    so, Eo = o.init_population(dim, L, J, 5, R0)
    assert np.array_equal(s, so) and np.array_equal(E, Eo)


# regimes: 0 (beta < 1.39), 1 (1.39 .. 2.77), 2.  At beta = 1e-17 exp(-4 beta) rounds to 1 (class
# c = 4 always accepts) while c = 5, 6 have T64 = 2^64 - 2^11: first-look threshold 0xFFFF.  The
# fast cube kernel compares against top + 1 in 16 bits: at beta = 5e-6 the top of c = 4 is 0xFFFE
# (the largest it takes), at 3e-6 it is 0xFFFF and the generic kernel sweeps instead (as at 0 and
# 1e-17)
SWEEP_BETAS = [0.0, 1e-17, 3e-6, 5e-6, 0.35, 1.2, 2.0, 5.0]


@pytest.mark.parametrize("dim,L,layout,R0", INIT_CASES)
def test_sweep_parity(dim, L, layout, R0):
    J = o.couplings(dim, L, 3)
    for beta in SWEEP_BETAS:
        note(f"sweep dim={dim} L={L} {layout} R0={R0} beta={beta}")
        run = make_run(dim, L, R0, layout)
        sched = pa.Schedule([0.0, beta] if beta > 0 else [0.0, 0.0], 2, run.n_bins, device=DEV)
        step = sched.step(1)
        step.t0 = 3
        run.sweep(step)
        s, E = run.population()
        so, Eo = o.init_population(dim, L, J, 7, R0)
        o.sweep(dim, L, J, 7, beta, R0, so, Eo, 3, 2)
        assert np.array_equal(s, so), f"spins differ at beta={beta}"
        assert np.array_equal(E, Eo), f"energies differ at beta={beta}"


@pytest.mark.parametrize("L,layout,cap", [(16, "bits64", None), (16, "bits64", 640), (10, "bits64", None), (8, "u8", None),
                                          (12, "u8", None)])
def test_sweep_launch_shapes_agree(L, layout, cap):
    # every launch shape (lanes per replica, waves per block) gives the same sample; shapes whose
    # block holds one whole 64-replica group move it block-wide, and with capacity 640 whole
    # blocks lie past the population
    R0 = 200
    J = o.couplings(3, L, 3)
    so, Eo = o.init_population(3, L, J, 7, R0)
    o.sweep(3, L, J, 7, 0.8, R0, so, Eo, 0, 3)
    try:
        # (0, 0): the default, for the bit-packed L = 16 cube the colour-packed kernel
        for lpr, wpb in ((0, 0), (1, 1), (1, 4), (2, 2), (2, 4), (4, 1), (4, 3), (4, 4)):
            note(f"sweep shape L={L} {layout} lpr={lpr} wpb={wpb}")
            pa.set_sweep_config(lpr, wpb)
            run = make_run(3, L, R0, layout, capacity=cap)
            sched = pa.Schedule([0.0, 0.8], 3, run.n_bins, device=DEV)
            run.sweep(sched.step(1))
            s, E = run.population()
            assert np.array_equal(s, so) and np.array_equal(E, Eo), f"lpr={lpr} wpb={wpb}"
    finally:
        pa.set_sweep_config(0, 0)


@pytest.mark.parametrize("L,R0", [(16, 20_000), (10, 3_001), (8, 5_000), (6, 4_111), (4, 9_000)])
def test_colour_kernels_match_row_pair_kernel(L, R0):
    # the default sweeps of bit-packed cubes (L = 16: words of one colour; L = 4..10: one string of
    # each colour per replica) against the row-pair kernel (taken when a launch shape is forced),
    # many groups, the last one partial: the same sample bit for bit, in every first-look regime
    for beta in (0.05, 0.5, 1.2, 1.5, 2.5, 3.0, 6.0):
        note(f"colour vs row-pair kernel L={L} R0={R0} beta={beta}")
        out = []
        try:
            for cfg in ((0, 0), (4, 4) if L % 4 == 0 else (1, 2)):
                pa.set_sweep_config(*cfg)
                run = make_run(3, L, R0, "bits64", seed=11, dseed=2)
                sched = pa.Schedule([0.0, beta], 4, run.n_bins, device=DEV)
                step = sched.step(1)
                step.t0 = 17
                run.sweep(step)
                out.append(run.population())
        finally:
            pa.set_sweep_config(0, 0)
        (s0, E0), (s1, E1) = out
        assert np.array_equal(s0, s1) and np.array_equal(E0, E1), f"beta={beta}"


RESAMPLE_CASES = [(1, 64, "u8", 300), (1, 64, "bits64", 300), (3, 4, "bits64", 500), (3, 6, "u8", 400),
                  (3, 8, "bits64", 700), (3, 10, "u8", 200), (3, 16, "bits64", 150)]


@pytest.mark.parametrize("dim,L,layout,R0", RESAMPLE_CASES)
def test_resample_parity(dim, L, layout, R0):
    J = o.couplings(dim, L, 3)
    for b0, b1 in ((0.0, 0.1), (0.6, 0.75), (2.0, 3.5)):
        note(f"resample dim={dim} L={L} {layout} R0={R0} {b0}->{b1}")
        run = make_run(dim, L, R0, layout, n_records=4)
        sched = pa.Schedule([b0, b1], 2, run.n_bins, device=DEV)
        step = sched.step(1)
        so, Eo = o.init_population(dim, L, J, 7, R0, capacity=run.capacity)
        if b0 > 0:
            run.sweep(pa.Schedule([0.0, b0], 2, run.n_bins, device=DEV).step(1))
            o.sweep(dim, L, J, 7, b0, R0, so, Eo, 0, 2)
        run.resample(step)
        r = o.resample(dim, L, 7, 1, b0, b1, R0, R0, so, Eo, run.capacity)
        assert r["status"] == 0
        info = run.query()
        assert info.status == 0 and info.R == r["R_new"] and info.k == 1
        c, off = run.counts_offsets(R0)
        assert np.array_equal(c, r["counts"]) and np.array_equal(off, r["offsets"])
        s, E = run.population()
        assert np.array_equal(s, r["s"][: r["R_new"]]) and np.array_equal(E, r["E"][: r["R_new"]])
        rec = run.records()[1]
        assert rec[5] == r["E_lo"] and rec[3] == r["S"], "S must be bit-identical (fixed summation order)"
        assert close(rec[1], r["lnQ"]) and rec[4] == r["R_new"]
        assert close(rec[2], o.num_sites(dim, L) * math.log(2.0) + r["lnQ"])


@pytest.mark.parametrize("L", [18, 20, 24, 32])
@pytest.mark.parametrize("layout", ["bits64", "u8"])
def test_largest_cubes_match_oracle(L, layout):
    # the largest sides the library takes (the generic kernel; 32^3 = 32768 sites): initial
    # population, two sweeps and a resample against the oracle
    R0 = 70
    note(f"largest cubes L={L} {layout}")
    J = o.couplings(3, L, 3)
    run = make_run(3, L, R0, layout, n_records=4)
    so, Eo = o.init_population(3, L, J, 7, R0, capacity=run.capacity)
    s, E = run.population()
    assert np.array_equal(s, so[:R0]) and np.array_equal(E, Eo[:R0])
    sched = pa.Schedule([0.0, 0.8, 1.0], 2, run.n_bins, device=DEV)
    run.sweep(sched.step(1))
    o.sweep(3, L, J, 7, 0.8, R0, so, Eo, 0, 2)
    s, E = run.population()
    assert np.array_equal(s, so[:R0]) and np.array_equal(E, Eo[:R0])
    run.resample(sched.step(2))
    r = o.resample(3, L, 7, 2, 0.8, 1.0, R0, R0, so, Eo, run.capacity)
    assert r["status"] == 0 and run.query().R == r["R_new"]
    s, E = run.population()
    assert np.array_equal(s, r["s"][: r["R_new"]]) and np.array_equal(E, r["E"][: r["R_new"]])


def test_unsupported_cube_side_is_rejected():
    # even sides the buffers allow but no sweep kernel takes (22, 26, 28, 30): PA_ERR_ARG, the
    # population untouched
    note("unsupported cube side")
    run = make_run(3, 22, 64, "bits64", n_records=4)
    s0, E0 = run.population()
    sched = pa.Schedule([0.0, 0.5], 2, run.n_bins, device=DEV)
    with pytest.raises(pa.PAError):
        run.sweep(sched.step(1))
    s1, E1 = run.population()
    assert np.array_equal(s0, s1) and np.array_equal(E0, E1)


def test_copy_numbers_in_the_hundreds():
    # one step of beta 0 -> 0.1 from the random start of 5000 replicas of the L = 8 cube: the lowest
    # energies get copy numbers up to ~700, i.e. many Poisson(64) blocks and every ladder level
    # (the binary-search inversion), every copy number against the oracle
    dim, L, R0 = 3, 8, 5000
    note("copy numbers in the hundreds")
    J = o.couplings(dim, L, 3)
    run = make_run(dim, L, R0, "bits64", n_records=4)
    sched = pa.Schedule([0.0, 0.1], 2, run.n_bins, device=DEV)
    so, Eo = o.init_population(dim, L, J, 7, R0, capacity=run.capacity)
    run.resample(sched.step(1))
    r = o.resample(dim, L, 7, 1, 0.0, 0.1, R0, R0, so, Eo, run.capacity)
    assert r["status"] == 0 and run.query().status == 0
    c, off = run.counts_offsets(R0)
    assert c.max() >= 256, "the case must reach several Poisson(64) blocks"
    assert np.array_equal(c, r["counts"]) and np.array_equal(off, r["offsets"])
    s, E = run.population()
    assert np.array_equal(s, r["s"][: r["R_new"]]) and np.array_equal(E, r["E"][: r["R_new"]])


@pytest.mark.parametrize("R0", [1, 63, 64, 65, 129])
@pytest.mark.parametrize("L,layout", [(8, "u8"), (8, "bits64"), (16, "bits64")])
def test_population_sizes_at_group_edges(L, layout, R0):
    # a single replica, one short of a 64-replica group, exactly one group, one past it, two groups
    # and one: initial population, two sweeps and a resample against the oracle (a population that
    # dies out must be flagged on both sides and left as it was)
    dim = 3
    note(f"group edges L={L} {layout} R0={R0}")
    J = o.couplings(dim, L, 3)
    run = make_run(dim, L, R0, layout, n_records=4)
    so, Eo = o.init_population(dim, L, J, 7, R0, capacity=run.capacity)
    s, E = run.population()
    assert np.array_equal(s, so[:R0]) and np.array_equal(E, Eo[:R0])
    sched = pa.Schedule([0.0, 0.9, 1.0], 2, run.n_bins, device=DEV)
    run.sweep(sched.step(1))
    o.sweep(dim, L, J, 7, 0.9, R0, so, Eo, 0, 2)
    s, E = run.population()
    assert np.array_equal(s, so[:R0]) and np.array_equal(E, Eo[:R0])
    r = o.resample(dim, L, 7, 2, 0.9, 1.0, R0, R0, so, Eo, run.capacity)
    run.resample(sched.step(2))
    if r["status"] == o.ERR_EXTINCT:
        code, flags = run.status()
        assert code == pa.PA_ERR_EXTINCT and flags & pa.PA_FLAG_EXTINCT
        assert run.query().R == R0
        s1, E1 = run.population()
        assert np.array_equal(s1, s) and np.array_equal(E1, E)
        return
    assert r["status"] == 0
    info = run.query()
    assert info.status == 0 and info.R == r["R_new"]
    c, off = run.counts_offsets(R0)
    assert np.array_equal(c, r["counts"]) and np.array_equal(off, r["offsets"])
    s, E = run.population()
    assert np.array_equal(s, r["s"][: r["R_new"]]) and np.array_equal(E, r["E"][: r["R_new"]])


RUN_CASES = [
    ("ring C1", 1, 64, "u8", 1000, 51, 5),
    ("ring C1 bits", 1, 64, "bits64", 1000, 51, 5),
    ("cube L8 reduced", 3, 8, "u8", 1500, 21, 10),
    ("cube L6 bits", 3, 6, "bits64", 900, 16, 4),
    ("cube L10 bits", 3, 10, "bits64", 400, 11, 4),
    ("cube L16 bits reduced", 3, 16, "bits64", 260, 7, 10),
]


@pytest.mark.parametrize("name,dim,L,layout,R0,nT,ns", RUN_CASES)
def test_full_run_parity(name, dim, L, layout, R0, nT, ns):
    note(f"full run {name}")
    betas = [5.0 * k / (nT - 1) for k in range(nT)]
    seed, dseed = 2024, 5
    run = pa.Run(dim, L, R0, seed, dseed, n_records=nT, layout=layout, device=DEV)
    run.init()
    sched = pa.Schedule(betas, ns, run.n_bins, device=DEV)
    for k in range(1, nT):
        st = sched.step(k)
        run.resample(st)
        run.sweep(st)
        pa.measure([run])
    J = o.couplings(dim, L, dseed)
    st_o, rec_o, s_o, E_o = o.run(dim, L, J, seed, R0, betas, ns, capacity=run.capacity)
    assert st_o == 0
    code, flags = run.status()
    assert code == pa.PA_OK and flags == 0
    rec = run.records()
    for k in range(nT):
        assert rec[k, 4] == rec_o[k, 1], f"R differs at k={k}"
        assert close(rec[k, 1], rec_o[k, 2]), f"ln Q differs at k={k}"
        assert close(rec[k, 2], rec_o[k, 3]), f"-beta F differs at k={k}"
        if k > 0:
            assert rec[k, 6] == rec_o[k, 4], f"E mean differs at k={k}"
            assert close(rec[k, 7], rec_o[k, 5], rtol=1e-12, atol=1e-12), f"E var differs at k={k}"
            assert close(rec[k, 8], rec_o[k, 6], rtol=1e-9, atol=1e-9), f"E skew differs at k={k}"
    s, E = run.population()
    assert np.array_equal(s, s_o) and np.array_equal(E, E_o)
    fe = torch.zeros(1, dtype=torch.float64, device=DEV)
    run.free_energy(fe)
    assert close(float(fe.cpu()[0]), rec_o[-1, 3])


def seeded_run_configs(n, seed=20261203):
    """Whole-run configurations drawn from a fixed seed: every lattice shape the sweep kernels
    specialise (cube sides 2-16, rings of 16-256 sites), both layouts, uneven populations and
    schedules of uneven beta steps reaching every first-look regime."""
    g = np.random.default_rng(seed)
    out = []
    for c in range(n):
        if g.random() < 0.7:
            dim, L = 3, int(g.choice([2, 4, 6, 8, 10, 12, 14, 16]))
        else:
            dim, L = 1, int(g.choice([16, 64, 100, 256]))
        layout = str(g.choice(["u8", "bits64"]))
        R0 = int(g.integers(20, 600))
        nT = int(g.integers(3, 7))
        ns = int(g.integers(1, 5))
        steps = g.uniform(0.05, 1.0, nT - 1)
        betas = [0.0] + list(np.cumsum(steps / steps.sum() * g.uniform(0.5, 4.0)))
        out.append((c, dim, L, layout, R0, [float(b) for b in betas], ns, int(g.integers(1, 1 << 30))))
    return out


@pytest.mark.parametrize("c,dim,L,layout,R0,betas,ns,seed", seeded_run_configs(20))
def test_seeded_random_runs_match_oracle(c, dim, L, layout, R0, betas, ns, seed):
    note(f"seeded run {c}: dim={dim} L={L} {layout} R0={R0} nT={len(betas)} ns={ns} seed={seed}")
    nT = len(betas)
    dseed = seed ^ 0x5A5A
    run = pa.Run(dim, L, R0, seed, dseed, n_records=nT, layout=layout, device=DEV)
    run.init()
    sched = pa.Schedule(betas, ns, run.n_bins, device=DEV)
    for k in range(1, nT):
        st = sched.step(k)
        run.resample(st)
        run.sweep(st)
        pa.measure([run])
    J = o.couplings(dim, L, dseed)
    st_o, rec_o, s_o, E_o = o.run(dim, L, J, seed, R0, betas, ns, capacity=run.capacity)
    assert st_o == 0
    code, flags = run.status()
    assert code == pa.PA_OK and flags == 0
    rec = run.records()
    for k in range(nT):
        assert rec[k, 4] == rec_o[k, 1], f"R differs at k={k}"
        assert close(rec[k, 1], rec_o[k, 2]) and close(rec[k, 2], rec_o[k, 3]), f"ln Q or -beta F differs at k={k}"
        if k > 0:
            assert rec[k, 6] == rec_o[k, 4], f"E mean differs at k={k}"
    s, E = run.population()
    assert np.array_equal(s, s_o) and np.array_equal(E, E_o)


@pytest.mark.parametrize("dim,L,layout", [(1, 64, "u8"), (3, 8, "bits64"), (3, 6, "u8"), (3, 16, "bits64")])
def test_overlap_parity(dim, L, layout):
    note(f"overlap dim={dim} L={L} {layout}")
    nT, ns = 6, 3
    betas = [1.5 * k / (nT - 1) for k in range(nT)]
    RA, RB = 330, 270
    a = pa.Run(dim, L, RA, 101, 9, n_records=nT, layout=layout, device=DEV).init()
    b = pa.Run(dim, L, RB, 202, 9, n_records=nT, layout=layout, device=DEV).init()
    sa = pa.Schedule(betas, ns, a.n_bins, device=DEV)
    for k in range(1, nT):
        for run in (a, b):
            st = sa.step(k)
            run.resample(st)
            run.sweep(st)
        pa.measure([a, b], [1, 0])
    J = o.couplings(dim, L, 9)
    _, rec_a, s_a, _ = o.run(dim, L, J, 101, RA, betas, ns, capacity=a.capacity)
    _, rec_b, s_b, _ = o.run(dim, L, J, 202, RB, betas, ns, capacity=b.capacity)
    h, P = o.overlap_hist(o.num_sites(dim, L), s_a, s_b)
    q2, q4, g = o.overlap_stats(o.num_sites(dim, L), h)
    for run in (a, b):
        rec = run.records()[nT - 1]
        assert rec[12] == P
        assert close(rec[9], q2) and close(rec[10], q4) and close(rec[11], g)


def test_overlap_long_chain_counts_in_global_memory():
    # a chain of 9000 sites: its N + 1 overlap bins exceed the bit-packed overlap kernel's LDS
    # histogram, which then counts in global memory; the overlap of the two initial populations
    # against the oracle's
    N, RA, RB = 9000, 300, 250
    note(f"overlap long chain N={N}")
    a = pa.Run(1, N, RA, 101, 9, n_records=2, layout="bits64", device=DEV).init()
    b = pa.Run(1, N, RB, 202, 9, n_records=2, layout="bits64", device=DEV).init()
    pa.measure([a, b], [1, 0])
    J = o.couplings(1, N, 9)
    s_a, _ = o.init_population(1, N, J, 101, RA)
    s_b, _ = o.init_population(1, N, J, 202, RB)
    h, P = o.overlap_hist(N, s_a, s_b)
    q2, q4, g = o.overlap_stats(N, h)
    for run in (a, b):
        rec = run.records()[0]
        assert rec[12] == P
        assert close(rec[9], q2) and close(rec[10], q4) and close(rec[11], g)


def test_capacity_and_extinction_flags_leave_state_unchanged():
    dim, L, R0 = 3, 6, 200
    note("capacity overflow")
    run = make_run(dim, L, R0, "bits64", capacity=256)
    s0, E0 = run.population()
    rec0 = run.records()
    sched = pa.Schedule([0.0, 0.1], 1, run.n_bins, device=DEV, R_targets=[0, 5000.0])
    run.resample(sched.step(1))
    code, flags = run.status()
    assert code == pa.PA_ERR_CAPACITY and flags & pa.PA_FLAG_CAPACITY
    info = run.query()
    assert info.R == R0 and info.k == 0 and info.R_new > 256
    s1, E1 = run.population()
    assert np.array_equal(s0, s1) and np.array_equal(E0, E1)
    assert np.array_equal(run.records(), rec0), "a refused step must not write its record"
    # sticky: later calls do nothing
    run.sweep(sched.step(1))
    s2, _ = run.population()
    assert np.array_equal(s0, s2)
    note("extinction")
    run = make_run(dim, L, R0, "u8")
    sched = pa.Schedule([0.0, 0.1], 1, run.n_bins, device=DEV, R_targets=[0, 1e-9])
    rec0 = run.records()
    run.resample(sched.step(1))
    code, flags = run.status()
    assert code == pa.PA_ERR_EXTINCT and flags & pa.PA_FLAG_EXTINCT
    assert run.query().R == R0
    assert np.array_equal(run.records(), rec0)


def test_bad_step_rejected_on_host():
    run = make_run(3, 4, 64, "u8")
    with pytest.raises(pa.PAError):
        pa.Schedule([0.5, 0.2], 1, run.n_bins, device=DEV)  # no weight table for a negative step
    sched = pa.Schedule([0.2, 0.5], 1, run.n_bins, device=DEV)
    st = sched.step(1)
    st.beta_from, st.beta_to = 0.5, 0.2  # beta decreases
    with pytest.raises(pa.PAError) as e:
        run.resample(st)
    assert e.value.code == pa.PA_ERR_ARG
    st = sched.step(1)
    st.k = 0
    with pytest.raises(pa.PAError):
        run.resample(st)
    assert run.query().k == 0 and run.status()[0] == pa.PA_OK


def test_device_weighted_average_matches_host():
    note("device weighted average")
    rng = np.random.default_rng(5)
    n_sets, M, n_obs = 3, 17, 2
    x = rng.normal(size=(n_sets, M)) + 500
    A = rng.normal(size=(n_sets, M, n_obs))
    R = rng.uniform(1e4, 1e5, (n_sets, M))
    xd = torch.tensor(x, device=DEV)
    Ad = torch.tensor(A, device=DEV)
    Rd = torch.tensor(R, device=DEV)
    out = torch.zeros((n_sets, n_obs + 3), dtype=torch.float64, device=DEV)
    pa.check(pa.lib().pa_weighted_average_dev(n_sets, M, xd.data_ptr(), Rd.data_ptr(), Ad.data_ptr(), n_obs,
                                              out.data_ptr(), torch.cuda.current_stream().cuda_stream))
    res = out.cpu().numpy()
    for s_ in range(n_sets):
        ref = o.weighted_average(x[s_], A[s_], R[s_])
        assert np.allclose(res[s_, :n_obs], ref["A_bar"], rtol=1e-12)
        assert close(res[s_, n_obs], ref["minus_betaF_bar"])
        assert close(res[s_, n_obs + 1], ref["var"]) and close(res[s_, n_obs + 2], ref["mean"])


def test_device_overlap_average_matches_oracle():
    # pair-weighted overlap observables and the Binder ratio (Sec. IV, eqs. pqs and omegaprime) on
    # seeded inputs, with and without target sizes, against the oracle
    from tests import inputs

    for n_sets, n_pairs, use_R in ((3, 50, True), (5, 1, False), (1, 7, False)):
        note(f"device overlap average sets={n_sets} pairs={n_pairs} R={use_R}")
        x, R, Q = inputs.overlap_pair_sets(17 + n_pairs, n_sets, n_pairs)
        out = torch.zeros((n_sets, 4), dtype=torch.float64, device=DEV)
        xd, Rd, Qd = (torch.tensor(a, device=DEV) for a in (x, R, Q))
        pa.check(pa.lib().pa_overlap_average_dev(n_sets, n_pairs, xd.data_ptr(), Rd.data_ptr() if use_R else None,
                                                 Qd.data_ptr(), out.data_ptr(),
                                                 torch.cuda.current_stream().cuda_stream))
        res = out.cpu().numpy()
        for s_ in range(n_sets):
            ref = o.overlap_average(x[s_], Q[s_], R[s_] if use_R else None)
            for v in range(4):
                assert close(res[s_, v], ref[v]), f"set {s_} value {v}: {res[s_, v]} vs {ref[v]}"
    assert pa.lib().pa_overlap_average_dev(1, 0, xd.data_ptr(), None, Qd.data_ptr(), out.data_ptr(), None) == pa.PA_ERR_ARG


def test_full_size_c4_sampled():
    # the throughput configuration at its real size: L = 16, R0 = 1e6, bit-packed.  The oracle sweeps
    # sampled replicas one by one from its own initial spins (a replica's sweep depends only on its
    # own spins and index); the resampling of 1e6 energies is checked through properties that hold
    # at any size (conservation, the scan, the gather, the mean population size)
    dim, L, R0 = 3, 16, 1_000_000
    seed, dseed = 77, 1
    note("C4 full size: init")
    run = pa.Run(dim, L, R0, seed, dseed, n_records=4, layout="bits64", device=DEV)
    run.init()
    J = o.couplings(dim, L, dseed)
    assert np.array_equal(run.couplings(), J)
    sample = np.array([0, 1, 63, 64, 65, 4097, 123457, 500000, 999935, 999936, R0 - 2, R0 - 1])
    s = run.replica_spins(sample)
    E = run.energies()
    assert len(E) == R0
    init_o = [o.init_replicas(dim, L, J, seed, int(r), 1) for r in sample]
    for n, r in enumerate(sample):
        assert np.array_equal(s[n], init_o[n][0][0]) and E[r] == init_o[n][1][0]
    # ten sweeps at beta = 1, 2 and 4 in turn: the three first-look regimes of the sweep kernel
    # (general thresholds; only dE = 4 with a non-zero top; all tops zero)
    betas = [0.0, 4.0, 4.0 + 1.0 / 60.0]
    sched = pa.Schedule(betas, 10, run.n_bins, device=DEV)
    for t0, beta in ((120, 1.0), (130, 2.0), (140, 4.0)):
        note(f"C4 full size: sweep beta={beta}")
        st = sched.step(1)
        st.beta_to = beta
        st.t0 = t0
        run.sweep(st)
        s1 = run.replica_spins(sample)
        E1 = run.energies()
        for n, r in enumerate(sample):
            so, Eo = init_o[n]
            o.sweep_replicas(dim, L, J, seed, beta, int(r), so, Eo, t0, 10)
            assert np.array_equal(s1[n], so[0]) and E1[r] == Eo[0], f"replica {r} at beta={beta}"
    note("C4 full size: resample 4.0 -> 4.0 + 1/60")
    old_buf = run.query().cur
    run.resample(sched.step(2))
    code, _ = run.status()
    assert code == pa.PA_OK
    c, off = run.counts_offsets(R0)
    E2 = run.energies()
    assert np.all(c >= 0) and off[0] == 0 and np.array_equal(np.diff(off), c) and off[-1] == len(E2)
    assert abs(len(E2) - R0) < 6 * math.sqrt(R0)           # E[sum of copies] = R_target
    rec = run.records()[2]
    assert rec[4] == len(E2) and rec[5] == E1.min()
    dbeta = betas[2] - betas[1]
    assert close(rec[1], -dbeta * rec[5] + math.log(rec[3]) - math.log(R0))
    src = np.searchsorted(off, np.arange(len(E2)), side="right") - 1
    assert np.array_equal(E2, E1[src])
    pick = np.unique(np.concatenate([np.arange(0, len(E2), 99991), [len(E2) - 1]]))
    new_s = run.replica_spins(pick)
    old_s = run.replica_spins(src[pick], buf=old_buf)
    assert np.array_equal(new_s, old_s)


@pytest.mark.parametrize("layout", ["u8", "bits64"])
def test_full_size_c2(layout):
    # the L = 8 cube at its real size, R0 = 5e4: resampling from the seeded initial population
    # (every copy number, S, ln Q and the gathered energies against the oracle), then 10 sweeps at
    # beta = 0.05 checked on sampled replicas, whose parents come from the oracle's copy numbers
    dim, L, R0, seed, dseed, db = 3, 8, 50_000, 91, 2, 0.05
    note(f"C2 full size {layout}: init + resample")
    run = pa.Run(dim, L, R0, seed, dseed, n_records=4, layout=layout, device=DEV).init()
    J = o.couplings(dim, L, dseed)
    s0_o, E0_o = o.init_replicas(dim, L, J, seed, 0, R0)
    sched = pa.Schedule([0.0, db], 10, run.n_bins, device=DEV)
    st = sched.step(1)
    run.resample(st)
    code, _ = run.status()
    assert code == pa.PA_OK
    stc, counts_o, S_o, lnQ_o, Elo_o = o.copy_numbers(seed, 1, 0.0, db, R0, E0_o)
    assert stc == 0
    c, off = run.counts_offsets(R0)
    assert np.array_equal(c, counts_o)
    rec = run.records()[1]
    assert rec[3] == S_o and rec[5] == Elo_o and close(rec[1], lnQ_o)
    src = np.repeat(np.arange(R0), counts_o)
    assert np.array_equal(run.energies(), E0_o[src])
    note(f"C2 full size {layout}: sweep")
    run.sweep(st)
    Rn = len(src)
    sample = np.unique(np.array([0, 1, 63, 64, 127, 128, Rn // 3, Rn // 2, Rn - 65, Rn - 64, Rn - 1]))
    s1 = run.replica_spins(sample)
    E1 = run.energies()
    for n, r in enumerate(sample):
        so = s0_o[src[r]][None, :].copy()          # a copy: the oracle sweeps in place
        Eo = np.array([E0_o[src[r]]], dtype=np.int32)
        o.sweep_replicas(dim, L, J, seed, db, int(r), so, Eo, 0, 10)
        assert np.array_equal(s1[n], so[0]) and E1[r] == Eo[0], f"replica {r}"
