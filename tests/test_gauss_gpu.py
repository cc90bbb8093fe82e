"""Gaussian couplings (the model of Sec. IV) on the GPU against the oracle: couplings, initial
populations, sweeps, copy numbers and whole runs bit for bit (spins, FP64 energies, copy
numbers, population sizes); ln Q, -beta F~ and the energy moments within 1e-12."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import oracle as o

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1006_0252_amd import pa  # noqa: E402

DEV = "cuda:0"


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def gauss_run(dim, L, R0, seed, ds, n_records=4, capacity=None):
    return pa.Run(dim, L, R0, seed, ds, n_records, capacity=capacity, layout="u8", device=DEV,
                  couplings="gauss").init()


@pytest.mark.parametrize("dim,L", [(1, 16), (3, 4), (3, 6)])
def test_couplings_and_initial_population(dim, L):
    note(f"gauss init dim={dim} L={L}")
    run = gauss_run(dim, L, 200, 11, 3)
    J = run.couplings()
    assert np.array_equal(J, o.couplings_gauss(dim, L, 3))
    s, E = run.population()
    s_o, E_o = o.init_replicas_gauss(dim, L, J, 11, 0, 200)
    assert np.array_equal(s, s_o) and np.array_equal(E, E_o)


# cubes of side 4 and 8 and chains of 16 k sites take the tabled kernel (ragged last tiles, several
# blocks; a single replica; chains of an odd and an even number of 16-site segments); side 6 and the
# chain of 40 take the per-replica kernel
SWEEP_CASES = [(1, 16, 130, 0.7), (3, 4, 300, 0.7), (3, 4, 77, 3.0), (3, 6, 65, 0.0), (3, 6, 130, 1.3),
               (3, 8, 1000, 0.7), (3, 8, 2100, 2.5), (3, 8, 64, 0.0), (1, 256, 300, 5.0), (1, 40, 90, 1.0),
               (3, 8, 1, 1.0), (3, 4, 1, 1.0), (1, 48, 129, 0.9), (1, 32, 63, 0.9), (1, 1024, 70, 1.5)]


@pytest.mark.parametrize("dim,L,R,beta", SWEEP_CASES)
def test_sweep_matches_oracle(dim, L, R, beta):
    note(f"gauss sweep dim={dim} L={L} R={R} beta={beta}")
    run = gauss_run(dim, L, R, 5, 9)
    sched = pa.Schedule([0.0, beta], 3, run.n_bins, device=DEV)
    st = sched.step(1)
    run.sweep(st)
    code, _ = run.status()
    assert code == pa.PA_OK
    s, E = run.population()
    J = o.couplings_gauss(dim, L, 9)
    s_o, E_o = o.init_replicas_gauss(dim, L, J, 5, 0, R)
    o.sweep_replicas_gauss(dim, L, J, 5, beta, 0, s_o, E_o, 0, 3)
    assert np.array_equal(s, s_o), np.nonzero((s != s_o).any(axis=1))[0][:10]
    assert np.array_equal(E, E_o)


# beta 0.3 -> 1.1: one replica takes 687 of the copies (ten Poisson(64) blocks); 0.3 -> 0.5: copy
# numbers up to 87, 18 of them from Poisson(2^m >= 16) draws (the copies the whole wave draws)
@pytest.mark.parametrize("b1", [1.1, 0.5])
def test_copy_numbers_match_oracle(b1):
    note(f"gauss resample 0.3 -> {b1}")
    R = 700
    run = gauss_run(3, 4, R, 8, 2, capacity=1536)
    run.sweep(pa.Schedule([0.0, 0.3], 2, run.n_bins, device=DEV).step(1))
    run.resample(pa.Schedule([0.3, b1], 2, run.n_bins, device=DEV).step(1))
    code, _ = run.status()
    assert code == pa.PA_OK
    J = o.couplings_gauss(3, 4, 2)
    s_o, E_o = o.init_replicas_gauss(3, 4, J, 8, 0, R)
    o.sweep_replicas_gauss(3, 4, J, 8, 0.3, 0, s_o, E_o, 0, 2)
    st, counts_o, S_o, lnQ_o, E_lo_o = o.copy_numbers_gauss(8, 1, 0.3, b1, float(R), E_o)
    assert st == 0
    c, _ = run.counts_offsets(R)
    assert np.array_equal(c, counts_o)
    rec = run.records()[1]
    assert rec[3] == S_o and rec[5] == E_lo_o and rec[4] == counts_o.sum()
    assert abs(rec[1] - lnQ_o) <= 1e-12 * max(1.0, abs(lnQ_o))
    s, E = run.population()
    keep = np.repeat(np.arange(R), counts_o)
    assert np.array_equal(s, s_o[keep]) and np.array_equal(E, E_o[keep])


@pytest.mark.parametrize("dim,L,R0,nT", [(3, 4, 200, 7), (1, 32, 300, 9), (3, 8, 500, 9), (1, 256, 400, 11)])
def test_whole_run_matches_oracle(dim, L, R0, nT):
    note(f"gauss run dim={dim} L={L} R0={R0}")
    betas = [2.5 * k / (nT - 1) for k in range(nT)]
    ns = 3
    cap = int(np.ceil(R0 * 1.6 / 64)) * 64
    run = gauss_run(dim, L, R0, 21, 4, n_records=nT, capacity=cap)
    sched = pa.Schedule(betas, ns, run.n_bins, device=DEV)
    for k in range(1, nT):
        st = sched.step(k)
        run.resample(st)
        run.sweep(st)
        pa.measure([run])
    code, _ = run.status()
    assert code == pa.PA_OK
    J = o.couplings_gauss(dim, L, 4)
    st_o, rec_o, s_o, E_o = o.run_gauss(dim, L, J, 21, R0, betas, ns, capacity=cap)
    assert st_o == 0
    s, E = run.population()
    assert np.array_equal(s, s_o) and np.array_equal(E, E_o)
    rec = run.records()
    assert np.array_equal(rec[:, 4], rec_o[:, 1])
    for k in range(nT):
        assert abs(rec[k, 1] - rec_o[k, 2]) <= 1e-12 * max(1.0, abs(rec_o[k, 2])), k
        assert abs(rec[k, 2] - rec_o[k, 3]) <= 1e-12 * max(1.0, abs(rec_o[k, 3])), k
        if k > 0:
            # FP64 sums over the population in another order: rounding only
            assert abs(rec[k, 6] - rec_o[k, 4]) <= 1e-12 * max(1.0, abs(rec_o[k, 4])), k
            assert abs(rec[k, 7] - rec_o[k, 5]) <= 1e-12 * max(1.0, abs(rec_o[k, 5])), k
            assert abs(rec[k, 8] - rec_o[k, 6]) <= 1e-9 * max(1.0, abs(rec_o[k, 6])), k
    fe = torch.zeros(1, dtype=torch.float64, device=DEV)
    run.free_energy(fe)
    assert abs(fe.item() - rec_o[-1, 3]) <= 1e-12 * abs(rec_o[-1, 3])


def seeded_gauss_configs(n, seed=1203):
    """Whole Gaussian runs drawn from a fixed seed: the tabled shapes (cube sides 4 and 8, chains of
    one, two, three and sixteen 16-site segments) and the per-replica ones (side 6, a chain of 40),
    uneven populations and schedules of uneven beta steps."""
    g = np.random.default_rng(seed)
    shapes = [(3, 4), (3, 8), (3, 6), (1, 16), (1, 32), (1, 48), (1, 256), (1, 40)]
    out = []
    for c in range(n):
        dim, L = shapes[int(g.integers(len(shapes)))]
        R0 = int(g.integers(20, 500))
        nT = int(g.integers(3, 7))
        steps = g.uniform(0.05, 1.0, nT - 1)
        betas = [0.0] + [float(b) for b in np.cumsum(steps / steps.sum() * g.uniform(0.5, 3.0))]
        out.append((c, dim, L, R0, betas, int(g.integers(1, 4)), int(g.integers(1, 1 << 30))))
    return out


@pytest.mark.parametrize("c,dim,L,R0,betas,ns,seed", seeded_gauss_configs(12))
def test_seeded_random_gauss_runs_match_oracle(c, dim, L, R0, betas, ns, seed):
    note(f"seeded gauss run {c}: dim={dim} L={L} R0={R0} nT={len(betas)} ns={ns} seed={seed}")
    nT = len(betas)
    ds = seed ^ 0x3C3C
    cap = int(np.ceil(R0 * 1.6 / 64)) * 64
    run = gauss_run(dim, L, R0, seed, ds, n_records=nT, capacity=cap)
    sched = pa.Schedule(betas, ns, run.n_bins, device=DEV)
    for k in range(1, nT):
        st = sched.step(k)
        run.resample(st)
        run.sweep(st)
        pa.measure([run])
    code, _ = run.status()
    assert code == pa.PA_OK
    J = o.couplings_gauss(dim, L, ds)
    st_o, rec_o, s_o, E_o = o.run_gauss(dim, L, J, seed, R0, betas, ns, capacity=cap)
    assert st_o == 0
    s, E = run.population()
    assert np.array_equal(s, s_o) and np.array_equal(E, E_o)
    rec = run.records()
    assert np.array_equal(rec[:, 4], rec_o[:, 1])
    for k in range(nT):
        assert abs(rec[k, 1] - rec_o[k, 2]) <= 1e-12 * max(1.0, abs(rec_o[k, 2])), k
        assert abs(rec[k, 2] - rec_o[k, 3]) <= 1e-12 * max(1.0, abs(rec_o[k, 3])), k


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle(graph):
    # one launch per kernel over four consecutive runs (two realizations, pairs (0,1) and (2,3)),
    # stepped eagerly or replayed once from a captured graph
    note(f"gauss batch of 4, L=8, graph={graph}")
    specs = [dict(dim=3, L=8, R0=R0, seed=40 + i, disorder_seed=1 + (i >> 1), couplings="gauss")
             for i, R0 in enumerate((300, 700, 1000, 64))]
    nT, ns = 6, 2
    betas = [3.0 * k / (nT - 1) for k in range(nT)]
    batch = pa.Batch(specs, nT, layout="u8", device=DEV)
    batch.init()
    sched = pa.Schedule(betas, ns, batch.runs[0].n_bins, device=DEV)
    if graph:
        g = batch.capture(sched, range(1, nT), pairs=True)
        g.launch()
    else:
        for k in range(1, nT):
            batch.step(sched, k, pairs=True)
    code, flags = batch.status()
    assert code == pa.PA_OK and not flags.any()
    pops = []
    for sp, run in zip(specs, batch.runs):
        J = o.couplings_gauss(3, 8, sp["disorder_seed"])
        st_o, rec_o, s_o, E_o = o.run_gauss(3, 8, J, sp["seed"], sp["R0"], betas, ns, capacity=run.capacity)
        assert st_o == 0
        s, E = run.population()
        assert np.array_equal(s, s_o) and np.array_equal(E, E_o)
        rec = run.records()
        assert np.array_equal(rec[:, 4], rec_o[:, 1])
        for k in range(1, nT):
            assert abs(rec[k, 2] - rec_o[k, 3]) <= 1e-12 * max(1.0, abs(rec_o[k, 3]))
            assert abs(rec[k, 6] - rec_o[k, 4]) <= 1e-12 * max(1.0, abs(rec_o[k, 4]))
        pops.append(s_o)
    for r, run in enumerate(batch.runs):
        h, P = o.overlap_hist(512, pops[r], pops[r ^ 1])
        q2, q4, gm = o.overlap_stats(512, h)
        rec = run.records()[nT - 1]
        assert rec[12] == P
        for got, want in zip(rec[9:12], (q2, q4, gm)):
            assert abs(got - want) <= 1e-12 * max(1.0, abs(want))


def test_ensemble_sizes_match_oracle():
    # the 3D ensemble's sizes (R = 2000, 100 sweeps per step, eight runs in one launch so that runs
    # are spread over the XCDs) for a start at T = 2 and five steps: about 10^9 attempts per run, so
    # that the rare first-look ties (one attempt in 2^16) are decided exactly many times over
    from paper_1006_0252_amd import gauss3d

    M, R0, ns, K = 8, 2000, 100, 5
    betas = gauss3d.schedule(100)
    note(f"gauss ensemble sizes: {M} runs, R0={R0}, {ns} sweeps, {K} steps")
    specs = [dict(dim=3, L=8, R0=R0, seed=1 + i, disorder_seed=1, couplings="gauss") for i in range(M)]
    batch = pa.Batch(specs, len(betas), layout="u8", device=DEV, capacity_factor=1.25)
    batch.init()
    sched = pa.Schedule(betas, ns, batch.runs[0].n_bins, device=DEV)
    batch.sweep(sched.start_sweeps())
    for k in range(1, K + 1):
        st = sched.step(k)
        batch.resample(st)
        batch.sweep(st)
    code, flags = batch.status()
    assert code == pa.PA_OK and not flags.any()
    J = o.couplings_gauss(3, 8, 1)
    for r in (0, 5):
        s_o, E_o = o.init_replicas_gauss(3, 8, J, 1 + r, 0, R0)
        o.sweep_replicas_gauss(3, 8, J, 1 + r, betas[0], 0, s_o, E_o, (len(betas) - 1) * ns, ns)
        rec = batch.runs[r].records()
        for k in range(1, K + 1):
            st_o, c, S, lnQ, _ = o.copy_numbers_gauss(1 + r, k, betas[k - 1], betas[k], float(R0), E_o)
            assert st_o == 0
            keep = np.repeat(np.arange(len(E_o)), c)
            s_o, E_o = np.ascontiguousarray(s_o[keep]), np.ascontiguousarray(E_o[keep])
            o.sweep_replicas_gauss(3, 8, J, 1 + r, betas[k], 0, s_o, E_o, (k - 1) * ns, ns)
            assert abs(rec[k][1] - lnQ) <= 1e-12 * max(1.0, abs(lnQ)), (r, k)
        s, E = batch.runs[r].population()
        assert np.array_equal(s, s_o) and np.array_equal(E, E_o), r


def test_overlap_of_gaussian_pair():
    note("gauss overlap pair")
    RA, RB = 150, 170
    a = gauss_run(3, 4, RA, 31, 6)
    b = gauss_run(3, 4, RB, 32, 6)
    sched = pa.Schedule([0.0, 1.5], 2, a.n_bins, device=DEV)
    for r in (a, b):
        r.sweep(sched.step(1))
    pa.measure([a, b], [1, 0])
    J = o.couplings_gauss(3, 4, 6)
    pops = []
    for seed, R in ((31, RA), (32, RB)):
        s_o, E_o = o.init_replicas_gauss(3, 4, J, seed, 0, R)
        o.sweep_replicas_gauss(3, 4, J, seed, 1.5, 0, s_o, E_o, 0, 2)
        pops.append(s_o)
    h, P = o.overlap_hist(64, pops[0], pops[1])
    q2, q4, g = o.overlap_stats(64, h)
    for run in (a, b):
        rec = run.records()[0]
        assert rec[12] == P
        for got, want in zip(rec[9:12], (q2, q4, g)):
            assert abs(got - want) <= 1e-12 * max(1.0, abs(want))


def test_gaussian_rejected_where_unsupported():
    r = pa.pa_sizes()
    assert pa.lib().pa_buffer_sizes(3, 4, pa.PA_BITS64, pa.PA_GAUSS, 64, 4, ctypes.byref(r)) == pa.PA_ERR_ARG
    run = gauss_run(3, 4, 64, 1, 1)
    t = np.array([0.2])
    out = torch.zeros(1, dtype=torch.float64, device=DEV)
    assert pa.lib().pa_rho_steps(ctypes.byref(run.desc), 1, pa._np(t), 1, 1.0, 1, out.data_ptr()) == pa.PA_ERR_ARG


def test_start_sweeps_then_steps_match_oracle():
    # a schedule that starts at T = 2: the random start is swept there first, with sweep indices
    # after those of the steps, then annealed
    note("gauss start at T=2")
    betas = 1.0 / np.linspace(2.0, 0.5, 5)
    ns, R0 = 3, 400
    run = gauss_run(3, 8, R0, 77, 5, n_records=len(betas), capacity=768)
    sched = pa.Schedule(betas, ns, run.n_bins, device=DEV)
    run.sweep(sched.start_sweeps())
    J = o.couplings_gauss(3, 8, 5)
    s_o, E_o = o.init_replicas_gauss(3, 8, J, 77, 0, R0)
    o.sweep_replicas_gauss(3, 8, J, 77, betas[0], 0, s_o, E_o, (len(betas) - 1) * ns, ns)
    s, E = run.population()
    assert np.array_equal(s, s_o) and np.array_equal(E, E_o)
    for k in range(1, len(betas)):
        st = sched.step(k)
        run.resample(st)
        run.sweep(st)
    code, _ = run.status()
    assert code == pa.PA_OK
    for k in range(1, len(betas)):
        st_o, c, S, lnQ, _ = o.copy_numbers_gauss(77, k, betas[k - 1], betas[k], float(R0), E_o)
        assert st_o == 0
        keep = np.repeat(np.arange(len(E_o)), c)
        s_o, E_o = np.ascontiguousarray(s_o[keep]), np.ascontiguousarray(E_o[keep])
        o.sweep_replicas_gauss(3, 8, J, 77, betas[k], 0, s_o, E_o, (k - 1) * ns, ns)
        assert abs(run.records()[k][1] - lnQ) <= 1e-12 * max(1.0, abs(lnQ))
    s, E = run.population()
    assert np.array_equal(s, s_o) and np.array_equal(E, E_o)


def test_ensemble_harness_small():
    # the 3D ensemble driver on a small case: 4 runs (2 pairs), 5 temperatures from T = 2 to 0.5;
    # its free energies are the sums of the recorded ln Q, its attempts the swept populations
    from paper_1006_0252_amd import gauss3d

    note("gauss ensemble harness, small")
    r = gauss3d.run(M=4, R=300, n_temps=5, n_sweeps=3)
    assert r["n_steps"] == 4 and len(r["sweep_ms"]) == 5
    assert r["attempts"] == float(r["attempts_per_sweep_step"].sum())
    assert r["attempts_per_sweep_step"][0] == 4 * 300 * 512 * 3
    assert r["var_betaF"] >= 0 and np.isfinite(r["minus_betaF_bar"])
    assert r["minus_betaF_bar"] >= r["mean_minus_betaF"] - 1e-9   # log-mean-exp >= mean
    assert 0.0 <= r["gamma_bar"] <= 1.0


def test_ensemble_harness_stepped_targets():
    # R_beta stepped up at the third temperature: the start has R_targets[0] replicas, the work
    # counts the swept populations, and the populations follow the new target
    from paper_1006_0252_amd import gauss3d

    note("gauss ensemble harness, stepped targets")
    Rt = [200.0, 200.0, 600.0, 600.0, 600.0]
    r = gauss3d.run(M=4, n_temps=5, n_sweeps=2, R_targets=Rt)
    assert r["attempts_per_sweep_step"][0] == 4 * 200 * 512 * 2
    assert np.all(np.abs(r["R_final"] - 600) < 6 * np.sqrt(600))
    assert len(r["var_profile"]) == 4 and np.all(r["var_profile"] >= 0)
