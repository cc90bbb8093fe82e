"""Batched runs (one launch per kernel for many runs of uneven size), HIP graph capture of
a schedule, and the persistent sweep's schedule options: all must give exactly the sample
that the runs give one by one, and the oracle's sample."""
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


def specs_mixed():
    # pairs (0,1), (2,3), ... share the lattice and couplings (overlap partners)
    Ls = [6, 6, 10, 10, 8, 8, 16, 16, 12, 12, 4, 4]
    R0s = [300, 21, 130, 200, 257, 64, 70, 130, 95, 66, 64, 100]
    return [dict(dim=3, L=L, R0=R, seed=100 + i, disorder_seed=7 + i // 2) for i, (L, R) in enumerate(zip(Ls, R0s))]


def solo_runs(specs, n_records, layout, caps):
    runs = []
    for sp, cap in zip(specs, caps):
        r = pa.Run(sp["dim"], sp["L"], sp["R0"], sp["seed"], sp["disorder_seed"], n_records, capacity=cap,
                   layout=layout, device=DEV)
        r.init()
        runs.append(r)
    return runs


def compare(batch, solos, k):
    for i, (b, s) in enumerate(zip(batch.runs, solos)):
        sb, Eb = b.population()
        ss, Es = s.population()
        assert np.array_equal(sb, ss) and np.array_equal(Eb, Es), f"run {i} population differs after step {k}"
        rb, rs = b.records(), s.records()
        assert np.array_equal(rb, rs), f"run {i} records differ after step {k}"


@pytest.mark.parametrize("layout", ["bits64", "u8"])
def test_batch_equals_solo_mixed_sizes(layout):
    specs = specs_mixed()
    nT, ns = 9, 3
    betas = [3.5 * k / (nT - 1) for k in range(nT)]  # crosses all three first-look regimes
    note(f"batch vs solo {layout}")
    batch = pa.Batch(specs, nT, layout=layout, device=DEV).init()
    solos = solo_runs(specs, nT, layout, [r.capacity for r in batch.runs])
    n_bins = max(r.n_bins for r in batch.runs)
    sched = pa.Schedule(betas, ns, n_bins, device=DEV)
    for k in range(1, nT):
        batch.step(sched, k, pairs=True)
        st = sched.step(k)
        for i, r in enumerate(solos):
            r.resample(st)
            r.sweep(st)
        pa.measure(solos, [i ^ 1 for i in range(len(solos))])
        if k in (1, 4, nT - 1):
            compare(batch, solos, k)
    code, flags = batch.status()
    assert code == pa.PA_OK and not flags.any()
    fe = torch.zeros(len(specs), dtype=torch.float64, device=DEV)
    batch.free_energy(fe)
    rec = batch.records()
    assert np.allclose(fe.cpu().numpy(), rec[:, -1, 2], rtol=1e-15)


def seeded_batches(n, seed=4242):
    """Batches drawn from a fixed seed: 2-10 runs in pairs (overlap partners share the lattice and
    couplings), mixed cube sides 2-16, populations of 1-400 replicas, both layouts."""
    g = np.random.default_rng(seed)
    out = []
    for c in range(n):
        n_pairs = int(g.integers(1, 6))
        specs = []
        for p in range(n_pairs):
            L = int(g.choice([2, 4, 6, 8, 10, 12, 14, 16]))
            for h in range(2):
                specs.append(dict(dim=3, L=L, R0=int(g.integers(1, 400)), seed=int(g.integers(1, 1 << 30)),
                                  disorder_seed=int(g.integers(1, 1 << 30)) if h == 0 else None))
            specs[-1]["disorder_seed"] = specs[-2]["disorder_seed"]
        out.append((c, str(g.choice(["bits64", "u8"])), specs))
    return out


@pytest.mark.parametrize("c,layout,specs", seeded_batches(6))
def test_seeded_batches_equal_solo(c, layout, specs):
    nT, ns = 5, 2
    betas = [3.0 * k / (nT - 1) for k in range(nT)]
    note(f"seeded batch {c}: {layout}, L {[sp['L'] for sp in specs]}, R0 {[sp['R0'] for sp in specs]}")
    batch = pa.Batch(specs, nT, layout=layout, device=DEV).init()
    solos = solo_runs(specs, nT, layout, [r.capacity for r in batch.runs])
    n_bins = max(r.n_bins for r in batch.runs)
    sched = pa.Schedule(betas, ns, n_bins, device=DEV)
    for k in range(1, nT):
        batch.step(sched, k, pairs=True)
        st = sched.step(k)
        for r in solos:
            r.resample(st)
            r.sweep(st)
        pa.measure(solos, [i ^ 1 for i in range(len(solos))])
    code, flags = batch.status()
    solo_flags = [r.status() for r in solos]
    if code == pa.PA_OK:
        assert all(sc == pa.PA_OK for sc, _ in solo_flags)
    compare(batch, solos, nT - 1)


def test_batch_matches_oracle():
    specs = [dict(dim=3, L=6, R0=150, seed=31, disorder_seed=4), dict(dim=3, L=10, R0=90, seed=32, disorder_seed=5),
             dict(dim=3, L=8, R0=130, seed=33, disorder_seed=4)]
    nT, ns = 6, 4
    betas = [2.0 * k / (nT - 1) for k in range(nT)]
    note("batch vs oracle")
    batch = pa.Batch(specs, nT, layout="bits64", device=DEV).init()
    sched = pa.Schedule(betas, ns, max(r.n_bins for r in batch.runs), device=DEV)
    for k in range(1, nT):
        batch.step(sched, k)
    for sp, run in zip(specs, batch.runs):
        J = o.couplings(3, sp["L"], sp["disorder_seed"])
        st, rec_o, s_o, E_o = o.run(3, sp["L"], J, sp["seed"], sp["R0"], betas, ns, capacity=run.capacity)
        assert st == 0
        s, E = run.population()
        assert np.array_equal(s, s_o) and np.array_equal(E, E_o)
        rec = run.records()
        assert np.allclose(rec[:, 2], rec_o[:, 3], rtol=1e-12, atol=0)


@pytest.mark.parametrize("specs,ns", [
    ([dict(dim=3, L=8, R0=300, seed=41, disorder_seed=2), dict(dim=3, L=24, R0=150, seed=42, disorder_seed=3)], 2),
    ([dict(dim=1, L=64, R0=400, seed=43, disorder_seed=4), dict(dim=1, L=40000, R0=120, seed=44, disorder_seed=5)], 0),
], ids=["cube_8_24", "chain_64_40000"])
def test_batch_histogram_of_runs_with_and_without_lds_bins(specs, ns):
    # the histogram kernel counts a run's energies in LDS when its bins fit the call's LDS table and
    # in global memory otherwise: a batch that mixes both (the larger lattice has more than 16384
    # bins) must equal the runs stepped one by one, and the oracle's first resampling (the chain
    # steps without sweeps: a 40000-site chain row does not fit the sweep's LDS)
    nT = 4
    betas = [0.0, 0.3, 0.9, 1.6]
    note(f"mixed histogram batch L={[sp['L'] for sp in specs]}")
    batch = pa.Batch(specs, nT, layout="bits64", device=DEV).init()
    solos = solo_runs(specs, nT, "bits64", [r.capacity for r in batch.runs])
    sched = pa.Schedule(betas, ns, max(r.n_bins for r in batch.runs), device=DEV)
    for k in range(1, nT):
        batch.step(sched, k)
        st = sched.step(k)
        for r in solos:
            r.resample(st)
            r.sweep(st)
        pa.measure(solos)
        compare(batch, solos, k)
        if k == 1:
            for sp, run in zip(specs, batch.runs):
                J = o.couplings(sp["dim"], sp["L"], sp["disorder_seed"])
                _, E0 = o.init_population(sp["dim"], sp["L"], J, sp["seed"], sp["R0"])
                stc, counts_o, S_o, _, Elo_o = o.copy_numbers(sp["seed"], 1, betas[0], betas[1], sp["R0"], E0)
                assert stc == 0
                c, _ = run.counts_offsets(sp["R0"])
                assert np.array_equal(c, counts_o)
                rec = run.records()[1]
                assert rec[3] == S_o and rec[5] == Elo_o
    code, flags = batch.status()
    assert code == pa.PA_OK and not flags.any()


def test_graph_replays_equal_eager():
    specs = specs_mixed()[:8]
    nT, ns = 6, 2
    betas = [3.0 * k / (nT - 1) for k in range(nT)]
    note("graph capture")
    stream = torch.cuda.Stream(DEV)
    gb = pa.Batch(specs, nT, layout="bits64", device=DEV, stream=stream)
    eb = pa.Batch(specs, nT, layout="bits64", device=DEV)
    sched = pa.Schedule(betas, ns, max(r.n_bins for r in gb.runs), device=DEV)
    gb.init()
    torch.cuda.synchronize()
    graph = gb.capture(sched, range(1, nT), pairs=True)
    for replay in range(3):
        note(f"graph replay {replay}")
        gb.init()  # eager work between replays
        graph.launch()
        eb.init()
        for k in range(1, nT):
            eb.step(sched, k, pairs=True)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(gb.runs, eb.runs)):
            sa, Ea = a.population()
            sb, Eb = b.population()
            assert np.array_equal(sa, sb) and np.array_equal(Ea, Eb), f"replay {replay} run {i}"
            assert np.array_equal(a.records(), b.records()), f"replay {replay} run {i} records"


def test_batch_schedules_give_same_sample():
    specs = specs_mixed()
    nT = 3
    betas = [0.0, 0.6, 1.4]
    ref = None
    try:
        for bpc, order, launch in ((8, 1, 0), (1, 0, 1), (3, 1, 2), (16, 0, 0), (2, 0, 1), (5, 1, 1)):
            note(f"batch schedule blocks_per_cu={bpc} order={order} launch={launch}")
            pa.set_batch_config(bpc, order, launch)
            b = pa.Batch(specs, nT, layout="bits64", device=DEV).init()
            sched = pa.Schedule(betas, 3, max(r.n_bins for r in b.runs), device=DEV)
            for k in range(1, nT):
                b.step(sched, k)
            pops = [r.population() for r in b.runs]
            if ref is None:
                ref = pops
            else:
                for (s1, e1), (s2, e2) in zip(ref, pops):
                    assert np.array_equal(s1, s2) and np.array_equal(e1, e2)
    finally:
        pa.set_batch_config(0, 0, 0)


def test_batch_error_is_isolated():
    # one run overflows its capacity: it freezes with the flag, the others carry on
    specs = [dict(dim=3, L=8, R0=200, seed=5, disorder_seed=1), dict(dim=3, L=8, R0=200, seed=6, disorder_seed=1)]
    note("batch error isolation")
    b = pa.Batch(specs, 3, layout="bits64", device=DEV, capacity_factor=1.0).init()
    sched = pa.Schedule([0.0, 0.1, 0.2], 2, b.runs[0].n_bins, device=DEV, R_targets=[0, 200.0, 200.0])
    st = sched.step(1)
    b.resample(st)
    b.sweep(st)
    code, flags = b.status()
    # R_target = 200 with capacity 320: both fit; now ask one run for too many by a solo step
    assert code == pa.PA_OK
    big = pa.Schedule([0.1, 0.2], 1, b.runs[0].n_bins, device=DEV, R_targets=[0, 5000.0])
    b.runs[0].resample(big.step(1))
    s1_before, _ = b.runs[1].population()
    st2 = sched.step(2)
    b.resample(st2)
    b.sweep(st2)
    code, flags = b.status()
    assert flags[0] & pa.PA_FLAG_CAPACITY and flags[1] == 0
    assert b.runs[1].query().k == 2


def test_ensemble_weighted_averages_and_autotuner():
    # a reduced batched configuration: 3 realisations x 4 seeds, graph-captured schedule,
    # tuned persistent schedule.  The device weighted average itself is checked against the
    # oracle on seeded inputs elsewhere; here the run records are GPU outputs, so they go only
    # to the library's own host weighted average (the grouping by realization and by pair) and
    # to the properties a weighted average has (a convex combination, a non-negative variance)
    from paper_1006_0252_amd import ensemble, workloads

    specs = workloads.batched_specs(n_realizations=3, R0_range=(300, 900), gen_seed=11)
    note("ensemble reduced batched configuration")
    r = ensemble.run_batched(specs, 11, 3, device=DEV, tune=True, graph=True)
    rec = r["records"]
    w = r["weighted"]
    k = 10
    for n, d in enumerate(w["realizations"]):
        idx = [i for i, sp in enumerate(specs) if sp["realization"] == d]
        x = rec[idx, k, 2]
        R = np.array([specs[i]["R0"] for i in idx], dtype=np.float64)
        E = rec[idx, k, 6]
        ref = pa.weighted_average(x, E[:, None], R)
        assert abs(w["E_bar"][n] - ref["A_bar"][0]) <= 1e-12 * abs(ref["A_bar"][0])
        assert abs(w["minus_betaF_bar"][n] - ref["minus_betaF_bar"]) <= 1e-12 * abs(ref["minus_betaF_bar"])
        assert abs(w["var_betaF"][n] - ref["var"]) <= 1e-12 * max(1.0, ref["var"])
        xp = x[0::2] + x[1::2]
        Rp = R[0::2] * R[1::2]
        Q = rec[np.array(idx)[0::2], k, 9:12]
        q2 = Q[:, 0]
        refq = pa.weighted_average(xp, Q, Rp)
        for v, name in enumerate(("q2", "q4", "gamma")):
            assert abs(w[name][n] - refq["A_bar"][v]) <= 1e-12, name
        g = 0.5 * (3.0 - refq["A_bar"][1] / refq["A_bar"][0] ** 2)
        assert abs(w["binder"][n] - g) <= 1e-12 * max(1.0, abs(g))
        assert E.min() - 1e-9 <= w["E_bar"][n] <= E.max() + 1e-9 and w["var_betaF"][n] >= 0.0
        assert q2.min() - 1e-12 <= w["q2"][n] <= q2.max() + 1e-12
    from paper_1006_0252_amd import autotune

    assert r["tuned"] in autotune.BATCH_CANDIDATES


def test_full_batched_configuration_sampled_parity():
    # the batched configuration at full size (256 runs, L in {6, 8, 10}, R0 in [1e4, 1e5]): one
    # batched resampling from the seeded initial populations, then one persistent sweep launch.
    # Every 16th run: all copy numbers and S against the oracle (from its own initial energies), and
    # sampled replicas after the sweep, whose parents come from the oracle's copy numbers
    from paper_1006_0252_amd import workloads

    specs = workloads.batched_specs()
    note("full batched configuration: init + resample")
    b = pa.Batch(specs, 3, layout="bits64", device=DEV).init()
    betas = [0.0, 0.05]
    sched = pa.Schedule(betas, 10, max(r.n_bins for r in b.runs), device=DEV)
    st = sched.step(1)
    b.resample(st)
    code, _ = b.status()
    assert code == pa.PA_OK
    parents = {}
    for i in range(0, len(specs), 16):
        sp = specs[i]
        J = o.couplings(3, sp["L"], sp["disorder_seed"])
        s0, E0 = o.init_replicas(3, sp["L"], J, sp["seed"], 0, sp["R0"])
        stc, counts_o, S_o, _, _ = o.copy_numbers(sp["seed"], 1, betas[0], betas[1], sp["R0"], E0)
        assert stc == 0
        c, _ = b.runs[i].counts_offsets(sp["R0"])
        assert np.array_equal(c, counts_o), f"copy numbers of run {i}"
        assert b.runs[i].records()[1][3] == S_o
        src = np.repeat(np.arange(sp["R0"]), counts_o)
        idx = np.unique(np.array([0, 63, 64, 129, len(src) // 2, len(src) - 1]))
        parents[i] = (J, idx, s0[src[idx]].copy(), E0[src[idx]].copy())   # the sampled replicas' parents
    note("full batched configuration: sweep")
    b.sweep(st)
    code, _ = b.status()
    assert code == pa.PA_OK
    for i, (J, idx, sp0, Ep0) in parents.items():
        sp = specs[i]
        sg = b.runs[i].replica_spins(idx)
        Eg = b.runs[i].energies()
        for k, r in enumerate(idx):
            so = sp0[k][None, :].copy()
            Eo = np.array([Ep0[k]], dtype=np.int32)
            o.sweep_replicas(3, sp["L"], J, sp["seed"], betas[1], int(r), so, Eo, 0, 10)
            assert np.array_equal(sg[k], so[0]) and Eg[r] == Eo[0], f"run {i} replica {r}"


@pytest.mark.parametrize("layout,N", [("u8", 64), ("bits64", 64), ("u8", 100), ("bits64", 100)])
def test_chain_batch_matches_oracle(layout, N):
    # chains of one length sweep in one launch (grid row = run): each run against the oracle
    note(f"chain batch {layout} N={N}")
    R0s = (300, 77, 1000, 130)
    nT, ns = 7, 3
    betas = [5.0 * k / (nT - 1) for k in range(nT)]
    specs = [dict(dim=1, L=N, R0=R0, seed=60 + i, disorder_seed=2 + (i & 1)) for i, R0 in enumerate(R0s)]
    batch = pa.Batch(specs, nT, layout=layout, device=DEV).init()
    sched = pa.Schedule(betas, ns, batch.runs[0].n_bins, device=DEV)
    for k in range(1, nT):
        batch.step(sched, k)
    code, flags = batch.status()
    assert code == pa.PA_OK and not flags.any()
    for sp, run in zip(specs, batch.runs):
        J = o.couplings(1, N, sp["disorder_seed"])
        st_o, rec_o, s_o, E_o = o.run(1, N, J, sp["seed"], sp["R0"], betas, ns, capacity=run.capacity)
        assert st_o == 0
        s, E = run.population()
        assert np.array_equal(s, s_o) and np.array_equal(E, E_o)
        assert np.array_equal(run.records()[:, 4], rec_o[:, 1])
