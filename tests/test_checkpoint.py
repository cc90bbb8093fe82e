"""Checkpoint and resume: a run stopped after step K, saved to a file, and continued in fresh
buffers ends bit for bit where the uninterrupted run ends.  This holds because every draw is keyed
by (seed, replica, sweep or step index) (Sec. II's sweeps and resampling read no other state): the
state between steps is the couplings, the population's spins and energies, its size, the
accumulated sum of ln Q and the step index.

CPU: the oracle, stepped by its own resample and sweep calls, against its own whole run.
GPU: pa_resume through the C ABI, against an uninterrupted library run and the oracle."""
import numpy as np
import pytest

from oracle import oracle as o


def _oracle_steps(dim, L, J, seed, R0, betas, ns, cap, k_from, k_to, s, E, R, acc):
    for k in range(k_from, k_to + 1):
        r = o.resample(dim, L, seed, k, betas[k - 1], betas[k], R0, R, s, E, cap)
        assert r["status"] == 0
        s, E, R = r["s"], r["E"], r["R_new"]
        acc += r["lnQ"]
        o.sweep(dim, L, J, seed, betas[k], R, s, E, (k - 1) * ns, ns)
    return s, E, R, acc


@pytest.mark.parametrize("dim,L,K", [(3, 4, 4), (1, 32, 1), (3, 6, 7)])
def test_oracle_resume_from_saved_arrays_is_bit_identical(tmp_path, dim, L, K):
    R0, nT, ns, seed, dseed = 300, 9, 3, 77, 4
    betas = [2.0 * k / (nT - 1) for k in range(nT)]
    J = o.couplings(dim, L, dseed)
    cap = 512
    st, rec, s_ref, E_ref = o.run(dim, L, J, seed, R0, betas, ns, capacity=cap)
    assert st == 0
    s, E = o.init_population(dim, L, J, seed, R0, capacity=cap)
    s, E, R, acc = _oracle_steps(dim, L, J, seed, R0, betas, ns, cap, 1, K, s, E, R0, 0.0)
    np.savez(tmp_path / "ck.npz", s=s[:R], E=E[:R], R=R, acc=acc, k=K)
    del s, E
    ck = np.load(tmp_path / "ck.npz")
    R, acc, K2 = int(ck["R"]), float(ck["acc"]), int(ck["k"])
    s = np.zeros((cap, o.num_sites(dim, L)), np.uint8)
    E = np.zeros(cap, np.int32)
    s[:R], E[:R] = ck["s"], ck["E"]
    s, E, R, acc = _oracle_steps(dim, L, J, seed, R0, betas, ns, cap, K2 + 1, nT - 1, s, E, R, acc)
    assert R == int(rec[-1, 1])
    assert np.array_equal(s[:R], s_ref) and np.array_equal(E[:R], E_ref)
    assert o.num_sites(dim, L) * np.log(2.0) + acc == rec[-1, 3]


@pytest.mark.gpu
@pytest.mark.parametrize("dim,L,layout,R0", [(3, 8, "bits64", 3000), (3, 16, "bits64", 1000), (1, 64, "u8", 700),
                                             (3, 6, "u8", 500)])
def test_resume_from_checkpoint_is_bit_identical(tmp_path, dim, L, layout, R0):
    import torch

    from paper_1006_0252_amd import pa

    dev = "cuda:0"
    nT, ns, K, seed, dseed = 12, 4, 5, 31, 6
    betas = [3.0 * k / (nT - 1) for k in range(nT)]
    print(f"resume dim={dim} L={L} {layout} R0={R0}", flush=True)

    def steps(run, sched, k_from, k_to):
        for k in range(k_from, k_to + 1):
            st = sched.step(k)
            run.resample(st)
            run.sweep(st)
            pa.measure([run])

    ref = pa.Run(dim, L, R0, seed, dseed, n_records=nT, layout=layout, device=dev).init()
    sched = pa.Schedule(betas, ns, ref.n_bins, device=dev)
    steps(ref, sched, 1, nT - 1)

    a = pa.Run(dim, L, R0, seed, dseed, n_records=nT, layout=layout, device=dev).init()
    steps(a, sched, 1, K)
    np.savez(tmp_path / "ck.npz", **a.checkpoint())
    del a
    torch.cuda.empty_cache()
    ck = dict(np.load(tmp_path / "ck.npz"))
    b = pa.Run(dim, L, R0, seed, dseed, n_records=nT, layout=layout, device=dev).resume(ck)
    assert b.query().k == K
    steps(b, sched, K + 1, nT - 1)

    code, flags = b.status()
    assert code == pa.PA_OK and flags == 0
    assert np.array_equal(b.records(), ref.records())
    s, E = b.population()
    s_ref, E_ref = ref.population()
    assert np.array_equal(s, s_ref) and np.array_equal(E, E_ref)
    fe, fe_ref = (torch.zeros(1, dtype=torch.float64, device=dev) for _ in range(2))
    b.free_energy(fe)
    ref.free_energy(fe_ref)
    assert float(fe.cpu()[0]) == float(fe_ref.cpu()[0])
    # and the resumed run is the oracle's
    st_o, rec_o, s_o, E_o = o.run(dim, L, o.couplings(dim, L, dseed), seed, R0, betas, ns, capacity=b.capacity)
    assert st_o == 0 and np.array_equal(s, s_o) and np.array_equal(E, E_o)


@pytest.mark.gpu
def test_resume_rejects_a_mismatched_checkpoint_and_invalid_state():
    from paper_1006_0252_amd import pa

    dev = "cuda:0"
    a = pa.Run(3, 8, 200, 1, 1, n_records=4, layout="bits64", device=dev).init()
    ck = a.checkpoint()
    with pytest.raises(ValueError):
        pa.Run(3, 8, 200, 2, 1, n_records=4, layout="bits64", device=dev).resume(ck)  # another seed
    bad = dict(ck)
    bad["info_k"] = np.asarray(4)  # k must be below n_records
    with pytest.raises(pa.PAError):
        pa.Run(3, 8, 200, 1, 1, n_records=4, layout="bits64", device=dev).resume(bad)
