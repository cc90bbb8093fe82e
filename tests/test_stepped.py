"""Per-temperature target sizes R_beta: the equal-work step profile (host) and, on the GPU, that
the population follows the targets and that the variance profile comes out per temperature."""
import numpy as np
import pytest

from paper_1006_0252_amd import pa, stepped


def test_equal_work_step_profile():
    betas = pa.linear_schedule(101)
    Rt, R_lo = stepped.equal_work_step(betas, 2000, 0.9)
    assert abs(Rt[1:].sum() - 2000 * 100) <= 100              # rounding of 100 targets
    assert np.all(Rt[1:][betas[1:] < 0.9] == round(R_lo)) and np.all(Rt[betas >= 0.9] == round(3 * R_lo))


@pytest.mark.gpu
def test_population_follows_stepped_targets():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[case] stepped targets L=6", flush=True)
    betas = pa.linear_schedule(21)
    Rt = np.where(betas < 1.0, 500.0, 1500.0)
    rec, T, att = stepped.ensemble(betas, Rt, 16, 6, 3, 4, R_init=500, device="cuda:0")
    R = rec[:, 1:, stepped.REC["R"]]
    m = R.mean(axis=0)
    assert np.all(np.abs(m - Rt[1:]) < 6 * np.sqrt(Rt[1:] * 2 / 16))   # Poisson sizes, 16 runs
    var, fbar = stepped.var_profile(rec, device="cuda:0")
    x = rec[:, :, stepped.REC["minus_betaF"]]
    assert np.allclose(var, x.var(axis=0, ddof=1), rtol=1e-10, atol=1e-12)
    assert abs(var[0]) < 1e-20 and np.all(var[1:] > 0)   # every run starts at N ln 2


@pytest.mark.gpu
@pytest.mark.parametrize("layout", ["bits64", "u8"])
def test_stepped_targets_match_oracle(layout):
    # per-step target sizes (growing and shrinking) on the GPU give the oracle's sample bit for bit
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as o

    print(f"[case] stepped targets vs oracle {layout}", flush=True)
    betas = [0.0, 0.2, 0.5, 0.9, 1.4, 2.0]
    Rt = [0.0, 300.0, 900.0, 900.0, 450.0, 700.0]
    L, seed, ds, ns = 6, 21, 4, 3
    cap = 1280
    run = pa.Run(3, L, 300, seed, ds, len(betas), capacity=cap, layout=layout, device="cuda:0").init()
    sched = pa.Schedule(betas, ns, run.n_bins, device="cuda:0", R_targets=Rt)
    for k in range(1, len(betas)):
        st = sched.step(k)
        run.resample(st)
        run.sweep(st)
    code, _ = run.status()
    assert code == pa.PA_OK
    J = o.couplings(3, L, ds)
    st_o, rec_o, s_o, E_o = o.run(3, L, J, seed, 300, betas, ns, capacity=cap, R_targets=Rt)
    assert st_o == 0
    s, E = run.population()
    assert np.array_equal(s, s_o) and np.array_equal(E, E_o)
    rec = run.records()
    assert np.array_equal(rec[:, 4], rec_o[:, 1])                  # population sizes
    assert np.allclose(rec[:, 2], rec_o[:, 3], rtol=1e-12, atol=0)  # -beta F~
