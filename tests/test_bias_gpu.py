"""Device bootstrap errors against the oracle, and the ring bias measurement of Sec. IV at a
reduced size: weighted estimates unbiased within their bootstrap errors against the exact
chain, the plain free-energy mean biased low."""
import sys

import numpy as np
import pytest

from oracle import oracle as o

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1006_0252_amd import bias, exact, pa  # noqa: E402

DEV = "cuda:0"


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def test_bootstrap_matches_oracle():
    note("bootstrap parity")
    g = np.random.default_rng(3)
    n_sets, M, n_obs, n_boot = 5, 37, 2, 50
    x = 500.0 + 2.0 * g.standard_normal((n_sets, M))
    R = g.integers(1000, 5000, (n_sets, M)).astype(np.float64)
    A = g.standard_normal((n_sets, M, n_obs))
    idx = g.integers(0, M, (n_boot, M)).astype(np.int32)
    idx[7, 3] = M  # out of range: that replicate is NaN, no read outside the set
    d = lambda a: torch.tensor(np.ascontiguousarray(a), device=DEV)  # noqa: E731
    xd, Rd, Ad, idd = d(x), d(R), d(A), d(idx)
    rep = torch.zeros((n_sets, n_boot, n_obs + 3), dtype=torch.float64, device=DEV)
    err = torch.zeros((n_sets, n_obs + 3), dtype=torch.float64, device=DEV)
    pa.check(pa.lib().pa_bootstrap_dev(n_sets, M, xd.data_ptr(), Rd.data_ptr(), Ad.data_ptr(), n_obs, n_boot,
                                       idd.data_ptr(), rep.data_ptr(), err.data_ptr(),
                                       torch.cuda.current_stream(DEV).cuda_stream), "pa_bootstrap_dev")
    rep, err = rep.cpu().numpy(), err.cpu().numpy()
    good = np.array([b for b in range(n_boot) if b != 7])
    for s in range(n_sets):
        assert np.all(np.isnan(rep[s, 7])) and np.all(np.isnan(err[s]))
        reps_o, err_o = o.bootstrap(x[s], idx[good], A[s], R[s])
        assert np.allclose(rep[s, good], reps_o, rtol=1e-12, atol=1e-12)
    # the error rows themselves, on the valid replicates only
    idx2 = idx[good]
    rep2 = torch.zeros((n_sets, len(good), n_obs + 3), dtype=torch.float64, device=DEV)
    err2 = torch.zeros((n_sets, n_obs + 3), dtype=torch.float64, device=DEV)
    pa.check(pa.lib().pa_bootstrap_dev(n_sets, M, xd.data_ptr(), Rd.data_ptr(), Ad.data_ptr(), n_obs, len(good),
                                       d(idx2).data_ptr(), rep2.data_ptr(), err2.data_ptr(),
                                       torch.cuda.current_stream(DEV).cuda_stream), "pa_bootstrap_dev")
    err2 = err2.cpu().numpy()
    for s in range(n_sets):
        _, err_o = o.bootstrap(x[s], idx2, A[s], R[s])
        assert np.allclose(err2[s], err_o, rtol=1e-10, atol=1e-13)


def test_ring_bias_reduced():
    # 4 realizations x 40 runs: the weighted free energy and energy agree with the exact chain
    # within 4 bootstrap errors; the plain mean of -beta F~ lies below the exact value
    note("ring bias, reduced")
    r = bias.run(n_real=4, M=40, n_boot=100, betas=(5.0,), device=DEV)["by_beta"][5.0]
    for p in r["per_realization"]:
        assert abs(p["F_w"] - p["F_exact"]) < 4 * p["F_w_err"] + 0.02
        assert abs(p["E_w"] - p["E_exact"]) < 4 * p["E_w_err"] + 0.05
    fb, fe = r["free_energy_bias_plain"]
    assert fb < 0
    mu1 = r["mu_k"][1][0]
    assert abs(mu1 - r["energy_bias_plain"][0]) < 1e-9   # blocks of one run are the plain mean


def test_gaussian_chain_bias_reduced():
    # the paper's 1D chain (Gaussian bonds, N = 256, R = 1000, its 100-temperature schedule, 50
    # sweeps), 2 realizations x 40 runs: weighted estimates agree with the exact transfer-matrix
    # values within 4 bootstrap errors at T = 0.2
    note("gaussian chain bias, reduced")
    r = bias.run(n_real=2, M=40, n_boot=100, betas=(5.0,), device=DEV, chain="gauss")["by_beta"][5.0]
    assert r["beta_grid"] == 5.0
    for p in r["per_realization"]:
        assert abs(p["F_w"] - p["F_exact"]) < 4 * p["F_w_err"] + 0.02
        assert abs(p["E_w"] - p["E_exact"]) < 4 * p["E_w_err"] + 0.05
        assert p["var"] > 0


@pytest.mark.parametrize("couplings,N", [("pm1", 64), ("gauss", 256)])
def test_chain_ensemble_graph_equals_eager(couplings, N):
    # the chain ensembles are timed as one captured HIP graph: its replay gives the records of
    # stepping eagerly, bit for bit
    note(f"chain ensemble graph vs eager {couplings} N={N}")
    betas = np.linspace(0.0, 2.0, 9)
    kw = dict(R0=300, n_sweeps=3, device=DEV, N=N, couplings=couplings, betas=betas)
    Xg, Eg, _, _, _, ag = bias.ring_ensemble(3, 6, graph=True, **kw)
    Xe, Ee, _, _, _, ae = bias.ring_ensemble(3, 6, graph=False, **kw)
    assert np.array_equal(Xg, Xe) and np.array_equal(Eg, Ee) and ag == ae
