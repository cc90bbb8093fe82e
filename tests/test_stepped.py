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
