"""Pins of the oracle's Gaussian-coupling path (the model of Sec. IV) against facts that do not
come from the oracle: libm's exp, the normal distribution, energy identities, the exact
checkerboard transition matrix on 2x2x2, and the exact transfer-matrix free energy of a ring
with Gaussian bonds."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as o


def test_expd_against_libm():
    xs = np.concatenate([-np.exp(np.linspace(-30, np.log(744.0), 4000)), [-0.0, -1e-300, -0.5 * math.log(2)]])
    for x in xs:
        want = math.exp(x)
        got = o.expd(x)
        assert abs(got - want) <= 4 * 2.0 ** -52 * want + 5e-324, (x, got, want)
    assert o.expd(0.0) == 1.0 and o.expd(-745.5) == 0.0 and o.expd(-1e4) == 0.0
    v = [o.expd(x) for x in np.linspace(-50, 0, 20001)]
    assert np.all(np.diff(v) >= 0)


def test_couplings_are_standard_normal():
    J = o.couplings_gauss(3, 16, 7)
    n = len(J)
    assert abs(J.mean()) < 4 / math.sqrt(n) and abs(J.var() - 1) < 4 * math.sqrt(2 / n)
    assert stats.kstest(J, "norm").pvalue > 1e-3
    J2 = o.couplings_gauss(3, 16, 8)
    assert abs(np.corrcoef(J, J2)[0, 1]) < 4 / math.sqrt(n)
    assert np.array_equal(J, o.couplings_gauss(3, 16, 7))


@pytest.mark.parametrize("dim,L", [(1, 12), (3, 4)])
def test_energy_identities(dim, L):
    J = o.couplings_gauss(dim, L, 3)
    s, E = o.init_replicas_gauss(dim, L, J, 5, 0, 3)
    N = L if dim == 1 else L ** 3
    for q in range(3):
        x = s[q].copy()
        dEs = []
        for i in range(N):
            dE = o.delta_energy_gauss(dim, L, J, x, i)
            y = x.copy()
            y[i] ^= 1
            assert abs(o.energy_gauss(dim, L, J, y) - E[q] - dE) < 1e-10
            dEs.append(dE)
        # each bond enters the single-flip changes of both its ends
        assert abs(sum(dEs) + 4 * E[q]) < 1e-9
        # energy by direct summation, independent of the oracle's bond bookkeeping
        sig = 1 - 2 * x.astype(float)
        if dim == 1:
            ref = float(np.sum(J * sig * np.roll(sig, -1)))
        else:
            g = sig.reshape(L, L, L)  # [z][y][x]
            Jg = J.reshape(L, L, L, 3)
            ref = float(np.sum(Jg[..., 0] * g * np.roll(g, -1, 2)) + np.sum(Jg[..., 1] * g * np.roll(g, -1, 1))
                        + np.sum(Jg[..., 2] * g * np.roll(g, -1, 0)))
        assert abs(E[q] - ref) < 1e-10


def _half_sweep_matrix_gauss(L, J, beta, colour, states, index):
    n = len(states)
    P = np.zeros((n, n))
    sites = [i for i in range(states.shape[1]) if o.colour(3, L, i) == colour]
    for a, s in enumerate(states):
        probs = []
        for i in sites:
            dE = o.delta_energy_gauss(3, L, J, s, i)
            if dE <= 0:
                probs.append(1.0)
            else:
                p = o.expd(-(beta * dE))
                probs.append(1.0 if p >= 1.0 else math.floor(math.ldexp(p, 64)) / 2.0 ** 64)
        for flips in itertools.product([0, 1], repeat=len(sites)):
            t = s.copy()
            pr = 1.0
            for f, i, p in zip(flips, sites, probs):
                if f:
                    t[i] ^= 1
                    pr *= p
                else:
                    pr *= 1 - p
            P[a, index[t.tobytes()]] += pr
    return P


@pytest.mark.parametrize("beta", [0.4, 2.0])
def test_checkerboard_sweep_stationary_gaussian_2x2x2(beta):
    L, N = 2, 8
    J = o.couplings_gauss(3, L, 9)
    states = np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.uint8)
    index = {s.tobytes(): a for a, s in enumerate(states)}
    E = np.array([o.energy_gauss(3, L, J, s) for s in states])
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    P0 = _half_sweep_matrix_gauss(L, J, beta, 0, states, index)
    P1 = _half_sweep_matrix_gauss(L, J, beta, 1, states, index)
    assert np.max(np.abs(pi @ (P0 @ P1) - pi)) < 1e-12
    F = pi[:, None] * P0
    assert np.max(np.abs(F - F.T)) < 1e-12


def test_sweep_samples_boltzmann_gaussian_2x2x2():
    L, N = 2, 8
    J = o.couplings_gauss(3, L, 9)
    beta = 0.7
    states = np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.uint8)
    E_all = np.array([o.energy_gauss(3, L, J, s) for s in states])
    p = np.exp(-beta * (E_all - E_all.min()))
    p /= p.sum()
    R = 20000
    s, E = o.init_replicas_gauss(3, L, J, 77, 0, R)
    o.sweep_replicas_gauss(3, L, J, 77, beta, 0, s, E, 0, 30)
    codes = s.astype(np.int64) @ (1 << np.arange(N - 1, -1, -1))
    obs = np.bincount(codes, minlength=2 ** N)
    m = R * p > 5
    chi2 = ((obs[m] - R * p[m]) ** 2 / (R * p[m])).sum()
    assert stats.chi2.sf(chi2, m.sum() - 1) > 1e-4
    assert np.allclose(E, E_all[codes], rtol=0, atol=1e-12)


def test_resampling_special_cases():
    E = np.array([-3.25, 1.5, 0.125, 7.0, -3.25])
    st, c, S, lnQ, E_lo = o.copy_numbers_gauss(1, 1, 0.7, 0.7, 5.0, E)
    assert st == 0 and S == 5.0 and lnQ == 0.0 and E_lo == -3.25
    E1 = np.full(17, -12.375)
    st, c, S, lnQ, _ = o.copy_numbers_gauss(1, 1, 0.2, 0.9, 17.0, E1)
    assert st == 0 and abs(lnQ - (0.9 - 0.2) * 12.375) < 1e-14 * 8.7   # Q = exp(-dbeta E) up to the rounding of ln S - ln R
    # ln Q against the definition with libm exp
    g = np.random.default_rng(4)
    E = g.standard_normal(1000) * 20
    st, c, S, lnQ, _ = o.copy_numbers_gauss(3, 2, 1.0, 1.1, 1000.0, E)
    want = math.log(math.fsum(math.exp(-0.1 * e) for e in E) / len(E))
    assert abs(lnQ - want) < 1e-12 * abs(want) + 1e-13
    assert abs(c.sum() - 1000) < 5 * math.sqrt(1000)


def test_weighted_free_energy_matches_exact_gaussian_ring():
    # the paper's 1D test with its own model: a ring of Gaussian bonds, exact Z by transfer
    # matrices; weighted -beta F_bar within bootstrap error at several temperatures
    N, R, M = 32, 600, 32
    J = o.couplings_gauss(1, N, 2)
    betas = np.array([4.0 * k / 40 for k in range(41)])
    runs = [o.run_gauss(1, N, J, 500 + m, R, betas, 4)[1] for m in range(M)]
    assert all(r[-1, 7] == 0 for r in runs)
    x = np.array([r[:, 3] for r in runs])
    rng = np.random.default_rng(1)
    idx = rng.integers(0, M, (100, M))
    for k in (10, 20, 40):
        _, err = o.bootstrap(x[:, k], idx)
        w = o.weighted_average(x[:, k])
        lnZ, _ = o.ring_exact(J, betas[k])
        assert abs(w["minus_betaF_bar"] - lnZ) < 4 * max(err[1], 2e-3), (k, w["minus_betaF_bar"], lnZ, err[1])
