"""Pins of the oracle's bootstrap errors (Sec. III) and of the exact ring results the bias
measurements use: special resamplings with known answers, the exact bootstrap variance of a
plain mean, and both exact-ring implementations against brute-force enumeration."""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as o
from paper_1006_0252_amd import exact


def test_identity_and_constant_resamples():
    g = np.random.default_rng(1)
    M = 9
    x = 1000.0 + g.standard_normal(M)
    A = g.standard_normal((M, 2))
    R = g.integers(100, 1000, M).astype(float)
    idx = np.array([np.arange(M), np.full(M, 4), np.full(M, 0)])
    reps, err = o.bootstrap(x, idx, A, R)
    w = o.weighted_average(x, A, R)
    assert np.allclose(reps[0], np.concatenate([w["A_bar"], [w["minus_betaF_bar"], w["var"], w["mean"]]]), rtol=1e-14)
    for row, r in ((1, 4), (2, 0)):
        assert np.allclose(reps[row][:2], A[r], rtol=1e-14)      # one run carries all the weight
        assert abs(reps[row][2] - x[r]) < 1e-10                  # -beta F_bar of M copies of run r
        assert abs(reps[row][3]) < 1e-20 and abs(reps[row][4] - x[r]) < 1e-12
    assert np.all(err >= 0)


def test_bootstrap_error_of_plain_mean():
    # equal free energies: every replicate is a plain mean of resampled values, whose exact
    # bootstrap variance is sum (A - mean)^2 / M^2
    g = np.random.default_rng(2)
    M, n_boot = 40, 4000
    A = g.standard_normal(M) * 3.0
    idx = g.integers(0, M, (n_boot, M))
    reps, err = o.bootstrap(np.zeros(M), idx, A[:, None])
    want = math.sqrt(((A - A.mean()) ** 2).sum()) / M
    assert abs(err[0] - want) < 0.05 * want


@pytest.mark.parametrize("N", [6, 9, 12])
def test_ring_exact_against_enumeration(N):
    g = np.random.default_rng(N)
    J = g.choice([-1, 1], N)
    states = np.array(list(itertools.product([-1, 1], repeat=N)))
    E = (J * states * np.roll(states, -1, axis=1)).sum(axis=1).astype(float)
    for beta in (0.2, 1.0, 3.0):
        w = np.exp(-beta * (E - E.min()))
        lnZ = math.log(w.sum()) - beta * E.min()
        Em = (E * w).sum() / w.sum()
        lz, e = o.ring_exact(J, beta)
        assert abs(lz - lnZ) < 1e-12 * abs(lnZ) + 1e-12 and abs(e - Em) < 1e-10
        assert abs(exact.ring_lnZ(J, beta) - lnZ) < 1e-12 * abs(lnZ) + 1e-12
        assert abs(exact.ring_energy(J, beta) - Em) < 1e-10


def test_ring_exact_large_chain_agrees():
    g = np.random.default_rng(5)
    J = g.choice([-1, 1], 64)
    for beta in (0.5, 2.0, 5.0):
        lz, e = o.ring_exact(J, beta)
        assert abs(lz - exact.ring_lnZ(J, beta)) < 1e-12 * lz
        assert abs(e - exact.ring_energy(J, beta)) < 1e-10


@pytest.mark.parametrize("N", [6, 9, 12])
def test_ring_exact_real_couplings_against_enumeration(N):
    # Gaussian bonds: both exact-ring implementations against the 2^N states
    g = np.random.default_rng(100 + N)
    J = g.standard_normal(N)
    states = np.array(list(itertools.product([-1, 1], repeat=N)))
    E = (J * states * np.roll(states, -1, axis=1)).sum(axis=1)
    for beta in (0.2, 1.0, 5.0):
        w = np.exp(-beta * (E - E.min()))
        lnZ = math.log(w.sum()) - beta * E.min()
        Em = (E * w).sum() / w.sum()
        lz, e = o.ring_exact(J, beta)
        assert abs(lz - lnZ) < 1e-12 * abs(lnZ) + 1e-12 and abs(e - Em) < 1e-10
        assert abs(exact.ring_lnZ(J, beta) - lnZ) < 1e-12 * abs(lnZ) + 1e-12
        assert abs(exact.ring_energy(J, beta) - Em) < 1e-10


def test_ring_exact_real_couplings_large_chain():
    # N = 256 Gaussian bonds (the paper's 1D size): closed form against transfer matrices
    J = o.couplings_gauss(1, 256, 3)
    for beta in (0.5, 2.0, 5.0):
        lz, e = o.ring_exact(J, beta)
        assert abs(lz - exact.ring_lnZ(J, beta)) < 1e-12 * lz
        assert abs(e - exact.ring_energy(J, beta)) < 1e-9 * abs(e)
