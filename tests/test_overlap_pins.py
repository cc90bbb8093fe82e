"""Pins of the oracle's measurement functions: energy moments, the overlap histogram and its
statistics <q^2>, <q^4>, Gamma = Prob(|q| < 0.2) (Sec. IV), and the pair-weighted overlap
averages with the Binder ratio (Sec. IV, eqs. pqs and omegaprime).

The expected values come from hand computation (small histograms and energy lists whose
moments are written out below as exact fractions), closed forms (a Gaussian overlap has
Binder ratio 0, a frozen one 1) and exact enumeration of the 2 x 2 x 2 lattice (256 x 256
state pairs with Boltzmann weights), never from the oracle itself.  No GPU is needed.
"""
import math

import numpy as np
import pytest

from oracle import oracle as o


# ----------------------------------------------------------------------------
# overlap statistics on hand-built histograms
# ----------------------------------------------------------------------------
def test_overlap_stats_hand_histogram_with_q_at_the_gamma_edge():
    # N = 10: counts at Hamming distances d = 0, 3, 4, 5, 6, 10, i.e. q = (N - 2d)/N =
    # 1, 0.4, 0.2, 0, -0.2, -1.  By hand: P = 16, sum c q^2 = 1 + 0.32 + 0.12 + 0 + 0.2 + 1 = 2.64,
    # sum c q^4 = 1 + 0.0512 + 0.0048 + 0 + 0.008 + 1 = 2.064, and only q = 0 has |q| < 0.2
    # (|q| = 0.2 exactly, at d = 4 and d = 6, is not counted): 4 of 16.
    N = 10
    hist = np.zeros(N + 1, np.int64)
    hist[[0, 3, 4, 5, 6, 10]] = [1, 2, 3, 4, 5, 1]
    q2, q4, g = o.overlap_stats(N, hist)
    assert abs(q2 - 0.165) < 1e-15
    assert abs(q4 - 0.129) < 1e-15
    assert g == 0.25


def test_overlap_stats_hand_histograms_odd_lattices():
    # N = 5, all pairs at d = 2 (q = 0.2, on the edge): q^2 = 0.04, q^4 = 0.0016, Gamma = 0
    h = np.zeros(6, np.int64)
    h[2] = 7
    q2, q4, g = o.overlap_stats(5, h)
    assert abs(q2 - 0.04) < 1e-16 and abs(q4 - 0.0016) < 1e-17 and g == 0.0
    # N = 25: d = 11 gives q = 3/25 = 0.12 (inside), d = 15 gives q = -0.2 (edge), d = 20 q = -0.6.
    # counts 3, 1, 4 over 8 pairs: q^2 sum = 3 (0.0144) + 0.04 + 4 (0.36) = 1.5232 -> 0.1904;
    # q^4 sum = 3 (0.00020736) + 0.0016 + 4 (0.1296) = 0.52062208 -> 0.06507776; Gamma = 3/8
    h = np.zeros(26, np.int64)
    h[[11, 15, 20]] = [3, 1, 4]
    q2, q4, g = o.overlap_stats(25, h)
    assert abs(q2 - 0.1904) < 1e-15 and abs(q4 - 0.06507776) < 1e-15 and g == 0.375


def test_overlap_hist_counts_hamming_distance_of_aligned_pairs():
    # replica j of A with replica j of B only; d is the number of sites where the spins differ
    N = 6
    A = np.array([[0, 0, 0, 0, 0, 0], [1, 1, 1, 0, 0, 0], [0, 1, 0, 1, 0, 1]], np.uint8)
    B = np.array([[0, 0, 0, 0, 0, 1], [1, 1, 1, 0, 0, 0], [1, 0, 1, 0, 1, 0], [1, 1, 1, 1, 1, 1]], np.uint8)
    h, P = o.overlap_hist(N, A, B)
    assert P == 3
    assert list(h) == [1, 1, 0, 0, 0, 0, 1]   # d = 1, 0, 6


# ----------------------------------------------------------------------------
# energy moments on hand-made lists
# ----------------------------------------------------------------------------
def test_energy_moments_hand_lists():
    # E = (-4, 0, 0, 8): mean 1; deviations -5, -1, -1, 7: variance (25 + 1 + 1 + 49)/4 = 19,
    # third moment (-125 - 1 - 1 + 343)/4 = 54, skewness 54 / 19^1.5
    m = o.energy_moments(np.array([-4, 0, 0, 8], np.int32))
    assert m[0] == 1.0 and abs(m[1] - 19.0) < 1e-13
    assert abs(m[2] - 54.0 / (19.0 * math.sqrt(19.0))) < 1e-14
    # mirrored list: skewness changes sign, mean and variance follow
    m = o.energy_moments(np.array([4, 0, 0, -8], np.int32))
    assert m[0] == -1.0 and abs(m[1] - 19.0) < 1e-13 and abs(m[2] + 54.0 / (19.0 * math.sqrt(19.0))) < 1e-14
    # symmetric list: skewness 0; a single energy: variance and skewness 0
    m = o.energy_moments(np.array([-12, -4, -4, 4, 4, 12], np.int32))
    assert m[0] == 0.0 and abs(m[1] - 176.0 / 3.0) < 1e-12 and m[2] == 0.0
    m = o.energy_moments(np.array([-20] * 5, np.int32))
    assert tuple(m) == (-20.0, 0.0, 0.0)
    # Gaussian-coupling twin on real energies: (0.5, 1.5, 4.0) mean 2, deviations -1.5, -0.5, 2:
    # variance (2.25 + 0.25 + 4)/3 = 13/6, third moment (-3.375 - 0.125 + 8)/3 = 1.5
    m = o.energy_moments_gauss(np.array([0.5, 1.5, 4.0]))
    assert m[0] == 2.0 and abs(m[1] - 13.0 / 6.0) < 1e-15
    assert abs(m[2] - 1.5 / (13.0 / 6.0) ** 1.5) < 1e-14


# ----------------------------------------------------------------------------
# pair weights and the Binder ratio
# ----------------------------------------------------------------------------
def test_overlap_average_pair_weights_and_binder_closed_forms():
    # Gaussian overlap: <q^4> = 3 <q^2>^2 gives g = 0; a frozen overlap (q = +-1) gives g = 1
    s2 = 0.25
    out = o.overlap_average([3.0, 4.0, 3.5, 3.5], [[s2, 3 * s2 * s2, 0.5], [s2, 3 * s2 * s2, 0.5]])
    assert out[0] == s2 and out[1] == 3 * s2 * s2 and out[2] == 0.5 and out[3] == 0.0
    out = o.overlap_average([1.0, 2.0], [[1.0, 1.0, 0.0]])
    assert tuple(out) == (1.0, 1.0, 0.0, 1.0)
    # eq. omegaprime weighs a pair by exp(x^(1) + x^(2)): pairs (0, 10) and (5, 5) have equal weight
    # (a slip that used one run of the pair would weigh them 1 : e^5); a third pair at (10, 10)
    # has e^10 times the weight of the others
    Q = np.array([[0.2, 0.1, 0.3], [0.4, 0.3, 0.1], [0.6, 0.5, 0.0]])
    out = o.overlap_average([0.0, 10.0, 5.0, 5.0], Q[:2])
    assert np.allclose(out[:3], Q[:2].mean(0), rtol=1e-15, atol=0)
    w = np.array([1.0, 1.0, math.exp(10.0)])
    w /= w.sum()
    out = o.overlap_average([0.0, 10.0, 5.0, 5.0, 10.0, 10.0], Q)
    assert np.allclose(out[:3], w @ Q, rtol=1e-14, atol=0)
    assert abs(out[3] - 0.5 * (3 - out[1] / out[0] ** 2)) < 1e-15
    # unequal target sizes: the pair weight carries R^(1) R^(2) (Sec. III)
    out = o.overlap_average([0.0, 0.0, 0.0, 0.0], Q[:2], R=[1.0, 3.0, 2.0, 1.0])
    assert np.allclose(out[:3], (3 * Q[0] + 2 * Q[1]) / 5, rtol=1e-15, atol=0)


# ----------------------------------------------------------------------------
# exact enumeration of the 2 x 2 x 2 lattice
# ----------------------------------------------------------------------------
L2, N2 = 2, 8


def _states():
    """all 256 states, one byte per spin (1 = sigma -1), and their +-1 spin values"""
    b = ((np.arange(256)[:, None] >> np.arange(N2)[None, :]) & 1).astype(np.uint8)
    return b, 1 - 2 * b.astype(np.int64)


def _energies(J, sig):
    """E = + sum_b J_b s_i s_j, bond b = 3 i + a joining site i = x + 2 (y + 2 z) and its +a
    neighbour; on the periodic 2-cube the +a neighbour is the site with coordinate a flipped, so
    every neighbour pair carries two bonds"""
    E = np.zeros(256, np.int64)
    for i in range(N2):
        for a in range(3):
            j = i ^ (1 << a)
            E += J[3 * i + a] * sig[:, i] * sig[:, j]
    return E


def _exact(J, beta):
    """Boltzmann probabilities, exact energy moments and the exact overlap distribution of two
    independent replicas"""
    b, sig = _states()
    E = _energies(J, sig)
    w = np.exp(-beta * (E - E.min()))
    p = w / w.sum()
    mu = p @ E
    var = p @ (E - mu) ** 2
    skew = (p @ (E - mu) ** 3) / var ** 1.5
    q = (sig @ sig.T) / N2                      # [256][256] overlap of every state pair
    pq = np.outer(p, p)
    ex = dict(p=p, b=b, E=E, mean=mu, var=var, skew=skew,
              q2=(pq * q ** 2).sum(), q4=(pq * q ** 4).sum(), q8=(pq * q ** 8).sum(),
              gamma=pq[np.abs(q) < 0.2].sum())
    ex["g"] = 0.5 * (3 - ex["q4"] / ex["q2"] ** 2)
    return ex


def _se_from_influence(p, infl, n):
    """standard error of an estimator over n independent draws from p, by its influence function"""
    return math.sqrt(p @ (infl - p @ infl) ** 2 / n)


@pytest.mark.parametrize("beta", [0.3, 1.0, 3.0])
def test_overlap_and_moments_of_exact_boltzmann_samples_2x2x2(beta):
    # two independent populations drawn exactly from the Boltzmann distribution (numpy, not the
    # oracle); the oracle's histogram, statistics, Binder ratio and energy moments must fall within
    # five standard errors of the exact values, the errors taken from the exact distribution
    J = np.where(np.random.default_rng(11).random(3 * N2) < 0.5, -1, 1).astype(np.int8)
    ex = _exact(J, beta)
    R = 200_000
    rng = np.random.default_rng(int(beta * 1000) + 5)
    a = rng.choice(256, size=R, p=ex["p"])
    c = rng.choice(256, size=R, p=ex["p"])
    hist, P = o.overlap_hist(N2, ex["b"][a], ex["b"][c])
    assert P == R and hist.sum() == R
    q2, q4, g = o.overlap_stats(N2, hist)
    # per-pair overlap distribution of one draw: P(q) = sum over state pairs with that q
    _, sig = _states()
    qq = (sig @ sig.T) / N2
    pq = np.outer(ex["p"], ex["p"]).ravel()
    qv = qq.ravel()
    se_q2 = _se_from_influence(pq, qv ** 2, R)
    se_q4 = _se_from_influence(pq, qv ** 4, R)
    se_g = _se_from_influence(pq, (np.abs(qv) < 0.2).astype(float), R)
    assert abs(q2 - ex["q2"]) < 5 * se_q2 + 1e-12
    assert abs(q4 - ex["q4"]) < 5 * se_q4 + 1e-12
    assert abs(g - ex["gamma"]) < 5 * se_g + 1e-12
    b = o.overlap_average([0.0, 0.0], [[q2, q4, g]])[3]
    infl_b = -0.5 * ((qv ** 4 - ex["q4"]) / ex["q2"] ** 2 - 2 * ex["q4"] * (qv ** 2 - ex["q2"]) / ex["q2"] ** 3)
    assert abs(b - ex["g"]) < 5 * _se_from_influence(pq, infl_b, R) + 1e-12
    # energy moments of population A
    m = o.energy_moments(ex["E"][a].astype(np.int32))
    p, E, mu, var = ex["p"], ex["E"].astype(float), ex["mean"], ex["var"]
    sd = math.sqrt(var)
    z = (E - mu) / sd
    assert abs(m[0] - mu) < 5 * _se_from_influence(p, E, R)
    assert abs(m[1] - var) < 5 * _se_from_influence(p, (E - mu) ** 2, R) + 1e-12
    infl_skew = z ** 3 - 3 * z - 1.5 * ex["skew"] * (z ** 2 - 1)
    assert abs(m[2] - ex["skew"]) < 5 * _se_from_influence(p, infl_skew, R) + 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("beta", [0.5, 2.0])
def test_population_annealing_overlap_and_binder_2x2x2(beta):
    # end to end through the oracle's algorithm: pairs of independent runs annealed to beta, their
    # overlaps (eq. pqs with the pair weights of eq. omegaprime), Binder ratio and energy moments
    # against exact enumeration, within five standard errors across the pairs
    J = o.couplings(3, L2, 6)
    ex = _exact(J, beta)
    betas = np.linspace(0.0, beta, 9)
    n_pairs, R = 8, 6000
    x, Q, mom = [], [], []
    for p_ in range(n_pairs):
        runs = [o.run(3, L2, J, 500 + 2 * p_ + h, R, betas, 3) for h in (0, 1)]
        assert all(r[0] == 0 for r in runs)
        hist, _ = o.overlap_hist(N2, runs[0][2], runs[1][2])
        Q.append(o.overlap_stats(N2, hist))
        x += [runs[0][1][-1, 3], runs[1][1][-1, 3]]
        mom.append(runs[0][1][-1, 4:7])
    Q, mom = np.array(Q), np.array(mom)
    out = o.overlap_average(np.array(x), Q)
    tol = lambda v: 5 * v.std(ddof=1) / math.sqrt(len(v)) + 2e-3  # noqa: E731
    assert abs(out[0] - ex["q2"]) < tol(Q[:, 0])
    assert abs(out[1] - ex["q4"]) < tol(Q[:, 1])
    assert abs(out[2] - ex["gamma"]) < tol(Q[:, 2])
    g_pairs = 0.5 * (3 - Q[:, 1] / Q[:, 0] ** 2)
    assert abs(out[3] - ex["g"]) < tol(g_pairs) + 0.01
    assert abs(mom[:, 0].mean() - ex["mean"]) < tol(mom[:, 0])
    assert abs(mom[:, 1].mean() - ex["var"]) < tol(mom[:, 1]) + 0.01 * ex["var"]
    assert abs(mom[:, 2].mean() - ex["skew"]) < tol(mom[:, 2]) + 0.02
