"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks the oracle against a published value, a closed form, an exact
enumeration, an invariant or an independent library routine (scipy), chosen so
that a plausible slip (a dropped term, a wrong sign, a wrong index, a swapped
operand) in the corresponding oracle function fails.  No GPU is needed.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.special
import scipy.stats

from oracle import oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# helpers that state definitions of the problem (not the oracle's code paths)
# ----------------------------------------------------------------------------
def all_states(N):
    """every microstate of N Ising spins, one byte per spin (1 = sigma -1)"""
    return np.array(list(itertools.product([0, 1], repeat=N)), dtype=np.uint8)[:, ::-1].copy()


def ring_lnZ(beta, J):
    """exact periodic-chain partition function by transfer matrices (Sec. IV):
    Z = (2 cosh b)^N + (-1)^N prod(J) (2 sinh b)^N for E = + sum J s s."""
    N = len(J)
    s = (-1) ** N * int(np.prod(J.astype(np.int64)))
    return N * math.log(2 * math.cosh(beta)) + math.log1p(s * math.tanh(beta) ** N)


def ring_mean_energy(beta, J):
    N = len(J)
    s = (-1) ** N * int(np.prod(J.astype(np.int64)))
    t = math.tanh(beta)
    return -N * t - s * N * t ** (N - 1) * (1 - t * t) / (1 + s * t ** N)


def ring_q2(beta, J):
    """<q^2> between two independent replicas of the ring: (1/N) sum_d corr(d)^2"""
    N = len(J)
    s = (-1) ** N * int(np.prod(J.astype(np.int64)))
    t = math.tanh(beta)
    return sum(((t ** d + s * t ** (N - d)) / (1 + s * t ** N)) ** 2 for d in range(N)) / N


def cube_bond_list(L):
    """(i, j) ends of bond b = 3 i + a, the +a neighbour of site i = x + L (y + L z)"""
    ends = []
    for i in range(L ** 3):
        x, y, z = i % L, (i // L) % L, i // (L * L)
        for a in range(3):
            c = [x, y, z]
            c[a] = (c[a] + 1) % L
            ends.append((i, c[0] + L * (c[1] + L * c[2])))
    return ends


# ----------------------------------------------------------------------------
# Philox4x32-10
# ----------------------------------------------------------------------------
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        out = o.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_philox_bits_balanced():
    # each output bit of consecutive counters is set half of the time
    bits = np.array([o.philox([c, 7, 3, 2], [11, 13]) for c in range(2000)], dtype=np.uint32)
    ones = np.unpackbits(bits.view(np.uint8)).mean()
    assert abs(ones - 0.5) < 0.01


# ----------------------------------------------------------------------------
# lattice, couplings and energy (Sec. IV)
# ----------------------------------------------------------------------------
def test_couplings_pm1_and_balanced():
    J = o.couplings(3, 16, 1)
    assert J.shape == (3 * 16 ** 3,)
    assert set(np.unique(J)) <= {-1, 1}
    frac = (J == -1).mean()
    assert abs(frac - 0.5) < 5 * 0.5 / math.sqrt(len(J))
    assert np.array_equal(J, o.couplings(3, 16, 1))
    assert not np.array_equal(J, o.couplings(3, 16, 2))


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_ring_energy_matches_transfer_matrix(seed):
    # summing exp(-beta E) over all 2^12 states with the oracle's energy must give the
    # exact transfer-matrix Z: pins the + sign, the bond placement and the periodic wrap
    N = 12
    J = o.couplings(1, N, seed)
    states = all_states(N)
    E = np.array([o.energy(1, N, J, s) for s in states], dtype=np.float64)
    for beta in (0.3, 1.0, 2.5):
        lnZ = scipy.special.logsumexp(-beta * E)
        assert abs(lnZ - ring_lnZ(beta, J)) < 1e-11 * abs(lnZ)


def test_energy_ferro_and_neel():
    # with every J = +1 the all-up state costs +(number of bonds) and the two-sublattice
    # (Neel) state -(number of bonds): the energy carries a + sign (Sec. IV)
    for dim, L in ((1, 8), (3, 2), (3, 4)):
        N = L if dim == 1 else L ** 3
        B = L if dim == 1 else 3 * N
        J = np.ones(B, dtype=np.int8)
        up = np.zeros(N, dtype=np.uint8)
        neel = np.array([o.colour(dim, L, i) for i in range(N)], dtype=np.uint8)
        assert o.energy(dim, L, J, up) == B
        assert o.energy(dim, L, J, neel) == -B
        assert o.energy(dim, L, -J, neel) == B


@pytest.mark.parametrize("L", [2, 4, 6])
def test_energy_gauge_invariance(L):
    # E is unchanged by s_i -> g_i s_i, J_ij -> g_i g_j J_ij for any gauge g
    rng = np.random.default_rng(L)
    J = o.couplings(3, L, 5)
    ends = cube_bond_list(L)
    for _ in range(5):
        s = rng.integers(0, 2, L ** 3).astype(np.uint8)
        g = rng.integers(0, 2, L ** 3).astype(np.uint8)
        Jg = np.array([J[b] * (1 - 2 * int(g[i])) * (1 - 2 * int(g[j])) for b, (i, j) in enumerate(ends)], np.int8)
        assert o.energy(3, L, J, s) == o.energy(3, L, Jg, s ^ g)


def test_energy_sums_over_all_states_2x2x2():
    # over all 2^8 states: sum E = 0, and sum E^2 / 2^N = B + 2 sum over doubled pairs of
    # J_b J_b' (on L = 2 every neighbour pair carries two bonds, x+1 = x-1); every E is
    # congruent mod 4 to sum_b J_b
    L, N = 2, 8
    for seed in (1, 2, 3):
        J = o.couplings(3, L, seed)
        E = np.array([o.energy(3, L, J, s) for s in all_states(N)], dtype=np.int64)
        assert E.sum() == 0
        ends = cube_bond_list(L)
        pair = {}
        for b, (i, j) in enumerate(ends):
            pair.setdefault(frozenset((i, j)), []).append(int(J[b]))
        expect = sum(sum(v) ** 2 for v in pair.values())
        assert (E ** 2).sum() == expect * 2 ** N
        assert np.all((E - int(J.sum())) % 4 == 0)


@pytest.mark.parametrize("dim,L", [(1, 10), (3, 2), (3, 4), (3, 6)])
def test_single_flip_identities(dim, L):
    # dE_i equals E(after flip) - E(before), and sum_i dE_i = -4 E (every bond counted twice)
    rng = np.random.default_rng(dim * 100 + L)
    N = L if dim == 1 else L ** 3
    J = o.couplings(dim, L, 9)
    for _ in range(4):
        s = rng.integers(0, 2, N).astype(np.uint8)
        E = o.energy(dim, L, J, s)
        tot = 0
        for i in range(N):
            dE = o.delta_energy(dim, L, J, s, i)
            t = s.copy()
            t[i] ^= 1
            assert o.energy(dim, L, J, t) - E == dE
            assert dE % 4 == 0
            tot += dE
        assert tot == -4 * E


def test_checkerboard_colours_bipartite():
    # no bond joins two sites of the same colour (so a colour class can be updated in any order)
    for L in (2, 4, 6, 8):
        for (i, j) in cube_bond_list(L):
            assert o.colour(3, L, i) != o.colour(3, L, j)
    for i in range(16):
        assert o.colour(1, 16, i) != o.colour(1, 16, (i + 1) % 16)


def test_initial_population_uniform():
    # at beta = 0 each spin is an independent fair coin (Sec. II): mean energy 0, and
    # the replica energies have variance = number of bonds
    L = 4
    J = o.couplings(3, L, 2)
    s, E = o.init_population(3, L, J, 77, 4000)
    assert abs(s.mean() - 0.5) < 0.01
    B = 3 * L ** 3
    assert abs(E.mean()) < 5 * math.sqrt(B / 4000)
    assert abs(E.var() / B - 1) < 0.1
    assert all(o.energy(3, L, J, s[r]) == E[r] for r in range(0, 4000, 97))


# ----------------------------------------------------------------------------
# Metropolis acceptance and sweeps (Sec. II)
# ----------------------------------------------------------------------------
def test_threshold_values():
    for beta in (0.05, 0.5, 1.0, 5.0):
        for dE in (4, 8, 12):
            T, always = o.threshold(beta, dE)
            assert not always
            p = math.exp(-beta * dE)
            assert abs(T / 2.0 ** 64 - p) <= p * 2.0 ** -50 + 2.0 ** -64
        for dE in (-4, 0):
            assert o.threshold(beta, dE)[1]
    assert o.threshold(0.0, 12)[1]
    # e^{-40} 2^64 = 78.4...: a 64-bit threshold keeps acceptances a 32-bit one rounds away
    assert o.threshold(5.0, 8)[0] == 78
    # near beta = 0 the probabilities sit next to 1: e^{-4e-17} is within half an ulp of 1, so it
    # is 1 (always accept); e^{-8e-17} and e^{-1.2e-16} round to 1 - 2^-53, whose threshold is
    # (1 - 2^-53) 2^64 = 2^64 - 2^11 (first 16 bits 0xFFFF)
    assert o.threshold(1e-17, 4) == (0, True)
    assert o.threshold(1e-17, 8) == (2 ** 64 - 2 ** 11, False)
    assert o.threshold(1e-17, 12) == (2 ** 64 - 2 ** 11, False)


def _half_sweep_matrix(dim, L, J, beta, colour, states, index):
    n = len(states)
    P = np.zeros((n, n))
    sites = [i for i in range(states.shape[1]) if o.colour(dim, L, i) == colour]
    for a, s in enumerate(states):
        probs = []
        for i in sites:
            dE = o.delta_energy(dim, L, J, s, i)
            T, always = o.threshold(beta, dE)
            probs.append(1.0 if (dE <= 0 or always) else T / 2.0 ** 64)
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


@pytest.mark.parametrize("beta", [0.3, 1.0, 5.0])
def test_checkerboard_sweep_leaves_boltzmann_invariant_2x2x2(beta):
    # exact 256 x 256 transition matrix of one checkerboard sweep with the oracle's dE and
    # acceptance T64/2^64: the Boltzmann vector of the oracle's energy is stationary
    L, N = 2, 8
    J = o.couplings(3, L, 4)
    states = all_states(N)
    index = {s.tobytes(): a for a, s in enumerate(states)}
    E = np.array([o.energy(3, L, J, s) for s in states], dtype=np.float64)
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    P0 = _half_sweep_matrix(3, L, J, beta, 0, states, index)
    P1 = _half_sweep_matrix(3, L, J, beta, 1, states, index)
    assert np.allclose(P0.sum(1), 1, atol=1e-13) and np.allclose(P1.sum(1), 1, atol=1e-13)
    P = P0 @ P1
    assert np.max(np.abs(pi @ P - pi)) < 1e-12
    # each half sweep satisfies detailed balance on its own
    F = pi[:, None] * P0
    assert np.max(np.abs(F - F.T)) < 1e-12


def test_sweep_samples_boltzmann_2x2x2():
    # the oracle's actual sweep loop (with its Philox streams): energy histogram of many
    # replicas after sweeps at beta vs the exact Boltzmann distribution by enumeration
    L, N = 2, 8
    J = o.couplings(3, L, 4)
    beta = 0.6
    E_all = np.array([o.energy(3, L, J, s) for s in all_states(N)])
    levels, mult = np.unique(E_all, return_counts=True)
    p = mult * np.exp(-beta * (levels - levels.min()))
    p /= p.sum()
    R = 20000
    s, E = o.init_population(3, L, J, 12345, R)
    o.sweep(3, L, J, 12345, beta, R, s, E, 0, 30)
    assert all(o.energy(3, L, J, s[r]) == E[r] for r in range(0, R, 331))
    obs = np.array([(E == e).sum() for e in levels])
    m = R * p > 5
    chi2 = ((obs[m] - R * p[m]) ** 2 / (R * p[m])).sum()
    assert scipy.stats.chi2.sf(chi2, m.sum() - 1) > 1e-4


def test_sweep_keeps_ring_boltzmann_sample():
    # ring N = 12: replicas drawn exactly from the Boltzmann distribution (by enumeration)
    # stay Boltzmann-distributed under the oracle's sweeps.  (Started from a uniform state
    # the +-J ring does not reach Boltzmann: with zero-cost flips always accepted, domain
    # walls move deterministically under the checkerboard order, so the chain is not
    # ergodic on the ring; invariance is what population annealing relies on.)
    N = 12
    J = o.couplings(1, N, 6)
    beta = 0.8
    states = all_states(N)
    E_all = np.array([o.energy(1, N, J, s) for s in states])
    p = np.exp(-beta * (E_all - E_all.min()))
    p /= p.sum()
    R = 20000
    pick = np.random.default_rng(5).choice(len(states), size=R, p=p)
    s = states[pick].copy()
    E = E_all[pick].astype(np.int32)
    o.sweep(1, N, J, 99, beta, R, s, E, 0, 25)
    assert all(o.energy(1, N, J, s[r]) == E[r] for r in range(0, R, 173))
    levels = np.unique(E_all)
    pl = np.array([p[E_all == e].sum() for e in levels])
    obs = np.array([(E == e).sum() for e in levels])
    m = R * pl > 5
    chi2 = ((obs[m] - R * pl[m]) ** 2 / (R * pl[m])).sum()
    assert scipy.stats.chi2.sf(chi2, m.sum() - 1) > 1e-4
    assert abs(E.mean() - ring_mean_energy(beta, J)) < 5 * E.std() / math.sqrt(R)


def test_met_uniform_acceptance_rate():
    # the accept decision for threshold T is taken with probability T/2^64 (first look + tie)
    seed = 2024
    for T in (2 ** 63, 3 * 2 ** 60 + 12345, 2 ** 48 * 7 + 5):
        hits = sum(o.lib().orc_met_accept(seed, r, 3, 1, i, T) for r in range(200) for i in range(100))
        p = T / 2.0 ** 64
        n = 20000
        assert abs(hits - n * p) < 5 * math.sqrt(n * p * (1 - p)) + 1


def test_sweep_deterministic_and_seed_dependent():
    L = 4
    J = o.couplings(3, L, 1)
    a, Ea = o.init_population(3, L, J, 5, 64)
    b, Eb = a.copy(), Ea.copy()
    o.sweep(3, L, J, 5, 1.0, 64, a, Ea, 0, 3)
    o.sweep(3, L, J, 5, 1.0, 64, b, Eb, 0, 3)
    assert np.array_equal(a, b) and np.array_equal(Ea, Eb)
    c, Ec = o.init_population(3, L, J, 5, 64)
    o.sweep(3, L, J, 5, 1.0, 64, c, Ec, 1, 3)  # other sweep indices, other stream
    assert not np.array_equal(a, c)


# ----------------------------------------------------------------------------
# Poisson copy numbers (Sec. II)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("m", [-20, -7, -1, 0, 1, 3, 6])
def test_ladder_table_is_poisson_cdf(m):
    # C[n] = floor(CDF_{2^m}(n) 2^32), checked against scipy's Poisson CDF
    C = o.ladder_table(m)
    lam = 2.0 ** m
    assert C[-1] == 2 ** 32
    assert np.all(np.diff(C.astype(np.float64)) >= 0)
    n = np.arange(len(C) - 1)
    ref = scipy.stats.poisson.cdf(n, lam) * 2.0 ** 32
    assert np.all(np.abs(C[:-1].astype(np.float64) - np.floor(ref)) <= 2)
    assert C[0] == math.floor(math.exp(-lam) * 2 ** 32)
    # the tail beyond the table is below 2^-32
    assert scipy.stats.poisson.sf(len(C) - 1, lam) < 2.0 ** -32


@pytest.mark.parametrize("lam", [1e-7, 0.3, 1.0, 2.5, 7.25, 64.0, 100.0, 1000.5])
def test_poisson_sampler_distribution(lam):
    n = 20000 if lam < 200 else 4000
    x = np.array([o.poisson(lam, 31337, j, 9) for j in range(n)])
    assert abs(x.mean() - lam) < 5 * math.sqrt(lam / n) + 1e-9
    if lam >= 0.3:
        assert abs(x.var() / lam - 1) < 5 * math.sqrt(2.0 / n) + 0.02
        ks = np.arange(x.max() + 1)
        p = scipy.stats.poisson.pmf(ks, lam)
        obs = np.bincount(x, minlength=len(ks))
        mk = n * p > 5
        chi2 = ((obs[mk] - n * p[mk]) ** 2 / (n * p[mk])).sum()
        assert scipy.stats.chi2.sf(chi2, max(mk.sum() - 1, 1)) > 1e-4
    assert o.poisson(0.0, 1, 0, 0) == 0


# ----------------------------------------------------------------------------
# resampling, Q and the free energy (Sec. II, eqs. Q, wn, sumQ)
# ----------------------------------------------------------------------------
def _pop(dim, L, seed, R, beta=0.0, ns=0):
    J = o.couplings(dim, L, 1)
    s, E = o.init_population(dim, L, J, seed, R)
    if ns:
        o.sweep(dim, L, J, seed, beta, R, s, E, 0, ns)
    return J, s, E


def test_resample_zero_step_gives_Q_one():
    J, s, E = _pop(3, 4, 3, 500)
    r = o.resample(3, 4, 3, 1, 0.7, 0.7, 500, 500, s, E, 2000)
    assert r["status"] == 0 and r["lnQ"] == 0.0


def test_resample_single_energy_gives_exact_Q():
    # a population all at one energy: Q = exp(-dbeta E) exactly
    L, N = 4, 64
    J = o.couplings(3, L, 1)
    s = np.zeros((300, N), np.uint8)
    E = np.full(300, o.energy(3, L, J, s[0]), np.int32)
    r = o.resample(3, L, 1, 1, 0.2, 0.45, 300, 300, s, E, 2000)
    assert r["lnQ"] == -(0.45 - 0.2) * float(E[0])


def test_resample_lnQ_is_log_mean_weight():
    # ln Q = ln[(1/R) sum_j exp(-dbeta E_j)] (eq. Q), evaluated independently with fsum
    J, s, E = _pop(3, 6, 8, 3000, beta=0.5, ns=3)
    for b0, b1 in ((0.5, 0.55), (0.5, 0.9), (0.5, 3.0)):
        r = o.resample(3, 6, 8, 2, b0, b1, 3000, 3000, s, E, 10000)
        Emin = int(E.min())
        ref = -(b1 - b0) * Emin + math.log(math.fsum(math.exp(-(b1 - b0) * (e - Emin)) for e in E.tolist())) - math.log(3000)
        assert abs(r["lnQ"] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_resample_conservation_and_gather():
    L, N = 4, 64
    J, s, E = _pop(3, L, 21, 2000, beta=0.4, ns=2)
    r = o.resample(3, L, 21, 5, 0.4, 0.6, 2000, 2000, s, E, 5000)
    assert r["status"] == 0
    c, off = r["counts"], r["offsets"]
    assert off[0] == 0 and np.array_equal(np.diff(off), c) and off[-1] == r["R_new"] == c.sum()
    src = np.repeat(np.arange(2000), c)
    assert np.array_equal(r["s"][: r["R_new"]], s[src])
    assert np.array_equal(r["E"][: r["R_new"]], E[src])
    assert all(o.energy(3, L, J, r["s"][k]) == r["E"][k] for k in range(0, r["R_new"], 53))
    assert r["E_lo"] == E.min()


def test_resample_mean_size_is_target():
    # E[R~'] = R_target: sum_j lambda_j = R_target (z-test over steps)
    J, s, E = _pop(3, 4, 4, 1000, beta=0.3, ns=2)
    sizes = [o.resample(3, 4, 4, k, 0.3, 0.5, 1500, 1000, s, E, 10000)["R_new"] for k in range(1, 301)]
    assert abs(np.mean(sizes) - 1500) < 5 * math.sqrt(1500 / 300)


def test_resample_copy_counts_are_poisson_in_tau():
    # two energy levels: copies ~ Poisson(R_target w_j / S) with w = exp(-dbeta (E - E_lo))
    N, R = 16, 4000
    J = o.couplings(1, N, 1)
    s = np.zeros((R, N), np.uint8)
    s[R // 2:, 0] = 1  # second half has one flipped spin: higher or lower energy
    E = np.array([o.energy(1, N, J, x) for x in s], np.int32)
    dbeta = 0.3
    r = o.resample(1, N, 1, 7, 1.0, 1.0 + dbeta, R, R, s, E, 4 * R)
    Elo = E.min()
    w = np.exp(-dbeta * (E - Elo))
    lam = R * w / w.sum()
    for level in np.unique(E):
        sel = E == level
        cnt = r["counts"][sel]
        lm = lam[sel][0]
        assert abs(cnt.mean() - lm) < 5 * math.sqrt(lm / sel.sum())


def test_resample_errors():
    J, s, E = _pop(1, 16, 2, 100)
    assert o.resample(1, 16, 2, 1, 0.0, 0.1, 100, 100, s, E, 50)["status"] == o.ERR_CAPACITY
    assert o.resample(1, 16, 2, 1, 0.0, 0.1, 1e-12, 100, s, E, 500)["status"] == o.ERR_EXTINCT
    assert o.resample(1, 16, 2, 1, 0.5, 0.1, 100, 100, s, E, 500)["status"] == o.ERR_ARG


def test_free_energy_starts_at_ln_omega():
    st, rec, _, _ = o.run(1, 16, o.couplings(1, 16, 1), 5, 100, [0.0, 0.1], 1)
    assert st == 0 and rec[0, 3] == 16 * math.log(2.0)
    assert abs(rec[1, 3] - (16 * math.log(2.0) + rec[1, 2])) < 1e-14 * rec[1, 3]


@pytest.mark.slow
def test_weighted_free_energy_and_energy_match_exact_ring():
    # the paper's 1D check (Sec. IV) on a +-J ring with an exact Z: weighted -beta F_bar and
    # E_bar within statistical error of the transfer-matrix values at every sampled beta
    N, R, M = 64, 1000, 48
    J = o.couplings(1, N, 1)
    betas = np.array([5.0 * k / 50 for k in range(51)])
    runs = [o.run(1, N, J, 1000 + m, R, betas, 5)[1] for m in range(M)]
    x = np.array([r[:, 3] for r in runs])
    Es = np.array([r[:, 4] for r in runs])
    rng = np.random.default_rng(0)
    for k in (10, 25, 50):
        w = o.weighted_average(x[:, k], Es[:, k:k + 1])
        boot = []
        for _ in range(100):  # bootstrap over runs (Sec. III)
            idx = rng.integers(0, M, M)
            bw = o.weighted_average(x[idx, k], Es[idx, k:k + 1])
            boot.append((bw["minus_betaF_bar"], bw["A_bar"][0]))
        boot = np.array(boot)
        errF = max(boot[:, 0].std(), 1e-3)
        errE = max(boot[:, 1].std(), 1e-4)
        assert abs(w["minus_betaF_bar"] - ring_lnZ(betas[k], J)) < 4 * errF
        assert abs(w["A_bar"][0] - ring_mean_energy(betas[k], J)) < 4 * errE + 1e-9


@pytest.mark.slow
def test_unweighted_mean_biased_weighted_not_small_R():
    # small populations: the plain mean of -beta F~ sits below ln Z by about Var/2, the
    # weighted estimate (eq. bestf) does not (Sec. III)
    N, R, M = 32, 40, 300
    J = o.couplings(1, N, 3)
    betas = np.array([3.0 * k / 30 for k in range(31)])
    x = np.array([o.run(1, N, J, 5000 + m, R, betas, 2)[1][-1, 3] for m in range(M)])
    exact = ring_lnZ(3.0, J)
    w = o.weighted_average(x)
    se = math.sqrt(w["var"] / M)
    assert w["var"] > 0.05
    assert exact - w["mean"] > 4 * se  # plain mean visibly biased low
    assert abs((exact - w["mean"]) - w["var"] / 2) < 0.5 * w["var"] + 3 * se
    assert abs(w["minus_betaF_bar"] - exact) < abs(exact - w["mean"]) / 2


@pytest.mark.slow
def test_variance_scales_inversely_with_population():
    # Var(beta F~) roughly proportional to 1/R (Sec. IV: R x5 gave Var / 4.7)
    N, M = 32, 160
    J = o.couplings(1, N, 4)
    betas = np.array([3.0 * k / 30 for k in range(31)])
    v = []
    for R in (60, 300):
        x = np.array([o.run(1, N, J, 7000 + m, R, betas, 2)[1][-1, 3] for m in range(M)])
        v.append(x.var(ddof=1))
    assert 2.5 < v[0] / v[1] < 9


# ----------------------------------------------------------------------------
# overlap (Sec. IV)
# ----------------------------------------------------------------------------
def test_overlap_hist_extremes():
    N = 64
    a = np.random.default_rng(1).integers(0, 2, (10, N)).astype(np.uint8)
    h, P = o.overlap_hist(N, a, a)
    assert P == 10 and h[0] == 10
    h, P = o.overlap_hist(N, a, 1 - a)
    assert h[N] == 10
    h, P = o.overlap_hist(N, a[:4], a)  # pairs j < min(R_A, R_B)
    assert P == 4
    q2, q4, g = o.overlap_stats(N, np.bincount([N // 2], minlength=N + 1))
    assert q2 == 0 and q4 == 0 and g == 1


@pytest.mark.slow
def test_overlap_q2_matches_exact_ring():
    # pairs of independent runs on the ring: weighted <q^2> (pair weights, eq. omegaprime)
    # against the exact two-replica value
    N, R, M = 32, 400, 24
    J = o.couplings(1, N, 2)
    betas = np.array([1.2 * k / 12 for k in range(13)])
    q2s, xs = [], []
    for m in range(M):
        sta, ra, sa, _ = o.run(1, N, J, 100 + 2 * m, R, betas, 3)
        stb, rb, sb, _ = o.run(1, N, J, 101 + 2 * m, R, betas, 3)
        h, P = o.overlap_hist(N, sa, sb)
        q2s.append(o.overlap_stats(N, h)[0])
        xs.append(ra[-1, 3] + rb[-1, 3])
    w = o.weighted_average(np.array(xs), np.array(q2s)[:, None])
    exact = ring_q2(1.2, J)
    se = np.std(q2s) / math.sqrt(M)
    assert abs(w["A_bar"][0] - exact) < 5 * se + 0.01 * exact


# ----------------------------------------------------------------------------
# weighted averages (Sec. III)
# ----------------------------------------------------------------------------
def test_weighted_average_special_cases():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(7, 3))
    w = o.weighted_average(np.full(7, 3.5), A)
    assert np.allclose(w["A_bar"], A.mean(0), rtol=1e-14) and np.allclose(w["omega"], 1 / 7)
    assert abs(w["minus_betaF_bar"] - 3.5) < 1e-14
    x = np.array([0.0, 0.0, 800.0, 0.0])
    w = o.weighted_average(x, A[:4])
    assert np.allclose(w["A_bar"], A[2]) and w["omega"][2] == 1.0
    assert abs(w["minus_betaF_bar"] - (800.0 - math.log(4))) < 1e-12
    x = rng.normal(size=7) + 1000.0
    w = o.weighted_average(x, A)
    perm = rng.permutation(7)
    wp = o.weighted_average(x[perm], A[perm])
    assert np.allclose(w["A_bar"], wp["A_bar"], rtol=1e-13)
    assert abs(w["minus_betaF_bar"] - (scipy.special.logsumexp(x) - math.log(7))) < 1e-12
    assert abs(w["var"] - np.var(x, ddof=1)) < 1e-12
    # unequal target sizes: weights R^(r) exp(x_r) (Sec. III)
    Rr = rng.uniform(1e4, 1e5, 7)
    wr = o.weighted_average(x, A, Rr)
    ref_w = np.exp(x - x.max()) * Rr
    ref_w /= ref_w.sum()
    assert np.allclose(wr["omega"], ref_w, rtol=1e-12)
    assert abs(wr["minus_betaF_bar"] - (scipy.special.logsumexp(x, b=Rr) - math.log(Rr.sum()))) < 1e-12
    wq = o.weighted_average(x, A, np.full(7, 5e4))
    assert np.allclose(wq["A_bar"], w["A_bar"], rtol=1e-13)
