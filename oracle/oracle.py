"""ctypes front end of the CPU oracle (``pa_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the library.  Arrays are numpy
arrays owned by the caller; every function forwards to the plain C oracle.

Spins are stored one byte per spin, 1 meaning sigma = -1, replica-major
([R][N]).  Couplings are int8 +-1, one per bond (bond i joins sites i and i+1
on the chain; bond 3 i + a joins site i and its +a neighbour on the cube).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pa_oracle.c")
_LIB = os.path.join(_HERE, "libpa_oracle.so")

OK, ERR_ARG, ERR_CAPACITY, ERR_EXTINCT, ERR_NONFINITE = 0, 1, 2, 3, 4
REC_W = 8  # beta, R, lnQ, -beta F, E mean, E var, E skew, status


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11 + OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
             "-o", tmp, _SRC, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.orc_philox.argtypes = [P, P, P]
        L.orc_num_sites.argtypes = [i32, i32]
        L.orc_num_bonds.argtypes = [i32, i32]
        L.orc_colour.argtypes = [i32, i32, i32]
        L.orc_couplings.argtypes = [i32, i32, u64, P]
        L.orc_energy.argtypes = [i32, i32, P, P]
        L.orc_energy.restype = i64
        L.orc_delta_energy.argtypes = [i32, i32, P, P, i32]
        L.orc_init_population.argtypes = [i32, i32, P, u64, i64, P, P]
        L.orc_init_range.argtypes = [i32, i32, P, u64, i64, i64, P, P]
        L.orc_sweep_range.argtypes = [i32, i32, P, u64, f64, i64, i64, P, P, i64, i32]
        L.orc_copy_numbers.argtypes = [u64, i64, f64, f64, f64, i64, P, P, P]
        L.orc_threshold.argtypes = [f64, i32, P]
        L.orc_threshold.restype = u64
        L.orc_met_accept.argtypes = [u64, i64, i64, i32, i32, u64]
        L.orc_sweep.argtypes = [i32, i32, P, u64, f64, i64, P, P, i64, i32]
        L.orc_ladder_table.argtypes = [i32, P]
        L.orc_poisson.argtypes = [f64, u64, i64, i64]
        L.orc_poisson.restype = i64
        L.orc_resample.argtypes = [i32, i32, u64, i64, f64, f64, f64, i64, P, P, i64, P, P, P, P, P, P]
        L.orc_energy_moments.argtypes = [i64, P, P]
        L.orc_overlap_hist.argtypes = [i32, i64, P, i64, P, P]
        L.orc_overlap_hist.restype = i64
        L.orc_overlap_stats.argtypes = [i32, P, P]
        L.orc_weighted_average.argtypes = [i32, P, P, P, i32, P, P, P, P, P]
        L.orc_overlap_average.argtypes = [i32, P, P, P, P]
        L.orc_run.argtypes = [i32, i32, P, u64, i64, i32, P, P, i32, i64, P, P, P, P]
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.argtypes = [i32]
        L.orc_set_num_threads.restype = None
        L.orc_expd.argtypes = [f64]
        L.orc_expd.restype = f64
        L.orc_couplings_gauss.argtypes = [i32, i32, u64, P]
        L.orc_energy_gauss.argtypes = [i32, i32, P, P]
        L.orc_energy_gauss.restype = f64
        L.orc_delta_energy_gauss.argtypes = [i32, i32, P, P, i32]
        L.orc_delta_energy_gauss.restype = f64
        L.orc_init_range_gauss.argtypes = [i32, i32, P, u64, i64, i64, P, P]
        L.orc_sweep_range_gauss.argtypes = [i32, i32, P, u64, f64, i64, i64, P, P, i64, i32]
        L.orc_copy_numbers_gauss.argtypes = [u64, i64, f64, f64, f64, i64, P, P, P]
        L.orc_energy_moments_gauss.argtypes = [i64, P, P]
        L.orc_run_gauss.argtypes = [i32, i32, P, u64, i64, i32, P, P, i32, i64, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def num_sites(dim, L):
    return L if dim == 1 else L ** 3


def num_bonds(dim, L):
    return L if dim == 1 else 3 * L ** 3


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(c), _p(k), _p(out))
    return out


def couplings(dim, L, disorder_seed):
    J = np.zeros(num_bonds(dim, L), dtype=np.int8)
    lib().orc_couplings(dim, L, disorder_seed, _p(J))
    return J


def energy(dim, L, J, s):
    return int(lib().orc_energy(dim, L, _p(np.ascontiguousarray(J, np.int8)), _p(np.ascontiguousarray(s, np.uint8))))


def delta_energy(dim, L, J, s, i):
    return int(lib().orc_delta_energy(dim, L, _p(np.ascontiguousarray(J, np.int8)),
                                      _p(np.ascontiguousarray(s, np.uint8)), i))


def colour(dim, L, i):
    return int(lib().orc_colour(dim, L, i))


def init_population(dim, L, J, seed, R, capacity=None):
    N = num_sites(dim, L)
    cap = capacity or R
    s = np.zeros((cap, N), dtype=np.uint8)
    E = np.zeros(cap, dtype=np.int32)
    lib().orc_init_population(dim, L, _p(J), seed, R, _p(s), _p(E))
    return s, E


def init_replicas(dim, L, J, seed, r_first, count):
    """replicas r_first .. r_first + count - 1 of the initial population"""
    N = num_sites(dim, L)
    s = np.zeros((count, N), dtype=np.uint8)
    E = np.zeros(count, dtype=np.int32)
    lib().orc_init_range(dim, L, _p(np.ascontiguousarray(J, np.int8)), seed, r_first, count, _p(s), _p(E))
    return s, E


def sweep_replicas(dim, L, J, seed, beta, r_first, s, E, t0, ns):
    """In place: ns sweeps of replicas with population indices r_first .. r_first + len(E) - 1."""
    assert s.dtype == np.uint8 and E.dtype == np.int32 and s.flags.c_contiguous and E.flags.c_contiguous
    lib().orc_sweep_range(dim, L, _p(np.ascontiguousarray(J, np.int8)), seed, beta, r_first, len(E), _p(s), _p(E),
                          t0, ns)


def copy_numbers(seed, k, beta_from, beta_to, R_target, E):
    """Q and the Poisson copy numbers of a population with energies E: (status, counts, S, lnQ, E_lo)."""
    E = np.ascontiguousarray(E, np.int32)
    counts = np.zeros(len(E), dtype=np.int32)
    out = np.zeros(3)
    st = lib().orc_copy_numbers(seed, k, beta_from, beta_to, float(R_target), len(E), _p(E), _p(counts), _p(out))
    return st, counts, out[0], out[1], int(out[2])


def threshold(beta, dE):
    always = ctypes.c_int(0)
    T = lib().orc_threshold(beta, dE, ctypes.byref(always))
    return int(T), bool(always.value)


def sweep(dim, L, J, seed, beta, R, s, E, t0, ns):
    """In place: ns checkerboard sweeps of the first R replicas."""
    assert s.dtype == np.uint8 and E.dtype == np.int32 and s.flags.c_contiguous
    lib().orc_sweep(dim, L, _p(J), seed, beta, R, _p(s), _p(E), t0, ns)


def ladder_table(m):
    C = np.zeros(512, dtype=np.uint64)
    n = lib().orc_ladder_table(m, _p(C))
    return C[:n].copy()


def poisson(lam, seed, j, k):
    return int(lib().orc_poisson(lam, seed, j, k))


def resample(dim, L, seed, k, beta_from, beta_to, R_target, R, s, E, capacity):
    """Returns (status, s_new, E_new, counts, offsets, S, lnQ, E_lo, R_new)."""
    N = num_sites(dim, L)
    s_new = np.zeros((capacity, N), dtype=np.uint8)
    E_new = np.zeros(capacity, dtype=np.int32)
    counts = np.zeros(max(R, 1), dtype=np.int32)
    offsets = np.zeros(R + 1, dtype=np.int64)
    out = np.zeros(3, dtype=np.float64)
    R_new = ctypes.c_int64(0)
    st = lib().orc_resample(dim, L, seed, k, beta_from, beta_to, float(R_target), R, _p(s), _p(E), capacity,
                            _p(s_new), _p(E_new), _p(counts), _p(offsets), _p(out), ctypes.byref(R_new))
    return dict(status=st, s=s_new, E=E_new, counts=counts[:R], offsets=offsets, S=out[0], lnQ=out[1],
                E_lo=int(out[2]), R_new=R_new.value)


def energy_moments(E):
    E = np.ascontiguousarray(E, np.int32)
    out = np.zeros(3)
    lib().orc_energy_moments(len(E), _p(E), _p(out))
    return out


def overlap_hist(N, sA, sB):
    sA = np.ascontiguousarray(sA, np.uint8)
    sB = np.ascontiguousarray(sB, np.uint8)
    hist = np.zeros(N + 1, dtype=np.int64)
    P = lib().orc_overlap_hist(N, sA.shape[0], _p(sA), sB.shape[0], _p(sB), _p(hist))
    return hist, int(P)


def overlap_stats(N, hist):
    hist = np.ascontiguousarray(hist, np.int64)
    out = np.zeros(3)
    lib().orc_overlap_stats(N, _p(hist), _p(out))
    return out  # q2, q4, Gamma


def weighted_average(x, A=None, R=None):
    """x: [M] of -beta F~_r; A: [M][n_obs]; R: [M] target sizes or None."""
    x = np.ascontiguousarray(x, np.float64)
    M = len(x)
    if A is None:
        A = np.zeros((M, 0))
    A = np.ascontiguousarray(np.asarray(A, np.float64).reshape(M, -1))
    n_obs = A.shape[1]
    Rr = None if R is None else np.ascontiguousarray(R, np.float64)
    A_bar = np.zeros(max(n_obs, 1))
    omega = np.zeros(M)
    mbF = ctypes.c_double(0)
    var = ctypes.c_double(0)
    mean = ctypes.c_double(0)
    st = lib().orc_weighted_average(M, _p(x), _p(Rr), _p(A), n_obs, _p(A_bar), _p(omega),
                                    ctypes.byref(mbF), ctypes.byref(var), ctypes.byref(mean))
    assert st == OK
    return dict(A_bar=A_bar[:n_obs], omega=omega, minus_betaF_bar=mbF.value, var=var.value, mean=mean.value)


def overlap_average(x, Q, R=None):
    """Weighted overlap observables over pairs of runs (Sec. IV, eqs. pqs and omegaprime).
    x: [2 n_pairs] of -beta F~ per run (pair p = runs 2p, 2p + 1); Q: [n_pairs][3] of the pair's
    (<q^2>, <q^4>, Gamma); R: [2 n_pairs] target sizes or None.  Returns ([q^2], [q^4], [Gamma], g)
    with the Binder ratio g = (3 - [q^4] / [q^2]^2) / 2."""
    x = np.ascontiguousarray(x, np.float64)
    Q = np.ascontiguousarray(np.asarray(Q, np.float64).reshape(-1, 3))
    n = Q.shape[0]
    assert len(x) == 2 * n
    Rr = None if R is None else np.ascontiguousarray(R, np.float64)
    out = np.zeros(4)
    st = lib().orc_overlap_average(n, _p(x), _p(Rr), _p(Q), _p(out))
    assert st == OK
    return out


def run(dim, L, J, seed, R0, betas, ns, capacity=None, R_targets=None):
    """A whole run; returns (status, rec[nT][8], final spins, final E)."""
    N = num_sites(dim, L)
    betas = np.ascontiguousarray(betas, np.float64)
    nT = len(betas)
    cap = capacity or int(R0 * 1.5 + 64)
    rec = np.zeros((nT, REC_W))
    s = np.zeros((cap, N), dtype=np.uint8)
    E = np.zeros(cap, dtype=np.int32)
    R_out = ctypes.c_int64(0)
    Rt = None if R_targets is None else np.ascontiguousarray(R_targets, np.float64)
    st = lib().orc_run(dim, L, _p(np.ascontiguousarray(J, np.int8)), seed, R0, nT, _p(betas), _p(Rt), ns, cap,
                       _p(rec), _p(s), _p(E), ctypes.byref(R_out))
    R = R_out.value
    return st, rec, s[:R], E[:R]


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n):
    """Threads of the oracle's OpenMP loops from now on."""
    lib().orc_set_num_threads(int(n))


def bootstrap(x, idx, A=None, R=None):
    """Bootstrap errors of the weighted averages (Sec. III: the error is the standard deviation
    over resampled ensembles of size M).  idx [n_boot][M]: run indices drawn with replacement,
    one resampled ensemble per row.  Returns (replicates [n_boot][n_obs + 3], errors [n_obs + 3]):
    each replicate row is (A_bar[0..n_obs-1], -beta F_bar, Var, mean) of weighted_average on the
    resampled runs; errors are the standard deviations over the rows (1 / (n_boot - 1))."""
    x = np.asarray(x, np.float64)
    M = len(x)
    A = np.zeros((M, 0)) if A is None else np.asarray(A, np.float64).reshape(M, -1)
    idx = np.asarray(idx, np.int64)
    reps = []
    for row in idx:
        w = weighted_average(x[row], A[row], None if R is None else np.asarray(R, np.float64)[row])
        reps.append(np.concatenate([w["A_bar"], [w["minus_betaF_bar"], w["var"], w["mean"]]]))
    reps = np.array(reps)
    n = len(reps)
    mean = reps.sum(axis=0) / n
    err = np.sqrt(((reps - mean) ** 2).sum(axis=0) / (n - 1)) if n > 1 else np.zeros(reps.shape[1])
    return reps, err


def ring_exact(J, beta):
    """ln Z and the mean energy of the periodic +-J chain with E = + sum_i J_i s_i s_(i+1) (the sign
    of Sec. IV), from the 2 x 2 transfer matrices T_i = [[e^(-b J_i), e^(b J_i)], [e^(b J_i),
    e^(-b J_i)]]: Z = trace of their product, E = -d ln Z / d beta by the product rule (each
    factor rescaled by its largest entry to keep the product finite)."""
    J = np.asarray(J, np.float64)
    P = np.eye(2)
    dP = np.zeros((2, 2))
    lnc = 0.0
    for j in J:
        T = np.array([[np.exp(-beta * j), np.exp(beta * j)], [np.exp(beta * j), np.exp(-beta * j)]])
        dT = np.array([[-j * np.exp(-beta * j), j * np.exp(beta * j)], [j * np.exp(beta * j), -j * np.exp(-beta * j)]])
        c = np.abs(T).max()
        dP = dP @ (T / c) + P @ (dT / c)
        P = P @ (T / c)
        lnc += np.log(c)
    Z = np.trace(P)
    return lnc + np.log(Z), -np.trace(dP) / Z


# ------------------------------------------------------------------ Gaussian couplings (Sec. IV)

def expd(x):
    """exp written out (Cody-Waite reduction, Taylor series to r^13, exact scaling)."""
    return lib().orc_expd(float(x))


def couplings_gauss(dim, L, disorder_seed):
    J = np.zeros(num_bonds(dim, L), dtype=np.float64)
    lib().orc_couplings_gauss(dim, L, disorder_seed, _p(J))
    return J


def energy_gauss(dim, L, J, s):
    return lib().orc_energy_gauss(dim, L, _p(np.ascontiguousarray(J, np.float64)), _p(np.ascontiguousarray(s, np.uint8)))


def delta_energy_gauss(dim, L, J, s, i):
    return lib().orc_delta_energy_gauss(dim, L, _p(np.ascontiguousarray(J, np.float64)),
                                        _p(np.ascontiguousarray(s, np.uint8)), i)


def init_replicas_gauss(dim, L, J, seed, r_first, count):
    N = num_sites(dim, L)
    s = np.zeros((count, N), dtype=np.uint8)
    E = np.zeros(count, dtype=np.float64)
    lib().orc_init_range_gauss(dim, L, _p(np.ascontiguousarray(J, np.float64)), seed, r_first, count, _p(s), _p(E))
    return s, E


def sweep_replicas_gauss(dim, L, J, seed, beta, r_first, s, E, t0, ns):
    """In place: ns sweeps of replicas r_first .. r_first + len(s) - 1; energies recomputed after."""
    assert s.flags.c_contiguous and E.flags.c_contiguous and E.dtype == np.float64
    lib().orc_sweep_range_gauss(dim, L, _p(np.ascontiguousarray(J, np.float64)), seed, beta, r_first, len(s), _p(s),
                                _p(E), t0, ns)


def copy_numbers_gauss(seed, k, beta_from, beta_to, R_target, E):
    E = np.ascontiguousarray(E, np.float64)
    counts = np.zeros(len(E), dtype=np.int32)
    out = np.zeros(3)
    st = lib().orc_copy_numbers_gauss(seed, k, beta_from, beta_to, R_target, len(E), _p(E), _p(counts), _p(out))
    return st, counts, out[0], out[1], out[2]


def energy_moments_gauss(E):
    E = np.ascontiguousarray(E, np.float64)
    out = np.zeros(3)
    lib().orc_energy_moments_gauss(len(E), _p(E), _p(out))
    return out


def run_gauss(dim, L, J, seed, R0, betas, ns, capacity=None, R_targets=None):
    """A whole run with Gaussian couplings; returns (status, rec[nT][8], final spins, final E)."""
    N = num_sites(dim, L)
    betas = np.ascontiguousarray(betas, np.float64)
    nT = len(betas)
    cap = capacity or int(R0 * 1.5 + 64)
    rec = np.zeros((nT, REC_W))
    s = np.zeros((cap, N), dtype=np.uint8)
    E = np.zeros(cap, dtype=np.float64)
    R_out = ctypes.c_int64(0)
    Rt = None if R_targets is None else np.ascontiguousarray(R_targets, np.float64)
    st = lib().orc_run_gauss(dim, L, _p(np.ascontiguousarray(J, np.float64)), seed, R0, nT, _p(betas), _p(Rt), ns,
                             cap, _p(rec), _p(s), _p(E), ctypes.byref(R_out))
    R = R_out.value
    return st, rec, s[:R], E[:R]
