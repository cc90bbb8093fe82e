"""Seeded synthetic inputs shared by the GPU tests and the oracle tests.

Only random numbers and shapes live here, none of the method's arithmetic: both sides
receive the same arrays and compute from them independently.
"""
from __future__ import annotations

import numpy as np


def mlp_theta(seed, scale=1.0):
    """FP32 parameter vector of the 6-64-64-64-1 network (8833 values): weights uniform in
    +-scale * sqrt(6 / (fan_in + fan_out)), biases uniform in +-0.1 scale."""
    g = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((6, 64), (64, 64), (64, 64), (64, 1)):
        a = scale * np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(g.uniform(-a, a, fan_in * fan_out))
        parts.append(g.uniform(-0.1 * scale, 0.1 * scale, fan_out))
    return np.concatenate(parts).astype(np.float32)


def mlp_features(seed, B, zero_var_every=0):
    """[B][6] FP32 feature rows (beta, ln N, ln R, E/N, var/N, skew) over the ranges the
    configurations produce; every zero_var_every-th row has var/N = 0."""
    g = np.random.default_rng(seed)
    X = np.empty((B, 6), np.float32)
    X[:, 0] = g.uniform(0.0, 5.0, B)
    X[:, 1] = np.log(g.choice([64.0, 216.0, 512.0, 1728.0, 4096.0], B))
    X[:, 2] = g.uniform(6.9, 13.8, B)
    X[:, 3] = g.uniform(-1.8, 0.0, B)
    X[:, 4] = np.exp(g.uniform(np.log(1e-3), np.log(3.0), B))
    X[:, 5] = g.uniform(-2.0, 2.0, B)
    if zero_var_every:
        X[::zero_var_every, 4] = 0.0
    return X


def mlp_targets(seed, B, bad_every=0):
    """[B] FP64 step labels, log-uniform in [1e-3, 1]; every bad_every-th is 0."""
    g = np.random.default_rng(seed)
    t = np.exp(g.uniform(np.log(1e-3), 0.0, B))
    if bad_every:
        t[::bad_every] = 0.0
    return t


def float32_values(seed, n):
    """FP32 values for rounding tests: random magnitudes over the normal range plus ties,
    subnormals, zeros, infinities and NaN."""
    g = np.random.default_rng(seed)
    x = (g.standard_normal(n) * np.exp(g.uniform(-30, 30, n))).astype(np.float32)
    u = x.view(np.uint32)
    u[: n // 8] = (u[: n // 8] & 0xFFFF0000) | 0x8000          # exact ties
    u[n // 8: n // 4] = (u[n // 8: n // 4] & 0xFFFF0000) | 0x7FFF
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-40, -1e-40, 3.4e38, -3.4e38], np.float32)
    x[-len(special):] = special
    return x


def overlap_pair_sets(seed, n_sets, n_pairs):
    """Inputs of a pair-weighted overlap average: -beta F~ per run [n_sets][2 n_pairs] (spread over
    a few units around 900, so the weights differ widely), target sizes [n_sets][2 n_pairs] and
    per-pair (<q^2>, <q^4>, Gamma) [n_sets][n_pairs][3] with <q^2>^2 <= <q^4> <= <q^2>."""
    g = np.random.default_rng(seed)
    x = 900.0 + 3.0 * g.standard_normal((n_sets, 2 * n_pairs))
    R = g.uniform(1e4, 1e5, (n_sets, 2 * n_pairs))
    q2 = g.uniform(0.05, 0.9, (n_sets, n_pairs))
    q4 = q2 * q2 + g.uniform(0.0, 1.0, (n_sets, n_pairs)) * (q2 - q2 * q2)
    gam = g.uniform(0.0, 0.3, (n_sets, n_pairs))
    return x, R, np.stack([q2, q4, gam], axis=-1)
