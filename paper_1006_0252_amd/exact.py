"""Exact results of the periodic chain, the reference the bias measurements are taken against.

With E = + sum_i J_i s_i s_(i+1) (the sign printed in Sec. IV), each bond factor is
exp(-beta J s s') = cosh(beta J) (1 - s s' tanh(beta J)); summing over the spins of a ring of N
sites leaves the terms with no bond or with every bond:
    Z = prod_i 2 cosh(beta J_i) (1 + P),   P = prod_i (-tanh(beta J_i)),
    E = -d ln Z / d beta = -sum_i J_i tanh(beta J_i) - (dP / d beta) / (1 + P),
    dP / d beta = sum_i (-J_i sech^2(beta J_i)) prod_(k != i) (-tanh(beta J_k)).
For J_i = +-1 this is Z = (2 cosh beta)^N (1 + s t^N) with t = tanh beta, s = (-1)^N prod_i J_i.
"""
from __future__ import annotations

import math

import numpy as np


def _log_cosh(x):
    a = abs(x)
    return a + math.log1p(math.exp(-2.0 * a)) - math.log(2.0)


def ring_lnZ(J, beta):
    J = np.asarray(J, np.float64)
    N = len(J)
    P = float(np.prod(-np.tanh(beta * J)))
    return N * math.log(2.0) + sum(_log_cosh(beta * j) for j in J) + math.log1p(P)


def ring_energy(J, beta):
    J = np.asarray(J, np.float64)
    t = -np.tanh(beta * J)                       # factors of P
    P = float(np.prod(t))
    dt = -J / np.cosh(beta * J) ** 2             # their derivatives in beta
    # prod over k != i by prefix and suffix products (no division by a vanishing tanh)
    pre = np.concatenate([[1.0], np.cumprod(t)[:-1]])
    suf = np.concatenate([np.cumprod(t[::-1])[:-1][::-1], [1.0]])
    dP = float(np.sum(dt * pre * suf))
    return -float(np.sum(J * np.tanh(beta * J))) - dP / (1.0 + P)
