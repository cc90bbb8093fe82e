"""Exact results of the periodic +-J chain, the reference the bias measurements are taken against.

With E = + sum_i J_i s_i s_(i+1) (the sign printed in Sec. IV) and J_i = +-1, each bond factor
exp(-beta J s s') = cosh(beta) (1 - J s s' tanh(beta)); summing over the spins of a ring of N
sites leaves the terms with no or all bonds:
    Z = (2 cosh beta)^N (1 + s t^N),   t = tanh beta,  s = (-1)^N prod_i J_i,
    E = -d ln Z / d beta = -N t - s N t^(N-1) (1 - t^2) / (1 + s t^N).
"""
from __future__ import annotations

import math

import numpy as np


def ring_lnZ(J, beta):
    J = np.asarray(J)
    N = len(J)
    s = (-1) ** N * int(np.prod(np.sign(J)))
    t = math.tanh(beta)
    return N * (math.log(2.0) + math.log(math.cosh(beta))) + math.log1p(s * t ** N)


def ring_energy(J, beta):
    J = np.asarray(J)
    N = len(J)
    s = (-1) ** N * int(np.prod(np.sign(J)))
    t = math.tanh(beta)
    return -N * t - s * N * t ** (N - 1) * (1.0 - t * t) / (1.0 + s * t ** N)
