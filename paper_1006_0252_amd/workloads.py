"""Synthetic workloads: sizes, seeds and schedules of the benchmark configurations.

Seeded input descriptions only (no arithmetic of the method): both the CPU oracle and the
GPU library take these and draw every random number themselves from the seeds.
Couplings are +-1 equiprobable from a disorder seed (the paper's own disorder
realisations were Gaussian and are not published).
"""
from __future__ import annotations

from dataclasses import dataclass, field


def linear_betas(n_temps: int, beta_max: float = 5.0):
    """beta_k = beta_max k / (n_temps - 1), k = 0 .. n_temps - 1 (starts at beta = 0)."""
    return [beta_max * k / (n_temps - 1) for k in range(n_temps)]


@dataclass
class Workload:
    name: str
    dim: int
    L: int
    R0: int
    n_temps: int
    n_sweeps: int
    layout: str = "u8"
    disorder_seed: int = 1
    run_seeds: list = field(default_factory=lambda: [1])

    @property
    def N(self):
        return self.L if self.dim == 1 else self.L ** 3

    @property
    def betas(self):
        return linear_betas(self.n_temps)

    @property
    def attempts_per_run(self):
        return self.R0 * self.N * self.n_sweeps * (self.n_temps - 1)


# ring N = 64 with an exact partition function; 18 disorder seeds mirror the paper's 18 1D realisations
C1 = Workload("ring_N64_R1000", dim=1, L=64, R0=1000, n_temps=51, n_sweeps=5, layout="u8",
              run_seeds=list(range(1, 201)))
# 3D L = 8, R0 = 5e4, 101 temperatures, 10 sweeps
C2 = Workload("cube_L8_R50000", dim=3, L=8, R0=50000, n_temps=101, n_sweeps=10, layout="u8")
# throughput configuration: 3D L = 16, R0 = 1e6 bit-packed, 301 temperatures, 10 sweeps
C4 = Workload("cube_L16_R1e6_bits", dim=3, L=16, R0=1_000_000, n_temps=301, n_sweeps=10, layout="bits64")
# learned-schedule target: 3D L = 12, R0 = 2e5
C5 = Workload("cube_L12_R2e5", dim=3, L=12, R0=200_000, n_temps=101, n_sweeps=10, layout="bits64")


def batched_specs(n_realizations: int = 64, seeds_per_realization: int = 4, gen_seed: int = 3,
                  Ls=(6, 8, 10), R0_range=(10_000, 100_000)):
    """The batched configuration: realisations with L uniform in Ls and R0 uniform in R0_range
    (integers, both drawn from a numpy generator seeded with gen_seed), each run with
    seeds_per_realization independent run seeds.  Runs (d, 0), (d, 1) and (d, 2), (d, 3) are
    overlap pairs.  Returns a list of dicts (dim, L, R0, seed, disorder_seed, realization)."""
    import numpy as np

    rng = np.random.default_rng(gen_seed)
    L_d = rng.choice(np.asarray(Ls), size=n_realizations)
    specs = []
    for d in range(n_realizations):
        for s in range(seeds_per_realization):
            R0 = int(rng.integers(R0_range[0], R0_range[1] + 1))
            specs.append(dict(dim=3, L=int(L_d[d]), R0=R0, seed=1000 * (d + 1) + s, disorder_seed=d + 1,
                              realization=d))
    return specs


# 256 runs: 64 realisations x 4 seeds, beta linear 0 -> 5 in 101 temperatures, 10 sweeps
C3_TEMPS, C3_SWEEPS = 101, 10
