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
