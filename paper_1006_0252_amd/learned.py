"""Learned temperature steps: a small network proposes each dbeta of the annealing schedule.

The paper's method is exact for any schedule (Sec. II), and the variance of beta F~ over
independent runs tells how well a schedule worked (Sec. III); Sec. IV simply spaces the
temperatures evenly.  This module learns the spacing instead:

1. traces -- fixed-schedule runs (the ring of N = 64 spins with R0 = 1000 and 51
   temperatures, the L = 8 cube with R0 = 5e4 and 101 temperatures) record at every
   temperature the population features (pa_features) and, for each target rho*, the step at
   which resampling would replace the fraction rho* of the population (pa_rho_steps);
2. training -- one network per rho* (6 -> 64 -> 64 -> 64 -> 1, BF16 weights, FP32
   arithmetic) fits ln dbeta* by full-batch Adam, all of it in the library's kernels
   (pa_mlp_grad, pa_mlp_adam);
3. pilot -- one run of the target system anneals with the network choosing every step
   (pa_features -> pa_mlp_forward), the last step clamped to land on beta_max; the betas it
   visited are the schedule, frozen from then on;
4. production -- the M runs of the ensemble use the frozen schedule like any fixed one
   (one batch, the whole schedule one HIP graph), so the weighted averages of Sec. III hold.

If the pilot fails (a raised status bit, a step budget exhausted) the fixed linear schedule
is returned instead, flagged.  Everything numeric runs in libpa; this module moves buffers,
launches calls and keeps the schedule's list of betas.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import pa

N_PARAMS = 8833
N_FEATURES = 6
RHO_TARGETS = (0.1, 0.2, 0.3, 0.5)
LABEL_CAP = 1.0


def glorot_theta(seed):
    """Initial FP32 parameters: weights uniform in +-sqrt(6 / (fan_in + fan_out)) (Glorot and
    Bengio, 2010), biases zero; drawn on the host from a seeded generator."""
    g = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((6, 64), (64, 64), (64, 64), (64, 1)):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(g.uniform(-a, a, fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def _stream(device):
    import torch

    return torch.cuda.current_stream(device).cuda_stream


class Network:
    """Device parameters of one step-proposing network: FP32 master copy and Adam moments,
    BF16 weights used by the forward and backward kernels."""

    def __init__(self, theta0, device="cuda"):
        import torch

        theta0 = np.ascontiguousarray(theta0, np.float32)
        assert theta0.shape == (N_PARAMS,)
        self.device = device
        self.theta = torch.from_numpy(theta0.copy()).to(device)
        self.m = torch.zeros(N_PARAMS, dtype=torch.float32, device=device)
        self.v = torch.zeros(N_PARAMS, dtype=torch.float32, device=device)
        self.grad = torch.zeros(N_PARAMS, dtype=torch.float32, device=device)
        self.w = torch.zeros(N_PARAMS, dtype=torch.int16, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.t = 0
        self._work = None
        self._work_B = 0
        pa.check(pa.lib().pa_bf16_round(self.theta.data_ptr(), self.w.data_ptr(), N_PARAMS, _stream(device)),
                 "pa_bf16_round")

    def forward(self, x, dmin, dmax, out=None):
        """Proposed steps for feature rows x (device FP32 [B][6])."""
        import torch

        B = x.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float32, device=self.device)
        pa.check(pa.lib().pa_mlp_forward(self.w.data_ptr(), x.data_ptr(), B, float(dmin), float(dmax), out.data_ptr(),
                                          _stream(self.device)), "pa_mlp_forward")
        return out

    def _work_for(self, B):
        import torch

        if self._work is None or self._work_B < B:
            nb = ctypes.c_int64()
            pa.check(pa.lib().pa_mlp_work_bytes(B, ctypes.byref(nb)), "pa_mlp_work_bytes")
            self._work = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
            self._work_B = B
        return self._work

    def gradient(self, x, target):
        """Loss (device [1]) and gradient (device [N_PARAMS]) on a batch; target FP64 dbeta*."""
        B = x.shape[0]
        work = self._work_for(B)
        pa.check(pa.lib().pa_mlp_grad(self.w.data_ptr(), x.data_ptr(), target.data_ptr(), B, work.data_ptr(),
                                       self.grad.data_ptr(), self.loss.data_ptr(), _stream(self.device)),
                 "pa_mlp_grad")
        return self.loss, self.grad

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        pa.check(pa.lib().pa_mlp_adam(self.theta.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                       self.grad.data_ptr(), self.w.data_ptr(), N_PARAMS, self.t, float(lr),
                                       float(beta1), float(beta2), float(eps), _stream(self.device)), "pa_mlp_adam")

    def train(self, x, target, steps, lr=3e-3, lr_final=3e-4, x_val=None, target_val=None, log_every=0):
        """Full-batch Adam with a geometric learning-rate decay from lr to lr_final.  Returns
        the loss history [(step, train loss, validation loss or None)] at log points."""
        hist = []
        for s in range(steps):
            a = lr * (lr_final / lr) ** (s / max(1, steps - 1))
            self.gradient(x, target)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(self.loss.item()), self.evaluate(x_val, target_val) if x_val is not None else None))
            self.adam(a)
        return hist

    def evaluate(self, x, target):
        """Loss on a batch, without touching the gradient used by training."""
        import torch

        keep = self.grad.clone()
        loss, _ = self.gradient(x, target)
        out = float(loss.item())
        self.grad.copy_(keep)
        torch.cuda.current_stream(self.device).synchronize()
        return out

    def weights_bits(self):
        return self.w.cpu().numpy().view(np.uint16).copy()


# ------------------------------------------------------------------ traces

def trace_specs(kind, n_realizations, seeds_per_realization, first_seed=1):
    """Fixed-schedule trace runs: kind 'ring' (N = 64, R0 = 1000, 51 temperatures, 5 sweeps,
    one byte per spin) or 'cube8' (L = 8, R0 = 5e4, 101 temperatures, 10 sweeps, bit-packed)."""
    dim, L, R0 = (1, 64, 1000) if kind == "ring" else (3, 8, 50000)
    specs = []
    for d in range(first_seed, first_seed + n_realizations):
        for s in range(seeds_per_realization):
            specs.append(dict(dim=dim, L=L, R0=R0, seed=1000 * d + s + 1, disorder_seed=d))
    return specs


TRACE_SHAPE = {"ring": dict(n_temps=51, n_sweeps=5, layout="u8"),
               "cube8": dict(n_temps=101, n_sweeps=10, layout="bits64")}


def collect_traces(kind, specs, targets=RHO_TARGETS, cap=LABEL_CAP, device="cuda"):
    """Run the fixed linear schedule of `kind` on every spec (one batch) and record, at every
    temperature k = 0 .. n_temps-1, features X [n_temps * n][6] (row k * n + r) and step labels
    D [n_targets][n_temps * n] for the targets rho*."""
    import torch

    shape = TRACE_SHAPE[kind]
    nT = shape["n_temps"]
    betas = pa.linear_schedule(nT, 5.0)
    batch = pa.Batch(specs, nT, layout=shape["layout"], device=device)
    batch.init()
    n = batch.n
    sched = pa.Schedule(betas, shape["n_sweeps"], max(r.n_bins for r in batch.runs), device=device)
    S = nT * n
    X = torch.empty((S, N_FEATURES), dtype=torch.float32, device=device)
    D = torch.empty((len(targets), S), dtype=torch.float64, device=device)
    tg = np.ascontiguousarray(targets, np.float64)
    torch.cuda.synchronize()
    for k in range(nT):
        if k == 0:
            batch.measure()
        else:
            batch.step(sched, k)
        pa.check(pa.lib().pa_features(batch.arr, n, X.data_ptr() + 4 * N_FEATURES * k * n), "pa_features")
        pa.check(pa.lib().pa_rho_steps(batch.arr, n, pa._np(tg), len(tg), float(cap), S, D.data_ptr() + 8 * k * n),
                 "pa_rho_steps")
    code, flags = batch.status()
    if code != pa.PA_OK:
        raise RuntimeError(f"trace runs failed: status {code}, runs {np.nonzero(flags)[0].tolist()}")
    batch.stream.synchronize()
    return X, D


def training_set(device="cuda", ring_real=(1, 15), ring_val=(16, 18), cube_real=(1, 20), cube_val=(21, 25),
                 ring_seeds=8, cube_seeds=2):
    """Train / validation features and labels from ring and L = 8 cube traces; realizations
    (disorder seeds) ring_real and cube_real train, ring_val and cube_val validate."""
    import torch

    def part(kind, lohi, seeds):
        return collect_traces(kind, trace_specs(kind, lohi[1] - lohi[0] + 1, seeds, lohi[0]), device=device)

    tr = [part("ring", ring_real, ring_seeds), part("cube8", cube_real, cube_seeds)]
    va = [part("ring", ring_val, ring_seeds), part("cube8", cube_val, cube_seeds)]
    Xt = torch.cat([t[0] for t in tr]).contiguous()
    Dt = torch.cat([t[1] for t in tr], dim=1).contiguous()
    Xv = torch.cat([t[0] for t in va]).contiguous()
    Dv = torch.cat([t[1] for t in va], dim=1).contiguous()
    return Xt, Dt, Xv, Dv


def train_networks(Xt, Dt, Xv=None, Dv=None, targets=RHO_TARGETS, steps=3000, seed=1, device="cuda", log_every=0):
    """One network per target rho* (row j of Dt), all from the same initial parameters."""
    nets, logs = {}, {}
    for j, rs in enumerate(targets):
        net = Network(glorot_theta(seed), device=device)
        tv = Dv[j].contiguous() if Dv is not None else None
        logs[rs] = net.train(Xt, Dt[j].contiguous(), steps, x_val=Xv, target_val=tv, log_every=log_every)
        nets[rs] = net
    return nets, logs


# ------------------------------------------------------------------ pilot and production

def pilot_schedule(net, L, R0, seed, disorder_seed, n_sweeps, dmin=1e-4, dmax=0.25, beta_max=5.0, max_steps=3000,
                   layout="bits64", device="cuda"):
    """Anneal one run of the 3D system with the network choosing every step.  Returns
    (betas, info); betas is the fixed linear schedule of 101 temperatures when the pilot fails."""
    import torch

    t_start = time.perf_counter()
    run = pa.Run(3, L, R0, seed, disorder_seed, max_steps + 1, capacity=int(np.ceil(R0 * 1.25 / 64)) * 64 + 64,
                 layout=layout, device=device)
    run.init()
    pa.measure([run])
    x = torch.empty((1, N_FEATURES), dtype=torch.float32, device=device)
    d = torch.empty(1, dtype=torch.float32, device=device)
    wtab = torch.empty(run.n_bins, dtype=torch.float64, device=device)
    betas = [0.0]
    ok = True
    with torch.cuda.stream(run.stream):
        for k in range(1, max_steps + 1):
            pa.check(pa.lib().pa_features(ctypes.byref(run.desc), 1, x.data_ptr()), "pa_features")
            net.forward(x, dmin, dmax, out=d)
            dbeta = float(d.item())                      # waits for the run's stream
            b_next = betas[-1] + dbeta
            if not np.isfinite(b_next):
                ok = False
                break
            if b_next >= beta_max - dmin:
                b_next = beta_max                        # the last step lands on beta_max
            wtab.copy_(torch.from_numpy(pa.fill_weights(b_next - betas[-1], run.n_bins)))
            st = pa.pa_step()
            st.beta_from, st.beta_to, st.R_target = betas[-1], b_next, 0.0
            st.k, st.n_sweeps, st.t0 = k, n_sweeps, (k - 1) * n_sweeps
            st.weights, st.n_weights = wtab.data_ptr(), run.n_bins
            run.resample(st)
            run.sweep(st)
            pa.measure([run])
            betas.append(b_next)
            if b_next >= beta_max:
                break
    code, flags = run.status()
    if code != pa.PA_OK or betas[-1] < beta_max:
        ok = False
    info = dict(seconds=time.perf_counter() - t_start, steps=len(betas) - 1, ok=ok, status=code)
    if not ok:
        return pa.linear_schedule(101, beta_max), info
    return np.array(betas, dtype=np.float64), info


def ensemble(betas, M, L, R0, n_sweeps, disorder_seed=1, seed0=1, layout="bits64", device="cuda", graph=True):
    """M independent runs on one schedule (one batch, the whole schedule one HIP graph).
    Returns the per-run -beta F~ at the last temperature, its weighted and plain averages and
    Var(beta F~) (pa_weighted_average), and the wall time per run."""
    import torch

    specs = [dict(dim=3, L=L, R0=R0, seed=seed0 + i, disorder_seed=disorder_seed) for i in range(M)]
    nT = len(betas)
    batch = pa.Batch(specs, nT, layout=layout, device=device)
    batch.init()
    sched = pa.Schedule(betas, n_sweeps, max(r.n_bins for r in batch.runs), device=device)
    torch.cuda.synchronize()
    if graph:
        g = batch.capture(sched, range(1, nT))   # recorded, not run: the state is still at beta = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.launch()
        batch.stream.synchronize()
        T = time.perf_counter() - t0
    else:
        t0 = time.perf_counter()
        for k in range(1, nT):
            batch.step(sched, k)
        batch.stream.synchronize()
        T = time.perf_counter() - t0
    code, flags = batch.status()
    if code != pa.PA_OK:
        raise RuntimeError(f"ensemble failed: status {code}, runs {np.nonzero(flags)[0].tolist()}")
    rec = batch.records()
    x = rec[:, nT - 1, 2].copy()
    wa = pa.weighted_average(x)
    attempts = float(np.sum(rec[:, 1:, 4]) * L ** 3 * n_sweeps)
    return dict(minus_betaF=x, minus_betaF_bar=wa["minus_betaF_bar"], mean=wa["mean"], var=wa["var"],
                seconds=T, seconds_per_run=T / M, n_temps=nT, attempts=attempts)


def time_to_target(var, seconds_per_run, target=1e-3, overhead=0.0):
    """Wall time of an ensemble whose weighted free energy has variance <= target:
    ceil(var / target) runs (Var(beta F_bar) ~ Var(beta F~) / M, Sec. III) plus a one-off overhead."""
    return overhead + seconds_per_run * float(np.ceil(var / target))
