"""Python binding of libpa (the C ABI in include/pa.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
torch provides the device buffers (caller-owned, as the ABI requires) and the stream.
The library must be built (``python -m paper_1006_0252_amd.build``); importing this module
on a machine without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpa.so")

PA_OK, PA_ERR_ARG, PA_ERR_CAPACITY, PA_ERR_EXTINCT, PA_ERR_NONFINITE, PA_ERR_HIP, PA_ERR_NOT_INIT, PA_ERR_SIZE = range(8)
PA_MLP_STATIC_MAX_B = 4096
PA_FLAG_CAPACITY, PA_FLAG_EXTINCT, PA_FLAG_NONFINITE = 1, 2, 4
PA_U8, PA_BITS64 = 0, 1
LAYOUTS = {"u8": PA_U8, "bits64": PA_BITS64}
PA_PM1, PA_GAUSS = 0, 1
COUPLINGS = {"pm1": PA_PM1, "gauss": PA_GAUSS}

P = ctypes.c_void_p


class pa_record(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "beta", "lnQ", "minus_betaF", "S", "R", "E_lo", "E_mean", "E_var", "E_skew",
        "q2", "q4", "gamma", "n_pairs", "r0", "r1", "r2")]


RECORD_FIELDS = [f[0] for f in pa_record._fields_][:13]


class pa_run(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("L", ctypes.c_int32), ("layout", ctypes.c_int32), ("n_records", ctypes.c_int32),
        ("couplings", ctypes.c_int32), ("reserved", ctypes.c_int32), ("capacity", ctypes.c_int64), ("R0", ctypes.c_int64), ("seed", ctypes.c_uint64),
        ("disorder_seed", ctypes.c_uint64), ("J", P), ("spins", P * 2), ("energy", P * 2), ("counts", P),
        ("offsets", P), ("work", P), ("record", P), ("state", P), ("stream", P),
    ]


class pa_step(ctypes.Structure):
    _fields_ = [
        ("beta_from", ctypes.c_double), ("beta_to", ctypes.c_double), ("R_target", ctypes.c_double),
        ("k", ctypes.c_int32), ("n_sweeps", ctypes.c_int32), ("t0", ctypes.c_int64), ("weights", P),
        ("n_weights", ctypes.c_int64),
    ]


class pa_sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "N", "n_bonds", "n_bins", "row_stride", "J_bytes", "spins_bytes", "energy_bytes", "counts_bytes",
        "offsets_bytes", "work_bytes", "record_bytes", "state_bytes")]


class pa_info(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int64), ("R_new", ctypes.c_int64), ("cur", ctypes.c_int32),
                ("status", ctypes.c_int32), ("E_lo", ctypes.c_int32), ("E_hi", ctypes.c_int32),
                ("k", ctypes.c_int32), ("initialised", ctypes.c_int32), ("acc", ctypes.c_double),
                ("ln_omega", ctypes.c_double), ("beta", ctypes.c_double)]


_lib = None

# every entry point declared in include/pa.h, with its ctypes signature
SIGNATURES = {
    "pa_buffer_sizes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                        ctypes.POINTER(pa_sizes)]),
    "pa_init_couplings": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, P]),
    "pa_sweep": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, ctypes.POINTER(pa_step)]),
    "pa_resample": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, ctypes.POINTER(pa_step)]),
    "pa_measure": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, P]),
    "pa_free_energy": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, P]),
    "pa_weighted_average": (ctypes.c_int, [ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, P, P]),
    "pa_weighted_average_dev": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P]),
    "pa_status": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, P]),
    "pa_query": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.POINTER(pa_info)]),
    "pa_resume": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, ctypes.POINTER(pa_info)]),
    "pa_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pa_fill_weights": (ctypes.c_int, [ctypes.c_double, ctypes.c_int64, P]),
    "pa_thresholds": (ctypes.c_int, [ctypes.c_double, ctypes.c_int, P, P]),
    "pa_ladder_table": (ctypes.c_int, [ctypes.c_int, P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "pa_set_sweep_config": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "pa_set_batch_config": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "pa_graph_begin": (ctypes.c_int, [P]),
    "pa_graph_end": (ctypes.c_int, [P, ctypes.POINTER(P)]),
    "pa_graph_launch": (ctypes.c_int, [P, P]),
    "pa_graph_destroy": (ctypes.c_int, [P]),
    "pa_features": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, P]),
    "pa_resampled_fraction": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, P, ctypes.c_int, P]),
    "pa_rho_steps": (ctypes.c_int, [ctypes.POINTER(pa_run), ctypes.c_int, P, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int64, P]),
    "pa_mlp_forward": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_float, ctypes.c_float, P, P]),
    "pa_mlp_work_bytes": (ctypes.c_int, [ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "pa_mlp_grad": (ctypes.c_int, [P, P, P, ctypes.c_int64, P, P, P, P]),
    "pa_mlp_grad_static": (ctypes.c_int, [P, P, P, ctypes.c_int64, P, P, P]),
    "pa_mlp_adam": (ctypes.c_int, [P, P, P, P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float, P]),
    "pa_bf16_round": (ctypes.c_int, [P, P, ctypes.c_int64, P]),
    "pa_overlap_average_dev": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, P, P, P, P, P]),
    "pa_bootstrap_dev": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_int, P, P, P, P]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libpa.so not built ({LIB_PATH}); run python -m paper_1006_0252_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class PAError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = lib().pa_strerror(code).decode()
        super().__init__(f"{where}: {msg} (status {code})")


def check(code, where=""):
    if code != PA_OK:
        raise PAError(code, where)


def _np(a):
    return a.ctypes.data_as(P)


# ------------------------------------------------------------------ host tables
def fill_weights(dbeta, n):
    w = np.zeros(n, dtype=np.float64)
    check(lib().pa_fill_weights(float(dbeta), n, _np(w)), "pa_fill_weights")
    return w


def thresholds(beta, z):
    T = np.zeros(z + 1, dtype=np.uint64)
    a = np.zeros(z + 1, dtype=np.uint8)
    check(lib().pa_thresholds(float(beta), z, _np(T), _np(a)), "pa_thresholds")
    return T, a


def ladder_table(m, cap=512):
    C = np.zeros(cap, dtype=np.uint64)
    n = ctypes.c_int(0)
    check(lib().pa_ladder_table(m, _np(C), cap, ctypes.byref(n)), "pa_ladder_table")
    return C[: n.value].copy()


def buffer_sizes(dim, L, layout, capacity, n_records, couplings=0):
    s = pa_sizes()
    check(lib().pa_buffer_sizes(dim, L, layout, couplings, capacity, n_records, ctypes.byref(s)), "pa_buffer_sizes")
    return s


def weighted_average(x, A=None, R=None):
    """Host FP64 weighted average over runs (Sec. III): dict like the oracle's."""
    x = np.ascontiguousarray(x, np.float64)
    M = len(x)
    A = np.zeros((M, 0)) if A is None else np.ascontiguousarray(np.asarray(A, np.float64).reshape(M, -1))
    n_obs = A.shape[1]
    Rr = None if R is None else np.ascontiguousarray(R, np.float64)
    A_bar = np.zeros(max(n_obs, 1))
    omega = np.zeros(M)
    out = np.zeros(3)
    check(lib().pa_weighted_average(M, _np(x), None if Rr is None else _np(Rr), _np(A), n_obs, _np(A_bar),
                                    _np(omega), _np(out[0:1]), _np(out[1:2]), _np(out[2:3])),
          "pa_weighted_average")
    return dict(A_bar=A_bar[:n_obs], omega=omega, minus_betaF_bar=out[0], var=out[1], mean=out[2])


def set_sweep_config(lanes_per_replica=0, waves_per_block=0):
    check(lib().pa_set_sweep_config(lanes_per_replica, waves_per_block), "pa_set_sweep_config")


def set_batch_config(blocks_per_cu=0, order=0, launch=0):
    check(lib().pa_set_batch_config(blocks_per_cu, order, launch), "pa_set_batch_config")


# ------------------------------------------------------------------ runs
def linear_schedule(n_temps, beta_max=5.0):
    """beta_k = beta_max k / (n_temps - 1), k = 0 .. n_temps - 1 (beta_0 = 0)."""
    return np.array([beta_max * k / (n_temps - 1) for k in range(n_temps)], dtype=np.float64)


class Schedule:
    """Temperature steps with their device weight tables w_d = exp(-dbeta 4 d)."""

    def __init__(self, betas, n_sweeps, n_bins, device="cuda", R_targets=None):
        import torch

        self.betas = np.asarray(betas, np.float64)
        self.n_sweeps = int(n_sweeps)
        self.n_bins = int(n_bins)
        self.R_targets = None if R_targets is None else np.asarray(R_targets, np.float64)
        tabs = np.stack([fill_weights(self.betas[k] - self.betas[k - 1], n_bins) for k in range(1, len(self.betas))]) \
            if len(self.betas) > 1 else np.zeros((0, n_bins))
        self.weights = torch.from_numpy(tabs).to(device)
        # the tables are read by kernels on the runs' streams: finish the copy first
        torch.cuda.current_stream(device).synchronize()

    def __len__(self):
        return len(self.betas)

    def step(self, k):
        """pa_step for the step into temperature k (k >= 1)."""
        s = pa_step()
        s.beta_from = float(self.betas[k - 1])
        s.beta_to = float(self.betas[k])
        s.R_target = float(self.R_targets[k]) if self.R_targets is not None else 0.0
        s.k = k
        s.n_sweeps = self.n_sweeps
        s.t0 = (k - 1) * self.n_sweeps
        s.weights = self.weights[k - 1].data_ptr()
        s.n_weights = self.n_bins
        return s

    def start_sweeps(self):
        """pa_step (for pa_sweep only) of n_sweeps at betas[0], for a schedule that starts at a
        finite temperature: the random initial population is equilibrated there first.  Its sweep
        indices follow those of the schedule's steps, so its draws are distinct from theirs."""
        s = self.step(1)
        s.beta_from = s.beta_to = float(self.betas[0])
        s.t0 = (len(self.betas) - 1) * self.n_sweeps
        return s


class Run:
    """One population-annealing run: caller-owned torch buffers described by a pa_run."""

    def __init__(self, dim, L, R0, seed, disorder_seed, n_records, capacity=None, layout="u8", device="cuda",
                 stream=None, state_ptr=None, couplings="pm1"):
        import torch

        self.dim, self.L, self.R0 = dim, L, int(R0)
        self.layout = LAYOUTS[layout] if isinstance(layout, str) else layout
        self.couplings_kind = COUPLINGS[couplings] if isinstance(couplings, str) else int(couplings)
        cap = capacity if capacity is not None else int(np.ceil(self.R0 * 1.5 / 64.0)) * 64 + 64
        self.capacity = int(cap)
        self.sizes = buffer_sizes(dim, L, self.layout, self.capacity, n_records, self.couplings_kind)
        s = self.sizes
        self.N = int(s.N)
        self.n_bonds = int(s.n_bonds)
        self.n_bins = int(s.n_bins)
        self.device = device

        def buf(nbytes):
            return torch.zeros(int(nbytes) + 256, dtype=torch.uint8, device=device)

        self.J = buf(s.J_bytes)
        self.spins = [buf(s.spins_bytes), buf(s.spins_bytes)]
        self.energy = [buf(s.energy_bytes), buf(s.energy_bytes)]
        self.counts = buf(s.counts_bytes)
        self.offsets = buf(s.offsets_bytes)
        self.work = buf(s.work_bytes)
        self.record = buf(s.record_bytes)
        self.state = None if state_ptr is not None else buf(s.state_bytes)
        alloc_stream = torch.cuda.current_stream(device)
        self.stream = stream if stream is not None else alloc_stream
        if self.stream != alloc_stream:
            # the zero fills of the buffers above run on the allocating stream: order them first
            self.stream.wait_stream(alloc_stream)
        r = pa_run()
        r.dim, r.L, r.layout, r.n_records = dim, L, self.layout, n_records
        r.couplings = self.couplings_kind
        r.capacity, r.R0 = self.capacity, self.R0
        r.seed, r.disorder_seed = int(seed), int(disorder_seed)
        r.J = self.J.data_ptr()
        r.spins[0], r.spins[1] = self.spins[0].data_ptr(), self.spins[1].data_ptr()
        r.energy[0], r.energy[1] = self.energy[0].data_ptr(), self.energy[1].data_ptr()
        r.counts = self.counts.data_ptr()
        r.offsets = self.offsets.data_ptr()
        r.work = self.work.data_ptr()
        r.record = self.record.data_ptr()
        r.state = state_ptr if state_ptr is not None else self.state.data_ptr()
        r.stream = self.stream.cuda_stream
        self.desc = r
        self.n_records = n_records

    # -- ABI calls (asynchronous)
    def init(self, J=None):
        if J is None:
            check(lib().pa_init_couplings(ctypes.byref(self.desc), 1, None), "pa_init_couplings")
        else:
            Jh = np.ascontiguousarray(J, np.int8)
            arr = (P * 1)(Jh.ctypes.data_as(P).value)
            check(lib().pa_init_couplings(ctypes.byref(self.desc), 1, ctypes.cast(arr, P)), "pa_init_couplings")
            self._J_host = Jh
        return self

    def sweep(self, step):
        check(lib().pa_sweep(ctypes.byref(self.desc), 1, ctypes.byref(step)), "pa_sweep")

    def resample(self, step):
        check(lib().pa_resample(ctypes.byref(self.desc), 1, ctypes.byref(step)), "pa_resample")

    def free_energy(self, out_tensor):
        check(lib().pa_free_energy(ctypes.byref(self.desc), 1, out_tensor.data_ptr()), "pa_free_energy")

    def query(self):
        info = pa_info()
        check(lib().pa_query(ctypes.byref(self.desc), ctypes.byref(info)), "pa_query")
        return info

    # -- checkpoint and resume (host copies of the run's whole state between steps)
    CHECKPOINT_META = ("dim", "L", "layout", "couplings_kind", "capacity", "n_records", "R0", "seed", "disorder_seed")

    def checkpoint(self):
        """The run's state between steps as host arrays (savable with numpy.savez): the couplings,
        the current buffer's spins and energies, the records and pa_query's dynamic state."""
        info = self.query()  # synchronises the stream
        out = {k: np.asarray(getattr(self, k) if hasattr(self, k) else getattr(self.desc, k)) for k in self.CHECKPOINT_META}
        out.update({f"info_{name}": np.asarray(getattr(info, name)) for name, _ in pa_info._fields_})
        out["J"] = self.J.cpu().numpy().copy()
        out["spins"] = self.spins[info.cur].cpu().numpy().copy()
        out["energy"] = self.energy[info.cur].cpu().numpy().copy()
        out["record"] = self.record.cpu().numpy().copy()
        return out

    def resume(self, ckpt):
        """Continue a checkpointed run in this run's buffers (same geometry, layout, couplings
        kind, seeds, capacity and record count): pa_init_couplings, the checkpoint's arrays copied
        in, then pa_resume."""
        import torch

        for k in self.CHECKPOINT_META:
            mine = getattr(self, k) if hasattr(self, k) else getattr(self.desc, k)
            if int(np.asarray(ckpt[k])) != int(mine):
                raise ValueError(f"checkpoint {k} = {int(np.asarray(ckpt[k]))}, this run has {int(mine)}")
        self.init()
        info = pa_info(**{name: np.asarray(ckpt[f"info_{name}"]).item() for name, _ in pa_info._fields_})
        with torch.cuda.stream(self.stream):
            for dst, key in ((self.J, "J"), (self.spins[info.cur], "spins"), (self.energy[info.cur], "energy"),
                             (self.record, "record")):
                dst.copy_(torch.from_numpy(np.ascontiguousarray(ckpt[key], np.uint8)))
        check(lib().pa_resume(ctypes.byref(self.desc), 1, ctypes.byref(info)), "pa_resume")
        return self

    def status(self):
        flags = np.zeros(1, np.int32)
        code = lib().pa_status(ctypes.byref(self.desc), 1, _np(flags))
        return code, int(flags[0])

    # -- host copies for inspection (synchronise)
    def _sync(self):
        self.stream.synchronize()

    def couplings(self):
        self._sync()
        if self.couplings_kind == PA_GAUSS:
            return self.J[: 8 * self.n_bonds].cpu().numpy().view(np.float64).copy()
        return self.J[: self.n_bonds].cpu().numpy().view(np.int8).copy()

    def records(self):
        self._sync()
        raw = self.record[: self.n_records * 128].cpu().numpy().view(np.float64).reshape(self.n_records, 16)
        return raw[:, :13].copy()

    def population(self, buf=None):
        """(spins u8 [R][N], energies int32 [R]) of the current population."""
        info = self.query()
        R = int(info.R)
        b = info.cur if buf is None else buf
        E = self._energy_view(self.energy[b], R)
        raw = self.spins[b].cpu().numpy()
        return unpack_spins(raw, self.dim, self.L, self.layout, R, int(self.sizes.row_stride)), E

    def energies(self):
        info = self.query()
        return self._energy_view(self.energy[info.cur], int(info.R))

    def _energy_view(self, buf, R):
        if self.couplings_kind == PA_GAUSS:
            return buf[: 8 * R].cpu().numpy().view(np.float64).copy()
        return buf[: 4 * R].cpu().numpy().view(np.int32).copy()

    def replica_spins(self, indices, buf=None):
        """u8 spins [len(indices)][N] of selected replicas of the current population."""
        info = self.query()
        b = info.cur if buf is None else buf
        idx = np.asarray(indices, dtype=np.int64)
        raw = self.spins[b].cpu().numpy()
        return select_spins(raw, self.dim, self.L, self.layout, idx, int(self.sizes.row_stride))

    def counts_offsets(self, R):
        self._sync()
        c = self.counts[: 4 * R].cpu().numpy().view(np.int32).copy()
        o = self.offsets[: 8 * (R + 1)].cpu().numpy().view(np.int64).copy()
        return c, o


class Batch:
    """Many runs whose device states are consecutive: every pa_* call covers all of them with
    one launch per kernel (the sweep as one persistent launch over (run, tile) work items)."""

    def __init__(self, specs, n_records, layout="bits64", device="cuda", stream=None, capacity_factor=1.25):
        """specs: list of dicts with dim, L, R0, seed, disorder_seed."""
        import torch

        self.n = len(specs)
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        self.states = torch.zeros(self.n * 256 + 256, dtype=torch.uint8, device=device)
        base = self.states.data_ptr()
        self.runs = []
        for r, sp in enumerate(specs):
            cap = int(np.ceil(sp["R0"] * capacity_factor / 64.0)) * 64 + 64
            self.runs.append(Run(sp["dim"], sp["L"], sp["R0"], sp["seed"], sp["disorder_seed"], n_records,
                                 couplings=sp.get("couplings", "pm1"),
                                 capacity=cap, layout=layout, device=device, stream=self.stream,
                                 state_ptr=base + 256 * r))
        self.arr = (pa_run * self.n)(*[r.desc for r in self.runs])
        self.n_records = n_records

    def init(self, J_list=None):
        if J_list is None:
            check(lib().pa_init_couplings(self.arr, self.n, None), "pa_init_couplings")
        else:
            self._J = [np.ascontiguousarray(J, np.int8) for J in J_list]
            ptrs = (P * self.n)(*[J.ctypes.data_as(P).value for J in self._J])
            check(lib().pa_init_couplings(self.arr, self.n, ctypes.cast(ptrs, P)), "pa_init_couplings")
        return self

    def resample(self, step):
        check(lib().pa_resample(self.arr, self.n, ctypes.byref(step)), "pa_resample")

    def sweep(self, step):
        check(lib().pa_sweep(self.arr, self.n, ctypes.byref(step)), "pa_sweep")

    def measure(self, pairs=False):
        if pairs:
            p = np.array([r ^ 1 for r in range(self.n)], dtype=np.int32)
            check(lib().pa_measure(self.arr, self.n, _np(p)), "pa_measure")
        else:
            check(lib().pa_measure(self.arr, self.n, None), "pa_measure")

    def free_energy(self, out_tensor):
        check(lib().pa_free_energy(self.arr, self.n, out_tensor.data_ptr()), "pa_free_energy")

    def status(self):
        flags = np.zeros(self.n, np.int32)
        code = lib().pa_status(self.arr, self.n, _np(flags))
        return code, flags

    def records(self):
        return np.stack([r.records() for r in self.runs])

    def step(self, sched, k, pairs=False):
        st = sched.step(k)
        self.resample(st)
        self.sweep(st)
        self.measure(pairs)

    def capture(self, sched, ks, pairs=False):
        """HIP graph of the steps ks (resample, sweep, measure each) on the batch's stream."""
        import torch

        with torch.cuda.stream(self.stream):
            check(lib().pa_graph_begin(self.stream.cuda_stream), "pa_graph_begin")
            try:
                for k in ks:
                    self.step(sched, k, pairs)
            finally:
                g = P()
                rc = lib().pa_graph_end(self.stream.cuda_stream, ctypes.byref(g))
            check(rc, "pa_graph_end")
        return Graph(g, self.stream)


class Graph:
    def __init__(self, handle, stream):
        self.handle = handle
        self.stream = stream

    def launch(self):
        check(lib().pa_graph_launch(self.handle, self.stream.cuda_stream), "pa_graph_launch")

    def __del__(self):
        if getattr(self, "handle", None):
            lib().pa_graph_destroy(self.handle)
            self.handle = None


def measure(runs, partner=None):
    """pa_measure over a list of Run objects (same call), partner: list of indices or None."""
    arr = (pa_run * len(runs))(*[r.desc for r in runs])
    if partner is None:
        check(lib().pa_measure(arr, len(runs), None), "pa_measure")
    else:
        p = np.ascontiguousarray(partner, np.int32)
        check(lib().pa_measure(arr, len(runs), _np(p)), "pa_measure")


def _rows_geometry(dim, L):
    N = L if dim == 1 else L ** 3
    if dim == 1:
        return N, (N + 31) // 32, 32, 32
    return N, L * L, (8 if L <= 8 else (16 if L <= 16 else 32)), L


def select_spins(raw, dim, L, layout, idx, row_stride):
    """Decode replicas idx of a population buffer (numpy uint8 view) into u8 spins."""
    N, n_rows, W, rowsites = _rows_geometry(dim, L)
    if layout == PA_U8:
        return raw.reshape(-1)[: (int(idx.max()) + 1) * row_stride].reshape(-1, row_stride)[idx, :N].copy()
    dt = {8: np.uint8, 16: np.uint16, 32: np.uint32}[W]
    words = raw.view(dt)
    pos = ((idx[:, None] >> 6) * n_rows + np.arange(n_rows)[None, :]) * 64 + (idx[:, None] & 63)
    w = words[pos].astype(np.uint64)
    bits = ((w[:, :, None] >> np.arange(rowsites, dtype=np.uint64)) & 1).astype(np.uint8)
    return bits.reshape(len(idx), n_rows * rowsites)[:, :N].copy()


def unpack_spins(raw, dim, L, layout, R, row_stride):
    """Decode a population buffer (numpy uint8 view) into u8 spins [R][N]."""
    N = L if dim == 1 else L ** 3
    if layout == PA_U8:
        return raw[: R * row_stride].reshape(R, row_stride)[:, :N].copy()
    if dim == 1:
        n_rows, W, rowsites = (N + 31) // 32, 32, 32
    else:
        n_rows, W, rowsites = L * L, (8 if L <= 8 else (16 if L <= 16 else 32)), L
    dt = {8: np.uint8, 16: np.uint16, 32: np.uint32}[W]
    G = (R + 63) // 64
    words = raw.view(dt)[: G * n_rows * 64].reshape(G, n_rows, 64)
    words = words.transpose(0, 2, 1).reshape(G * 64, n_rows)[:R].astype(np.uint64)
    bits = ((words[:, :, None] >> np.arange(rowsites, dtype=np.uint64)) & 1).astype(np.uint8)
    return bits.reshape(R, n_rows * rowsites)[:, :N].copy()
