"""Parity of the learned-step kernels with the oracle: BF16 rounding (bit-exact), network
forward and loss gradient (same BF16 weights; FP32 on the GPU against FP64, 1e-4 relative),
Adam, population features and resampled-fraction labels (from bit-identical populations),
and training end to end."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import learned as ol
from oracle import oracle as o
from tests import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1006_0252_amd import learned, pa  # noqa: E402

DEV = "cuda:0"


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def stream():
    return torch.cuda.current_stream(DEV).cuda_stream


def gpu_bf16(x32):
    x = torch.from_numpy(np.ascontiguousarray(x32, np.float32)).to(DEV)
    out = torch.zeros(len(x32), dtype=torch.int16, device=DEV)
    pa.check(pa.lib().pa_bf16_round(x.data_ptr(), out.data_ptr(), len(x32), stream()), "pa_bf16_round")
    return out


def test_bf16_rounding_bit_exact():
    note("bf16 rounding")
    x = inputs.float32_values(3, 5001)
    got = gpu_bf16(x).cpu().numpy().view(np.uint16)
    assert np.array_equal(got, ol.bf16_bits(x))


@pytest.mark.parametrize("B", [1, 63, 777])
def test_forward_matches_oracle(B):
    note(f"mlp forward B={B}")
    theta = inputs.mlp_theta(21, scale=1.5)
    w = gpu_bf16(theta)
    assert np.array_equal(w.cpu().numpy().view(np.uint16), ol.bf16_bits(theta))
    X = inputs.mlp_features(22 + B, B, zero_var_every=50 if B > 1 else 0)
    Xd = torch.from_numpy(X).to(DEV)
    out = torch.empty(B, dtype=torch.float32, device=DEV)
    dmin, dmax = 1e-4, 0.5
    pa.check(pa.lib().pa_mlp_forward(w.data_ptr(), Xd.data_ptr(), B, dmin, dmax, out.data_ptr(), stream()), "fwd")
    got = out.cpu().numpy().astype(np.float64)
    want = ol.forward(ol.bf16_values(ol.bf16_bits(theta)), X.astype(np.float64), np.float32(dmin), np.float32(dmax))
    assert np.allclose(got, want, rtol=1e-5, atol=0), np.max(np.abs(got / want - 1))
    if B >= 50:
        assert got[0] == np.float32(dmax)  # row 0 has var = 0


@pytest.mark.parametrize("B", [5, 1500])
def test_gradient_matches_oracle(B):
    note(f"mlp gradient B={B}")
    theta = inputs.mlp_theta(31, scale=1.5)
    w = gpu_bf16(theta)
    X = inputs.mlp_features(32, B, zero_var_every=41)
    t = inputs.mlp_targets(33, B, bad_every=37)
    if B > 10:
        t[5] = np.nan
    Xd = torch.from_numpy(X).to(DEV)
    td = torch.from_numpy(t).to(DEV)
    nb = ctypes.c_int64()
    pa.check(pa.lib().pa_mlp_work_bytes(B, ctypes.byref(nb)), "work")
    work = torch.full((int(nb.value),), 0x7F, dtype=torch.uint8, device=DEV)  # garbage: must be overwritten
    grad = torch.empty(learned.N_PARAMS, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    pa.check(pa.lib().pa_mlp_grad(w.data_ptr(), Xd.data_ptr(), td.data_ptr(), B, work.data_ptr(), grad.data_ptr(),
                                  loss.data_ptr(), stream()), "grad")
    g = grad.cpu().numpy().astype(np.float64)
    L_o, g_o = ol.loss_and_grad(ol.bf16_values(ol.bf16_bits(theta)), X.astype(np.float64), t)
    assert abs(float(loss.item()) - L_o) <= 1e-5 * L_o
    for name, lo in ol.OFF.items():
        hi = lo + {"W1": 384, "b1": 64, "W2": 4096, "b2": 64, "W3": 4096, "b3": 64, "w4": 64, "b4": 1}[name]
        a, b = g[lo:hi], g_o[lo:hi]
        scale = np.abs(b).max()
        assert np.abs(a - b).max() <= 1e-4 * scale, (name, np.abs(a - b).max() / scale)
        big = np.abs(b) > 1e-2 * scale
        assert np.all(np.abs(a[big] - b[big]) <= 1e-4 * np.abs(b[big])), name
    # the same call again gives the same bits (fixed summation order)
    g1 = grad.clone()
    pa.check(pa.lib().pa_mlp_grad(w.data_ptr(), Xd.data_ptr(), td.data_ptr(), B, work.data_ptr(), grad.data_ptr(),
                                  loss.data_ptr(), stream()), "grad")
    assert torch.equal(g1, grad)


def test_adam_matches_oracle():
    note("adam")
    n = learned.N_PARAMS
    g = np.random.default_rng(41)
    theta = inputs.mlp_theta(42)
    m = (g.standard_normal(n) * 1e-2).astype(np.float32)
    v = (g.random(n) * 1e-3).astype(np.float32)
    grad = (g.standard_normal(n) * 3e-2).astype(np.float32)
    dev = [torch.from_numpy(a.copy()).to(DEV) for a in (theta, m, v, grad)]
    w = torch.empty(n, dtype=torch.int16, device=DEV)
    lr, b1, b2, eps, t = 2e-3, 0.9, 0.999, 1e-8, 3
    pa.check(pa.lib().pa_mlp_adam(dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(), dev[3].data_ptr(),
                                  w.data_ptr(), n, t, lr, b1, b2, eps, stream()), "adam")
    # the kernel receives the hyperparameters as FP32: the oracle takes those same values
    lr, b1, b2, eps = (float(np.float32(a)) for a in (lr, b1, b2, eps))
    th_o, m_o, v_o = ol.adam(theta, m, v, grad, t, lr, b1, b2, eps)
    th, mg, vg = (d.cpu().numpy().astype(np.float64) for d in dev[:3])
    m64, v64, g64 = m.astype(np.float64), v.astype(np.float64), grad.astype(np.float64)
    # FP32 rounding of the two terms of each moment (a few ulps of the larger term)
    dm = 2.4e-7 * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64))
    dv = 2.4e-7 * (b2 * v64 + (1 - b2) * g64 * g64)
    assert np.all(np.abs(mg - m_o) <= dm + 1e-30)
    assert np.all(np.abs(vg - v_o) <= dv + 1e-30)
    bc1, bc2 = 1 - b1 ** t, 1 - b2 ** t
    denom = np.sqrt(v_o / bc2) + eps
    u_o = theta.astype(np.float64) - th_o
    du = 1e-5 * np.abs(u_o) + lr * (dm / bc1) / denom + 0.5 * lr * np.abs(m_o / bc1) * (dv / bc2) / (denom ** 2 * np.sqrt(v_o / bc2) + 1e-300)
    assert np.all(np.abs((theta - th) - u_o) <= du + 2.4e-7 * np.abs(theta))
    wb = w.cpu().numpy().view(np.uint16)
    assert np.array_equal(wb, ol.bf16_bits(dev[0].cpu().numpy()))        # BF16 of the new master copy
    ob = ol.bf16_bits(th_o.astype(np.float32)).astype(np.int32)
    assert np.all(np.abs(wb.astype(np.int32) - ob) <= 1)


@pytest.mark.parametrize("dim,L,R0,layout,nT", [(3, 6, 3000, "bits64", 5), (1, 64, 1000, "u8", 6), (3, 8, 2000, "u8", 4)])
def test_features_and_labels_match_oracle(dim, L, R0, layout, nT):
    note(f"features and labels dim={dim} L={L} R0={R0} {layout}")
    betas = [0.1 * k for k in range(nT)]
    ns = 3
    run = pa.Run(dim, L, R0, seed=77, disorder_seed=5, n_records=nT, layout=layout, device=DEV).init()
    sched = pa.Schedule(betas, ns, run.n_bins, device=DEV)
    for k in range(1, nT):
        st = sched.step(k)
        run.resample(st)
        run.sweep(st)
    pa.measure([run])
    x = torch.empty((1, 6), dtype=torch.float32, device=DEV)
    pa.check(pa.lib().pa_features(ctypes.byref(run.desc), 1, x.data_ptr()), "pa_features")
    targets = np.array([0.05, 0.1, 0.3, 0.5, 0.9], np.float64)
    lab = torch.empty((len(targets), 3), dtype=torch.float64, device=DEV)
    pa.check(pa.lib().pa_rho_steps(ctypes.byref(run.desc), 1, pa._np(targets), len(targets), 1.0, 3,
                                   lab.data_ptr() + 8), "pa_rho_steps")
    dbs = np.array([0.0, 0.01, 0.1, 0.7], np.float64)
    rho = torch.empty(len(dbs), dtype=torch.float64, device=DEV)
    pa.check(pa.lib().pa_resampled_fraction(ctypes.byref(run.desc), 1, pa._np(dbs), len(dbs), rho.data_ptr()), "rho")
    J = o.couplings(dim, L, 5)
    st_o, rec_o, s_o, E_o = o.run(dim, L, J, 77, R0, betas, ns, capacity=run.capacity)
    assert st_o == 0
    s, E = run.population()
    assert np.array_equal(E, E_o)
    N = L if dim == 1 else L ** 3
    f_o = ol.features(betas[-1], N, E_o)
    f = x.cpu().numpy()[0].astype(np.float64)
    assert np.allclose(f, f_o, rtol=2e-7, atol=1e-7)
    vals, h = ol.histogram(E_o)
    rho_o = np.array([ol.rho(vals, h, d) for d in dbs])
    assert np.allclose(rho.cpu().numpy(), rho_o, rtol=1e-12, atol=1e-14)
    lab_o = np.array([ol.step_label(vals, h, rs, 1.0) for rs in targets])
    got = lab.cpu().numpy()[:, 1]
    assert np.allclose(got, lab_o, rtol=1e-9, atol=0)


def test_training_reduces_loss_and_is_reproducible():
    note("training on ring traces")
    specs = learned.trace_specs("ring", 4, 4)
    X, D = learned.collect_traces("ring", specs, device=DEV)
    assert X.shape == (51 * 16, 6) and D.shape == (4, 51 * 16)
    t = D[2].contiguous()
    assert torch.all(torch.isfinite(t)) and torch.all(t > 0)
    losses = []
    for rep in range(2):
        net = learned.Network(learned.glorot_theta(3), device=DEV)
        hist = net.train(X, t, 300, log_every=299)
        losses.append((hist[0][1], hist[-1][1], net.weights_bits()))
    first, last, w0 = losses[0]
    assert last < 0.2 * first
    assert losses[1][1] == last and np.array_equal(losses[1][2], w0)


def test_pilot_schedule_is_valid():
    note("pilot schedule")
    net = learned.Network(learned.glorot_theta(5), device=DEV)
    betas, info = learned.pilot_schedule(net, 6, 2000, seed=9, disorder_seed=2, n_sweeps=2, dmin=0.01, dmax=0.3,
                                         device=DEV)
    assert info["ok"], info
    assert betas[0] == 0.0 and betas[-1] == 5.0
    d = np.diff(betas)
    assert np.all(d > 0) and np.all(d[:-1] >= 0.01 * (1 - 1e-6)) and np.all(d[:-1] <= 0.3 * (1 + 1e-6))
    assert d[-1] <= 0.31 * (1 + 1e-6)  # the landing step may absorb a remainder below dmin


def test_learned_schedule_beats_fixed_at_equal_steps():
    # what the trained network gains: a network trained on ring and L = 8 traces towards
    # rho* = 0.3 picks the schedule of an L = 6 cube on a pilot run; with the same number of
    # temperatures, the fixed linear schedule's Var(beta F~) is far larger, and the learned
    # ensemble's weighted free energy agrees with a long fixed-schedule ensemble's
    note("learned vs fixed at equal steps")
    Xr, Dr = learned.collect_traces("ring", learned.trace_specs("ring", 6, 4), device=DEV)
    Xc, Dc = learned.collect_traces("cube8", learned.trace_specs("cube8", 6, 1), device=DEV)
    X = torch.cat([Xr, Xc]).contiguous()
    D = torch.cat([Dr, Dc], dim=1).contiguous()
    j = learned.RHO_TARGETS.index(0.3)
    net = learned.Network(learned.glorot_theta(1), device=DEV)
    hist = net.train(X, D[j].contiguous(), 1500, log_every=1499)
    assert hist[-1][1] < 0.02
    L, R0, ns, M = 6, 5000, 10, 32
    betas, info = learned.pilot_schedule(net, L, R0, seed=10 ** 6, disorder_seed=3, n_sweeps=ns, device=DEV)
    assert info["ok"], info
    K = len(betas)
    e_l = learned.ensemble(betas, M, L, R0, ns, disorder_seed=3, device=DEV)
    e_f = learned.ensemble(pa.linear_schedule(K), M, L, R0, ns, disorder_seed=3, device=DEV)
    ref = learned.ensemble(pa.linear_schedule(401), M, L, R0, ns, disorder_seed=3, seed0=5000, device=DEV)
    note(f"K={K} var learned {e_l['var']:.4g} fixed {e_f['var']:.4g} long fixed {ref['var']:.4g}; "
         f"-bF learned {e_l['minus_betaF_bar']:.4f} long fixed {ref['minus_betaF_bar']:.4f}")
    assert e_l["var"] < 0.2 * e_f["var"]
    se = np.sqrt(e_l["var"] / M + ref["var"] / M)
    assert abs(e_l["minus_betaF_bar"] - ref["minus_betaF_bar"]) < 5 * se + 0.01
