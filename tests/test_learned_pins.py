"""Pins of the learned-step oracle against facts that do not come from the oracle itself:
exact distributions (the exponential tilt of a binomial), closed forms of two-level
populations and of Adam's first steps, library moments and library BF16 rounding,
finite differences of the loss, and symmetries of the network."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import learned as ol
from tests import inputs

torch = pytest.importorskip("torch")


# ------------------------------------------------------------------ resampled fraction

def test_rho_zero_step_monotone_and_limit():
    g = np.random.default_rng(1)
    E = -4 * g.binomial(40, 0.4, 5000) + 12
    vals, h = ol.histogram(E)
    assert ol.rho(vals, h, 0.0) == 0.0
    grid = np.linspace(0, 3, 61)
    r = np.array([ol.rho(vals, h, d) for d in grid])
    assert np.all(np.diff(r) >= -1e-15)
    # for a large step everything but the lowest energy is resampled away
    assert abs(ol.rho(vals, h, 50.0) - (1.0 - h[0] / h.sum())) < 1e-12


@pytest.mark.parametrize("n,p,dbeta", [(40, 0.3, 0.05), (400, 0.3, 0.01), (2500, 0.7, 0.002), (60, 0.45, 0.4)])
def test_rho_of_binomial_equals_total_variation_of_tilt(n, p, dbeta):
    # energies 4k with binomial weights: reweighting by exp(-dbeta 4k) gives the binomial
    # with p' = p e / (1 - p + p e), e = exp(-4 dbeta); rho is the total-variation distance
    k = np.arange(n + 1)
    h = stats.binom.pmf(k, n, p)
    e = math.exp(-4 * dbeta)
    p2 = p * e / (1 - p + p * e)
    tv = 0.5 * np.abs(stats.binom.pmf(k, n, p) - stats.binom.pmf(k, n, p2)).sum()
    assert abs(ol.rho(4 * k, h, dbeta) - tv) < 1e-12


def test_rho_and_label_two_levels_closed_form():
    a, b = 700.0, 300.0
    vals, h = np.array([-8, -4]), np.array([a, b])
    p0 = a / (a + b)
    for d in (0.01, 0.2, 1.5):
        w = math.exp(-4 * d)
        assert abs(ol.rho(vals, h, d) - (a / (a + b * w) - p0)) < 1e-14
    for rs in (0.05, 0.1, 0.2):
        w = (a / (rs + p0) - a) / b
        assert abs(ol.step_label(vals, h, rs, 5.0) - (-math.log(w) / 4)) < 1e-12
    # rho never exceeds b / (a + b): the target 0.35 is out of reach, the label is the cap
    assert ol.step_label(vals, h, 0.35, 2.0) == 2.0


def test_label_solves_target():
    g = np.random.default_rng(5)
    E = 4 * g.binomial(300, 0.5, 20000)
    vals, h = ol.histogram(E)
    for rs in (0.1, 0.2, 0.3, 0.5):
        d = ol.step_label(vals, h, rs, 1.0)
        assert 0 < d < 1 and abs(ol.rho(vals, h, d) - rs) < 1e-12
    # a single energy: nothing can be resampled
    assert ol.step_label(np.array([12]), np.array([9.0]), 0.1, 0.7) == 0.7


def test_features_match_library_moments():
    g = np.random.default_rng(2)
    E = 4 * g.binomial(200, 0.3, 3001) - 500
    f = ol.features(1.25, 512, E)
    assert f[0] == 1.25 and f[1] == math.log(512) and f[2] == math.log(3001)
    assert abs(f[3] - np.mean(E) / 512) < 1e-15
    assert abs(f[4] - np.var(E) / 512) < 1e-12 * f[4]
    assert abs(f[5] - stats.skew(E, bias=True)) < 1e-10
    assert ol.features(0.0, 64, np.full(10, -64))[5] == 0.0


# ------------------------------------------------------------------ BF16 rounding

def test_bf16_rounding_matches_torch():
    x = inputs.float32_values(3, 4096)
    mine = ol.bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    nan = np.isnan(x)
    assert np.array_equal(mine[~nan], ref[~nan])
    assert np.all(mine[nan] == 0x7FC0)
    vals = ol.bf16_values(mine[~nan])
    assert np.array_equal(vals, torch.from_numpy(ref[~nan].view(np.int16)).view(torch.bfloat16).double().numpy())


# ------------------------------------------------------------------ network

def _theta(seed, scale=1.0):
    return ol.bf16_values(ol.bf16_bits(inputs.mlp_theta(seed, scale)))


def test_loss_gradient_matches_finite_differences():
    theta = _theta(7, scale=2.0)
    X = inputs.mlp_features(8, 6).astype(np.float64)
    t = inputs.mlp_targets(9, 6)
    L, g = ol.loss_and_grad(theta, X, t)
    assert abs(L - ol.loss(theta, X, t)) < 1e-14 * L
    rng = np.random.default_rng(0)
    idx = set(rng.choice(ol.N_PARAMS, 300, replace=False).tolist())
    for off in ol.OFF.values():  # every block, first and second entries
        idx.update(i for i in (off, off + 1) if i < ol.N_PARAMS)
    idx.update([ol.OFF["b1"] - 1, ol.OFF["b2"] - 1, ol.OFF["b3"] - 1, ol.OFF["w4"] - 1, ol.N_PARAMS - 1])
    gmax = np.abs(g).max()
    eps = 1e-5
    for i in sorted(idx):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (ol.loss(tp, X, t) - ol.loss(tm, X, t)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * gmax + 1e-6 * abs(g[i]), (i, fd, g[i])


def test_invalid_samples_do_not_contribute():
    theta = _theta(11)
    X = inputs.mlp_features(12, 8).astype(np.float64)
    t = inputs.mlp_targets(13, 8)
    X[2, 4] = 0.0
    t[5] = 0.0
    t[6] = np.nan
    keep = [0, 1, 3, 4, 7]
    L, g = ol.loss_and_grad(theta, X, t)
    L2, g2 = ol.loss_and_grad(theta, X[keep], t[keep])
    assert abs(L * 8 - L2 * 5) < 1e-12 and np.allclose(g * 8, g2 * 5, rtol=1e-12, atol=1e-15)


def test_hidden_unit_permutation_invariance():
    theta = _theta(17)
    p = ol.unpack(theta)
    g = np.random.default_rng(3)
    p1, p2, p3 = g.permutation(64), g.permutation(64), g.permutation(64)
    q = dict(W1=p["W1"][p1], b1=p["b1"][p1], W2=p["W2"][p2][:, p1], b2=p["b2"][p2],
             W3=p["W3"][p3][:, p2], b3=p["b3"][p3], w4=p["w4"][p3], b4=p["b4"])
    X = inputs.mlp_features(18, 50).astype(np.float64)
    a = ol.forward(theta, X, 0.0, np.inf)
    b = ol.forward(ol.pack(q), X, 0.0, np.inf)
    assert np.allclose(a, b, rtol=1e-13, atol=0)
    # a wrong permutation (columns of W3 not following W2's rows) changes the output
    bad = dict(q, W3=p["W3"][p3])
    assert not np.allclose(a, ol.forward(ol.pack(bad), X, 0.0, np.inf), rtol=1e-6)


def test_single_path_network_closed_form():
    theta = np.zeros(ol.N_PARAMS)
    p = ol.unpack(theta)
    p["W1"][3, 0], p["W2"][5, 3], p["W3"][7, 5], p["w4"][7], p["b4"] = 0.8, -1.3, 0.9, 2.0, -0.25
    p["b1"][3], p["b2"][5] = 0.1, -0.2
    theta = ol.pack(p)
    x = np.array([3.0, math.log(512), 10.0, -1.2, 0.5, 0.3])
    u = (3.0 - 2.5) / 2.5
    z = 2.0 * math.tanh(0.9 * math.tanh(-1.3 * math.tanh(0.8 * u + 0.1) - 0.2)) - 0.25
    want = math.log1p(math.exp(z)) / math.sqrt(512 * 0.5)
    assert abs(ol.forward(theta, [x], 0.0, 10.0)[0] - want) < 1e-15
    assert ol.forward(theta, [x], 0.0, want / 2)[0] == want / 2          # clamp above
    assert ol.forward(theta, [x], 2 * want, 10.0)[0] == 2 * want          # clamp below
    x0 = x.copy()
    x0[4] = 0.0
    assert ol.forward(theta, [x0], 0.0, 0.3)[0] == 0.3                     # var = 0 -> dmax


# ------------------------------------------------------------------ Adam

def test_adam_constant_gradient_moves_by_lr():
    # with a constant gradient the bias-corrected moments are g and g^2 at every step:
    # each step moves theta by lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = np.array([1.0, 1.0, -1.0, 0.5]), np.zeros(4), np.zeros(4)
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        th_new, m, v = ol.adam(th, m, v, g, t, lr, 0.9, 0.999, eps)
        assert np.allclose(th - th_new, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)
        th = th_new


def test_adam_second_step_after_gradient_stops():
    g = np.array([0.5, -4.0])
    b1, b2, lr = 0.9, 0.999, 0.1
    th1, m, v = ol.adam(np.zeros(2), np.zeros(2), np.zeros(2), g, 1, lr, b1, b2, 0.0)
    th2, m, v = ol.adam(th1, m, v, np.zeros(2), 2, lr, b1, b2, 0.0)
    # m2^ = b1 g / (1 + b1), v2^ = b2 g^2 / (1 + b2)
    step = lr * (b1 / (1 + b1)) / math.sqrt(b2 / (1 + b2)) * np.sign(g)
    assert np.allclose(th1 - th2, step, rtol=1e-12)
