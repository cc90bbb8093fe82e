"""CPU oracle of the learned temperature step.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the library, and sharing
no code with it.  Plain numpy, FP64 throughout (the network's weights are whatever values
the caller passes, normally BF16-representable ones), one obvious loop or array
expression per formula.

The paper fixes the schedule by hand (Sec. II: any sequence of temperatures gives an
exact method; Sec. III: the variance of beta F~ measures how well a run equilibrated;
Sec. IV uses evenly spaced temperatures).  This extension proposes each step with a small
network and needs the following, none of which the paper defines:

* resampled fraction of a population for a step dbeta, built from the normalised
  weights tau_j of Sec. II (eq. wn):  rho(dbeta) = 1 - (1/R) sum_j min(1, tau_j),
  tau_j = exp(-dbeta E_j) / Q with Q the mean of exp(-dbeta E) (eq. Q).  It is the
  total-variation distance between the population and its reweighting, 0 at dbeta = 0
  and non-decreasing in dbeta;
* the step label: the dbeta in [0, cap] with rho(dbeta) = rho*, by bisection (64
  halvings of [0, cap]; cap itself when rho(cap) <= rho*);
* features of a population at beta: (beta, ln N, ln R, mean E / N, var E / N, skewness),
  variance with 1/R, skewness = third central moment / var^1.5 (0 when var = 0);
* the network 6 -> 64 -> 64 -> 64 -> 1 with tanh hidden units: inputs normalised by the
  fixed affine map xh = (x - SHIFT) / SCALE, output y = softplus(z) is the step in units
  of 1 / sigma_E (sigma_E = sqrt(N * var/N)), so dbeta = y / sigma_E, clamped to
  [dmin, dmax] (dmax when var = 0);
* loss: mean over the batch of (ln y - ln sigma_E - ln dbeta*)^2 (squared error of
  ln dbeta), samples with var <= 0 or a non-finite label contribute 0 and still count
  in the mean;
* Adam (Kingma and Ba, ICLR 2015) with bias-corrected moments;
* rounding of FP32 values to BF16, round to nearest, ties to even.

Parameter vector (row-major W[out][in]):
  W1[64][6] @0, b1[64] @384, W2[64][64] @448, b2 @4544, W3[64][64] @4608, b3 @8704,
  w4[64] @8768, b4 @8832; 8833 values.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, HIDDEN = 6, 64
SHIFT = np.array([2.5, 6.0, 10.0, -1.0, 1.0, 0.0])
SCALE = np.array([2.5, 2.0, 2.5, 1.0, 1.0, 2.0])
OFF = dict(W1=0, b1=384, W2=448, b2=4544, W3=4608, b3=8704, w4=8768, b4=8832)
N_PARAMS = 8833
BISECT_STEPS = 64


# ----------------------------------------------------------------- parameters

def unpack(theta):
    t = np.asarray(theta, np.float64)
    assert t.shape == (N_PARAMS,)
    return dict(
        W1=t[0:384].reshape(HIDDEN, N_IN), b1=t[384:448],
        W2=t[448:4544].reshape(HIDDEN, HIDDEN), b2=t[4544:4608],
        W3=t[4608:8704].reshape(HIDDEN, HIDDEN), b3=t[8704:8768],
        w4=t[8768:8832], b4=t[8832])


def pack(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"],
                           p["w4"], [p["b4"]]]).astype(np.float64)


# ----------------------------------------------------------------- BF16

def bf16_bits(x):
    """BF16 bit patterns of FP32 values: the top 16 bits after rounding the low 16 to
    nearest, ties to even; NaN -> 0x7FC0."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    out = np.empty(u.shape, np.uint16)
    for idx, b in np.ndenumerate(u):
        b = int(b)
        if (b & 0x7F800000) == 0x7F800000 and (b & 0x007FFFFF):
            out[idx] = 0x7FC0
            continue
        low = b & 0xFFFF
        hi = b >> 16
        if low > 0x8000 or (low == 0x8000 and (hi & 1)):
            hi += 1
        out[idx] = hi & 0xFFFF
    return out


def bf16_values(bits):
    """FP64 values of BF16 bit patterns."""
    b = np.asarray(bits, np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


# ----------------------------------------------------------------- population statistics

def histogram(E):
    """Distinct energies and their counts."""
    vals, counts = np.unique(np.asarray(E, np.int64), return_counts=True)
    return vals, counts.astype(np.float64)


def rho(vals, h, dbeta):
    """Resampled fraction 1 - (1/R) sum_j min(1, tau_j) of a population with h[i] replicas
    at energy vals[i] (h may be any non-negative weights)."""
    vals = np.asarray(vals, np.float64)
    h = np.asarray(h, np.float64)
    R = h.sum()
    w = np.exp(-dbeta * (vals - vals.min()))   # exp(-dbeta E) up to a common factor
    Q = (h * w).sum() / R
    tau = w / Q
    return 1.0 - (h * np.minimum(1.0, tau)).sum() / R


def step_label(vals, h, rho_target, cap):
    """dbeta in [0, cap] with rho(dbeta) = rho_target, by bisection; cap when unreachable."""
    if rho(vals, h, cap) <= rho_target:
        return cap
    lo, hi = 0.0, cap
    for _ in range(BISECT_STEPS):
        mid = 0.5 * (lo + hi)
        if rho(vals, h, mid) < rho_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def features(beta, N, E):
    """(beta, ln N, ln R, mean/N, var/N, skew) of a population with energies E."""
    E = np.asarray(E, np.float64)
    R = len(E)
    mean = E.mean()
    d = E - mean
    var = (d * d).mean()
    m3 = (d * d * d).mean()
    skew = m3 / var ** 1.5 if var > 0 else 0.0
    return np.array([beta, math.log(N), math.log(R), mean / N, var / N, skew])


# ----------------------------------------------------------------- network

def softplus(z):
    return max(z, 0.0) + math.log1p(math.exp(-abs(z)))


def sigmoid(z):
    return 1.0 / (1.0 + math.exp(-z)) if z >= 0 else math.exp(z) / (1.0 + math.exp(z))


def forward_one(p, x):
    """Activations of one sample x (6 raw features)."""
    xh = (np.asarray(x, np.float64) - SHIFT) / SCALE
    h1 = np.tanh(p["W1"] @ xh + p["b1"])
    h2 = np.tanh(p["W2"] @ h1 + p["b2"])
    h3 = np.tanh(p["W3"] @ h2 + p["b3"])
    z = float(p["w4"] @ h3 + p["b4"])
    return dict(xh=xh, h1=h1, h2=h2, h3=h3, z=z)


def log_sigma(x):
    """ln sigma_E = (ln N + ln(var/N)) / 2; None when var <= 0."""
    v = x[4]
    return None if not v > 0 else 0.5 * (x[1] + math.log(v))


def forward(theta, X, dmin, dmax):
    """dbeta proposed for every row of X [B][6]."""
    p = unpack(theta)
    out = np.empty(len(X))
    for b, x in enumerate(np.asarray(X, np.float64)):
        ls = log_sigma(x)
        if ls is None:
            out[b] = dmax
            continue
        a = forward_one(p, x)
        d = softplus(a["z"]) / math.exp(ls)
        out[b] = min(max(d, dmin), dmax)
    return out


def loss_and_grad(theta, X, dstar):
    """Mean squared error of ln dbeta over the batch and its gradient (backpropagation)."""
    p = unpack(theta)
    g = {k: np.zeros_like(v) if isinstance(v, np.ndarray) else 0.0 for k, v in p.items()}
    X = np.asarray(X, np.float64)
    B = len(X)
    total = 0.0
    for x, t in zip(X, np.asarray(dstar, np.float64)):
        ls = log_sigma(x)
        if ls is None or not (t > 0 and math.isfinite(t)):
            continue
        a = forward_one(p, x)
        z = a["z"]
        err = math.log(softplus(z)) - ls - math.log(t)
        total += err * err
        gz = (2.0 / B) * err * sigmoid(z) / softplus(z)
        g["b4"] += gz
        g["w4"] += gz * a["h3"]
        d3 = gz * p["w4"] * (1.0 - a["h3"] ** 2)
        g["W3"] += np.outer(d3, a["h2"])
        g["b3"] += d3
        d2 = (p["W3"].T @ d3) * (1.0 - a["h2"] ** 2)
        g["W2"] += np.outer(d2, a["h1"])
        g["b2"] += d2
        d1 = (p["W2"].T @ d2) * (1.0 - a["h1"] ** 2)
        g["W1"] += np.outer(d1, a["xh"])
        g["b1"] += d1
    return total / B, pack(g)


def loss(theta, X, dstar):
    p = unpack(theta)
    X = np.asarray(X, np.float64)
    total = 0.0
    for x, t in zip(X, np.asarray(dstar, np.float64)):
        ls = log_sigma(x)
        if ls is None or not (t > 0 and math.isfinite(t)):
            continue
        err = math.log(softplus(forward_one(p, x)["z"])) - ls - math.log(t)
        total += err * err
    return total / len(X)


# ----------------------------------------------------------------- Adam

def adam(theta, m, v, grad, t, lr, beta1, beta2, eps):
    """One Adam update (step number t >= 1): returns new (theta, m, v)."""
    theta, m, v, grad = (np.asarray(a, np.float64) for a in (theta, m, v, grad))
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
