"""FP64 CPU oracle of the learned warm start's network, loss, gradient and features.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only the tests, the smoke entry and the benchmark's CPU-baseline leg do.
It shares no code with the HIP path.

The learned warm start is not part of the paper's method (its contact solve
starts from the previous iterate, Alg. 1); it is an addition whose only effect
is the starting point of the first contact solve of a step.  What is fixed here:

* the network: 16 inputs -> three hidden layers of 128 ReLU units -> 3
  outputs, parameters packed as W1, b1, W2, b2, W3, b3, W4, b4 with every W
  stored out x in, row-major (35,587 values);
* "bf16 GEMM": both operands of every matrix product are rounded to bfloat16
  (8 significant bits, round to nearest, ties to even) and the products are
  summed exactly (here in FP64); biases and the ReLU act on the unrounded sums.
  With ``bf16=False`` every product is plain FP64;
* the loss: mean squared error over the n x 3 outputs, L = sum (y - t)^2 / (3n);
* backpropagation: dY = 2 (Y - T) / (3n); for a layer Z = A W^T + b:
  dW = dZ^T A, db = column sums of dZ, dA = dZ W; a ReLU passes dZ where its
  output is positive.  In bf16 mode dW and dA are bf16 GEMMs too.
* features (one row per contact, at the step start, contact frame of the
  step; delta_c = contact margin, s = h^2 / m_v, dobs the obstacle's
  displacement over the step, Gbar = Abar^-1):
  d0/delta_c, n.(h v + h^2 g)/delta_c, (h v - dobs).(n, t1, t2)/delta_c,
  s lambda_prev (3)/delta_c, had-previous flag, mu, log10(m_v Gbar_vv),
  log10(m_v / 1 g), number of contacts on the vertex among the list
  neighbours (1..3), (g.n) h^2/delta_c, (dobs.n)/delta_c, 1;
  label: s (lambda_1 - lambda_prev) / delta_c (contact frame), where lambda_1
  solves the step's first contact subproblem (first local-global iteration)
  and lambda_prev is the previous-step warm start of the features; the
  prediction is lambda_prev + output * delta_c / s, projected on the cone.

Pins (tests/test_mlp_oracle.py): central finite differences of the FP64 loss
for the backpropagation, hand-built networks with known outputs for the
forward pass, known bfloat16 roundings, and the bf16 gradient within the
format's precision of the FP64 one.
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT, N_HID, N_OUT = 16, 128, 3
SHAPES = [("W1", (N_HID, N_FEAT)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_OUT, N_HID)), ("b4", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray):
    """Splits the packed parameter vector into the dict of named arrays (views)."""
    out, off = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[off:off + k].reshape(shp)
        off += k
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(a) -> np.ndarray:
    """Rounds to bfloat16 (8 significant bits, nearest, ties to even), returned as FP64.

    Written from the definition: x = m 2^e with 0.5 <= |m| < 1, keep 8 bits of m.
    Values stay in FP32's normal range in every use here.
    """
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def _mm(A, B, rounded: bool):
    if rounded:
        return bf16(A) @ bf16(B)
    return A @ B


def forward(theta: np.ndarray, X: np.ndarray, rounded: bool = True):
    """Network outputs Y (n x 3) and the hidden activations (H1, H2, H3)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    H1 = np.maximum(_mm(X, p["W1"].T, rounded) + p["b1"], 0.0)
    H2 = np.maximum(_mm(H1, p["W2"].T, rounded) + p["b2"], 0.0)
    H3 = np.maximum(_mm(H2, p["W3"].T, rounded) + p["b3"], 0.0)
    Y = _mm(H3, p["W4"].T, rounded) + p["b4"]
    return Y, (H1, H2, H3)


def loss(theta, X, T, rounded: bool = True) -> float:
    Y, _ = forward(theta, X, rounded)
    return float(np.sum((Y - np.asarray(T, dtype=np.float64)) ** 2) / Y.size)


def loss_and_grad(theta, X, T, rounded: bool = True):
    """Mean-squared loss and its gradient by backpropagation (packed like theta)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    Y, (H1, H2, H3) = forward(theta, X, rounded)
    L = float(np.sum((Y - T) ** 2) / Y.size)
    g = {}
    dZ = 2.0 * (Y - T) / Y.size
    layers = [("W4", "b4", H3, None), ("W3", "b3", H2, H3), ("W2", "b2", H1, H2), ("W1", "b1", X, H1)]
    for k, (wn, bn, Ain, Aout) in enumerate(layers):
        if Aout is not None:
            dZ = dZ * (Aout > 0.0)
        g[wn] = _mm(dZ.T, Ain, rounded)
        g[bn] = dZ.sum(axis=0)
        if wn != "W1":
            dZ = _mm(dZ, p[wn], rounded)
    return L, pack(g)


def adam_step(theta, grad, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(oe, x, v, obstacles, params, contacts, lam_prev, has_prev):
    """Per-contact feature rows (c x 16) at the step start.

    contacts: the step's contact list (flash_oracle.detect), lam_prev (c x 3)
    the previous-step multipliers already expressed in this step's frames and
    projected onto the cone, has_prev (c,) bool.
    """
    c = contacts.count
    F = np.zeros((c, N_FEAT))
    if c == 0:
        return F
    h = params.h
    dc = params.contact_margin if params.contact_margin > 0 else 1e-3
    g = np.asarray(params.gravity, dtype=np.float64)
    for j in range(c):
        vi = int(contacts.vertex[j])
        fr = contacts.frame[j]          # columns n, t1, t2
        nrm = fr[:, 0]
        m = oe.mass[vi]
        s = h * h / m
        e = np.zeros((oe.n, 1))
        e[vi, 0] = 1.0
        gvv = float(oe.solve(e)[vi, 0])
        ut = h * v[vi] + h * h * g
        rel = h * v[vi] - contacts.dobs[j]
        nc = 1
        if j > 0 and contacts.vertex[j - 1] == vi:
            nc += 1
        if j + 1 < c and contacts.vertex[j + 1] == vi:
            nc += 1
        F[j, 0] = contacts.d0[j] / dc
        F[j, 1] = nrm @ ut / dc
        F[j, 2:5] = (fr.T @ rel) / dc
        F[j, 5:8] = s * np.asarray(lam_prev[j], dtype=np.float64) / dc
        F[j, 8] = 1.0 if has_prev[j] else 0.0
        F[j, 9] = oe.mu
        F[j, 10] = math.log10(max(gvv * m, 1e-30))
        F[j, 11] = math.log10(m / 1e-3)
        F[j, 12] = nc
        F[j, 13] = (g @ nrm) * h * h / dc
        F[j, 14] = (contacts.dobs[j] @ nrm) / dc
        F[j, 15] = 1.0
    return F


def labels(oe, params, contacts, lam_first, lam_prev):
    """s (lambda_1 - lambda_prev) / delta_c per contact (contact frame).

    lam_first (c x 3): solution of the step's first contact subproblem;
    lam_prev (c x 3): the previous-step warm start (zero for new contacts).
    """
    dc = params.contact_margin if params.contact_margin > 0 else 1e-3
    s = params.h * params.h / oe.mass[np.asarray(contacts.vertex, dtype=np.int64)]
    return s[:, None] * (np.asarray(lam_first, dtype=np.float64) - np.asarray(lam_prev, dtype=np.float64)) / dc
