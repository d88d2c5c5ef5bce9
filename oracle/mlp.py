"""FP64 reference of the learned warm-start network (test infrastructure).

The network maps 12 per-contact features to a 3-vector (a scaled impulse):
  z1 = W1 x + b1,  h1 = gelu(z1)      (128)
  z2 = W2 h1 + b2, h2 = gelu(z2)      (128)
  y  = W3 h2 + b3                      (3)
with the exact GELU, gelu(z) = z Phi(z), and the loss L = mean over samples and
outputs of (y - t)^2.  Parameters use the padded shapes of the GPU kernels:
W1 (128, 16) whose last 4 input columns multiply zero features, W3 (16, 128) whose
rows 3..15 are unused, b3 (16,).  Pins: the backward pass is checked against central
differences of the loss.

The learned warm start is not part of the paper; its inputs are built from quantities
the paper defines: the contact frame and normal gap (App. A), the previous impulse
re-expressed in the new frame (the plain warm start), and the Delassus diagonal K_jj
that sets r_n = h^2 K_jj (Sec. 5.4).  Per contact, with l the mean rest edge length of
the scene and x~ the predicted position:
  f0     (n . x~ - d_n) / l                  normal gap at the predicted state
  f1..3  n                                   contact normal (world)
  f4..6  h C (v_t - u_obstacle) / l          relative velocity in the contact frame
  f7..9  h^2 K_jj lambda_prev / l            previous impulse (contact frame), scaled
  f10    log K_jj
  f11    mu
  f12..15 0
and the target is h^2 K_jj lambda / l for the converged impulse lambda of the frame.
Adam follows Kingma and Ba (2015), bias-corrected moments.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SHAPES = {"W1": (128, 16), "b1": (128,), "W2": (128, 128), "b2": (128,), "W3": (16, 128), "b3": (16,)}
ORDER = ["W1", "b1", "W2", "b2", "W3", "b3"]


def n_params():
    return sum(int(np.prod(SHAPES[k])) for k in ORDER)


def unflatten(flat):
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = np.asarray(flat[o:o + n], np.float64).reshape(SHAPES[k])
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[k], np.float64).reshape(-1) for k in ORDER])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def pad_features(X):
    X = np.asarray(X, np.float64)
    out = np.zeros((len(X), 16))
    out[:, :X.shape[1]] = X
    return out


def forward(p, X):
    x = pad_features(X)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, :3], (x, z1, h1, z2, h2)


def loss(p, X, T):
    y, _ = forward(p, X)
    return float(np.mean((y - T) ** 2))


def grad(p, X, T):
    """Gradient of the mean-squared loss with respect to every parameter (FP64)."""
    y, (x, z1, h1, z2, h2) = forward(p, X)
    B = len(X)
    dy = np.zeros((B, 16))
    dy[:, :3] = 2.0 * (y - T) / (B * 3)
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    dh2 = dy @ p["W3"]
    dz2 = dh2 * gelu_grad(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * gelu_grad(z1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return g


def bf16_round(a):
    """Round float64 values to bfloat16 (round to nearest even) and back."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------------ bf16 rounding points

def _round_weights(p):
    return {k: (bf16_round(v) if k.startswith("W") else np.asarray(v, np.float64)) for k, v in p.items()}


def forward_bf16(p, X):
    """The network with the device's rounding points: weights, inputs and the
    activations h1, h2 rounded to bf16 (they are matrix-core operands); every sum and
    the GELU exact (float64)."""
    q = _round_weights(p)
    x = bf16_round(pad_features(X))
    z1 = x @ q["W1"].T + q["b1"]
    h1 = bf16_round(gelu(z1))
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = bf16_round(gelu(z2))
    y = h2 @ q["W3"].T + q["b3"]
    return y[:, :3], (x, z1, h1, z2, h2)


def grad_bf16(p, X, T):
    """Gradient of the mean-squared loss with the device's rounding points: the forward
    of forward_bf16, and dL/dy, dL/dz2, dL/dz1 rounded to bf16 (matrix-core operands);
    the bias gradients sum those rounded values."""
    y, (x, z1, h1, z2, h2) = forward_bf16(p, X)
    q = _round_weights(p)
    B = len(X)
    dy = np.zeros((B, 16))
    dy[:, :3] = 2.0 * (y - T) / (B * 3)
    dy = bf16_round(dy)
    dz2 = bf16_round((dy @ q["W3"]) * gelu_grad(z2))
    dz1 = bf16_round((dz2 @ q["W2"]) * gelu_grad(z1))
    return {"W3": dy.T @ h2, "b3": dy.sum(0), "W2": dz2.T @ h1, "b2": dz2.sum(0), "W1": dz1.T @ x,
            "b1": dz1.sum(0)}


# ------------------------------------------------------------------ warm-start data

def mean_edge_length(rest, tets):
    """Mean over tets of the six edge lengths at rest (an edge shared by k tets counts k
    times)."""
    rest = np.asarray(rest, np.float64)
    tets = np.asarray(tets, np.int64)
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    L = [np.linalg.norm(rest[tets[:, a]] - rest[tets[:, b]], axis=1) for a, b in pairs]
    return float(np.mean(np.concatenate(L)))


def features(C, d_n, mu, node, q_pred, v_t, obst_vel, lam_prev, K_diag, h, ell):
    """Input features (c, 16) per the definition in the module docstring.

    C (c,3,3) rows n, f1, f2; d_n (c,); mu (c,); node (c,) node per contact; q_pred,
    v_t (n,3); obst_vel (c,3) obstacle velocity per contact; lam_prev (c,3) in the
    contact frame; K_diag (c,) = K_jj."""
    C = np.asarray(C, np.float64)
    c = len(C)
    F = np.zeros((c, 16))
    if c == 0:
        return F
    xp = np.asarray(q_pred, np.float64)[node]
    rel = np.asarray(v_t, np.float64)[node] - np.asarray(obst_vel, np.float64)
    K_diag = np.asarray(K_diag, np.float64)
    F[:, 0] = (np.einsum("ji,ji->j", C[:, 0, :], xp) - np.asarray(d_n)) / ell
    F[:, 1:4] = C[:, 0, :]
    F[:, 4:7] = h * np.einsum("jai,ji->ja", C, rel) / ell
    F[:, 7:10] = (h * h * K_diag / ell)[:, None] * np.asarray(lam_prev, np.float64)
    F[:, 10] = np.log(K_diag)
    F[:, 11] = np.asarray(mu, np.float64)
    return F


def learned_impulse(y, K_diag, h, ell, mu, lam_plain, comp=None, persist=False):
    """Candidate start impulses from network outputs y (c,3): lambda = y l / (h^2 K_jj),
    then the normal part clamped at 0 and the friction part scaled onto the cone
    |lambda_f| <= mu lambda_n.  Contacts with a non-finite prediction, bilateral rows
    (comp >= 0) and, with persist, contacts whose plain start is zero keep lam_plain."""
    y = np.asarray(y, np.float64)
    lam_plain = np.asarray(lam_plain, np.float64)
    lam = y * (ell / (h * h * np.asarray(K_diag, np.float64)))[:, None]
    lam[:, 0] = np.maximum(lam[:, 0], 0.0)
    lf = np.sqrt((lam[:, 1:] ** 2).sum(1))
    cap = np.asarray(mu, np.float64) * lam[:, 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        sh = np.where(lf > cap, np.where(lf > 0, cap / lf, 0.0), 1.0)
    lam[:, 1:] *= sh[:, None]
    keep = ~np.all(np.isfinite(y), axis=1)
    if comp is not None:
        keep |= np.asarray(comp) >= 0.0
    if persist:
        keep |= np.all(lam_plain == 0.0, axis=1)
    lam[keep] = lam_plain[keep]
    return lam


def targets(lam, K_diag, h, ell):
    """Scaled converged impulse h^2 K_jj lambda / l (c, 3)."""
    return (h * h * np.asarray(K_diag, np.float64) / ell)[:, None] * np.asarray(lam, np.float64)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of flat parameters p with gradient g at step t >= 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
