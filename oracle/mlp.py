"""FP64 reference of the surrogate networks' training arithmetic (test infrastructure only).

The learned form replaces a tabulated potential function g (f, phi or F) inside an
input range [x_lo, x_hi] by a network with one input, two SiLU layers of H = 32
units and a linear output:

    t  = (x - c) s,           c = (x_lo + x_hi) / 2,  s = 2 / (x_hi - x_lo)
    z1 = W1 t + b1,           h1 = silu(z1)
    z2 = W2 h1 + b2,          h2 = silu(z2)
    y  = w3 . h2 + b3,        g(x) = y_shift + y_scale y

silu(z) = z sigma(z).  The force needs g'(x) = y_scale s dy/dt, so the forward pass
carries the tangent dh1 = silu'(z1) W1, dz2 = W2 dh1, dy = w3 . (silu'(z2) dz2).
A loss that depends on y and dy per sample is linearised as
sum_b c_val[b] y_b + c_der[b] dy_b; ``param_grad`` is its exact gradient with
respect to the parameters (reverse mode through the forward and tangent passes,
which brings in silu'').  Everything here is plain numpy in float64, written from
these definitions; the C oracle has its own evaluation of the same network.

Parameter vector layout (MLP_PARAMS = 1153): W1[32], b1[32], W2[32][32] (row =
output unit), b2[32], w3[32], b3.
"""
from __future__ import annotations

import numpy as np

H = 32
MLP_PARAMS = H * (H + 4) + 1


def split(p):
    p = np.asarray(p, dtype=np.float64)
    W1 = p[0:H]
    b1 = p[H:2 * H]
    W2 = p[2 * H:2 * H + H * H].reshape(H, H)
    b2 = p[2 * H + H * H:3 * H + H * H]
    w3 = p[3 * H + H * H:4 * H + H * H]
    b3 = p[4 * H + H * H]
    return W1, b1, W2, b2, w3, b3


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def d2silu(z):
    s = sigmoid(z)
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def scaling(x_lo, x_hi):
    return 0.5 * (x_lo + x_hi), 2.0 / (x_hi - x_lo)


def forward_t(p, t):
    """Normalised output y(t) and dy/dt for an array of t."""
    W1, b1, W2, b2, w3, b3 = split(p)
    t = np.asarray(t, dtype=np.float64)[:, None]
    z1 = t * W1[None, :] + b1[None, :]
    h1 = silu(z1)
    dh1 = dsilu(z1) * W1[None, :]
    z2 = h1 @ W2.T + b2[None, :]
    dz2 = dh1 @ W2.T
    y = silu(z2) @ w3 + b3
    dy = (dsilu(z2) * dz2) @ w3
    return y, dy


def evaluate(net, x):
    """g(x) and g'(x) of net = (x_lo, x_hi, y_shift, y_scale, params)."""
    lo, hi, sh, sc, p = net
    c, s = scaling(lo, hi)
    y, dy = forward_t(p, (np.asarray(x, dtype=np.float64) - c) * s)
    return sh + sc * y, sc * s * dy


def param_grad(p, t, c_val, c_der):
    """Gradient of sum_b c_val[b] y(t_b) + c_der[b] dy/dt(t_b) with respect to p."""
    W1, b1, W2, b2, w3, b3 = split(p)
    t = np.asarray(t, dtype=np.float64)[:, None]
    cv = np.asarray(c_val, dtype=np.float64)[:, None]
    cd = np.asarray(c_der, dtype=np.float64)[:, None]
    # forward with tangents
    z1 = t * W1[None, :] + b1[None, :]
    h1, a1 = silu(z1), dsilu(z1)
    dh1 = a1 * W1[None, :]
    z2 = h1 @ W2.T + b2[None, :]
    dz2 = dh1 @ W2.T
    h2, a2 = silu(z2), dsilu(z2)
    dh2 = a2 * dz2
    # reverse
    g_w3 = (cv * h2 + cd * dh2).sum(0)
    g_b3 = cv.sum()
    g_h2 = cv * w3[None, :]
    g_dh2 = cd * w3[None, :]
    g_a2 = g_dh2 * dz2
    g_dz2 = g_dh2 * a2
    g_z2 = g_h2 * a2 + g_a2 * d2silu(z2)
    g_W2 = g_z2.T @ h1 + g_dz2.T @ dh1
    g_b2 = g_z2.sum(0)
    g_h1 = g_z2 @ W2
    g_dh1 = g_dz2 @ W2
    g_a1 = g_dh1 * W1[None, :]
    g_W1 = (g_dh1 * a1).sum(0)
    g_z1 = g_h1 * a1 + g_a1 * d2silu(z1)
    g_W1 = g_W1 + (g_z1 * t).sum(0)
    g_b1 = g_z1.sum(0)
    return np.concatenate([g_W1, g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])


def sobolev_coefs(y, dy, y_ref, dy_ref, lam):
    """Per-sample c_val, c_der and the loss of mean((y - y_ref)^2 + lam (dy - dy_ref)^2)."""
    n = len(y)
    ey, ed = y - y_ref, dy - dy_ref
    loss = float(np.mean(ey * ey + lam * ed * ed))
    return 2.0 * ey / n, 2.0 * lam * ed / n, loss


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015); step counts from 1.  Returns p, m, v."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def round_bf16(x):
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def force_match(net_f, net_phi, r, dhat, fp_i, fp_j, f_ref):
    """Forces of sampled atoms from their pair lists with the networks' f' and phi'.

    r[n, K] (0 = no pair), dhat[n, K, 3] unit vectors from the atom to its partner,
    fp_i[n], fp_j[n, K] = F'(rho) of atom and partner, f_ref[n, 3].  Returns the
    predicted forces, the loss sum |F - F_ref|^2 / sum |F_ref|^2, and the per-pair
    coefficients of dy/dt for the f and phi networks (c_der of ``param_grad``).
    """
    mask = r > 0.0
    rr = np.where(mask, r, 1.0)
    _, dfr = evaluate(net_f, rr.ravel())
    _, dph = evaluate(net_phi, rr.ravel())
    dfr = dfr.reshape(r.shape) * mask
    dph = dph.reshape(r.shape) * mask
    w = fp_i[:, None] + fp_j
    s = w * dfr + dph
    F = (s[:, :, None] * dhat).sum(1)
    res = F - f_ref
    norm = float((f_ref * f_ref).sum())
    loss = float((res * res).sum()) / norm
    proj = (res[:, None, :] * dhat).sum(2) * mask * (2.0 / norm)   # dL/ds per pair
    _, _, _, sc_f, _ = net_f
    _, _, _, sc_p, _ = net_phi
    s_f = scaling(net_f[0], net_f[1])[1]
    s_p = scaling(net_phi[0], net_phi[1])[1]
    c_f = proj * w * sc_f * s_f      # ds/d(dy_f) = w * y_scale * s
    c_p = proj * sc_p * s_p
    return F, loss, c_f, c_p
