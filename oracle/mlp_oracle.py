"""FP64 CPU oracle of the coordinate-MLP surrogate.

TEST INFRASTRUCTURE ONLY: called by the test suite, never by the library.

The surrogate is not part of the paper (which has no learned component); it
is the library's stand-in for V(r) inside the QM region.  The network:

    gamma(r)  = [cos(2 pi B r), sin(2 pi B r)]          B: n_freq x 3, 2 n_freq inputs
    H_0       = bf16(gamma)
    Z_l       = H_{l-1} W_l^T + b_l,   H_l = bf16(silu(Z_l)),   l = 1..4
    y         = H_4 . w_out + b_out                       (output layer in FP32)
    V_hat(r)  = poly(r / R) + sigma * y

with W_l used as BF16 (their FP32 master copies are the parameters), silu(z) =
z / (1 + exp(-z)), and poly a polynomial baseline in the scaled coordinates
u = r / R (monomials u_x^a u_y^b u_z^c, a+b+c <= degree, ordered by total
degree, then a descending, then b descending).

Training loss on normalised targets t: L = mean((y - t)^2).  The backward pass
treats each BF16 rounding as the identity (straight-through) and rounds dZ to
BF16 where the GPU feeds it to its matrix cores: dW_l = bf16(dZ_l)^T H_{l-1},
dH_{l-1} = bf16(dZ_l) bf16(W_l), db_l = sum_n dZ_l.

``rounding=False`` runs the same network with no rounding at all, for the
finite-difference self-check of the backward formulas.

Parameter vector layout (float32): W1 (128 x 128, out x in), b1, W2, b2, W3, b3,
W4, b4, w_out (128), b_out (1): 66,177 values for 64 frequencies.
"""
from __future__ import annotations

import math

import numpy as np

N_LAYERS = 4
HIDDEN = 128


def bf16(x):
    """Round to bfloat16 (round to nearest even) through float32, as the GPU
    converts its FP32 values."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def n_params(n_in=128):
    return N_LAYERS * (HIDDEN * HIDDEN + HIDDEN) + HIDDEN + 1 if n_in == 128 else None


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for _ in range(N_LAYERS):
        W = p[o:o + HIDDEN * HIDDEN].reshape(HIDDEN, HIDDEN)
        o += HIDDEN * HIDDEN
        b = p[o:o + HIDDEN]
        o += HIDDEN
        out.append((W, b))
    w_out = p[o:o + HIDDEN]
    o += HIDDEN
    b_out = p[o]
    return out, w_out, b_out


def features(points, B):
    phi = 2.0 * math.pi * (np.asarray(points, dtype=np.float64) @ np.asarray(B, dtype=np.float64).T)
    return np.concatenate([np.cos(phi), np.sin(phi)], axis=1)


def hidden_pre(Hprev, W, b):
    """Pre-activation of one hidden layer from given inputs (FP64):
    Hprev bf16(W)^T + b, with its conditioning scale |Hprev| |bf16(W)|^T + |b|."""
    Wr = bf16(W)
    return Hprev @ Wr.T + b, np.abs(Hprev) @ np.abs(Wr).T + np.abs(b)


def hidden_act(Z):
    """H = bf16(silu(Z)) of given pre-activations."""
    return bf16(silu(np.asarray(Z, dtype=np.float64)))


def output(H4, w_out, b_out):
    """y = H4 . w_out + b_out (FP64) and its scale |H4| |w_out| + |b_out|."""
    return H4 @ w_out + b_out, np.abs(H4) @ np.abs(w_out) + abs(b_out)


def dz_of(dH, Z):
    """dL/dZ = dL/dH silu'(Z) (FP64, before any rounding)."""
    return dH * dsilu(np.asarray(Z, dtype=np.float64))


def weight_grad(dZr, Hprev):
    """dL/dW = dZ_r^T Hprev (dZ_r as fed to the product) and its scale."""
    return dZr.T @ Hprev, np.abs(dZr).T @ np.abs(Hprev)


def input_grad(dZr, W):
    """dL/dHprev = dZ_r bf16(W) and its scale."""
    Wr = bf16(W)
    return dZr @ Wr, np.abs(dZr) @ np.abs(Wr)


def forward(params, points, B, rounding=True):
    layers, w_out, b_out = unpack(params)
    r = bf16 if rounding else (lambda x: np.asarray(x, dtype=np.float64))
    H = r(features(points, B))
    cache = [(H, None)]
    for W, b in layers:
        Z = H @ r(W).T + b
        H = r(silu(Z))
        cache.append((H, Z))
    y = H @ w_out + b_out
    return y, cache


def loss_and_grads(params, points, t, B, rounding=True):
    """Loss mean((y - t)^2) and its gradient in the parameter layout."""
    layers, w_out, b_out = unpack(params)
    r = bf16 if rounding else (lambda x: np.asarray(x, dtype=np.float64))
    y, cache = forward(params, points, B, rounding)
    n = len(t)
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / n
    H4 = cache[-1][0]
    g_wout = H4.T @ dy
    g_bout = dy.sum()
    dH = np.outer(dy, w_out)
    grads = [None] * N_LAYERS
    for l in range(N_LAYERS - 1, -1, -1):
        W, b = layers[l]
        Z = cache[l + 1][1]
        Hprev = cache[l][0]
        dZ = dH * dsilu(Z)
        dZr = r(dZ)
        gW = dZr.T @ Hprev
        gb = dZ.sum(axis=0)
        grads[l] = (gW, gb)
        if l > 0:
            dH = dZr @ r(W)
    flat = []
    for gW, gb in grads:
        flat += [gW.ravel(), gb]
    flat += [g_wout, np.array([g_bout])]
    return loss, np.concatenate(flat)


def monomials(degree):
    out = []
    for k in range(degree + 1):
        for a in range(k, -1, -1):
            for b in range(k - a, -1, -1):
                out.append((a, b, k - a - b))
    return out


def poly_eval(points, coefs, degree, radius):
    u = np.asarray(points, dtype=np.float64) / radius
    v = np.zeros(u.shape[0])
    for c, (a, b, e) in zip(coefs, monomials(degree)):
        v += c * u[:, 0] ** a * u[:, 1] ** b * u[:, 2] ** e
    return v


def predict(params, points, B, coefs, degree, radius, sigma):
    y, _ = forward(params, points, B, rounding=True)
    return poly_eval(points, coefs, degree, radius) + sigma * y


def fd_check(params, points, t, B, idx, h=1e-6):
    """Central differences of the unrounded loss at parameter indices idx."""
    p = np.asarray(params, dtype=np.float64).copy()
    _, g = loss_and_grads(p, points, t, B, rounding=False)
    fd = []
    for i in idx:
        old = p[i]
        p[i] = old + h
        lp, _ = loss_and_grads(p, points, t, B, rounding=False)
        p[i] = old - h
        lm, _ = loss_and_grads(p, points, t, B, rounding=False)
        p[i] = old
        fd.append((lp - lm) / (2 * h))
    return g[np.asarray(idx)], np.array(fd)
