"""Pins of the MLP oracle (CPU).

The surrogate network has no counterpart in the paper, so its oracle is pinned
by what mathematics and independent libraries fix: bfloat16 rounding against
torch's own conversion, SiLU and its derivative against closed values and
central differences, the monomial basis against its count and against a known
polynomial, and the backward pass against central differences of the loss.
"""
import math

import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M


def test_bf16_matches_torch_rounding():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.integers(-8, 8, 4000),
                        [0.0, -0.0, 1.0, -1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: even mantissa (1) wins;
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: 1 + 2^-6 wins.
    assert M.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert M.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_silu_values_and_derivative():
    assert M.silu(np.array([0.0]))[0] == 0.0
    assert abs(M.silu(np.array([1.0]))[0] - 1.0 / (1.0 + math.exp(-1.0))) < 1e-16
    assert abs(M.silu(np.array([-40.0]))[0]) < 1e-15
    z = np.linspace(-6, 6, 41)
    h = 1e-5
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(M.dsilu(z), fd, rtol=0, atol=1e-9)
    assert M.dsilu(np.array([0.0]))[0] == 0.5


@pytest.mark.parametrize("degree", [0, 1, 3, 8])
def test_monomials_count_and_order(degree):
    mons = M.monomials(degree)
    assert len(mons) == math.comb(degree + 3, 3)
    assert len(set(mons)) == len(mons)
    assert mons[0] == (0, 0, 0)
    tot = [sum(m) for m in mons]
    assert tot == sorted(tot)
    if degree >= 1:
        assert mons[1:4] == [(1, 0, 0), (0, 1, 0), (0, 0, 1)]


def test_poly_eval_known_polynomial():
    # p(u) = 2 - u_x + 3 u_x u_z + u_y^2 with u = r / 2
    mons = M.monomials(2)
    c = np.zeros(len(mons))
    c[mons.index((0, 0, 0))] = 2.0
    c[mons.index((1, 0, 0))] = -1.0
    c[mons.index((1, 0, 1))] = 3.0
    c[mons.index((0, 2, 0))] = 1.0
    r = np.random.default_rng(1).uniform(-3, 3, (50, 3))
    u = r / 2.0
    ref = 2 - u[:, 0] + 3 * u[:, 0] * u[:, 2] + u[:, 1] ** 2
    np.testing.assert_allclose(M.poly_eval(r, c, 2, 2.0), ref, rtol=0, atol=1e-13)


def test_features_are_unit_circle_pairs():
    rng = np.random.default_rng(2)
    B = rng.standard_normal((64, 3))
    r = rng.uniform(-5, 5, (20, 3))
    f = M.features(r, B)
    assert f.shape == (20, 128)
    np.testing.assert_allclose(f[:, :64] ** 2 + f[:, 64:] ** 2, 1.0, atol=1e-14)
    # B = 0 gives cos = 1, sin = 0
    f0 = M.features(r, np.zeros((64, 3)))
    assert np.all(f0[:, :64] == 1.0) and np.all(f0[:, 64:] == 0.0)


def _small_params(seed):
    rng = np.random.default_rng(seed)
    p = []
    for _ in range(M.N_LAYERS):
        p += [rng.standard_normal(M.HIDDEN * M.HIDDEN) / math.sqrt(M.HIDDEN), 0.1 * rng.standard_normal(M.HIDDEN)]
    p += [rng.standard_normal(M.HIDDEN) / math.sqrt(M.HIDDEN), [0.3]]
    return np.concatenate(p)


def test_param_count():
    assert M.n_params() == 66177
    assert len(_small_params(0)) == 66177


def test_forward_unrounded_against_explicit_layers():
    params = _small_params(3)
    rng = np.random.default_rng(4)
    B = rng.standard_normal((64, 3)) * 0.25
    r = rng.uniform(-4, 4, (7, 3))
    y, _ = M.forward(params, r, B, rounding=False)
    # the same network written with torch in float64, layer by layer
    P = torch.tensor(params, dtype=torch.float64)
    phi = 2 * math.pi * torch.tensor(r) @ torch.tensor(B).T
    h = torch.cat([torch.cos(phi), torch.sin(phi)], dim=1)
    o = 0
    for _ in range(M.N_LAYERS):
        W = P[o:o + 128 * 128].reshape(128, 128)
        o += 128 * 128
        b = P[o:o + 128]
        o += 128
        h = torch.nn.functional.silu(torch.nn.functional.linear(h, W, b))
    yt = h @ P[o:o + 128] + P[o + 128]
    np.testing.assert_allclose(y, yt.numpy(), rtol=1e-13, atol=1e-13)


def test_backward_matches_central_differences():
    params = _small_params(6)
    rng = np.random.default_rng(7)
    B = rng.standard_normal((64, 3)) * 0.25
    r = rng.uniform(-4, 4, (24, 3))
    t = rng.standard_normal(24)
    L = M.HIDDEN * M.HIDDEN + M.HIDDEN
    # indices in every layer's weights and biases and in the output layer
    idx = []
    for l in range(M.N_LAYERS):
        idx += [l * L + 5, l * L + 1000, l * L + M.HIDDEN * M.HIDDEN + 3]
    idx += [M.N_LAYERS * L + 7, M.N_LAYERS * L + M.HIDDEN]
    g, fd = M.fd_check(params, r, t, B, idx)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-9)


def test_backward_matches_torch_autograd():
    params = _small_params(8)
    rng = np.random.default_rng(9)
    B = rng.standard_normal((64, 3)) * 0.25
    r = rng.uniform(-4, 4, (16, 3))
    t = rng.standard_normal(16)
    loss, g = M.loss_and_grads(params, r, t, B, rounding=False)
    P = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    phi = 2 * math.pi * torch.tensor(r) @ torch.tensor(B).T
    h = torch.cat([torch.cos(phi), torch.sin(phi)], dim=1)
    o = 0
    for _ in range(M.N_LAYERS):
        W = P[o:o + 128 * 128].reshape(128, 128)
        o += 128 * 128
        b = P[o:o + 128]
        o += 128
        h = torch.nn.functional.silu(torch.nn.functional.linear(h, W, b))
    yt = h @ P[o:o + 128] + P[o + 128]
    lt = torch.mean((yt - torch.tensor(t)) ** 2)
    lt.backward()
    assert abs(loss - lt.item()) < 1e-13 * max(1.0, abs(loss))
    np.testing.assert_allclose(g, P.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_rounded_loss_close_to_unrounded():
    params = _small_params(10)
    rng = np.random.default_rng(11)
    B = rng.standard_normal((64, 3)) * 0.25
    r = rng.uniform(-4, 4, (32, 3))
    y0, _ = M.forward(params, r, B, rounding=False)
    y1, _ = M.forward(params, r, B, rounding=True)
    # BF16 keeps 8 significant bits: the output moves by far less than its scale
    assert np.max(np.abs(y1 - y0)) < 0.05 * (np.max(np.abs(y0)) + 1.0)
    assert np.max(np.abs(y1 - y0)) > 0.0


def test_layer_helpers_chain_to_the_pinned_passes():
    """The per-layer steps (hidden_pre, hidden_act, output, dz_of,
    weight_grad, input_grad) chained together give exactly the forward pass
    and the gradient of loss_and_grads, which the tests above pin against
    torch autograd and central differences; their scales bound the terms."""
    from oracle import mlp_oracle as M
    rng = np.random.default_rng(21)
    p = rng.standard_normal(M.n_params()) * 0.1
    B = rng.standard_normal((64, 3)) * 0.3
    pts = rng.standard_normal((40, 3)) * 2.0
    t = rng.standard_normal(40)
    layers, w_out, b_out = M.unpack(p)
    H = [M.bf16(M.features(pts, B))]
    Z = []
    for W, b in layers:
        z, sc = M.hidden_pre(H[-1], W, b)
        assert np.all(np.abs(z) <= sc * (1 + 1e-12))
        Z.append(z)
        H.append(M.hidden_act(z))
    y, _ = M.output(H[-1], w_out, b_out)
    y_ref, _ = M.forward(p, pts, B, rounding=True)
    assert np.array_equal(y, y_ref)
    dy = 2.0 * (y - t) / len(t)
    dH = np.outer(dy, w_out)
    grads = []
    for l in range(3, -1, -1):
        dz = M.dz_of(dH, Z[l])
        gW, _ = M.weight_grad(M.bf16(dz), H[l])
        grads.append((l, gW, dz.sum(axis=0)))
        if l > 0:
            dH, _ = M.input_grad(M.bf16(dz), layers[l][0])
    _, g_ref = M.loss_and_grads(p, pts, t, B, rounding=True)
    for l, gW, gb in grads:
        o = l * (128 * 128 + 128)
        assert np.allclose(g_ref[o:o + 128 * 128], gW.ravel(), rtol=1e-12, atol=1e-15)
        assert np.allclose(g_ref[o + 128 * 128:o + 128 * 128 + 128], gb, rtol=1e-12, atol=1e-15)
