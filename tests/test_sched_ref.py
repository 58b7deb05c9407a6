"""Pins of the CPU reference for the learned schedule (no GPU).

The float64 network reference is checked against quantities it does not
compute itself: finite differences of its own loss, PyTorch autograd of the
same network, PyTorch's bfloat16 rounding and Adam, and features of
constructed queries whose values follow by hand.
"""
import math

import numpy as np
import pytest
import torch

from oracle import sched_ref as R


def _net(seed, n=200):
    rng = np.random.Generator(np.random.PCG64(seed))
    params = R.quantized(rng.normal(0.0, 0.3, R.N_PARAMS).astype(np.float32))
    feat = rng.normal(0.0, 2.0, (n, R.NF)).astype(np.float32)
    norm = np.concatenate([rng.normal(0.0, 0.5, R.NF), rng.uniform(0.5, 1.5, R.NF)]).astype(np.float32)
    label = rng.normal(0.0, 1.0, n)
    return params, R.normalize(feat, norm), label


def test_bf16_rounding_matches_torch():
    rng = np.random.Generator(np.random.PCG64(1))
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-30, 1000), rng.normal(0, 1e30, 1000)])
    x = x.astype(np.float32)
    # exact ties: the low 16 bits are 0x8000, with both parities of bit 16
    ties = (np.arange(1, 2001, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties, -ties, np.float32([0.0, -0.0])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(R.bf16(x), ref)


def test_quantized_rounds_only_the_weight_matrices():
    p = np.full(R.N_PARAMS, 1.0 + 2.0 ** -12, np.float32)
    q = R.unpack(R.quantized(p))
    assert np.all(q["W1"] == 1.0) and np.all(q["W2"] == 1.0)
    for k in ("b1", "b2", "w3", "b3"):
        assert np.all(q[k] == np.float32(1.0 + 2.0 ** -12))


def _pattern(params, x):
    p = R.unpack(params)
    z1 = x @ p["W1"] + p["b1"]
    z2 = np.maximum(z1, 0) @ p["W2"] + p["b2"]
    return z1 > 0, z2 > 0


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    params, x, label = _net(seed)
    g = R.grad(params, x, label)
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    idx = rng.choice(R.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [R.N_PARAMS - 1]])  # b3
    for i in idx:
        # Along one parameter the loss is piecewise quadratic, with kinks where a unit's activation flips.
        # A central difference over an interval without a kink is exact up to rounding, so shrink the step
        # until the activation pattern is the same at both ends.
        h = 1e-2
        while True:
            pp, pm = params.copy(), params.copy()
            pp[i] += h
            pm[i] -= h
            if all(np.array_equal(a, b) for a, b in zip(_pattern(pp, x), _pattern(pm, x))):
                break
            h /= 4
        fd = (R.loss(pp, x, label) - R.loss(pm, x, label)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, h, fd, g[i])


def test_forward_and_gradient_match_autograd():
    params, x, label = _net(2, n=333)
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in R.unpack(params).items()}
    X = torch.tensor(x, dtype=torch.float64)
    y = torch.relu(torch.relu(X @ p["W1"] + p["b1"]) @ p["W2"] + p["b2"]) @ p["w3"] + p["b3"][0]
    np.testing.assert_allclose(R.forward(params, x), y.detach().numpy(), rtol=1e-12, atol=1e-12)
    loss = torch.mean((y - torch.tensor(label)) ** 2)
    loss.backward()
    ref = np.concatenate([p[k].grad.numpy().ravel() for k, _ in R.SIZES])
    np.testing.assert_allclose(R.grad(params, x, label), ref, rtol=1e-10, atol=1e-13)
    assert abs(R.loss(params, x, label) - loss.item()) <= 1e-12 * loss.item()


def test_forward_special_case_by_hand():
    # one active path: x0 -> hidden 0 -> hidden 0 -> output, all weights 1/2, biases 1/4
    d = {k: np.zeros(s) for k, s in R.SIZES}
    d["W1"][0, 0] = 0.5
    d["W2"][0, 0] = 0.5
    d["w3"][0] = 0.5
    d["b1"][0] = d["b2"][0] = 0.25
    d["b3"][0] = 0.25
    params = R.pack(d)
    x = np.zeros((3, R.NF))
    x[:, 0] = [2.0, -2.0, 0.0]
    # x0 = 2: z1 = 1.25, z2 = 0.875, y = 0.6875; x0 = -2: z1 < 0, z2 = 0.25, y = 0.375
    np.testing.assert_array_equal(R.forward(params, x), [0.6875, 0.375, 0.25 + 0.5 * (0.25 + 0.5 * 0.25)])


def test_adam_matches_torch():
    rng = np.random.Generator(np.random.PCG64(3))
    p0 = rng.normal(0, 1, 50)
    grads = [rng.normal(0, 1, 50) for _ in range(5)]
    w = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-2, betas=(0.9, 0.99), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step, g in enumerate(grads, 1):
        w.grad = torch.tensor(g)
        opt.step()
        p, m, v = R.adam(p, g, m, v, step, 1e-2, 0.9, 0.99, 1e-8)
    np.testing.assert_allclose(p, w.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_features_vf_head_on_by_hand():
    # static triangle (0,0,0), (1,0,0), (0,1,0); vertex from (1/4, 1/4, h) to (1/4, 1/4, h - s)
    h, s, delta = 0.25, 1.0, 1e-6
    q = np.array([[0.25, 0.25, h], [0, 0, 0], [1, 0, 0], [0, 1, 0],
                  [0.25, 0.25, h - s], [0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float64).ravel()
    f = R.features(0, q, delta)
    lr = lambda x: np.float32(math.log2(1 + x / delta))
    assert f[0] == 0
    assert f[4] == lr(s) and f[5] == lr(1.0) and f[6] == lr(1.0)
    # F = p - a - u (b - a) - v (c - a) = (1/4 - u, 1/4 - v, h - s t): every side of the root box meets 0
    e = np.max(np.abs(R._eps(0, q)))
    assert f[10] == 3
    assert f[7] == -lr(0.25 + e) or abs(f[7] + lr(0.25)) < 1e-6
    assert f[8] == lr(min(1.0, s)) and f[9] == lr(max(1.0, s))
    c = 0.25 - 1.0 / 3.0
    n0, n1 = math.sqrt(2 * c * c + h * h), math.sqrt(2 * c * c + (h - s) ** 2)
    assert abs(f[11] - lr(n0)) < 1e-5 and abs(f[12] - lr(n1)) < 1e-5
    assert abs(f[13] - lr(math.sqrt(2 * c * c + (h - s / 2) ** 2))) < 1e-5
    assert f[14] == 1  # only z changes sign
    assert abs(f[15] - (2 * c * c + h * (h - s)) / (n0 * n1)) < 1e-6


def test_features_ee_crossing_by_hand():
    # edge along x at height z = h moving down by s; static edge along y at z = 0
    h, s, delta = 0.5, 1.0, 1e-6
    q = np.array([[-1, 0, h], [1, 0, h], [0, -1, 0], [0, 1, 0],
                  [-1, 0, h - s], [1, 0, h - s], [0, -1, 0], [0, 1, 0]], np.float64).ravel()
    f = R.features(1, q, delta)
    lr = lambda x: np.float32(math.log2(1 + x / delta))
    assert f[0] == 1
    assert f[4] == lr(s)            # max(|d0|, |d1|) + max(|d2|, |d3|) = s + 0
    assert f[5] == lr(2.0) and f[6] == lr(2.0)
    # F = a0 + u (a1 - a0) - b0 - v (b1 - b0) = (2u - 1, 1 - 2v, h - s t); at the centre (0, 0, h - s t)
    assert f[10] == 3
    assert f[11] == lr(h) and f[12] == lr(abs(h - s)) and f[13] == lr(0.0)
    assert f[14] == 1
    assert f[15] == -1.0
    # sides of the root box: 2, 2 and s
    assert f[8] == lr(min(2.0, s)) and f[9] == lr(2.0)


def test_features_separated_pair_has_positive_gap():
    # vertex far above a static triangle, moving parallel to it: every corner of F_z is >= 5
    q = np.array([[0.2, 0.2, 5.0], [0, 0, 0], [1, 0, 0], [0, 1, 0],
                  [0.3, 0.2, 5.0], [0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float64).ravel()
    f = R.features(0, q, 1e-6)
    assert f[7] > 0 and abs(f[7] - np.float32(math.log2(1 + 5.0 / 1e-6))) < 1e-4
    assert f[10] == 2 and f[14] == 0 and f[15] > 0.99
