"""Pins of the warm-start network oracle: bfloat16 rounding against torch's own
conversion, the backward pass against finite differences, Adam against torch.optim."""
import numpy as np
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def _small_problem(seed=0):
    rng = np.random.default_rng(seed)
    params = mlp.init_params(rng, n_in=12, n_hidden=8, n_out=5)
    params[4] = rng.standard_normal(params[4].shape) * 0.3     # non-zero last layer
    params[1] = rng.standard_normal(8) * 0.1
    x = rng.standard_normal((7, 12))
    y = rng.standard_normal((7, 5))
    return params, x, y


def test_backward_matches_finite_differences():
    """with unrounded activations the loss is smooth in the biases: finite differences
    pin the backward formulas; the rounded (straight-through) variant is pinned against
    torch autograd below"""
    params, x, y = _small_problem()
    loss, grads = mlp.loss_and_grad(params, x, y, round_hidden=False)
    # differentiate w.r.t. the bf16-rounded weights: perturb biases (fp64) exactly,
    # and weights through a copy that bypasses the rounding by using exact bf16 steps
    h = 1e-6
    for k in (1, 3, 5):
        p = params[k]
        for idx in [(0,), (p.size - 1,)]:
            pp = [q.copy() for q in params]
            pm = [q.copy() for q in params]
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (mlp.loss_and_grad(pp, x, y, round_hidden=False)[0]
                  - mlp.loss_and_grad(pm, x, y, round_hidden=False)[0]) / (2 * h)
            assert abs(fd - grads[k][idx]) < 1e-7 * (1 + abs(fd))
    # weights: rounded weights are piecewise constant in the raw weight, so check the
    # gradient against a torch autograd evaluation on the rounded values
    tp = [torch.tensor(mlp.bf16_round(q) if i % 2 == 0 else q, requires_grad=True) for i, q in enumerate(params)]
    xt = torch.tensor(mlp.bf16_round(x))

    def rnd(h):   # bfloat16 rounding, identity in the backward pass
        return h + (h.to(torch.bfloat16).to(torch.float64) - h).detach()

    h1 = rnd(torch.relu(xt @ tp[0].T + tp[1]))
    h2 = rnd(torch.relu(h1 @ tp[2].T + tp[3]))
    out = h2 @ tp[4].T + tp[5]
    lt = ((out - torch.tensor(y)) ** 2).mean()
    lt.backward()
    loss, grads = mlp.loss_and_grad(params, x, y)
    assert abs(lt.item() - loss) < 1e-12
    for i in range(6):
        assert np.allclose(tp[i].grad.numpy(), grads[i], rtol=1e-10, atol=1e-13)


def test_adam_matches_torch():
    params, x, y = _small_problem(1)
    tp = [torch.tensor(q.copy(), requires_grad=True) for q in params]
    opt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = [np.zeros_like(q) for q in params]
    v = [np.zeros_like(q) for q in params]
    p = [q.copy() for q in params]
    rng = np.random.default_rng(5)
    for step in range(1, 4):
        grads = [rng.standard_normal(q.shape) for q in params]
        p, m, v = mlp.adam_step(p, grads, m, v, step, 1e-2)
        for t, g in zip(tp, grads):
            t.grad = torch.tensor(g)
        opt.step()
    for a, t in zip(p, tp):
        assert np.allclose(a, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def _forward_f32(params, x, order):
    """the network evaluated with FP32 accumulation (products of bf16 values are exact
    in FP32), summing the K products in the given order of chunks"""
    W1, b1, W2, b2, W3, b3 = [mlp.bf16_round(p) if i % 2 == 0 else p for i, p in enumerate(params)]

    def pre(a, W, b):
        a32, W32 = a.astype(np.float32), W.astype(np.float32)
        z = np.zeros((a.shape[0], W.shape[0]), np.float32)
        for sl in order(a.shape[1]):
            z = z + a32[:, sl] @ W32[:, sl].T
        return (z + b.astype(np.float32)).astype(np.float64)
    x = mlp.bf16_round(x)
    h1 = mlp.bf16_round(np.maximum(pre(x, W1, b1), 0.0))
    h2 = mlp.bf16_round(np.maximum(pre(h1, W2, b2), 0.0))
    return pre(h2, W3, b3)


def test_fp32_accumulation_stays_within_the_flip_bound():
    """FP32 evaluations in two summation orders (whole rows; 8-wide chunks summed in
    reverse) differ from the FP64 oracle only where the bound of tests/mlp_bound.py
    admits one-step bf16 flips of ambiguous hidden activations (about one first-layer
    activation in a hundred is ambiguous; a flip there widens the second layer's
    intervals)"""
    from mlp_bound import flip_bound
    rng = np.random.default_rng(3)
    params = mlp.init_params(rng, n_in=968, n_out=96)
    params[3] = rng.standard_normal(128) * 0.1
    params[4] = rng.standard_normal(params[4].shape) * 0.05
    x = rng.standard_normal((129, 968))
    y64, _ = mlp.forward(params, x)
    bound, n_amb = flip_bound(params, x)
    assert 0 < n_amb <= 0.02 * 129 * 128
    tol = 1e-5 * np.max(np.abs(y64)) + bound
    for order in (lambda K: [slice(0, K)], lambda K: [slice(i, min(i + 8, K)) for i in range(0, K, 8)][::-1]):
        y32 = _forward_f32(params, x, order)
        assert np.all(np.abs(y32 - y64) <= tol)
    # a bound that ignored the flips would not hold in general: the rows the bound singles
    # out are the only ones allowed to move by more than the FP32 floor
    moved = np.abs(_forward_f32(params, x, lambda K: [slice(0, K)]) - y64) > 1e-5 * np.max(np.abs(y64))
    assert not np.any(moved & (bound == 0))
