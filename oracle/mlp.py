"""Per-element warm-start network: x (960) -> 128 -> 128 -> out (320), ReLU hidden layers.

Precision contract: weights, the input and both hidden activations are rounded to
bfloat16 (round to nearest even) where they enter a matrix product; biases and all
accumulation are full precision (FP64 here). The backward pass treats the
roundings as the identity (straight-through). Loss: mean squared error over the
batch and outputs.
Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; w -= lr mhat / (sqrt(vhat) + eps)
with the usual bias corrections.
"""
import numpy as np


def bf16_round(x):
    """round float64 -> nearest bfloat16 (ties to even) -> float64"""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, x, round_hidden=True):
    W1, b1, W2, b2, W3, b3 = [bf16_round(p) if i % 2 == 0 else p for i, p in enumerate(params)]
    rh = bf16_round if round_hidden else (lambda a: a)
    x = bf16_round(x)
    z1 = x @ W1.T + b1
    h1 = rh(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + b2
    h2 = rh(np.maximum(z2, 0.0))
    y = h2 @ W3.T + b3
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(params, x, target, round_hidden=True):
    W1, b1, W2, b2, W3, b3 = [bf16_round(p) if i % 2 == 0 else p for i, p in enumerate(params)]
    y, (xr, z1, h1, z2, h2) = forward(params, x, round_hidden)
    n = y.size
    diff = y - target
    loss = np.sum(diff * diff) / n
    dy = 2.0 * diff / n
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = dy @ W3
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ xr
    gb1 = dz1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** step)
        vh = vv / (1 - b2 ** step)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


def init_params(rng, n_in=960, n_hidden=128, n_out=320):
    W1 = rng.standard_normal((n_hidden, n_in)) * np.sqrt(2.0 / n_in)
    W2 = rng.standard_normal((n_hidden, n_hidden)) * np.sqrt(2.0 / n_hidden)
    W3 = np.zeros((n_out, n_hidden))
    return [W1, np.zeros(n_hidden), W2, np.zeros(n_hidden), W3, np.zeros(n_out)]
