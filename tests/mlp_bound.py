"""How far a correct FP32-accumulating evaluation of the warm-start network may sit from
the FP64 oracle.

The network rounds its hidden activations to bf16 after each product. A kernel that
accumulates in FP32 forms a pre-activation z that differs from the exact one by the
rounding of its running sums: for a chain of 8-product steps (the matrix-core step of
the kernel; the products of bf16 values are exact in FP32) at most 2^-24 times the sum of
the magnitudes of the partial sums, taken here with a factor 4 for other orders and
groupings, plus the rounding of the bias addition. Where [z - delta, z + delta]
straddles a bf16 rounding boundary (or the ReLU kink) the rounded activation may differ
from the oracle's by one bf16 step; elsewhere it must round the same way. (The
order-free worst case, K 2^-24 sum |a_i w_i|, would call about a third of all
activations ambiguous and bound nothing.) flip_bound
propagates those admissible one-step differences through the following layers (a flip in
the first hidden layer widens the second layer's interval by |W2| times its size) and
returns a per-output bound on |y_kernel - y_oracle| beyond FP32 rounding of the output
layer itself. Rows without an ambiguous activation get a zero bound.
"""
import numpy as np

from oracle import mlp

U32 = 2.0 ** -24


def _chain_error(a, W):
    """2^-24 sum_k |S_k| over the running sums S_k of 8-product steps, per (row, unit)"""
    K = a.shape[1]
    out = np.zeros((a.shape[0], W.shape[0]))
    acc = np.zeros_like(out)
    for k in range(0, K, 8):
        acc = acc + a[:, k:k + 8] @ W[:, k:k + 8].T
        out += np.abs(acc)
    return U32 * out


def _layer(a, W, b, widen=None):
    """(rounded activation, admissible deviation of it) for one hidden layer"""
    z = a @ W.T + b
    delta = 4.0 * _chain_error(a, W) + U32 * (np.abs(b) + np.abs(z))
    if widen is not None:
        delta = delta + widen
    lo = mlp.bf16_round(np.maximum(z - delta, 0.0))
    hi = mlp.bf16_round(np.maximum(z + delta, 0.0))
    h = mlp.bf16_round(np.maximum(z, 0.0))
    return h, hi - lo


def flip_bound(params, x):
    W1, b1, W2, b2, W3, b3 = [mlp.bf16_round(p) if i % 2 == 0 else p for i, p in enumerate(params)]
    xr = mlp.bf16_round(np.asarray(x, np.float64))
    h1, d1 = _layer(xr, W1, b1)
    h2, d2 = _layer(h1, W2, b2, widen=d1 @ np.abs(W2).T)
    return d2 @ np.abs(W3).T, int((d1 > 0).sum())
