"""Learned Newton warm start: recording method-generated stages, training the
per-element network on the GPU, and comparing the learned guess with the plain
extrapolated one. A workflow over the library's kernels: the stages come from
dg_implicit_step, the training from dg_mlp_grad / dg_mlp_adam_step, the inference
from the guess path of dg_implicit_step.
"""
from __future__ import annotations

import numpy as np

from . import Network, affine_rows


def init_params(rng, n_in, n_out, hidden=128):
    """He-scaled hidden layers, zero output layer: the untrained network returns the
    plain guess unchanged"""
    return [rng.standard_normal((hidden, n_in)) * np.sqrt(2.0 / n_in), np.zeros(hidden),
            rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden), np.zeros(hidden),
            np.zeros((n_out, hidden)), np.zeros(n_out)]


def record(mesh, u, t0, dt, n_steps, every, capacity, log=None, **opts):
    """run n_steps implicit steps from (u, t0) recording one element in `every` per
    converged stage; returns (X, Y, rows, per-step stats); u is advanced in place"""
    import torch
    N = mesh.n_dof // (mesh.n_fields * mesh.n_elem)
    X = torch.empty((capacity, 15 * N), dtype=torch.float32, device=u.device)
    Y = torch.empty((capacity, 5 * N), dtype=torch.float32, device=u.device)
    mesh.warmstart_record(X, Y, capacity, every)
    stats = []
    t = t0
    for k in range(n_steps):
        stats.append(mesh.implicit_step(u, t, dt, **opts))
        t += dt
        if log and (k + 1) % 25 == 0:
            win = stats[-25:]
            log("recorded %d of %d steps: Newton %.1f (max %d), GMRES %.1f per step" % (
                k + 1, n_steps, np.mean([sum(s["newton_its"]) for s in win]),
                max(max(s["newton_its"]) for s in win), np.mean([sum(s["gmres_its"]) for s in win])))
    rows = mesh.warmstart_recorded()
    mesh.warmstart_record(None, None, 0, 1)
    return X, Y, rows, stats


def standardise(X, Y, rows, sample=200000, rng=None):
    """per-column mean and scale from up to `sample` recorded rows (host), applied in
    place on the device (dg_affine_rows); returns (x_mean, x_scale, y_mean, y_scale)"""
    rng = rng or np.random.default_rng(0)
    idx = np.sort(rng.choice(rows, size=min(rows, sample), replace=False))
    xs = X[:rows][idx].double().cpu().numpy()
    ys = Y[:rows][idx].double().cpu().numpy()
    xm, xsd = xs.mean(0), xs.std(0)
    ym, ysd = ys.mean(0), ys.std(0)
    xsd = np.where(xsd > 1e-30, xsd, 1.0)
    ysd = np.where(ysd > 1e-30, ysd, 1.0)
    affine_rows(X[:rows], xm, xsd)
    affine_rows(Y[:rows], ym, ysd)
    return xm.astype(np.float32), xsd.astype(np.float32), ym.astype(np.float32), ysd.astype(np.float32)


def train(net: Network, X, Y, rows, epochs=20, batch=4096, lr=1e-3, rng=None, log=None, holdout=0.1):
    """Adam on contiguous mini-batches in a shuffled order; the last `holdout` fraction
    of the rows is kept for validation. Returns (train losses, validation losses)."""
    rng = rng or np.random.default_rng(0)
    n_val = int(rows * holdout)
    n_tr = rows - n_val
    starts = np.arange(0, n_tr, batch)
    tr, va = [], []
    for ep in range(epochs):
        acc = 0.0
        for s in rng.permutation(starts):
            e = min(s + batch, n_tr)
            acc += net.grad(X[s:e], Y[s:e]) * (e - s)
            net.adam_step(lr)
        tr.append(acc / n_tr)
        if n_val:
            va.append(net.grad(X[n_tr:rows], Y[n_tr:rows]))
        if log:
            log("epoch %d train %.4e val %.4e" % (ep, tr[-1], va[-1] if va else float("nan")))
    return tr, va


def compare(mesh, u, t0, dt, n_steps, log=None, **opts):
    """the same n_steps from the same state with the plain and with the learned guess;
    returns (plain stats, learned stats, plain final state, learned final state)"""
    out = {}
    for guess in (0, 1):
        x = u.clone()
        t = t0
        st = []
        for k in range(n_steps):
            st.append(mesh.implicit_step(x, t, dt, guess=guess, **opts))
            t += dt
            if log and (k + 1) % 25 == 0:
                log("%s guess: %d of %d steps" % ("learned" if guess else "plain", k + 1, n_steps))
        out[guess] = (st, x)
    return out[0][0], out[1][0], out[0][1], out[1][1]
