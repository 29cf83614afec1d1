"""The warm-start network on the GPU against the FP64 oracle (same bf16 rounding
contract): forward outputs and loss gradients to 1e-5 relative, one Adam step to
1e-6; and the learned guess inside the implicit step changes the cost of Newton,
never the converged answer."""
import numpy as np
import pytest

import synth
from gpu_common import need_gpu, shell_pair, to_dev, torch
from mlp_bound import flip_bound
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _problem(seed=0, n=150, n_in=960, n_out=320):
    rng = np.random.default_rng(seed)
    params = omlp.init_params(rng, n_in=n_in, n_out=n_out)
    params[4] = rng.standard_normal(params[4].shape) * 0.05
    params[1] = rng.standard_normal(128) * 0.1
    params[3] = rng.standard_normal(128) * 0.1
    params[5] = rng.standard_normal(n_out) * 0.1
    params = [p.astype(np.float32).astype(np.float64) for p in params]
    x = rng.standard_normal((n, n_in)).astype(np.float32)
    t = rng.standard_normal((n, n_out)).astype(np.float32)
    return params, x, t


def test_mlp_forward_and_gradients_match_oracle():
    need_gpu()
    from paper_2306_01085_amd import Network
    params, x, t = _problem(0)
    net = Network(960, 320, params)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    y = net.forward(xd).cpu().numpy()
    yref, _ = omlp.forward(params, x.astype(np.float64))
    assert _rel(y, yref) < 1e-5
    loss, grads = net.grad(xd, td, want_grads=True)
    lref, gref = omlp.loss_and_grad(params, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss / lref - 1) < 1e-5
    for g, gr in zip(grads, gref):
        assert _rel(g, gr) < 1e-5


@pytest.mark.parametrize("n,n_in,n_out", [(70, 200, 64), (1, 8, 32), (129, 968, 96)])
def test_mlp_forward_ragged_shapes(n, n_in, n_out):
    """row counts off the 64-row block, input widths with a partial last 64-column chunk,
    against the FP64 oracle: every output within 1e-5 of the output scale plus the
    admissible effect of one-step bf16 flips of hidden activations that lie within FP32
    accumulation error of a rounding boundary (tests/mlp_bound.py; one activation of the
    129 x 968 case is such a one)"""
    need_gpu()
    from paper_2306_01085_amd import DgError, Network
    params, x, _ = _problem(3, n=n, n_in=n_in, n_out=n_out)
    net = Network(n_in, n_out, params)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    yref, _ = omlp.forward(params, x.astype(np.float64))
    bound, _ = flip_bound(params, x.astype(np.float64))
    assert np.all(np.abs(y - yref) <= 1e-5 * np.max(np.abs(yref)) + bound)
    # an input that is not 16-byte aligned is refused
    xd = torch.from_numpy(np.concatenate([[0.0], x.ravel()]).astype(np.float32)).cuda()[1:].view(n, n_in)
    with pytest.raises(DgError):
        net.forward(xd)


def test_mlp_adam_step_matches_oracle():
    need_gpu()
    from paper_2306_01085_amd import Network
    params, x, t = _problem(1, n=64)
    net = Network(960, 320, params)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    _, g = net.grad(xd, td, want_grads=True)
    net.adam_step(1e-3)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    ref, _, _ = omlp.adam_step(params, [gi.astype(np.float64) for gi in g], m, v, 1, 1e-3)
    for a, b in zip(net.params(), ref):
        assert np.max(np.abs(a - b)) <= 1e-6 * max(1.0, np.max(np.abs(b)))


def test_learned_guess_keeps_the_answer():
    """record stages on a small shell, train briefly, then the same steps with the
    plain and the learned guess converge to the same states"""
    need_gpu()
    from paper_2306_01085_amd import Network
    from paper_2306_01085_amd import warmstart as ws
    w = synth.shell_workload(4, p=3, n_ang=2, n_rad=16)
    om, gm = shell_pair(w, 2, 16, 3)
    u = to_dev(np.moveaxis(w.state_fn()(om.X), 0, 1).copy())
    dt = synth.seconds_to_nondim(30.0)
    opts = dict(newton_rtol=1e-10, gmres_rtol=1e-6, precond=0)
    X, Y, rows, _ = ws.record(gm, u, 0.0, dt, 4, every=1, capacity=10 * gm.n_elem, **opts)
    assert rows == 4 * 3 * gm.n_elem - 2 * gm.n_elem  # no pairs before two stage solutions exist
    norms = ws.standardise(X, Y, rows)
    net = Network(960, 320, ws.init_params(np.random.default_rng(0), 960, 320))
    tr, va = ws.train(net, X, Y, rows, epochs=20, batch=256, lr=1e-3)
    assert tr[-1] < tr[0]
    gm.warmstart_set(net, *norms)
    sp, sl, up, ul = ws.compare(gm, u, 4 * dt, dt, 2, **opts)
    change = torch.linalg.norm(up - u).item()
    assert torch.linalg.norm(up - ul).item() < 1e-6 * change
    assert all(f in (0, 1) for s in sl for f in s["fallback"])
