"""The paper's own matrix-free product (section 3.2): J v as the one-sided difference
(R(u + h v) - R(u)) / h, h = sqrt(eps) (1 + |u|) / |v|, on the GPU (DG_F64_FD) against the
oracle's difference with the same step and against the exact product (complex step).
The difference's own error is 6e-7 (shell) to 1e-5 (column) of |J v| here (oracle against
oracle); the two R implementations differ by round-off amplified by 1/h, so the bound is
1e-4. Newton-GMRES with this product reaches the same converged step as the oracle's
dense solve."""
import numpy as np
import pytest

import synth
from gpu_common import need_gpu, shell_pair, to_dev, torch
from oracle import jac as ojac
from oracle import mesh as omesh
from oracle import timeint

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_shell_fd_jvp():
    need_gpu()
    w = synth.shell_workload(11, p=3, n_ang=2, n_rad=2)
    om, gm = shell_pair(w, 2, 2, 3)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    v = synth.tangent(u.shape, 4)
    ex = ojac.jvp_complex(om, w.phys, u, v, 0.1)
    fd = ojac.jvp_fd(om, w.phys, u, v, 0.1)
    got = gm.jvp(to_dev(u), to_dev(v), t=0.1, prec="f64_fd").cpu().numpy().reshape(u.shape)
    assert _rel(got, fd) < 1e-4
    assert _rel(got, ex) < 1e-4
    # the mesh's buffers are reused: a second call gives the same numbers
    again = gm.jvp(to_dev(u), to_dev(v), t=0.1, prec="f64_fd").cpu().numpy().reshape(u.shape)
    assert np.array_equal(got, again)


def test_columns_fd_jvp_and_zero_direction():
    need_gpu()
    from paper_2306_01085_amd import Mesh
    w = synth.config_column(3)
    om = omesh.columns_mesh([16], 3, w.r_bot, w.r_top)
    gm = Mesh.columns([16], [3], w.r_bot, w.r_top, 1.0, w.phys, w.col_phys)
    u = np.moveaxis(w.state(0, om.X[:, :, 0]), 0, 1).copy()
    v = synth.tangent(u.shape, 5)
    ex = ojac.jvp_complex(om, w.phys, u, v, 0.0)
    fd = ojac.jvp_fd(om, w.phys, u, v, 0.0)
    got = gm.jvp(to_dev(u), to_dev(v), prec="f64_fd").cpu().numpy().reshape(u.shape)
    assert _rel(got, fd) < 1e-4
    assert _rel(got, ex) < 1e-4
    zero = gm.jvp(to_dev(u), torch.zeros(u.size, dtype=torch.float64, device="cuda"), prec="f64_fd")
    assert torch.count_nonzero(zero).item() == 0


def test_implicit_step_with_fd_jvp():
    need_gpu()
    from paper_2306_01085_amd import Mesh
    w = synth.config_column(2)
    om = omesh.columns_mesh([8], 2, w.r_bot, w.r_top)
    gm = Mesh.columns([8], [2], w.r_bot, w.r_top, 1.0, w.phys, w.col_phys)
    u = np.moveaxis(w.state(0, om.X[:, :, 0]), 0, 1).copy()
    ref, _ = timeint.implicit_step_dense(om, w.phys, u, 0.0, w.dt, scheme=33, rtol=1e-13)
    ut = to_dev(u)
    st = gm.implicit_step(ut, 0.0, w.dt, newton_rtol=1e-10, gmres_rtol=1e-6, jvp_prec="f64_fd", precond=0)
    out = ut.cpu().numpy().reshape(u.shape)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref - u) < 1e-6, st


def test_shell_implicit_step_with_fd_jvp_and_line_preconditioner():
    need_gpu()
    w = synth.shell_workload(3, p=2, n_ang=1, n_rad=2)
    om, gm = shell_pair(w, 1, 2, 2)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    dt = synth.seconds_to_nondim(10.0)
    ref, _ = timeint.implicit_step_jfnk(om, w.phys, u, 0.0, dt, scheme=33, rtol=1e-12)
    ut = to_dev(u)
    st = gm.implicit_step(ut, 0.0, dt, newton_rtol=1e-10, gmres_rtol=1e-6, jvp_prec="f64_fd", precond=2)
    out = ut.cpu().numpy().reshape(u.shape)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref - u) < 1e-6, st
