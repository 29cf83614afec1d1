"""Properties of J(u)v that hold at any size, checked on the benchmark shell at full size
(6x16x16x16, p = 3, 7.9M DOF) in the launch configuration the benchmark uses: the
directional derivative is linear in v, and the dual-number arithmetic makes that exact for
a power-of-two scale (every operation on the derivative parts is linear, and scaling by 2
commutes with rounding), J(u) 0 = 0 exactly, and J(u)(v1 + v2) = J(u)v1 + J(u)v2 to
rounding. FP64, FP32 and the BF16-MFMA product (whose bf16 operand rounding also commutes
with the scale)."""
import numpy as np
import pytest

import synth
from gpu_common import need_gpu, to_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shell():
    need_gpu()
    from paper_2306_01085_amd import Mesh
    from paper_2306_01085_amd import autotune
    w = synth.config_shell_p3(0)
    gm = Mesh.shell(p=w.p, n_ang=w.n_ang, n_rad=w.n_rad, r_bot=w.r_bot, r_top=w.r_top, stretch=w.stretch,
                    phys=w.phys)
    X = gm.nodes().reshape(w.n_elem, -1, 3)
    u = to_dev(synth.shell_state_at(w, X))
    autotune.tune_shell_pass1(gm, u)
    g = torch.Generator(device="cuda").manual_seed(5)
    v1 = torch.randn(gm.n_dof, dtype=torch.float64, device="cuda", generator=g)
    v2 = torch.randn(gm.n_dof, dtype=torch.float64, device="cuda", generator=g)
    v1 /= torch.linalg.norm(v1)
    v2 /= torch.linalg.norm(v2)
    return gm, u, v1, v2


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_power_of_two_scaling_is_exact(shell, prec):
    gm, u, v1, _ = shell
    v = v1 if prec == "f64" else v1.float()
    a = gm.jvp(u, v, t=0.2, prec=prec)
    b = gm.jvp(u, 2 * v, t=0.2, prec=prec)
    assert torch.equal(b, 2 * a)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_zero_direction_gives_zero(shell, prec):
    gm, u, v1, _ = shell
    z = torch.zeros_like(v1 if prec == "f64" else v1.float())
    out = gm.jvp(u, z, t=0.2, prec=prec)
    assert torch.count_nonzero(out).item() == 0


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_additivity(shell, prec, tol):
    gm, u, v1, v2 = shell
    c = (lambda x: x) if prec == "f64" else (lambda x: x.float())
    j1 = gm.jvp(u, c(v1), t=0.2, prec=prec).double()
    j2 = gm.jvp(u, c(v2), t=0.2, prec=prec).double()
    j12 = gm.jvp(u, c(v1) + c(v2), t=0.2, prec=prec).double()
    assert (torch.linalg.norm(j12 - j1 - j2) / torch.linalg.norm(j12)).item() < tol
