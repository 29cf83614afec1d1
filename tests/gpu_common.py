"""Helpers for the GPU parity tests: build oracle meshes and library meshes from
the same synthetic workload, and compare."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).ravel()).to(dev())


def shell_pair(w, n_ang, n_rad, p):
    from oracle import mesh as omesh
    from paper_2306_01085_amd import Mesh
    om = omesh.shell_mesh(p, n_ang, n_rad, w.r_bot, w.r_top, w.stretch)
    gm = Mesh.shell(p=p, n_ang=n_ang, n_rad=n_rad, r_bot=w.r_bot, r_top=w.r_top, stretch=w.stretch, phys=w.phys)
    return om, gm


def rel_to_scale(a, b, scale):
    return float(np.max(np.abs(a - b)) / np.max(scale))
