"""dg_residual_noalloc (R(u) with the face traces in the library's per-GPU scratch array)
against dg_residual, its allocating counterpart, and the oracle: bitwise the same result on
shells and columns, on two calls in a row with the second on a smaller mesh, and a mesh
whose traces exceed the scratch array is refused before any device work."""
import numpy as np
import pytest

import synth
from gpu_common import need_gpu, rel_to_scale, shell_pair, to_dev, torch
from oracle import dg as odg
from oracle import mesh as omesh

pytestmark = pytest.mark.gpu


def _shell_case(seed, p, n_ang, n_rad):
    w = synth.shell_workload(seed, p=p, n_ang=n_ang, n_rad=n_rad)
    om, gm = shell_pair(w, n_ang, n_rad, p)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    u += 1e-3 * np.random.default_rng(seed).standard_normal(u.shape)
    return w.phys, om, gm, u


def _column_case(seed, nelem, p):
    from paper_2306_01085_amd import Mesh
    w = synth.column_batch_workload(seed, n_col=len(nelem))
    w.nelem = np.asarray(nelem, np.int32)
    w.p = np.asarray(p, np.int32)
    w.stretch = np.full(len(nelem), 1.1)
    gm = Mesh.columns(w.nelem, w.p, w.r_bot, w.r_top, w.stretch, w.phys, w.col_phys)
    parts = []
    for c in range(len(nelem)):
        om = omesh.columns_mesh([int(nelem[c])], int(p[c]), w.r_bot, w.r_top, 1.1)
        P = dict(w.phys)
        for k in w.col_phys:
            P[k] = float(w.col_phys[k][c])
        parts.append((om, P, np.moveaxis(w.state(c, om.X[:, :, 0]), 0, 1).copy()))
    return gm, parts


def test_noalloc_residual_matches_dg_residual_on_shells():
    need_gpu()
    t = 0.41
    for seed, p, n_ang, n_rad in [(1, 3, 2, 4), (2, 3, 1, 2)]:          # the second call is smaller
        print("noalloc shell case", seed, p, n_ang, n_rad, flush=True)
        phys, om, gm, u = _shell_case(seed, p, n_ang, n_rad)
        ud = to_dev(u)
        ref = gm.residual(ud, t=t)
        out = torch.full_like(ud, float("nan"))
        gm.residual_noalloc(ud, out, t=t)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        R, scale = odg.residual_parts(om, phys, u, t)
        assert rel_to_scale(out.cpu().numpy().reshape(u.shape), R, scale) < 1e-12


def test_noalloc_residual_matches_dg_residual_on_columns():
    need_gpu()
    for seed, nelem, p in [(3, [6, 9, 4], [2, 4, 3]), (4, [3, 5], [3, 2])]:
        print("noalloc column case", seed, nelem, p, flush=True)
        gm, parts = _column_case(seed, nelem, p)
        u0 = np.concatenate([c[2].ravel() for c in parts])
        ud = to_dev(u0)
        ref = gm.residual(ud, t=0.0)
        out = torch.full_like(ud, float("nan"))
        gm.residual_noalloc(ud, out, t=0.0)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        off = gm.col_offsets()
        got = out.cpu().numpy()
        for c, (om, P, u) in enumerate(parts):
            R, scale = odg.residual_parts(om, P, u, 0.0)
            assert rel_to_scale(got[off[c]:off[c + 1]].reshape(u.shape), R, scale) < 1e-12


def test_noalloc_residual_refuses_meshes_beyond_the_scratch():
    """6 x 17 x 17 x 16 at p = 3: 27,744 elements, 106.5 MB of traces > 96 MiB"""
    need_gpu()
    from paper_2306_01085_amd import DG_ERR_ARG, DgError, Mesh
    w = synth.shell_workload(0, p=3, n_ang=17, n_rad=16)
    gm = Mesh.shell(p=3, n_ang=17, n_rad=16, r_bot=w.r_bot, r_top=w.r_top, stretch=w.stretch, phys=w.phys)
    u = torch.zeros(gm.n_dof, dtype=torch.float64, device="cuda")
    out = torch.zeros_like(u)
    with pytest.raises(DgError) as ei:
        gm.residual_noalloc(u, out)
    assert ei.value.code == DG_ERR_ARG and "scratch" in str(ei.value)
