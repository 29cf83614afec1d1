"""Parity of the EUVAC heating (section 2.2, Table A) on the GPU with the oracle: R(u)
and J(u)v on a shell that holds day-side, night-side and shadowed nodes (sub-solar
latitude from the June-solstice declination), on uneven columns, and one implicit
column step. The heating is state dependent (density and scale height), so it enters
J v through the Chapman factor and the optical depths."""
import dataclasses

import numpy as np
import pytest

import synth
from gpu_common import need_gpu, rel_to_scale, shell_pair, to_dev, torch
from oracle import dg as odg
from oracle import jac as ojac
from oracle import mesh as omesh
from oracle import timeint

pytestmark = pytest.mark.gpu


def _euvac(phys, day=172.0):
    P = dict(phys)
    P.update(synth.euvac_physics(f107bar=150.0, day=day))
    P["heating_model"] = 1
    P["heat_amp"] = 0.0
    return P


@pytest.mark.parametrize("p,n_ang,n_rad", [(3, 2, 3), (2, 2, 2), (4, 1, 2)])
def test_shell_residual_and_jvp_with_euvac(p, n_ang, n_rad):
    need_gpu()
    w = synth.shell_workload(20 + p, p=p, n_ang=n_ang, n_rad=n_rad)
    w = dataclasses.replace(w, phys=_euvac(w.phys))
    om, gm = shell_pair(w, n_ang, n_rad, p)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    t = 0.37
    R, scale = odg.residual_parts(om, w.phys, u, t)
    r = gm.residual(to_dev(u), t=t).cpu().numpy().reshape(u.shape)
    assert rel_to_scale(r, R, scale) < 1e-12
    v = synth.tangent(u.shape, 5)
    ref, lscale = ojac.jvp_parts(om, w.phys, u, v, t)
    jv = gm.jvp(to_dev(u), to_dev(v), t=t).cpu().numpy().reshape(u.shape)
    assert np.linalg.norm(jv - ref) / np.linalg.norm(ref) < 1e-12
    assert rel_to_scale(jv, ref, lscale) < 1e-12
    jv32 = gm.jvp(to_dev(u), to_dev(v).float(), t=t, prec="f32").cpu().double().numpy().reshape(u.shape)
    assert np.linalg.norm(jv32 - ref) / np.linalg.norm(ref) < 1e-5


def test_euvac_heating_is_present():
    """the energy rows of R differ from the unheated residual by the oracle's heating
    source, on the day side only (a check that the term is switched on, not a parity)"""
    need_gpu()
    w = synth.shell_workload(31, p=2, n_ang=2, n_rad=2, heating=False)
    we = dataclasses.replace(w, phys=_euvac(w.phys))
    om, gm0 = shell_pair(w, 2, 2, 2)
    _, gme = shell_pair(we, 2, 2, 2)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    d = (gme.residual(to_dev(u), t=0.0) - gm0.residual(to_dev(u), t=0.0)).cpu().numpy().reshape(u.shape)
    assert np.max(np.abs(d[:, :4])) == 0.0
    assert np.max(d[:, 4]) > 0 and np.min(d[:, 4]) >= 0


def test_columns_with_euvac():
    need_gpu()
    from paper_2306_01085_amd import Mesh
    nelem, p, stretch = [6, 13, 24], [2, 3, 4], 1.1
    w = synth.column_batch_workload(3, n_col=len(nelem))
    phys = _euvac(w.phys)
    col_phys = dict(w.col_phys)
    col_phys["heat_amp"] = np.zeros(len(nelem))
    gm = Mesh.columns(np.asarray(nelem, np.int32), np.asarray(p, np.int32), w.r_bot, w.r_top, stretch, phys,
                      col_phys)
    off = gm.col_offsets()
    cols = []
    for c in range(len(nelem)):
        om = omesh.columns_mesh([nelem[c]], p[c], w.r_bot, w.r_top, stretch)
        P = dict(phys)
        for k in col_phys:
            P[k] = float(col_phys[k][c])
        cols.append((om, P, np.moveaxis(w.state(c, om.X[:, :, 0]), 0, 1).copy()))
    u = np.concatenate([c[2].ravel() for c in cols])
    v = synth.tangent(u.shape, 4)
    r = gm.residual(to_dev(u), t=0.1).cpu().numpy()
    jv = gm.jvp(to_dev(u), to_dev(v), t=0.1).cpu().numpy()
    for c, (om, P, uc) in enumerate(cols):
        R, scale = odg.residual_parts(om, P, uc, 0.1)
        assert rel_to_scale(r[off[c]:off[c + 1]].reshape(uc.shape), R, scale) < 1e-12, c
        ref = ojac.jvp_complex(om, P, uc, v[off[c]:off[c + 1]].reshape(uc.shape), 0.1)
        jc = jv[off[c]:off[c + 1]].reshape(uc.shape)
        assert np.linalg.norm(jc - ref) / np.linalg.norm(ref) < 1e-12, c


def test_implicit_column_step_with_euvac():
    need_gpu()
    from paper_2306_01085_amd import Mesh
    w = synth.config_column(5)
    phys = _euvac(w.phys)
    col_phys = dict(w.col_phys)
    col_phys["heat_amp"] = np.zeros(1)
    om = omesh.columns_mesh([8], 2, w.r_bot, w.r_top)
    gm = Mesh.columns([8], [2], w.r_bot, w.r_top, 1.0, phys, col_phys)
    u = np.moveaxis(w.state(0, om.X[:, :, 0]), 0, 1).copy()
    ref, _ = timeint.implicit_step_dense(om, phys, u, 0.0, w.dt, scheme=33, rtol=1e-13)
    ut = to_dev(u)
    gm.implicit_step(ut, 0.0, w.dt, newton_rtol=1e-10, gmres_rtol=1e-6, precond=0)
    out = ut.cpu().numpy().reshape(u.shape)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref - u) < 1e-6
