"""Parity of the variable composition (section 2.1.1: fitted mass fractions of N2, O2 and
He, O the balance; m(r), c_v = 1/m, the mole-fraction conductivity weight, the grad c_v
energy term of eq. fluxSWNondimensional) on the GPU with the oracle: R(u) and J(u)v on
shells (with the prescribed heating and with EUVAC, whose number densities then follow
the local mass fractions), on uneven columns, implicit steps of a column and of a shell,
the BF16 J v's error, and the host's rejection of fractions outside [0, 1]. Inputs: the
synthetic fits of the input generators, the rest state in hydrostatic balance with m(r)
plus the seeded perturbations."""
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


def _euvac(phys):
    P = dict(phys)
    P.update(synth.euvac_physics(f107bar=150.0, day=172.0))
    P["heating_model"] = 1
    P["heat_amp"] = 0.0
    return P


@pytest.mark.parametrize("p,n_ang,n_rad,euv", [(3, 2, 3, False), (2, 2, 2, False), (4, 1, 2, False),
                                               (3, 2, 2, True)])
def test_shell_residual_and_jvp(p, n_ang, n_rad, euv):
    need_gpu()
    w = synth.with_composition(synth.shell_workload(40 + p, p=p, n_ang=n_ang, n_rad=n_rad))
    if euv:
        w = dataclasses.replace(w, phys=_euvac(w.phys))
    om, gm = shell_pair(w, n_ang, n_rad, p)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    t = 0.29
    R, scale = odg.residual_parts(om, w.phys, u, t)
    r = gm.residual(to_dev(u), t=t).cpu().numpy().reshape(u.shape)
    assert rel_to_scale(r, R, scale) < 1e-12
    v = synth.tangent(u.shape, 6)
    ref, lscale = ojac.jvp_parts(om, w.phys, u, v, t)
    jv = gm.jvp(to_dev(u), to_dev(v), t=t).cpu().numpy().reshape(u.shape)
    assert np.linalg.norm(jv - ref) / np.linalg.norm(ref) < 1e-12
    assert rel_to_scale(jv, ref, lscale) < 1e-12
    jv32 = gm.jvp(to_dev(u), to_dev(v).float(), t=t, prec="f32").cpu().double().numpy().reshape(u.shape)
    assert np.linalg.norm(jv32 - ref) / np.linalg.norm(ref) < 1e-5


def test_shell_jvp_bf16_error_with_composition():
    """the BF16-MFMA J v keeps its error level (a few 1e-3 relative) with the mixture"""
    need_gpu()
    w = synth.with_composition(synth.shell_workload(45, p=3, n_ang=2, n_rad=2))
    om, gm = shell_pair(w, 2, 2, 3)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    v = synth.tangent(u.shape, 7)
    ref = ojac.jvp_complex(om, w.phys, u, v, 0.0)
    jb = gm.jvp(to_dev(u), to_dev(v).float(), t=0.0, prec="bf16").cpu().double().numpy().reshape(u.shape)
    assert np.linalg.norm(jb - ref) / np.linalg.norm(ref) < 3e-2


def test_pure_oxygen_matches_the_constant_mass_kernels():
    """fits that are all zero (pure O, m = 1) give the default model's R and J v"""
    need_gpu()
    w = synth.shell_workload(46, p=3, n_ang=2, n_rad=2)
    wo = dataclasses.replace(w, phys=dict(w.phys, composition=1, comp_a=[0.0] * 6, comp_b=[0.0] * 6))
    om, gm = shell_pair(w, 2, 2, 3)
    _, go = shell_pair(wo, 2, 2, 3)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    v = synth.tangent(u.shape, 8)
    a, b = gm.residual(to_dev(u)).cpu().numpy(), go.residual(to_dev(u)).cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
    a, b = gm.jvp(to_dev(u), to_dev(v)).cpu().numpy(), go.jvp(to_dev(u), to_dev(v)).cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


@pytest.mark.parametrize("euv", [False, True])
def test_columns(euv):
    need_gpu()
    from paper_2306_01085_amd import Mesh
    nelem, p, stretch = [7, 12, 21], [2, 3, 4], 1.1
    w = synth.with_composition(synth.column_batch_workload(8, n_col=len(nelem)))
    phys = _euvac(w.phys) if euv else w.phys
    col_phys = dict(w.col_phys)
    if euv:
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
        uc = np.moveaxis(w.state(c, om.X[:, :, 0]), 0, 1).copy()
        uc[:, 1] += 0.02 * np.sin(0.3 * om.X[:, :, 0])
        cols.append((om, P, uc))
    u = np.concatenate([c[2].ravel() for c in cols])
    v = synth.tangent(u.shape, 9)
    r = gm.residual(to_dev(u), t=0.1).cpu().numpy()
    jv = gm.jvp(to_dev(u), to_dev(v), t=0.1).cpu().numpy()
    for c, (om, P, uc) in enumerate(cols):
        R, scale = odg.residual_parts(om, P, uc, 0.1)
        assert rel_to_scale(r[off[c]:off[c + 1]].reshape(uc.shape), R, scale) < 1e-12, c
        ref = ojac.jvp_complex(om, P, uc, v[off[c]:off[c + 1]].reshape(uc.shape), 0.1)
        jc = jv[off[c]:off[c + 1]].reshape(uc.shape)
        assert np.linalg.norm(jc - ref) / np.linalg.norm(ref) < 1e-12, c


def test_implicit_column_step():
    need_gpu()
    from paper_2306_01085_amd import Mesh
    w = synth.with_composition(synth.config_column(6))
    om = omesh.columns_mesh([8], 2, w.r_bot, w.r_top)
    gm = Mesh.columns([8], [2], w.r_bot, w.r_top, 1.0, w.phys, w.col_phys)
    u = np.moveaxis(w.state(0, om.X[:, :, 0]), 0, 1).copy()
    ref, _ = timeint.implicit_step_dense(om, w.phys, u, 0.0, w.dt, scheme=33, rtol=1e-13)
    ut = to_dev(u)
    gm.implicit_step(ut, 0.0, w.dt, newton_rtol=1e-10, gmres_rtol=1e-6, precond=0)
    out = ut.cpu().numpy().reshape(u.shape)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref - u) < 1e-6


@pytest.mark.parametrize("precond,prec", [(2, "f64"), (2, "f32")])
def test_implicit_shell_step(precond, prec):
    need_gpu()
    w = synth.with_composition(synth.shell_workload(47, p=2, n_ang=1, n_rad=2))
    om, gm = shell_pair(w, 1, 2, 2)
    u = np.moveaxis(w.state_fn()(om.X), 0, 1).copy()
    dt = synth.seconds_to_nondim(10.0)
    ref, _ = timeint.implicit_step_jfnk(om, w.phys, u, 0.0, dt, scheme=33, rtol=1e-12)
    ut = to_dev(u)
    st = gm.implicit_step(ut, 0.0, dt, newton_rtol=1e-10, gmres_rtol=1e-6, jvp_prec=prec, precond=precond)
    out = ut.cpu().numpy().reshape(u.shape)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref - u) < 1e-6, st


def test_fractions_outside_the_unit_interval_are_rejected():
    need_gpu()
    from paper_2306_01085_amd import DgError, Mesh
    w = synth.shell_workload(48, p=2, n_ang=1, n_rad=2)
    bad = dict(w.phys, composition=1, comp_a=[1.5, 0, 0, 0, 0, 0], comp_b=[0.0] * 6)
    with pytest.raises(DgError):
        Mesh.shell(p=2, n_ang=1, n_rad=2, r_bot=w.r_bot, r_top=w.r_top, stretch=w.stretch, phys=bad)
    gm = Mesh.shell(p=2, n_ang=1, n_rad=2, r_bot=w.r_bot, r_top=w.r_top, stretch=w.stretch, phys=w.phys)
    with pytest.raises(DgError):
        gm.set_physics(bad)
