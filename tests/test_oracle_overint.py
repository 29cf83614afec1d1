"""Pins of the oracle's over-integrated 1D residual (dg.residual_overint: Gauss quadrature
of p + 2 points and the exact mass matrix in both equations of eq. (DGformulation)):
free-stream preservation, p + 1 convergence on a manufactured solution, agreement with a
much finer quadrature, and the property it exists for: the linearised hot column has no
growing intra-element mode, which the collocated GLL residual has."""
import math

import numpy as np
import pytest
import sympy as sp

import synth
from oracle import dg
from oracle import mesh as M
from oracle import physics as ph


def test_free_stream_overint():
    P = synth.base_physics(1)
    us = synth.uniform_state(1)
    P.update(r_ref=0.0, heat_amp=0.0, bc_mode=1, bc_state=list(us))
    for p in (2, 3, 4):
        m = M.columns_mesh([5], p, synth.R_BOT, synth.R_TOP, 1.2)
        u = np.broadcast_to(us[None, :, None], (m.E, 3, m.ref.N)).copy()
        assert np.max(np.abs(dg.residual_overint(m, P, u))) < 1e-13


def test_quadrature_converges():
    """p + 2 Gauss points integrate the non-polynomial fluxes and sources to within a small
    fraction of the residual: the result barely moves with p + 8 points"""
    w = synth.column_workload(3, n_elem=6, p=3)
    P = dict(w.phys)
    for k, v in w.col_phys.items():
        P[k] = float(np.asarray(v).ravel()[0])
    m = M.columns_mesh([6], 3, w.r_bot, w.r_top, 1.3)
    u = np.moveaxis(w.state(0, m.X[:, :, 0]), 0, 1).copy()
    u += 1e-3 * np.random.default_rng(1).standard_normal(u.shape)
    a = dg.residual_overint(m, P, u)
    b = dg.residual_overint(m, P, u, nq=m.ref.p + 8)
    assert np.linalg.norm(a - b) < 5e-3 * np.linalg.norm(b)
    assert np.linalg.norm(a - dg.residual(m, P, u)) > 0.1 * np.linalg.norm(b)   # not the collocated one


@pytest.mark.slow
def test_manufactured_solution_order_overint():
    """the steady manufactured solution of test_oracle_dg with the forcing projected by the
    same quadrature: L2 error decreases like h^(p+1)"""
    from oracle import jac
    P = dict(d=1, gamma=5 / 3, Gr=1e5, Pr=0.9, Fr=0.0, m=1.0, nu_r=1.0, alpha_r=0.5, alpha0c=1.0,
             lam=2.5, T_bot=1.0, r_ref=1.0, omega=[0, 0, 0], heat_amp=1.0, heat_qm=0.1, heat_rm=1.5,
             heat_H=0.2, sun_lat=0, sun_lon0=0, sun_rate=0, bc_mode=1, bc_state=[0] * 5)
    x = sp.Symbol("x")
    lr = 0.3 * sp.sin(2 * x) - 0.5
    uex = [lr, 0.3 * sp.cos(3 * x) + 0.2, sp.exp(lr / 2) * (1 + 0.2 * sp.sin(x))]
    q = [[sp.diff(c, x)] for c in uex]
    F = ph.flux(uex, q, P, sp)
    S = ph.source(uex, q, [x], 0.0, P, sp)
    forcing = sp.lambdify(x, [sp.diff(F[c][0], x) - S[c] for c in range(3)], "numpy")
    fu = sp.lambdify(x, uex, "numpy")
    U = lambda xx: np.array([np.broadcast_to(v, np.shape(xx)) for v in fu(xx)])
    P["bc_fn"] = lambda Xf: U(Xf[0])
    for p in (2, 3):
        errs = []
        for E in (8, 16, 32):
            m = M.columns_mesh([E], p, 1.0, 2.0)
            xg, wg, V, Dg, Mr = dg.gauss_tables(m.ref, p + 2)
            Jel = m.J[:, 0]
            xq = m.X[:, 0, 0][:, None] + (xg[None, :] + 1.0) * Jel[:, None]
            fq = np.array([np.broadcast_to(v, xq.shape) for v in forcing(xq)])          # [3, E, nq]
            fh = np.einsum("ij,cej->eci", np.linalg.inv(Mr), np.einsum("g,gi,ceg->cei", wg, V, fq))
            X = m.X[:, :, 0]
            ue = np.moveaxis(U(X), 0, 1)
            u = ue.copy()
            for _ in range(20):
                G = dg.residual_overint(m, P, u) + fh
                if np.max(np.abs(G)) < 1e-11:
                    break
                n = u.size
                Jm = np.zeros((n, n))
                for j in range(n):
                    e = np.zeros(n)
                    e[j] = 1e-30
                    Jm[:, j] = np.imag(dg.residual_overint(m, P, u + 1j * e.reshape(u.shape))).ravel() / 1e-30
                u = u - np.linalg.solve(Jm, G.ravel()).reshape(u.shape)
            eg = np.einsum("gj,ecj->ecg", V, u - ue)       # the error at the Gauss points
            errs.append(math.sqrt(np.sum(Jel[:, None, None] * wg[None, None, :] * eg ** 2)))
        rate = math.log2(errs[-2] / errs[-1])
        assert rate > p + 1 - 0.3, (p, errs)


def _top_growth(residual_fn, P, mesh, u):
    n = u.size
    Jm = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1e-30
        Jm[:, j] = np.imag(residual_fn(mesh, P, u + 1j * e.reshape(u.shape))).ravel() / 1e-30
    return np.max(np.linalg.eigvals(Jm).real)


@pytest.mark.parametrize("p", [2, 3])
def test_overint_removes_the_growing_mode(p):
    """the hot column (T_inf = 1300 K, graded 34-element mesh of the 1D model) at its Bates
    rest state: the collocated residual's Jacobian has real eigenvalues of 0.06 (p = 3) to
    0.15 (p = 2) per time unit, modes that alternate in sign inside the elements near the
    lower boundary; the over-integrated residual's spectrum stays in the closed left half
    plane up to round-off"""
    ne, T_inf = 34, 1300.0
    P = synth.base_physics(1)
    for k, v in synth._column_phys(T_inf, 200.0, 1.0).items():
        P[k] = float(v)
    mesh = M.columns_mesh([ne], p, synth.R_BOT, synth.R_TOP, synth.graded_stretch(ne))
    u = np.moveaxis(np.asarray(synth.column_state(mesh.X[:, :, 0], T_inf)), 0, 1).copy()
    g_col = _top_growth(dg.residual, P, mesh, u)
    g_oi = _top_growth(dg.residual_overint, P, mesh, u)
    assert g_col > 0.05
    assert g_oi < 1e-3
