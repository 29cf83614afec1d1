"""Pins of the LDG stabilisation of eq. (LDG2) and of the upper-boundary penalty.

sigma = lambda_max I + sigma_d, where the diffusive block sigma_d (section 3.1) holds the
two diffusivities of the transformed fluxes of eq. (fluxSWNondimensional): the factor in
front of the strain in the viscous momentum flux and the one in front of grad T in the
conductive energy flux. The tests below take those factors from the oracle's flux (itself
pinned symbolically to the Navier-Stokes equations in test_oracle_physics) by probing it
with a pure shear and a pure temperature gradient, so a sigma with m and 1/m swapped, a
dropped sqrt(gamma) or 1/Pr, or a wrong density power fails here. The residual-level tests
then fix how the residual applies sigma: at the trace u_hat of interior faces and at u_b on
the lower face, weighted by |Sn| and lifted by 1/(w_end J), and the upper-face penalty
lambda (U.n) n |Sn| on inflow and outflow nodes alike (the reading taken for the open top).
"""
import numpy as np
import pytest

import synth
from oracle import dg
from oracle import mesh as M
from oracle import physics as ph


def _phys(d, comp):
    P = synth.base_physics(d)
    P["lam"] = 1.7
    if comp:
        P.update(synth.composition_physics())
    return P


def _diffusivities(u, x, P):
    """(momentum, energy) diffusivities of the flux at state u and position x, read off
    the oracle's viscous flux: F_U = -c_m eps(v), F_Theta = -c_e grad T"""
    d = P["d"]
    f = d + 2
    zero = 0.0 * u[0]
    _, _, _, _, s, _, _ = ph.primitives(u, P, np)
    # pure shear: q_U[0][d-1] = 1 only (grad of log-density and of Theta zero), so
    # grad v = s e_0 (x) e_{d-1}; in 1D eps = (4/3) dv/dx, otherwise eps_{0,d-1} = s
    q = [[zero + 0.0 for _ in range(d)] for _ in range(f)]
    q[1][d - 1] = zero + 1.0
    Fv = ph.flux_viscous(u, q, P, np, x)
    eps01 = (4.0 / 3.0) * s if d == 1 else s
    c_m = -Fv[1][d - 1] / eps01
    # pure temperature gradient: q_Theta[0] = 1, so grad T = s e_0
    q = [[zero + 0.0 for _ in range(d)] for _ in range(f)]
    q[d + 1][0] = zero + 1.0
    Fv = ph.flux_viscous(u, q, P, np, x)
    c_e = -Fv[d + 1][0] / s
    # the flux probe itself: no other component responds to these gradients
    return c_m, c_e


def _sigma_expected(u, x, P):
    c_m, c_e = _diffusivities(u, x, P)
    d = P["d"]
    lam = P["lam"]
    return [lam + 0.0 * c_m] + [lam + c_m] * d + [lam + c_e]


def _random_state(rng, d, n):
    lr = rng.uniform(-12.0, 0.5, n)
    U = [rng.normal(0, 0.05, n) * np.exp(0.5 * lr) for _ in range(d)]
    Th = rng.uniform(0.8, 6.0, n) * np.exp(0.5 * lr)
    return [lr] + U + [Th]


@pytest.mark.parametrize("d", [1, 3])
@pytest.mark.parametrize("comp", [False, True])
def test_sigma_is_lambda_plus_flux_diffusivities(d, comp):
    P = _phys(d, comp)
    rng = np.random.default_rng(11 + d + 2 * comp)
    n = 64
    u = _random_state(rng, d, n)
    rad = rng.uniform(synth.R_BOT, synth.R_TOP, n)
    if d == 1:
        x = [rad]
    else:
        dirs = rng.normal(size=(3, n))
        dirs /= np.linalg.norm(dirs, axis=0)
        x = [rad * dirs[k] for k in range(3)]
    sig = ph.sigma(u, P, np, x)
    ref = _sigma_expected(u, x, P)
    for c in range(d + 2):
        np.testing.assert_allclose(np.broadcast_to(sig[c], (n,)), np.broadcast_to(ref[c], (n,)), rtol=1e-14)
    # the diffusive part is not negligible at these states (else the test says little)
    assert np.min(np.asarray(sig[1]) - P["lam"]) > 0 and np.min(np.asarray(sig[d + 1]) - P["lam"]) > 0
    if comp:
        # with the mixture, c_v = 1/m departs from 1 over the sampled heights
        m = ph.mixture(P, np, x)[0]
        assert np.max(np.abs(m - 1.0)) > 0.3


def test_sigma_depends_on_mass_as_the_paper_states():
    """sigma_d of the energy row is kappa/(Pr sqrt(rho) c_v) sqrt(gamma/Gr) with c_v = 1/m:
    at a fixed state its conduction part (alpha_r = 0, unit conductivity weight) grows
    linearly with m; the momentum row does not depend on m through c_v (only through
    the molecular viscosity sqrt(T m))"""
    P = _phys(1, False)
    P["alpha_r"] = 0.0
    P["nu_r"] = 0.0
    u = [np.array([-3.0]), np.array([0.0]), np.array([2.0 * np.exp(-1.5)])]
    out = []
    for m in (1.0, 2.0):
        P["m"] = m
        s = ph.sigma(u, P, np)
        out.append((float(s[1][0]) - P["lam"], float(s[2][0]) - P["lam"]))
    (vm1, e1), (vm2, e2) = out
    assert e2 / e1 == pytest.approx(2.0, rel=1e-9)
    assert vm2 / vm1 == pytest.approx(np.sqrt(2.0), rel=1e-9)


def _jump_state(mesh, P, rng):
    """smooth in each element, discontinuous across faces (a different offset per element)"""
    d = P["d"]
    E, N = mesh.E, mesh.ref.N
    r = np.linalg.norm(mesh.X, axis=-1)
    u = np.zeros((E, d + 2, N))
    u[:, 0] = -0.4 * (r - synth.R_BOT) + rng.normal(0, 0.05, (E, 1))
    for k in range(d):
        u[:, 1 + k] = rng.normal(0, 0.02, (E, 1)) + 0.01 * np.sin(r)
    u[:, d + 1] = (1.0 + 0.1 * (r - synth.R_BOT)) * np.exp(0.5 * u[:, 0]) * (1 + rng.normal(0, 0.03, (E, 1)))
    return u


def _penalty_by_hand(mesh, P, u):
    """the sigma terms of the residual written out from eq. (LDG2): on every face node
    -|Sn| sigma(u_hat) (u - u_hat) at interior faces, -|Sn| sigma(u_b) (u - u_b) on the lower
    face, lifted by 1/(w_end J); zero on the upper face (its penalty takes lambda directly)"""
    ref = mesh.ref
    d = P["d"]
    E, N = mesh.E, ref.N
    out = np.zeros_like(u)
    w_end = ref.w1[0]
    flat = np.moveaxis(u, 1, 0).reshape(d + 2, E * N)
    for e in range(E):
        for fi, (a, side, nodes, wf) in enumerate(ref.faces):
            tag = mesh.tag[e, fi]
            if tag == 2:
                continue
            for m_, j in enumerate(nodes):
                uo = u[e, :, j]
                if tag == 0:
                    un = flat[:, mesh.nbr[e, fi, m_]]
                    ut = 0.5 * (uo + un)
                else:
                    ut = np.array([uo[0]] + [0.0] * d + [P["T_bot"] * np.exp(0.5 * uo[0])])
                xs = [np.array([mesh.X[e, j, k]]) for k in range(d)]
                sg = np.array([float(np.asarray(v).ravel()[0])
                               for v in _sigma_expected([np.array([v]) for v in ut], xs, P)])
                Sn = side * mesh.Ja[e, j, a, :]
                out[e, :, j] -= np.linalg.norm(Sn) * sg * (uo - ut) / (w_end * mesh.J[e, j])
    return out


@pytest.mark.parametrize("geom", ["column", "shell"])
def test_residual_applies_sigma_at_the_trace(geom, monkeypatch):
    rng = np.random.default_rng(5)
    if geom == "column":
        P = _phys(1, True)
        mesh = M.columns_mesh([4], 2, synth.R_BOT, synth.R_TOP, 1.15)
    else:
        P = _phys(3, True)
        mesh = M.shell_mesh(2, 1, 2, synth.R_BOT, synth.R_TOP, 1.15)
    u = _jump_state(mesh, P, rng)
    R_full = dg.residual(mesh, P, u)
    zero_sigma = lambda uh, P_, xp, x=None: [0.0 * uh[0] for _ in range(P_["d"] + 2)]  # noqa: E731
    monkeypatch.setattr(ph, "sigma", zero_sigma)
    R_none = dg.residual(mesh, P, u)
    expect = _penalty_by_hand(mesh, P, u)
    scale = np.max(np.abs(expect), axis=(0, 2), keepdims=True)
    assert np.all(scale > 0)
    # (the difference of two residuals carries their rounding: 1e-9 of the penalty scale)
    np.testing.assert_allclose((R_full - R_none) / scale, expect / scale, rtol=0, atol=1e-9)


@pytest.mark.parametrize("direction", [+1.0, -1.0])
def test_upper_face_penalty_on_outflow_and_inflow(direction, monkeypatch):
    """the upper-face numerical flux is F_inviscid(u).n plus lambda (U.n) n |Sn| in the
    momentum rows: with sigma switched off, R is affine in lambda only through that term, so
    dR/dlambda at the top node is -(U.n) n |Sn| / (w_end J) in the momentum row and zero in
    the others; the same on an outflow (U.n > 0) and an inflow (U.n < 0) node"""
    P = _phys(1, False)
    mesh = M.columns_mesh([3], 2, synth.R_BOT, synth.R_TOP, 1.0)
    rng = np.random.default_rng(2)
    u = _jump_state(mesh, P, rng)
    u[-1, 1, -1] = direction * 0.03 * np.exp(0.5 * u[-1, 0, -1])
    monkeypatch.setattr(ph, "sigma", lambda uh, P_, xp, x=None: [0.0 * uh[0] for _ in range(P_["d"] + 2)])
    P1, P2 = dict(P, lam=1.0), dict(P, lam=3.5)
    dR = (dg.residual(mesh, P2, u) - dg.residual(mesh, P1, u)) / 2.5
    J_top = mesh.J[-1, -1]
    Sn = mesh.Ja[-1, -1, 0, 0]           # outward normal of the upper face (side +1)
    expect = -(u[-1, 1, -1] * Sn) * Sn / abs(Sn) / (mesh.ref.w1[-1] * J_top)
    assert np.sign(u[-1, 1, -1] * Sn) == direction
    assert dR[-1, 1, -1] == pytest.approx(expect, rel=1e-12)
    others = dR.copy()
    others[-1, 1, -1] = 0.0
    assert np.max(np.abs(others)) < 1e-12 * abs(expect)


def _top_mode_growth(P, mesh, u):
    """largest real part over the eigenmodes of the linearised column that live in its two
    top elements (at least 80% of the mode's squared norm there)"""
    from oracle import jac
    lam, V = np.linalg.eig(jac.dense_jacobian(mesh, P, u))
    E, f, N = u.shape
    w = (np.abs(V) ** 2).reshape(E, f * N, -1).sum(axis=1)
    w /= w.sum(axis=0)
    top = w[-2:].sum(axis=0) > 0.8
    return np.max(lam.real[top])


def test_upper_penalty_damps_the_top_element_mode(monkeypatch):
    """without the upper-face penalty the linearised hot column (T_inf = 1300 K, the graded
    34-element p = 2 mesh of the 1D model) has a growing oscillatory mode in its top
    elements; the penalty cuts its growth rate at least three-fold (it does not remove it
    at this temperature: the rate stays near 0.03 per time unit)"""
    ne, T_inf = 34, 1300.0
    P = synth.base_physics(1)
    for k, v in synth._column_phys(T_inf, 200.0, 1.0).items():
        P[k] = float(v)
    mesh = M.columns_mesh([ne], 2, synth.R_BOT, synth.R_TOP, synth.graded_stretch(ne))
    u = np.moveaxis(np.asarray(synth.column_state(mesh.X[:, :, 0], T_inf)), 0, 1).copy()
    with_pen = _top_mode_growth(P, mesh, u)
    monkeypatch.setattr(dg, "top_penalty", lambda P_, uin, Sn, Smag, d: np.zeros_like(uin))
    without = _top_mode_growth(P, mesh, u)
    assert without > 0.1
    assert with_pen < without / 3.0
