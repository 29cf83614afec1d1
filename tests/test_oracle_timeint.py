"""Pins of the time integrator and the solvers: DIRK order conditions and stability,
GMRES against a direct solve, Newton against scipy's root finder, and one oracle
implicit step against a sequence of tiny explicit steps (a reference integrator
that shares nothing with the DIRK code)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import root

import synth
from oracle import dg, jac, timeint
from oracle import mesh as M


@pytest.mark.parametrize("scheme,order", [(22, 2), (33, 3)])
def test_dirk_order_conditions(scheme, order):
    A, b, c = timeint.dirk_tableau(scheme)
    assert np.allclose(A.sum(axis=1), c, atol=1e-15)
    assert abs(b.sum() - 1) < 1e-15
    assert abs(b @ c - 0.5) < 1e-15
    if order == 3:
        assert abs(b @ c ** 2 - 1 / 3) < 1e-14
        assert abs(b @ (A @ c) - 1 / 6) < 1e-14
    # singly diagonal and stiffly accurate
    assert np.allclose(np.diag(A), A[0, 0])
    assert np.allclose(A[-1], b)
    # L-stability: stability function -> 0 at infinity
    z = -1e8
    I = np.eye(len(b))
    Rz = 1 + z * b @ np.linalg.solve(I - z * A, np.ones(len(b)))
    assert abs(Rz) < 1e-6


@pytest.mark.parametrize("scheme,order", [(22, 2), (33, 3)])
def test_dirk_observed_order(scheme, order):
    A, b, c = timeint.dirk_tableau(scheme)
    lam = -1.3 + 0.4j
    errs = []
    for n in (20, 40, 80):
        h = 1.0 / n
        y = 1.0 + 0j
        for _ in range(n):
            K = []
            for i in range(len(c)):
                rhs = y + h * sum(A[i, j] * K[j] for j in range(i))
                Y = rhs / (1 - h * A[i, i] * lam)
                K.append(lam * Y)
            y = y + h * sum(b[i] * K[i] for i in range(len(b)))
        errs.append(abs(y - np.exp(lam)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.15), rates


def test_gmres_matches_direct_solve():
    rng = np.random.default_rng(0)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.5
    b = rng.standard_normal(n)
    x, its = timeint.gmres(lambda v: A @ v, b, m=30, rtol=1e-12)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-9 * np.linalg.norm(np.linalg.solve(A, b))
    # right preconditioning with the exact inverse converges in one iteration
    Ainv = np.linalg.inv(A)
    x2, its2 = timeint.gmres(lambda v: A @ v, b, m=30, rtol=1e-12, M=lambda v: Ainv @ v)
    assert its2 <= 2 and np.allclose(x2, x, atol=1e-9)


def _tiny_column():
    w = synth.config_column(0)
    m = M.columns_mesh([4], 2, w.r_bot, w.r_top)
    u = np.moveaxis(w.state(0, m.X[:, :, 0]), 0, 1)
    return m, w.phys, u, w.dt


def test_newton_stage_matches_scipy_root():
    m, P, u, dt = _tiny_column()
    A, b, c = timeint.dirk_tableau(33)
    a = A[0, 0]
    G = lambda U: U - dt * a * dg.residual(m, P, U, 0.0) - u
    Jf = lambda U: np.eye(U.size) - dt * a * jac.dense_jacobian(m, P, U)
    U1, its, hist = timeint.newton_dense(G, Jf, u, np.linalg.norm(G(u)), rtol=1e-13)
    sol = root(lambda y: G(y.reshape(u.shape)).ravel(), u.ravel(), method="hybr", tol=1e-14)
    assert sol.success
    assert np.max(np.abs(U1.ravel() - sol.x)) < 1e-10 * np.max(np.abs(U1))
    assert its <= 8


def test_implicit_step_against_fine_explicit_integration():
    """one DIRK(3,3) step of a small dt agrees with an adaptive RK45 integration of the
    semi-discrete system to the step's local error (O(dt^4))"""
    m, P, u, dt = _tiny_column()
    h = dt * 0.05
    u1, _ = timeint.implicit_step_dense(m, P, u, 0.0, h, scheme=33)
    f = lambda t, y: dg.residual(m, P, y.reshape(u.shape), t).ravel()
    ref = solve_ivp(f, (0.0, h), u.ravel(), method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
    change = np.linalg.norm(ref - u.ravel())
    assert np.linalg.norm(u1.ravel() - ref) < 1e-3 * change


def test_jfnk_step_matches_dense_step():
    m, P, u, dt = _tiny_column()
    u1, _ = timeint.implicit_step_dense(m, P, u, 0.0, dt, scheme=33, rtol=1e-13)
    u2, _ = timeint.implicit_step_jfnk(m, P, u, 0.0, dt, scheme=33, rtol=1e-13)
    assert np.max(np.abs(u1 - u2)) < 1e-10 * np.max(np.abs(u1))


@pytest.mark.parametrize("p", [2, 3, 4])
def test_modal_filter_closed_form(p):
    """the filter keeps every tensor polynomial below degree p in each variable and
    multiplies the degree-p Legendre factor of each variable by sigma (closed form on
    the reference element, 3D and 1D)"""
    from numpy.polynomial import legendre as L
    from oracle import mesh as omesh
    sigma = 0.37
    Pp = lambda x: L.legval(x, np.r_[np.zeros(p), 1.0])
    om = omesh.shell_mesh(p, 1, 1, 1.0, 1.5)
    x1 = om.ref.x1
    a, b, c = (x1[i] for i in om.ref.idx)
    low = 0.3 + a ** (p - 1) * b - 0.7 * b * c ** (p - 1) + a * b * c
    u = np.stack([low, Pp(a) * b, Pp(a) * Pp(b) * Pp(c), Pp(c) + low, Pp(b) * a ** (p - 1)])[None]
    want = np.stack([low, sigma * Pp(a) * b, sigma ** 3 * Pp(a) * Pp(b) * Pp(c), sigma * Pp(c) + low,
                     sigma * Pp(b) * a ** (p - 1)])[None]
    got = timeint.modal_filter(om, u, sigma)
    assert np.max(np.abs(got - want)) < 1e-13
    col = omesh.columns_mesh([3], p, 1.0, 2.0)
    xc = col.ref.x1
    uc = np.tile(np.stack([xc ** (p - 1), Pp(xc), 1.0 + Pp(xc)]), (3, 1, 1))
    wc = np.tile(np.stack([xc ** (p - 1), sigma * Pp(xc), 1.0 + sigma * Pp(xc)]), (3, 1, 1))
    assert np.max(np.abs(timeint.modal_filter(col, uc, sigma) - wc)) < 1e-13
