"""Pins of the oracle's reduced-basis (RB) initial guess and preconditioner: exactness
on the span of the basis, the defining identity M^-1 A W = W, the base preconditioner
on the orthogonal complement, least-squares optimality with a rank-deficient basis
(against numpy's lstsq), and the converged DIRK step (the RB only changes the GMRES
path, so the step must equal the dense-Newton step)."""
import numpy as np

import synth
from oracle import mesh as M
from oracle import rb, timeint


def _system(n=40, k=5, seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n)
    W = rng.standard_normal((k, n))
    return rng, A, W, (A @ W.T).T


def test_guess_is_exact_on_the_span():
    rng, A, W, Z = _system()
    x = W.T @ rng.standard_normal(W.shape[0])
    x0 = rb.rb_guess(W, Z, A @ x)
    assert np.linalg.norm(x0 - x) < 1e-12 * np.linalg.norm(x)


def test_preconditioner_maps_AW_to_W():
    rng, A, W, Z = _system(seed=1)
    d = rng.uniform(1, 2, A.shape[0])
    base = lambda v: v / d
    for j in range(W.shape[0]):
        assert np.linalg.norm(rb.rb_precond(W, Z, Z[j], base) - W[j]) < 1e-11 * np.linalg.norm(W[j])


def test_preconditioner_is_the_base_one_off_the_span():
    rng, A, W, Z = _system(seed=2)
    v = rng.standard_normal(A.shape[0])
    Q, _ = np.linalg.qr(Z.T)
    v -= Q @ (Q.T @ v)
    d = rng.uniform(1, 2, A.shape[0])
    assert np.linalg.norm(rb.rb_precond(W, Z, v, lambda r: r / d) - v / d) < 1e-12 * np.linalg.norm(v)


def test_guess_is_the_least_squares_fit_with_a_dependent_basis():
    rng, A, W, Z = _system(seed=3)
    W = np.vstack([W, W[1] + 2 * W[3]])   # a dependent sixth update
    Z = (A @ W.T).T
    rhs = rng.standard_normal(A.shape[0])
    x0 = rb.rb_guess(W, Z, rhs)
    c_ls, *_ = np.linalg.lstsq(Z.T, rhs, rcond=None)
    r_ls = np.linalg.norm(rhs - Z.T @ c_ls)
    assert abs(np.linalg.norm(rhs - A @ x0) - r_ls) < 1e-10 * np.linalg.norm(rhs)


def test_rb_gmres_solves_the_system_in_fewer_iterations():
    """a right-hand side close to the span: the RB guess and preconditioner reach the
    direct solution, with fewer GMRES iterations than plain GMRES"""
    rng, A, W, Z = _system(n=60, k=6, seed=4)
    x = W.T @ rng.standard_normal(6) + 1e-3 * rng.standard_normal(60)
    b = A @ x
    xp, its_plain = timeint.gmres(lambda v: A @ v, b, m=60, rtol=1e-12)
    xr, its_rb = timeint.gmres(lambda v: A @ v, b, x0=rb.rb_guess(W, Z, b), m=60, rtol=1e-12,
                               M=lambda v: rb.rb_precond(W, Z, v))
    assert np.linalg.norm(xr - x) < 1e-9 * np.linalg.norm(x)
    assert np.linalg.norm(xp - x) < 1e-9 * np.linalg.norm(x)
    assert its_rb < its_plain


def test_rb_steps_match_dense_steps():
    w = synth.config_column(0)
    m = M.columns_mesh([4], 2, w.r_bot, w.r_top)
    u = np.moveaxis(w.state(0, m.X[:, :, 0]), 0, 1)
    win = rb.RBWindow(3)
    ud, ur = u, u
    for s in range(2):
        ud, _ = timeint.implicit_step_dense(m, w.phys, ud, s * w.dt, w.dt, scheme=33, rtol=1e-13)
        ur, _ = rb.implicit_step_jfnk_rb(m, w.phys, ur, s * w.dt, w.dt, win, scheme=33, rtol=1e-13)
    assert len(win.W) == 3
    assert np.max(np.abs(ur - ud)) < 1e-10 * np.max(np.abs(ud))
