"""Reduced-basis (RB) initial guess and preconditioner for the Newton-GMRES systems.

Test infrastructure only: the tests call it, the product path never does.

Section 3.2 names the construction without printing it. The linear system of each
Newton iteration is preconditioned by a low-rank approximation of the Jacobian
built on a reduced basis W spanned by the most recent Newton updates, and the same
basis yields GMRES's initial guess; the products J W come from Jacobian-vector
products. The reading written out here (and on the GPU):

  * W = [d_1 .. d_k]: the k = n_rb most recent Newton updates, carried across the
    Newton iterations, stages and steps of one run (the window is emptied when the
    stage operator's dt a_ii changes); Z = A W, with A = I - dt a_ii J the stage
    operator at the iterate where each update was solved;
  * c(v) = G^+ Z^T v with G = Z^T Z (a pseudo-inverse: eigenvalues of G below
    rcond times the largest are dropped): the coefficients of the least-squares fit
    of v by the columns of Z;
  * initial guess x0 = W c(rhs), the minimiser of |rhs - A x| over x in span W
    when Z = A W;
  * preconditioner M^-1 v = W c(v) + P^-1 (v - Z c(v)), P the base preconditioner
    (identity when none): exact on the span of Z, the base one on the rest.
"""
import numpy as np

from . import timeint


def rb_coef(Z, v, rcond=1e-10):
    """c = G^+ Z v with G = Z Z^T; Z holds the vectors A d_j as rows (k x n)"""
    G = Z @ Z.T
    lam, Q = np.linalg.eigh(G)
    keep = lam > rcond * max(lam.max(), 0.0) if lam.size else lam > 0
    inv = np.where(keep, 1.0 / np.where(keep, lam, 1.0), 0.0)
    return Q @ (inv * (Q.T @ (Z @ v)))


def rb_guess(W, Z, rhs, rcond=1e-10):
    """x0 = W^T c(rhs) (W, Z: k x n)"""
    return W.T @ rb_coef(Z, rhs, rcond)


def rb_precond(W, Z, v, base=None, rcond=1e-10):
    """M^-1 v = W^T c + P^-1 (v - Z^T c), c = c(v)"""
    c = rb_coef(Z, v, rcond)
    r = v - Z.T @ c
    return W.T @ c + (r if base is None else base(r))


class RBWindow:
    """the n_rb most recent (update, A update) pairs, oldest dropped first"""

    def __init__(self, n_rb):
        self.n_rb = n_rb
        self.W, self.Z = [], []
        self.aii_dt = None

    def push(self, d, z):
        self.W.append(d.copy())
        self.Z.append(z.copy())
        if len(self.W) > self.n_rb:
            self.W.pop(0)
            self.Z.pop(0)

    def arrays(self):
        return np.array(self.W), np.array(self.Z)


def newton_jfnk_rb(mesh, P, Gfun, U0, ti, aii_dt, ref_norm, window, rtol=1e-12, maxit=40, gmres_rtol=1e-12):
    """Newton with matrix-free GMRES (complex-step products) whose linear systems use the
    RB initial guess and preconditioner of the window; every update joins the window"""
    from . import jac
    if window.aii_dt != aii_dt:
        window.W, window.Z = [], []
        window.aii_dt = aii_dt
    U = U0.copy()
    gm = 0
    for it in range(maxit):
        G = Gfun(U)
        nG = np.linalg.norm(G)
        if nG <= rtol * ref_norm:
            return U, it, gm
        Aop = lambda v, U=U: v - aii_dt * jac.jvp_complex(mesh, P, U, v.reshape(U.shape), ti).ravel()
        rhs = -G.ravel()
        x0, M = None, None
        if window.W:
            Wa, Za = window.arrays()
            x0 = rb_guess(Wa, Za, rhs)
            M = lambda v, Wa=Wa, Za=Za: rb_precond(Wa, Za, v)
        dx, its = timeint.gmres(Aop, rhs, x0=x0, m=60, rtol=gmres_rtol, max_restarts=200, M=M)
        gm += its
        window.push(dx, Aop(dx))
        U = U + dx.reshape(U.shape)
    raise RuntimeError("JFNK Newton with the RB window did not converge")


def implicit_step_jfnk_rb(mesh, P, u, t, dt, window, scheme=33, rtol=1e-12):
    """one DIRK step, every stage solved by newton_jfnk_rb sharing the window (pass the
    same window to consecutive steps); returns (u_{n+1}, GMRES iterations)"""
    from . import dg
    A, b, c = timeint.dirk_tableau(scheme)
    Rs = []
    gm = 0
    Ui = u
    for i in range(len(c)):
        ti = t + c[i] * dt
        bi = u + dt * sum(A[i, j] * Rs[j] for j in range(i))
        aii = A[i, i]
        G = lambda U: U - dt * aii * dg.residual(mesh, P, U, ti) - bi
        Ui, _, its = newton_jfnk_rb(mesh, P, G, u, ti, dt * aii, np.linalg.norm(G(u)), window, rtol)
        gm += its
        Rs.append(dg.residual(mesh, P, Ui, ti))
    return Ui, gm
