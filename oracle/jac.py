"""Jacobian-vector products of the residual (section 3.2).

The method needs only J(u) v. The oracle offers three independent routes:
  * complex step:  J v = Im R(u + i h v) / h, h = 1e-30 -- exact to round-off
    (every operation in the residual is analytic in u along the path);
  * the finite difference of R that the paper uses, (R(u + eps v) - R(u)) / eps,
    with eps = sqrt(machine eps) (1 + |u|) / |v| (the step rule is not printed);
  * a dense Jacobian assembled column by column (tiny meshes only).
"""
import numpy as np

from . import dg


def jvp_complex(mesh, P, u, v, t=0.0, h=1e-30, residual=None):
    """residual: the residual function (dg.residual, the collocated one, by default)"""
    residual = dg.residual if residual is None else residual
    uc = u.astype(np.complex128) + 1j * h * v
    return np.imag(residual(mesh, P, uc, t)) / h


def jvp_parts(mesh, P, u, v, t=0.0, h=1e-30):
    """(J v, linearised term scale): the complex step of each part of R (volume divergence,
    face contribution, source) separately, the scale being |dV| + |dFc| + |dS| per node, so
    that a parity bound relative to it is not loosened or tightened by cancellation
    between the parts of J v"""
    uc = u.astype(np.complex128) + 1j * h * v
    R, V, Fc, S = dg.residual_terms(mesh, P, uc, t)
    scale = np.abs(np.imag(V)) / h
    del V
    scale += np.abs(np.imag(Fc)) / h
    del Fc
    scale += np.abs(np.imag(S)) / h
    del S
    return np.imag(R) / h, np.moveaxis(scale, 0, 1).copy()


def jvp_fd(mesh, P, u, v, t=0.0, eps=None, central=False):
    if eps is None:
        eps = np.sqrt(np.finfo(np.float64).eps) * (1.0 + np.linalg.norm(u)) / np.linalg.norm(v)
    if central:
        return (dg.residual(mesh, P, u + eps * v, t) - dg.residual(mesh, P, u - eps * v, t)) / (2 * eps)
    return (dg.residual(mesh, P, u + eps * v, t) - dg.residual(mesh, P, u, t)) / eps


def dense_jacobian(mesh, P, u, t=0.0, residual=None):
    n = u.size
    Jm = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        Jm[:, j] = jvp_complex(mesh, P, u, e.reshape(u.shape), t, residual=residual).ravel()
    return Jm
