"""A dense Jacobian of the oracle's residual for the implicit-step parity tests, assembled by
complex-step columns (as oracle.jac.dense_jacobian) K columns at a time: K independent
copies of the mesh form one larger mesh, copy c carrying the perturbation of column j0 + c.
The copies share no faces, so each one's residual is that of the original problem."""
import numpy as np

from oracle import dg
from oracle.mesh import Mesh


def tiled_mesh(mesh, K):
    """K disjoint copies of mesh in one Mesh (copy c holds elements c E .. (c + 1) E - 1)"""
    E, N = mesh.E, mesh.ref.N
    nbr = np.concatenate([np.where(mesh.nbr >= 0, mesh.nbr + c * E * N, -1) for c in range(K)])
    return Mesh(mesh.d, mesh.ref, np.tile(mesh.X, (K, 1, 1)), np.tile(mesh.Ja, (K, 1, 1, 1)),
                np.tile(mesh.J, (K, 1)), nbr, np.tile(mesh.tag, (K, 1)))


def dense_jacobian(mesh, P, u, t=0.0, K=48, h=1e-30):
    n = u.size
    E, f, N = u.shape
    big = tiled_mesh(mesh, K)
    Jm = np.empty((n, n))
    for j0 in range(0, n, K):
        k = min(K, n - j0)
        U = np.tile(u.reshape(1, n), (K, 1)).astype(np.complex128)
        U[np.arange(k), j0 + np.arange(k)] += 1j * h
        R = dg.residual(big, P, U.reshape(K * E, f, N), t)
        Jm[:, j0:j0 + k] = (np.imag(R).reshape(K, n)[:k] / h).T
    return Jm
