"""Nodal Lagrange basis on Gauss-Lobatto-Legendre points.

The DG spaces of section 3.1 are realised as tensor-product polynomials of degree
p per direction (the DOF counts of the convergence table, n_elem (k+1)^3 5, fix the
tensor space), collocated at the p+1 GLL points with GLL quadrature.
"""
import numpy as np
from numpy.polynomial import legendre as L


def gll(p):
    """nodes and weights of the (p+1)-point GLL rule on [-1, 1]: the end points and
    the roots of P_p', weights 2 / (p (p+1) P_p(x)^2)."""
    c = np.zeros(p + 1)
    c[p] = 1.0
    inner = np.sort(np.real(L.legroots(L.legder(c))))
    # polish the interior roots with Newton on P_p'
    d1, d2 = L.legder(c), L.legder(c, 2)
    for _ in range(3):
        inner = inner - L.legval(inner, d1) / L.legval(inner, d2)
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (p * (p + 1) * L.legval(x, c) ** 2)
    return x, w


def diff_matrix(x):
    """D[i, j] = l_j'(x_i) for the Lagrange basis on nodes x (barycentric form)."""
    n = len(x)
    lam = np.array([1.0 / np.prod([x[j] - x[k] for k in range(n) if k != j]) for j in range(n)])
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D


def lagrange_eval(x, xe):
    """matrix V[k, j] = l_j(xe[k])"""
    n = len(x)
    V = np.ones((len(xe), n))
    for j in range(n):
        for k in range(n):
            if k != j:
                V[:, j] *= (xe - x[k]) / (x[j] - x[k])
    return V


class RefElement:
    """tensor-product reference element [-1,1]^d with n = p+1 nodes per direction.
    Node (i1, .., id) has flat index i1 + n i2 + n^2 i3 (xi_1 fastest)."""

    def __init__(self, p, d):
        self.p, self.d, self.n = p, d, p + 1
        self.x1, self.w1 = gll(p)
        self.D1 = diff_matrix(self.x1)
        n = self.n
        self.N = n ** d
        I = np.eye(n)
        # multi-index of every node: idx[a][node] = index along direction a
        grid = np.indices((n,) * d)[::-1]          # grid[0] = i1 (fastest)
        self.idx = [g.ravel() for g in grid]
        self.W = np.ones(self.N)
        for a in range(d):
            self.W *= self.w1[self.idx[a]]
        # reference derivative matrices Dr[a][i, j] = d phi_j / d xi_a (x_i)
        self.Dr = []
        for a in range(d):
            mats = [I] * d
            mats[a] = self.D1
            M = np.ones((1, 1))
            for b in reversed(range(d)):          # direction d-1 is the slowest index
                M = np.kron(M, mats[b])
            self.Dr.append(M)
        # faces: (direction a, side -1/+1, node list ordered by the remaining
        # directions lexicographically, quadrature weights)
        self.faces = []
        for a in range(d):
            for side in (-1, 1):
                target = 0 if side < 0 else n - 1
                nodes = np.nonzero(self.idx[a] == target)[0]
                wf = np.ones(len(nodes))
                for b in range(d):
                    if b != a:
                        wf *= self.w1[self.idx[b][nodes]]
                self.faces.append((a, side, nodes, wf))
        self.Nf = n ** (d - 1)
