"""Meshes: batches of 1D radial columns and the cubed-sphere spherical shell.

Section 3.3: the shell between 100 and 600 km is split into the six panels of a
cube-sphere, each into n_ang x n_ang angular elements, times n_rad radial layers
whose thickness grows geometrically. Elements are curved of degree p
(isoparametric: nodes on the exact sphere). The angular map of a panel is the
equiangular gnomonic projection (the paper does not name the projection).

Metric terms J a^i = J grad(xi_i) use the invariant curl form (Kopriva 2006), so
that the discrete metric identities hold (a uniform state is preserved to round-off)
and the discrete operator commutes with rotations of the Cartesian axes. The oracle evaluates that formula directly on each element's nodes.

Element numbering of the shell: e = ((panel * n_ang + j) * n_ang + i) * n_rad + k
(radial layer fastest); nodes inside an element: xi_1 fastest (angular alpha),
then xi_2 (angular beta), then xi_3 (radius). Columns are concatenated, each
numbered from the bottom.

Boundary tags per element face: 0 interior, 1 lower boundary, 2 upper boundary.
"""
from dataclasses import dataclass

import numpy as np
from scipy.spatial import cKDTree

from .gll import RefElement


@dataclass
class Mesh:
    d: int
    ref: RefElement
    X: np.ndarray        # [E, N, d] node coordinates (nondimensional)
    Ja: np.ndarray       # [E, N, d(a), d(k)] contravariant metric J dxi_a/dx_k
    J: np.ndarray        # [E, N]
    nbr: np.ndarray      # [E, 2d, Nf] global index e'*N + j' of the matching node, -1 on boundaries
    tag: np.ndarray      # [E, 2d] boundary tag

    @property
    def E(self):
        return self.X.shape[0]


def radial_edges(r_bot, r_top, n, stretch):
    """layer interfaces with geometric growth h_{k+1} = stretch h_k"""
    if abs(stretch - 1.0) < 1e-15:
        h = np.full(n, (r_top - r_bot) / n)
    else:
        h1 = (r_top - r_bot) * (stretch - 1.0) / (stretch ** n - 1.0)
        h = h1 * stretch ** np.arange(n)
    edges = r_bot + np.concatenate([[0.0], np.cumsum(h)])
    edges[-1] = r_top
    return edges


def columns_mesh(nelem_list, p, r_bot, r_top, stretch=1.0):
    """several independent 1D columns of equal degree p"""
    ref = RefElement(p, 1)
    n = ref.n
    Xs, Js, nbrs, tags = [], [], [], []
    e0 = 0
    for ne in nelem_list:
        edges = radial_edges(r_bot, r_top, ne, stretch)
        h = np.diff(edges)
        X = edges[:-1, None] + 0.5 * (ref.x1[None, :] + 1.0) * h[:, None]
        Xs.append(X[:, :, None])
        Js.append(np.repeat(0.5 * h[:, None], n, axis=1))
        nbr = np.full((ne, 2, 1), -1, dtype=np.int64)
        tag = np.zeros((ne, 2), dtype=np.int64)
        for e in range(ne):
            if e > 0:
                nbr[e, 0, 0] = (e0 + e - 1) * n + (n - 1)
            else:
                tag[e, 0] = 1
            if e < ne - 1:
                nbr[e, 1, 0] = (e0 + e + 1) * n + 0
            else:
                tag[e, 1] = 2
        nbrs.append(nbr)
        tags.append(tag)
        e0 += ne
    X = np.concatenate(Xs)
    J = np.concatenate(Js)
    Ja = np.ones((X.shape[0], n, 1, 1))
    return Mesh(1, ref, X, Ja, J, np.concatenate(nbrs), np.concatenate(tags))


# ------------------------------------------------------------------ cubed sphere
def panel_point(panel, a, b):
    """point on the cube surface for tangent coordinates a = tan(alpha), b = tan(beta);
    every panel's (alpha, beta, outward) frame is right-handed"""
    one = np.ones_like(a)
    table = {
        0: (one, a, b),
        1: (-a, one, b),
        2: (-one, -a, b),
        3: (a, -one, b),
        4: (-b, a, one),
        5: (b, a, -one),
    }
    return np.stack(table[panel], axis=-1)


def curl_metrics(ref, X):
    """J a^i_n = -1/2 e_i . curl_xi( I^N( X_l grad_xi X_m - X_m grad_xi X_l ) ),
    (n, m, l) cyclic: the invariant curl form (Kopriva 2006). Being a discrete
    curl it satisfies the metric identities; being antisymmetric in (l, m) it does
    not depend on the orientation of the Cartesian axes.  X: [N, 3] nodes of one
    element.  Returns Ja[N, a, n]."""
    Dr = ref.Dr
    Ja = np.zeros((ref.N, 3, 3))
    for n_, m_, l_ in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        v = [0.5 * (X[:, l_] * (Dr[k] @ X[:, m_]) - X[:, m_] * (Dr[k] @ X[:, l_])) for k in range(3)]
        curl = [Dr[1] @ v[2] - Dr[2] @ v[1],
                Dr[2] @ v[0] - Dr[0] @ v[2],
                Dr[0] @ v[1] - Dr[1] @ v[0]]
        for a in range(3):
            Ja[:, a, n_] = -curl[a]
    return Ja


def shell_nodes(ref, n_ang, n_rad, r_bot, r_top, stretch):
    p1 = ref.n
    xi = ref.x1
    redges = radial_edges(r_bot, r_top, n_rad, stretch)
    ang = np.linspace(-np.pi / 4, np.pi / 4, n_ang + 1)
    E = 6 * n_ang * n_ang * n_rad
    X = np.zeros((E, ref.N, 3))
    i1, i2, i3 = ref.idx
    e = 0
    for panel in range(6):
        for j in range(n_ang):
            for i in range(n_ang):
                al = ang[i] + 0.5 * (xi[i1] + 1.0) * (ang[i + 1] - ang[i])
                be = ang[j] + 0.5 * (xi[i2] + 1.0) * (ang[j + 1] - ang[j])
                P = panel_point(panel, np.tan(al), np.tan(be))
                unit = P / np.linalg.norm(P, axis=-1, keepdims=True)
                for k in range(n_rad):
                    r = redges[k] + 0.5 * (xi[i3] + 1.0) * (redges[k + 1] - redges[k])
                    X[e] = r[:, None] * unit
                    e += 1
    assert p1 == ref.n
    return X


def shell_mesh(p, n_ang, n_rad, r_bot, r_top, stretch=1.0):
    ref = RefElement(p, 3)
    X = shell_nodes(ref, n_ang, n_rad, r_bot, r_top, stretch)
    E, N = X.shape[:2]
    Ja = np.zeros((E, N, 3, 3))
    J = np.zeros((E, N))
    for e in range(E):
        Ja[e] = curl_metrics(ref, X[e])
        dX = [ref.Dr[a] @ X[e] for a in range(3)]       # dX/dxi_a  [N, 3]
        J[e] = np.einsum("ij,ij->i", dX[0], np.cross(dX[1], dX[2]))
    nbr, tag = connect_by_coordinates(ref, X, n_rad)
    return Mesh(3, ref, X, Ja, J, nbr, tag)


def connect_by_coordinates(ref, X, n_rad):
    """pair faces by their centroids, then face nodes by coordinates"""
    E = X.shape[0]
    nf = len(ref.faces)
    cent = np.zeros((E, nf, 3))
    for f, (a, side, nodes, wf) in enumerate(ref.faces):
        cent[:, f] = X[:, nodes].mean(axis=1)
    flat = cent.reshape(-1, 3)
    scale = np.max(np.abs(X))
    tree = cKDTree(flat)
    pairs = tree.query_pairs(1e-9 * scale, output_type="ndarray")
    partner = np.full(E * nf, -1, dtype=np.int64)
    partner[pairs[:, 0]] = pairs[:, 1]
    partner[pairs[:, 1]] = pairs[:, 0]
    N = ref.N
    nbr = np.full((E, nf, ref.Nf), -1, dtype=np.int64)
    tag = np.zeros((E, nf), dtype=np.int64)
    for e in range(E):
        for f, (a, side, nodes, wf) in enumerate(ref.faces):
            pf = partner[e * nf + f]
            if pf < 0:
                # radial faces without partner: bottom or top of the shell
                assert a == 2, "angular faces are always interior"
                tag[e, f] = 1 if side < 0 else 2
                continue
            e2, f2 = divmod(pf, nf)
            nodes2 = ref.faces[f2][2]
            t2 = cKDTree(X[e2, nodes2])
            dist, loc = t2.query(X[e, nodes])
            assert np.all(dist < 1e-9 * scale)
            nbr[e, f] = e2 * N + nodes2[loc]
    return nbr, tag
