"""The LDG discretisation, eq. (DGformulation), in weak form with GLL quadrature.

Pass 1 (auxiliary gradient):  (q, p) = -(u, div p) + <u_hat, p.n>
Pass 2 (state):               (du/dt, w) = (F(u, q), grad w) - <F_hat.n, w> + (s(u, q), w)

Numerical trace and flux, eq. (LDG2), at interior faces:
    u_hat = (u + u^-)/2
    F_hat.n = (F(u, q) + F(u^-, q^-)).n / 2 + sigma(u_hat) (u - u_hat)
with sigma = lambda_max I + sigma_d(u_hat) (physics.sigma).

Boundary faces (section 2.3, the details being the stated reading):
  lower (tag 1): u_b = (varrho, 0, T_bot sqrt(rho)); u_hat = u_b;
                 F_hat.n = F(u_b, q).n + sigma(u_b) (u - u_b)
  upper (tag 2): u_hat = u; F_hat.n = F_inviscid(u).n (zero normal stress, adiabatic,
                 the advective fluxes open) plus the penalty sigma (u - u_b) of eq. (LDG2)
                 with u_b = u less its normal momentum and sigma = lambda_max on the
                 momentum: lambda (U.n) n |Sn|, which takes the acoustic energy leaving
                 through the open top out of the system
  bc_mode 1 (test problems): every boundary is a Dirichlet state u_D (a constant
                 vector, or P["bc_fn"](x)), treated like the lower boundary with u_b = u_D.

All integrals use the collocated GLL rule, so the mass matrix is diag(w_i J_i) and
R = M^{-1}(...) is the nodal time derivative du/dt.
"""
import numpy as np

from . import physics as ph


def _arr(lst, like):
    return np.array([np.broadcast_to(np.asarray(v, dtype=like.dtype), like.shape) for v in lst])


def _arr2(lst, like):
    return np.array([[np.broadcast_to(np.asarray(v, dtype=like.dtype), like.shape) for v in row] for row in lst])


def _dot_n(F, Sn, d):
    # F: [f, d, ...], Sn: [d, ...]
    return sum(F[:, k] * Sn[k] for k in range(d))


def boundary_value(mesh, P, uin, Xf):
    """state u_b imposed on a boundary face (before the tag decides how it is used)"""
    if P.get("bc_mode", 0) == 1:
        if "bc_fn" in P:
            return np.asarray(P["bc_fn"](Xf), dtype=uin.dtype)
        ud = np.asarray(P["bc_state"][: P["d"] + 2], dtype=uin.dtype)
        return np.broadcast_to(ud[:, None, None], uin.shape).copy()
    return _arr(ph.bottom_state(uin, P, np), uin[0])


def top_penalty(P, uin, Sn, Smag, d):
    """lambda (U.Sn) Sn / |Sn| in the momentum rows, zero elsewhere: the term
    sigma (u - u_b) |Sn| of the upper face with u_b = u less its normal momentum"""
    Un = sum(uin[1 + k] * Sn[k] for k in range(d)) / Smag
    out = np.zeros_like(uin)
    for k in range(d):
        out[1 + k] = P["lam"] * Un * Sn[k]
    return out


def traces(mesh, P, u):
    """u_hat on every face node: list over faces of [f, E, Nf]"""
    ref = mesh.ref
    f = P["d"] + 2
    E, N = mesh.E, ref.N
    unodes = np.moveaxis(u, 1, 0).reshape(f, E * N)
    out = []
    for fi, (a, side, nodes, wf) in enumerate(ref.faces):
        uin = np.moveaxis(u[:, :, nodes], 1, 0)          # [f, E, Nf]
        nb = mesh.nbr[:, fi, :]
        uout = unodes[:, np.where(nb >= 0, nb, 0)]
        uh = 0.5 * (uin + uout)
        tag = mesh.tag[:, fi][None, :, None]
        Xf = np.moveaxis(mesh.X[:, nodes, :], 2, 0)      # [d, E, Nf]
        ub = boundary_value(mesh, P, uin, Xf)
        if P.get("bc_mode", 0) == 1:
            uh = np.where(tag > 0, ub, uh)
        else:
            uh = np.where(tag == 1, ub, np.where(tag == 2, uin, uh))
        out.append(uh)
    return out


def gradient(mesh, P, u):
    """pass 1: q[e, c, k, j] (weak form with GLL quadrature)"""
    ref = mesh.ref
    d = P["d"]
    W = ref.W
    uh = traces(mesh, P, u)
    q = np.zeros(u.shape[:2] + (d, ref.N), dtype=u.dtype)
    for a in range(d):
        # T[e, c, k, i] = w_i Ja[e, i, a, k] u[e, c, i]
        JaT = np.transpose(mesh.Ja[:, :, a, :], (0, 2, 1))          # [E, k, i]
        T = u[:, :, None, :] * (W[None, None, None, :] * JaT[:, None, :, :])
        q -= T @ ref.Dr[a]
    for fi, (a, side, nodes, wf) in enumerate(ref.faces):
        Sn = side * mesh.Ja[:, nodes, a, :]                          # [E, Nf, k]
        q[:, :, :, nodes] += np.einsum("cem,emk,m->eckm", uh[fi], Sn, wf)
    q /= (W[None, :] * mesh.J)[:, None, None, :]
    return q


def residual(mesh, P, u, t=0.0, q=None):
    """R(u) = du/dt of the semi-discrete system, shape [E, f, N]"""
    ref = mesh.ref
    d = P["d"]
    f = d + 2
    E, N = mesh.E, ref.N
    W = ref.W
    if q is None:
        q = gradient(mesh, P, u)
    uh = traces(mesh, P, u)
    un = np.moveaxis(u, 1, 0)                         # [f, E, N]
    qn = np.moveaxis(q, 1, 0)                         # [f, E, d, N] -> index as [c][k]
    qn = np.moveaxis(qn, 2, 1)                        # [f, d, E, N]
    xn = np.moveaxis(mesh.X, 2, 0)                    # [d, E, N]
    F = _arr2(ph.flux(un, qn, P, np, xn), un[0])      # [f, d, E, N]
    S = _arr(ph.source(un, qn, xn, t, P, np), un[0])  # [f, E, N]
    R = np.zeros((f, E, N), dtype=u.dtype)
    for a in range(d):
        # contravariant flux G[c, e, i] = w_i sum_k Ja[e, i, a, k] F[c, k, e, i]
        G = W[None, None, :] * np.einsum("eik,ckei->cei", mesh.Ja[:, :, a, :], F)
        R += G @ ref.Dr[a]
    unodes = un.reshape(f, E * N)
    qnodes = qn.reshape(f, d, E * N)
    for fi, (a, side, nodes, wf) in enumerate(ref.faces):
        Sn = np.moveaxis(side * mesh.Ja[:, nodes, a, :], 2, 0)       # [d, E, Nf]
        Smag = np.sqrt(sum(Sn[k] ** 2 for k in range(d)))
        uin = un[:, :, nodes]
        qin = qn[:, :, :, nodes]
        Fin = F[:, :, :, nodes]
        nb = mesh.nbr[:, fi, :]
        safe = np.where(nb >= 0, nb, 0)
        uout = unodes[:, safe]
        qout = qnodes[:, :, safe]
        Xf = np.moveaxis(mesh.X[:, nodes, :], 2, 0)                  # [d, E, Nf]
        Fout = _arr2(ph.flux(uout, qout, P, np, Xf), uout[0])
        uhat = uh[fi]
        sig = _arr(ph.sigma(uhat, P, np, Xf), uhat[0])
        Fh_int = 0.5 * (_dot_n(Fin, Sn, d) + _dot_n(Fout, Sn, d)) + Smag * sig * (uin - uhat)
        # boundary versions
        ub = boundary_value(mesh, P, uin, Xf)
        Fb = _arr2(ph.flux(ub, qin, P, np, Xf), ub[0])
        sigb = _arr(ph.sigma(ub, P, np, Xf), ub[0])
        Fh_dir = _dot_n(Fb, Sn, d) + Smag * sigb * (uin - ub)
        Fi_top = _arr2(ph.flux_inviscid(uin, P, np, Xf), uin[0])
        Fh_top = _dot_n(Fi_top, Sn, d) + top_penalty(P, uin, Sn, Smag, d)
        tag = mesh.tag[:, fi][None, :, None]
        if P.get("bc_mode", 0) == 1:
            Fh = np.where(tag > 0, Fh_dir, Fh_int)
        else:
            Fh = np.where(tag == 1, Fh_dir, np.where(tag == 2, Fh_top, Fh_int))
        R[:, :, nodes] -= Fh * wf[None, None, :]
    R = R / (W[None, :] * mesh.J)[None] + S
    return np.moveaxis(R, 0, 1).copy()


def residual_terms(mesh, P, u, t=0.0):
    """R and its three parts, each [f, E, N]: the volume divergence V, the face
    contribution Fc (lifted numerical fluxes) and the source S, R = V + Fc + S (works on
    complex states as well, for the complex step)"""
    ref = mesh.ref
    d = P["d"]
    R = residual(mesh, P, u, t)
    q = gradient(mesh, P, u)
    un = np.moveaxis(u, 1, 0)
    qn = np.moveaxis(np.moveaxis(q, 1, 0), 2, 1)
    del q
    xn = np.moveaxis(mesh.X, 2, 0)
    S = _arr(ph.source(un, qn, xn, t, P, np), un[0])
    F = _arr2(ph.flux(un, qn, P, np, xn), un[0])
    del qn
    V = np.zeros_like(S)
    for a in range(d):
        G = ref.W[None, None, :] * np.einsum("eik,ckei->cei", mesh.Ja[:, :, a, :], F)
        V += G @ ref.Dr[a]
    del F
    V = V / (ref.W[None, :] * mesh.J)[None]
    Fc = np.moveaxis(R, 0, 1) - V - S
    return R, V, Fc, S


def residual_parts(mesh, P, u, t=0.0):
    """(R, term scale): the scale is |volume divergence| + |face lift| + |source| per
    node, used to express parity tolerances relative to the cancelling terms."""
    R, V, Fc, S = residual_terms(mesh, P, u, t)
    scale = np.abs(V) + np.abs(Fc) + np.abs(S)
    return R, np.moveaxis(scale, 0, 1).copy()


def conservation_terms(mesh, P, u, t=0.0):
    """(sum_i w_i J_i R_i, boundary flux + source integral) per field: equal for a
    conservative scheme since interior face fluxes are single valued."""
    ref = mesh.ref
    d = P["d"]
    q = gradient(mesh, P, u)
    R = residual(mesh, P, u, t, q=q)
    WJ = ref.W[None, :] * mesh.J
    lhs = np.einsum("ecj,ej->c", R, WJ)
    un = np.moveaxis(u, 1, 0)
    qn = np.moveaxis(np.moveaxis(q, 1, 0), 2, 1)
    xn = np.moveaxis(mesh.X, 2, 0)
    S = _arr(ph.source(un, qn, xn, t, P, np), un[0])
    rhs = np.einsum("cej,ej->c", S, WJ)
    mag = np.einsum("cej,ej->c", np.abs(S), WJ) + np.einsum("ecj,ej->c", np.abs(R), WJ)
    # boundary flux integrals
    for fi, (a, side, nodes, wf) in enumerate(ref.faces):
        tag = mesh.tag[:, fi]
        if not np.any(tag > 0):
            continue
        Sn = np.moveaxis(side * mesh.Ja[:, nodes, a, :], 2, 0)
        Smag = np.sqrt(sum(Sn[k] ** 2 for k in range(d)))
        uin = un[:, :, nodes]
        qin = qn[:, :, :, nodes]
        Xf = np.moveaxis(mesh.X[:, nodes, :], 2, 0)
        ub = boundary_value(mesh, P, uin, Xf)
        Fb = _arr2(ph.flux(ub, qin, P, np, Xf), ub[0])
        sigb = _arr(ph.sigma(ub, P, np, Xf), ub[0])
        Fh_dir = _dot_n(Fb, Sn, d) + Smag * sigb * (uin - ub)
        Fh_top = _dot_n(_arr2(ph.flux_inviscid(uin, P, np, Xf), uin[0]), Sn, d) + top_penalty(P, uin, Sn, Smag, d)
        t_ = tag[None, :, None]
        if P.get("bc_mode", 0) == 1:
            Fh = np.where(t_ > 0, Fh_dir, 0.0)
        else:
            Fh = np.where(t_ == 1, Fh_dir, np.where(t_ == 2, Fh_top, 0.0))
        rhs -= np.einsum("cem,m->c", Fh, wf)
        mag += np.einsum("cem,m->c", np.abs(Fh), wf)
    return lhs, rhs, mag


# ------------------------------------------------------------------ over-integration (1D)
def gauss_tables(ref, nq):
    """nq-point Gauss-Legendre rule on [-1, 1] and the nodal basis there: V[g, j] = l_j(x_g),
    Dg[g, j] = l_j'(x_g), and the exact reference mass matrix M[i, j] = int l_i l_j"""
    from .gll import lagrange_eval
    xg, wg = np.polynomial.legendre.leggauss(nq)
    V = lagrange_eval(ref.x1, xg)
    Dg = V @ ref.D1
    M = V.T @ (wg[:, None] * V)
    return xg, wg, V, Dg, M


def residual_overint(mesh, P, u, t=0.0, nq=None, parts=False):
    """R(u) of eq. (DGformulation) on 1D columns with the volume integrals evaluated by
    nq-point Gauss quadrature (default p + 2) and the exact mass matrix, instead of the
    collocated GLL rule: the gradient equation and the state equation are each
    M (.) = (weak volume terms) + (face terms), the fluxes and sources taken at the Gauss
    points from the interpolated u and q. The numerical trace and flux of eq. (LDG2) and
    the boundary treatment are those of `residual`, at the face points (the element's end
    nodes). Shape [E, f, N] like `residual`. With parts=True: (R, term scale), the scale
    being |volume and source part| + |face part| per node, each projected by M^-1."""
    if P["d"] != 1:
        raise ValueError("over-integration is implemented for 1D columns")
    ref = mesh.ref
    nq = ref.p + 2 if nq is None else nq
    xg, wg, V, Dg, Mr = gauss_tables(ref, nq)
    Mi = np.linalg.inv(Mr)
    E, f, N = u.shape
    Jel = mesh.J[:, 0]                              # h / 2 (affine elements)
    uh = traces(mesh, P, u)                         # u_hat on the two faces: [f, E, 1] each
    # gradient: J M q = -(u, dl/dxi) + <u_hat n, l>, exactly integrated (degree 2p - 1)
    ug = np.einsum("gj,ecj->ecg", V, u)
    rq = -np.einsum("g,gi,ecg->eci", wg, Dg, ug)
    for fi, (a, side, nodes, wf) in enumerate(ref.faces):
        rq[:, :, nodes[0]] += side * uh[fi][:, :, 0].T
    q = np.einsum("ij,ecj->eci", Mi, rq) / Jel[:, None, None]
    # state equation: J M R = (F, dl/dxi) + J (s, l) - <F_hat n, l>
    qg = np.einsum("gj,ecj->ecg", V, q)
    xq = mesh.X[:, 0, 0][:, None] + (xg[None, :] + 1.0) * Jel[:, None]     # Gauss point radii [E, nq]
    un = np.moveaxis(ug, 1, 0)                      # [f, E, nq]
    qn = np.moveaxis(qg, 1, 0)[:, None]             # [f, 1, E, nq]
    F = _arr2(ph.flux(un, qn, P, np, [xq]), un[0])[:, 0]     # [f, E, nq]
    S = _arr(ph.source(un, qn, [xq], t, P, np), un[0])        # [f, E, nq]
    rr = np.einsum("g,gi,ceg->eci", wg, Dg, F) + Jel[:, None, None] * np.einsum("g,gi,ceg->eci", wg, V, S)
    unodes = np.moveaxis(u, 1, 0).reshape(f, E * N)
    qnodes = np.moveaxis(q, 1, 0).reshape(f, E * N)
    rvol = rr.copy()
    for fi, (a, side, nodes, wf) in enumerate(ref.faces):
        j = nodes[0]
        Sn = np.full(E, float(side))                # outward normal of the face (1D)
        uin = u[:, :, j].T                          # [f, E]
        qin = q[:, :, j].T[:, None]                 # [f, 1, E]
        nb = mesh.nbr[:, fi, 0]
        safe = np.where(nb >= 0, nb, 0)
        uout, qout = unodes[:, safe], qnodes[:, safe][:, None]
        Xf = [mesh.X[:, j, 0]]
        Fin = _arr2(ph.flux(uin, qin, P, np, Xf), uin[0])[:, 0]
        Fout = _arr2(ph.flux(uout, qout, P, np, Xf), uout[0])[:, 0]
        uhat = uh[fi][:, :, 0]
        sig = _arr(ph.sigma(uhat, P, np, Xf), uhat[0])
        Fh_int = 0.5 * (Fin + Fout) * Sn + sig * (uin - uhat)
        ub = boundary_value(mesh, P, uin[:, :, None], [Xf[0][:, None]])[:, :, 0]
        Fb = _arr2(ph.flux(ub, qin, P, np, Xf), ub[0])[:, 0]
        sigb = _arr(ph.sigma(ub, P, np, Xf), ub[0])
        Fh_dir = Fb * Sn + sigb * (uin - ub)
        Fi_top = _arr2(ph.flux_inviscid(uin, P, np, Xf), uin[0])[:, 0]
        Fh_top = Fi_top * Sn + top_penalty(P, uin, [Sn], np.abs(Sn), 1)
        tag = mesh.tag[:, fi][None, :]
        if P.get("bc_mode", 0) == 1:
            Fh = np.where(tag > 0, Fh_dir, Fh_int)
        else:
            Fh = np.where(tag == 1, Fh_dir, np.where(tag == 2, Fh_top, Fh_int))
        rr[:, :, j] -= Fh.T
    R = np.einsum("ij,ecj->eci", Mi, rr) / Jel[:, None, None]
    if not parts:
        return R
    vol = np.einsum("ij,ecj->eci", Mi, rvol) / Jel[:, None, None]
    return R, np.abs(vol) + np.abs(R - vol)
