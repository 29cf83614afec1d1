"""Implicit time stepping: DIRK stages solved by Newton (eq. NewtonSolve).

DIRK(3,3) and DIRK(2,2) are Alexander's L-stable, stiffly accurate singly-diagonal
schemes (cited in section 3.1; the tableaux are not printed in the paper and are
restated here from their defining order conditions):
  DIRK(2,2): g = 1 - 1/sqrt(2); A = [[g, 0], [1-g, g]]; c = (g, 1)
  DIRK(3,3): g the root in (1/6, 1/2) of g^3 - 3 g^2 + 3/2 g - 1/6 = 0;
             c = (g, (1+g)/2, 1); a21 = (1-g)/2;
             b1 = -(6g^2 - 16g + 1)/4, b2 = (6g^2 - 20g + 5)/4, b3 = g.
Stage i solves G_i(U) = U - dt a_ii R(U, t + c_i dt) - b_i = 0 with
b_i = u_n + dt sum_{j<i} a_ij R(U_j, t + c_j dt); u_{n+1} = U_last.

The exact stage solution used for parity is a dense Newton (numpy LU on the
complex-step Jacobian) iterated to a residual of 1e-13 relative to |G(u_n)|.

Optional modal filter (not part of the paper's method): after a step, the
coefficient of the degree-p Legendre polynomial of every element, in every
direction, is multiplied by sigma = exp(-filter_rate dt); filter_rate = 0 is the
plain DIRK step.
"""
import numpy as np

from . import dg, jac


def dirk_tableau(scheme):
    if scheme == 22:
        g = 1.0 - 1.0 / np.sqrt(2.0)
        A = np.array([[g, 0.0], [1.0 - g, g]])
        return A, A[-1].copy(), np.array([g, 1.0])
    if scheme == 33:
        roots = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
        g = float(np.real([r for r in roots if abs(r.imag) < 1e-12 and 1 / 6 < r.real < 0.5][0]))
        a21 = 0.5 * (1.0 - g)
        b1 = -(6 * g * g - 16 * g + 1) / 4.0
        b2 = (6 * g * g - 20 * g + 5) / 4.0
        A = np.array([[g, 0, 0], [a21, g, 0], [b1, b2, g]])
        return A, A[-1].copy(), np.array([g, 0.5 * (1 + g), 1.0])
    raise ValueError(scheme)


def newton_dense(Gfun, Jfun, U0, ref_norm, rtol=1e-13, maxit=30):
    """Newton to |G| <= rtol |G(u_n)|; an iterate whose residual has stopped falling
    (the round-off floor of the residual evaluation) is accepted once it is below
    1e-10 |G(u_n)|"""
    U = U0.copy()
    hist = []
    for it in range(maxit):
        G = Gfun(U)
        nG = np.linalg.norm(G)
        hist.append(nG)
        if nG <= rtol * ref_norm:
            return U, it, hist
        if len(hist) >= 3 and nG > 0.5 * hist[-2] and nG <= 1e-10 * ref_norm:
            return U, it, hist
        Jm = Jfun(U)
        U = U - np.linalg.solve(Jm, G.ravel()).reshape(U.shape)
    raise RuntimeError("dense Newton did not converge: %s" % hist[-5:])


def filter_matrix(x, p, sigma):
    """1D nodal filter on the points x: to Legendre coefficients (Vandermonde inverse),
    scale the degree-p coefficient by sigma, back to nodal values"""
    V = np.polynomial.legendre.legvander(x, p)
    return V @ np.diag(np.r_[np.ones(p), sigma]) @ np.linalg.inv(V)


def modal_filter(mesh, u, sigma):
    """the tensor-product filter applied to every element of u [E, f, N]"""
    ref = mesh.ref
    F1 = filter_matrix(ref.x1, ref.p, sigma)
    n, d = ref.n, mesh.d
    v = u.reshape(u.shape[:2] + (n,) * d)          # node index a + n b + n^2 c -> axes (c, b, a)
    for ax in range(d):
        v = np.moveaxis(np.tensordot(v, F1, axes=([2 + ax], [1])), -1, 2 + ax)
    return v.reshape(u.shape)


def implicit_step_dense(mesh, P, u, t, dt, scheme=33, rtol=1e-13, guesses=None, filter_rate=0.0, residual=None):
    """one DIRK step with every stage solved by dense Newton, then the optional modal
    filter. residual: the spatial residual (dg.residual, collocated, by default).
    Returns (u_new, stages)."""
    residual = dg.residual if residual is None else residual
    A, b, c = dirk_tableau(scheme)
    s = len(c)
    Rs, Us = [], []
    for i in range(s):
        ti = t + c[i] * dt
        bi = u + dt * sum(A[i, j] * Rs[j] for j in range(i))
        aii = A[i, i]
        G = lambda U: U - dt * aii * residual(mesh, P, U, ti) - bi
        Jf = lambda U: np.eye(U.size) - dt * aii * jac.dense_jacobian(mesh, P, U, ti, residual=residual)
        ref = np.linalg.norm(G(u))
        U0 = u if guesses is None else guesses[i]
        Ui, _, _ = newton_dense(G, Jf, U0, ref, rtol)
        Us.append(Ui)
        Rs.append(residual(mesh, P, Ui, ti))
    un = modal_filter(mesh, Us[-1], np.exp(-filter_rate * dt)) if filter_rate > 0 else Us[-1]
    return un, Us


def gmres(Aop, rhs, x0=None, m=30, rtol=1e-10, max_restarts=50, M=None):
    """right-preconditioned restarted GMRES(m) with classical Gram-Schmidt applied
    twice (CGS2) and Givens rotations. Aop, M: callables on flat vectors."""
    n = rhs.size
    x = np.zeros(n) if x0 is None else x0.copy()
    Mf = (lambda z: z) if M is None else M
    bnorm = np.linalg.norm(rhs)
    total = 0
    for _ in range(max_restarts):
        r = rhs - Aop(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm:
            return x, total
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        V[0] = r / beta
        g = np.zeros(m + 1)
        g[0] = beta
        cs, sn = np.zeros(m), np.zeros(m)
        k_used = 0
        for j in range(m):
            w = Aop(Mf(V[j]))
            h = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h
            h2 = V[: j + 1] @ w
            w = w - V[: j + 1].T @ h2
            h = h + h2
            H[: j + 1, j] = h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t0 = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t0
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k_used = j + 1
            if abs(g[j + 1]) <= rtol * bnorm:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + Mf(V[:k_used].T @ y)
    return x, total


def newton_jfnk(mesh, P, Gfun, U0, ti, aii_dt, ref_norm, rtol=1e-12, maxit=40, gmres_rtol=1e-12, M=None):
    """Newton with matrix-free GMRES on complex-step products (for meshes too large for
    the dense Jacobian); same stage equation and stopping rule as newton_dense. A Newton
    step whose residual is not finite or has not fallen is halved (up to 12 times): large
    steps (dt = 60 s from the step's start state) can otherwise leave the physical states
    (negative temperature). The damping changes the path, not the solution G(U) = 0, and so
    does the optional right preconditioner M of GMRES (a callable on flat vectors)."""
    from . import jac
    U = U0.copy()
    G = Gfun(U)
    nG = np.linalg.norm(G)
    prev = np.inf
    for it in range(maxit):
        if nG <= rtol * ref_norm or (nG > 0.5 * prev and nG <= 1e-10 * ref_norm):
            return U, it
        prev = nG
        Aop = lambda v: v - aii_dt * jac.jvp_complex(mesh, P, U, v.reshape(U.shape), ti).ravel()
        dx, _ = gmres(Aop, -G.ravel(), m=60, rtol=gmres_rtol, max_restarts=200, M=M)
        dx = dx.reshape(U.shape)
        lam = 1.0
        for _ in range(13):
            with np.errstate(invalid="ignore", over="ignore"):
                Gt = Gfun(U + lam * dx)
            nt = np.linalg.norm(Gt)
            if np.isfinite(nt) and (nt < nG or lam == 1.0 and nG <= 1e-10 * ref_norm):
                break
            lam *= 0.5
        else:
            if nG <= 1e-10 * ref_norm:       # the round-off floor of the residual evaluation
                return U, it
            raise RuntimeError("JFNK Newton: no step lowers the residual")
        U = U + lam * dx
        G, nG = Gt, nt
    raise RuntimeError("JFNK Newton did not converge")


def implicit_step_jfnk(mesh, P, u, t, dt, scheme=33, rtol=1e-12, filter_rate=0.0, M=None):
    """one DIRK step with every stage solved by matrix-free Newton-GMRES to rtol, then
    the optional modal filter; M: optional right preconditioner of every GMRES solve (it
    steers the iterations only)"""
    A, b, c = dirk_tableau(scheme)
    Rs, Us = [], []
    for i in range(len(c)):
        ti = t + c[i] * dt
        bi = u + dt * sum(A[i, j] * Rs[j] for j in range(i))
        aii = A[i, i]
        G = lambda U: U - dt * aii * dg.residual(mesh, P, U, ti) - bi
        Ui, _ = newton_jfnk(mesh, P, G, u, ti, dt * aii, np.linalg.norm(G(u)), rtol, M=M)
        Us.append(Ui)
        Rs.append(dg.residual(mesh, P, Ui, ti))
    un = modal_filter(mesh, Us[-1], np.exp(-filter_rate * dt)) if filter_rate > 0 else Us[-1]
    return un, Us
