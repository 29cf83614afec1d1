"""Pointwise physics of the nondimensional thermosphere model.

State u = (varrho, U, Theta) with varrho = log(rho/rho0), U = sqrt(rho) v (d components)
and Theta = sqrt(rho) T (section 2.4). Fluxes and sources follow eq.
(fluxSWNondimensional); the acceleration follows the nondimensional form given right
after it (gravity / gamma, centripetal Fr^2/gamma, Coriolis 2 Fr/sqrt(gamma)); the
transport coefficients are the molecular + eddy laws of section 2.1.2 normalised by
their lower-boundary values: mu = sqrt(T m) + nu_r rho, kappa = alpha0c w T^0.69 +
alpha_r rho c_p, with c_v = c_p = 1/m. The mean molecular mass m is either a constant
(P["m"]; the conductivity's species weight w = 1 and the grad(c_v) source term vanishes)
or, with P["composition"], the chemically frozen mixture of section 2.1.1
(composition.py): m(r) and w(r) from the fitted mass fractions, and the energy equation
carries -(1/c_v)(Theta v - conductive flux) . grad c_v. Quantities that depend on m take
the node positions x.

Every function takes plain component lists and a math namespace `xp` (numpy for
numbers, including complex numbers for the complex step; sympy for the symbolic
check of the transformation from eq. (NS1)).
"""
import numpy as np

from . import composition


def mixture(P, xp, x):
    """(m, conductivity weight) at the points x (list of d coordinate arrays)"""
    if composition.enabled(P) and x is None:
        raise ValueError("the variable composition needs the node positions")
    return composition.at(x, P, xp) if x is not None else (P["m"], 1.0)


def _consts(P, xp, m):
    g = P["gamma"]
    return dict(
        inv_gm=1.0 / (g * m),
        c_visc=1.0 / xp.sqrt(g * P["Gr"]),
        c_cond=(1.0 / P["Pr"]) * xp.sqrt(g / P["Gr"]),
        c_diss=(g - 1.0) * xp.sqrt(g / P["Gr"]),
    )


def primitives(u, P, xp):
    d = P["d"]
    lr = u[0]
    U = [u[1 + i] for i in range(d)]
    Th = u[1 + d]
    rho = xp.exp(lr)
    s = xp.exp(-0.5 * lr)          # 1/sqrt(rho)
    v = [s * Ui for Ui in U]
    T = s * Th
    return lr, U, Th, rho, s, v, T


def transport(rho, T, P, xp, x=None):
    m, w = mixture(P, xp, x)
    mu = xp.sqrt(T * m) + P["nu_r"] * rho
    kap = P["alpha0c"] * w * T ** P.get("kappa_exp", 0.69) + P["alpha_r"] * rho * (1.0 / m)
    return mu, kap


def gradients(u, q, P, xp):
    """velocity gradient gv[i][k] = d v_i / d x_k and temperature gradient gT[k]
    recovered from the auxiliary variable q = grad u."""
    d = P["d"]
    lr, U, Th, rho, s, v, T = primitives(u, P, xp)
    gl = [q[0][k] for k in range(d)]
    gv = [[s * (q[1 + i][k] - 0.5 * U[i] * gl[k]) for k in range(d)] for i in range(d)]
    gT = [s * (q[1 + d][k] - 0.5 * Th * gl[k]) for k in range(d)]
    return gl, gv, gT


def strain(gv, d):
    div = sum(gv[i][i] for i in range(d))
    eps = [[gv[i][k] + gv[k][i] - (2.0 / 3.0 if i == k else 0.0) * div for k in range(d)] for i in range(d)]
    return eps, div


def flux_inviscid(u, P, xp, x=None):
    d = P["d"]
    C = _consts(P, xp, mixture(P, xp, x)[0])
    lr, U, Th, rho, s, v, T = primitives(u, P, xp)
    F = [[lr * v[k] for k in range(d)]]
    for i in range(d):
        F.append([U[i] * v[k] + (C["inv_gm"] * Th if i == k else 0.0) for k in range(d)])
    F.append([Th * v[k] for k in range(d)])
    return F


def flux_viscous(u, q, P, xp, x=None):
    """the diffusive part of F, returned with the sign it has inside F"""
    d = P["d"]
    m = mixture(P, xp, x)[0]
    C = _consts(P, xp, m)
    lr, U, Th, rho, s, v, T = primitives(u, P, xp)
    mu, kap = transport(rho, T, P, xp, x)
    gl, gv, gT = gradients(u, q, P, xp)
    eps, div = strain(gv, d)
    F = [[0.0 * lr for k in range(d)]]
    for i in range(d):
        F.append([-C["c_visc"] * mu * s * eps[i][k] for k in range(d)])
    F.append([-C["c_cond"] * kap * s * m * gT[k] for k in range(d)])
    return F


def flux(u, q, P, xp, x=None):
    Fi = flux_inviscid(u, P, xp, x)
    Fv = flux_viscous(u, q, P, xp, x)
    return [[Fi[c][k] + Fv[c][k] for k in range(P["d"])] for c in range(P["d"] + 2)]


def sun_unit(t, P):
    """sub-solar unit vector at nondimensional time t: latitude sun_lat, longitude
    sun_lon0 - sun_rate t (the Sun's apparent motion in the Earth-fixed frame)"""
    lon = P["sun_lon0"] - P["sun_rate"] * t
    lat = P["sun_lat"]
    return [np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)]


def column_cos_zenith(t, P):
    """cos chi of a 1D column: the Sun overhead, or, with P["site"] (unit vector of the
    column's Earth-fixed site), site . sub-solar direction (section 2.2: from the
    declination, the latitude and the local time)"""
    site = P.get("site")
    if site is None or not any(site):
        return 1.0
    sh = sun_unit(t, P)
    return float(sum(site[k] * sh[k] for k in range(3)))


def heating(x, t, P, xp):
    """prescribed Chapman-shaped EUV heating rate Q(x, t) (nondimensional, W/m^3 over
    rho0 c_vO T0 a0/H0): Q = amp qm exp(1 - z - e^{-z}/cos chi) on the day side,
    z = (|r| - rm)/H, zero where cos chi <= 0; 1D columns take cos chi from their site
    (column_cos_zenith: 1 without a site).
    The solar zenith angle follows section 2.2: cos chi = r_hat . s_hat(t), the
    sub-solar point moving in longitude at the nondimensional rotation rate."""
    d = P["d"]
    r = xp.sqrt(sum(x[k] * x[k] for k in range(d)))
    if d == 3:
        lon = P["sun_lon0"] - P["sun_rate"] * t
        lat = P["sun_lat"]
        sh = [xp.cos(lat) * xp.cos(lon), xp.cos(lat) * xp.sin(lon), xp.sin(lat)]
        cchi = sum(x[k] * sh[k] for k in range(3)) / r
    else:
        cchi = column_cos_zenith(t, P) + 0.0 * r
    z = (r - P["heat_rm"]) / P["heat_H"]
    if xp is np:
        cchi = np.asarray(cchi, dtype=np.float64)
        day = cchi > 0
        safe = np.where(day, cchi, 1.0)
        Q = P["heat_amp"] * P["heat_qm"] * np.exp(1.0 - z - np.exp(-z) / safe)
        return np.where(day, Q, 0.0)
    return P["heat_amp"] * P["heat_qm"] * xp.exp(1 - z - xp.exp(-z) / cchi)


def acceleration_times_sqrt_rho(u, x, P, xp):
    """sqrt(rho) a with a = g/gamma - Fr^2/gamma w x (w x r) - 2 Fr/sqrt(gamma) w x v,
    g = -(r_ref/|r|)^2 r_hat (gravity normalised at the lower boundary)."""
    d = P["d"]
    g = P["gamma"]
    lr, U, Th, rho, s, v, T = primitives(u, P, xp)
    sq = xp.exp(0.5 * lr)
    r2 = sum(x[k] * x[k] for k in range(d))
    r3 = r2 * xp.sqrt(r2)
    out = [sq * (-(P["r_ref"] ** 2) * x[k] / r3) / g for k in range(d)]
    if d == 3:
        w = P["omega"]
        wr = sum(w[k] * x[k] for k in range(3))
        ww = sum(w[k] * w[k] for k in range(3))
        wwr = [w[k] * wr - ww * x[k] for k in range(3)]             # w x (w x r)
        wU = [w[1] * U[2] - w[2] * U[1], w[2] * U[0] - w[0] * U[2], w[0] * U[1] - w[1] * U[0]]
        Fr = P["Fr"]
        for k in range(3):
            out[k] = out[k] - sq * (Fr ** 2 / g) * wwr[k] - (2.0 * Fr / xp.sqrt(g)) * wU[k]
    return out


def source(u, q, x, t, P, xp):
    d = P["d"]
    g = P["gamma"]
    m = mixture(P, xp, x)[0]
    C = _consts(P, xp, m)
    lr, U, Th, rho, s, v, T = primitives(u, P, xp)
    mu, kap = transport(rho, T, P, xp, x)
    gl, gv, gT = gradients(u, q, P, xp)
    eps, div = strain(gv, d)
    S = [(lr - 1.0) * div]
    acc = acceleration_times_sqrt_rho(u, x, P, xp)
    for i in range(d):
        eg = sum(eps[i][k] * gl[k] for k in range(d))
        S.append(acc[i] + 0.5 * div * U[i] - 0.5 * C["inv_gm"] * Th * gl[i]
                 + 0.5 * C["c_visc"] * mu * s * eg)
    if P.get("heating_model", 0) == 1:
        from . import euvac
        Q = euvac.heating(x, t, rho, T, P)
    else:
        Q = heating(x, t, P, xp)
    Tg = sum(gT[k] * gl[k] for k in range(d))
    ed = sum(eps[i][k] * gv[i][k] for i in range(d) for k in range(d))
    Se = Q * s * m + (1.5 - g) * Th * div + 0.5 * C["c_cond"] * kap * s * m * Tg + C["c_diss"] * mu * s * m * ed
    if composition.enabled(P):
        # -(1/c_v) (Theta v - sqrt(gamma/Gr)/Pr kappa/(sqrt(rho) c_v) grad T) . grad c_v
        r = xp.sqrt(sum(x[k] * x[k] for k in range(d)))
        cv = composition.specific_heat(r, P, xp)
        gcv = composition.grad_specific_heat(x, P, xp)
        Se = Se - sum((Th * v[k] - C["c_cond"] * kap * s / cv * gT[k]) * gcv[k] for k in range(d)) / cv
    S.append(Se)
    return S


def sigma(uhat, P, xp, x=None):
    """stabilisation of eq. (LDG2): sigma_c = lambda_max I plus the diffusive block
    diag(0, mu/(sqrt(rho) sqrt(gamma Gr)) I_d, kappa/(Pr sqrt(rho) c_v) sqrt(gamma/Gr)),
    evaluated at the numerical trace."""
    d = P["d"]
    m = mixture(P, xp, x)[0]
    C = _consts(P, xp, m)
    lr, U, Th, rho, s, v, T = primitives(uhat, P, xp)
    mu, kap = transport(rho, T, P, xp, x)
    lam = P["lam"]
    sig = [lam + 0.0 * lr]
    for i in range(d):
        sig.append(lam + C["c_visc"] * mu * s)
    sig.append(lam + C["c_cond"] * kap * s * m)
    return sig


def bottom_state(u, P, xp):
    """lower boundary (section 2.3): no slip, isothermal T = T_bot, log-density from the interior"""
    d = P["d"]
    lr = u[0]
    return [lr] + [0.0 * lr for _ in range(d)] + [P["T_bot"] * xp.exp(0.5 * lr)]
