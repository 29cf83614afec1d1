"""Pin of the transformed equations: the time derivatives implied by the
nondimensional Navier-Stokes system eq. (NS1) (scaled as in section 2.5), mapped
through the change of variables u = (log rho, sqrt(rho) v, sqrt(rho) T) of
section 2.4, must equal -div F(u, grad u) + s(u, grad u) of the oracle's flux and
source (eq. fluxSWNondimensional) identically. The NS1 side is written here
independently, in primitive variables, with a constant mean mass and with the variable
composition of section 2.1.1 (c_v = sum_s chi_s / m_s varying in space, so that the
energy equation's d(c_v T)/dt + v . grad(c_v T) brings the grad c_v term)."""
import math

import numpy as np
import pytest
import sympy as sp

from oracle import physics as ph


def _params(d, mixture=False):
    P = dict(d=d, gamma=5.0 / 3.0, Gr=37.0, Pr=1.7, Fr=0.31, m=1.0, nu_r=2.0, alpha_r=0.7,
             alpha0c=0.9, lam=1.0, T_bot=1.0, r_ref=3.0,
             omega=[0.2, -0.1, 1.0] if d == 3 else [0.0, 0.0, 0.0],
             heat_amp=1.3, heat_qm=0.4, heat_rm=4.0, heat_H=0.5,
             sun_lat=0.2, sun_lon0=0.1, sun_rate=0.05, bc_mode=0, bc_state=[0] * 5)
    if mixture:
        # N2, O2, He fractions of about 0.15, 0.03, 0.03 near |r| = 4, O the balance
        P.update(composition=1, comp_a=[0.5, 0.1, 0.2, 0.05, 0.001, 0.002],
                 comp_b=[-0.3, -0.8, -0.5, -1.0, 0.4, 0.6])
    return P


def _mixture(x, P):
    """(m, conductivity weight) of the NS1 side: mass fractions of N2, O2, He from their
    two-exponential fits, O the balance; m = 1 / sum chi_s / m_s, mole fractions
    m chi_s / m_s weighting alpha = 3.6e-4 (N2, O2), 5.6e-4 (O, He) over alpha_O"""
    if not P.get("composition"):
        return P["m"], 1
    r = sp.sqrt(sum(xx ** 2 for xx in x))
    a, b = P["comp_a"], P["comp_b"]
    n2, o2, he = [a[2 * i] * sp.exp(b[2 * i] * r) + a[2 * i + 1] * sp.exp(b[2 * i + 1] * r) for i in range(3)]
    o = 1 - n2 - o2 - he
    masses = [28.0134 / 15.9994, 31.9988 / 15.9994, 4.002602 / 15.9994, 1.0]
    fr = [n2, o2, he, o]
    m = 1 / sum(c / ms for c, ms in zip(fr, masses))
    w = sum(m * c / ms * al for c, ms, al in zip(fr, masses, [3.6, 3.6, 5.6, 5.6])) / 5.6
    return m, w


def _ns1_rates(rho, v, T, x, t, P, Q):
    """d(rho)/dt, d(v)/dt, d(T)/dt from eq. (NS1), nondimensional:
    rho Dv/Dt + grad p - div(tau)/sqrt(gamma Gr) = rho a,  p = rho T/(gamma m),
    rho c_v DT/Dt + (gamma-1) rho T/m div v = Q + sqrt(gamma/Gr)/Pr div(kappa grad T)
                                               + (gamma-1) sqrt(gamma/Gr) tau : grad v"""
    d = len(x)
    g = P["gamma"]
    m, wk = _mixture(x, P)
    D = lambda f, k: sp.diff(f, x[k])
    gv = [[D(v[i], k) for k in range(d)] for i in range(d)]
    div = sum(gv[i][i] for i in range(d))
    eps = [[gv[i][k] + gv[k][i] - sp.Rational(2, 3) * (1 if i == k else 0) * div for k in range(d)]
           for i in range(d)]
    mu = sp.sqrt(T * m) + P["nu_r"] * rho
    kap = P["alpha0c"] * wk * T ** 0.69 + P["alpha_r"] * rho / m
    tau = [[mu * eps[i][k] for k in range(d)] for i in range(d)]
    p = rho * T / (g * m)
    r = sp.sqrt(sum(xx ** 2 for xx in x))
    grav = [-(P["r_ref"] / r) ** 2 * x[k] / r for k in range(d)]
    acc = [grav[k] / g for k in range(d)]
    if d == 3:
        w = P["omega"]
        wxr = [w[1] * x[2] - w[2] * x[1], w[2] * x[0] - w[0] * x[2], w[0] * x[1] - w[1] * x[0]]
        wwxr = [w[1] * wxr[2] - w[2] * wxr[1], w[2] * wxr[0] - w[0] * wxr[2], w[0] * wxr[1] - w[1] * wxr[0]]
        wxv = [w[1] * v[2] - w[2] * v[1], w[2] * v[0] - w[0] * v[2], w[0] * v[1] - w[1] * v[0]]
        acc = [acc[k] - P["Fr"] ** 2 / g * wwxr[k] - 2 * P["Fr"] / math.sqrt(g) * wxv[k] for k in range(3)]
    drho = -sum(D(rho * v[k], k) for k in range(d))
    dv = [-sum(v[k] * gv[i][k] for k in range(d))
          + (-D(p, i) + sum(D(tau[i][k], k) for k in range(d)) / math.sqrt(g * P["Gr"])) / rho + acc[i]
          for i in range(d)]
    cv = 1.0 / m
    cond = sum(D(kap * D(T, k), k) for k in range(d)) * math.sqrt(g / P["Gr"]) / P["Pr"]
    diss = (g - 1) * math.sqrt(g / P["Gr"]) * sum(tau[i][k] * gv[i][k] for i in range(d) for k in range(d))
    # rho (d(c_v T)/dt + v . grad(c_v T)) = rho c_v DT/Dt + rho T v . grad c_v (c_v steady)
    cvadv = rho * T * sum(v[k] * D(cv, k) for k in range(d))
    dT = -sum(v[k] * D(T, k) for k in range(d)) + (
        -(g - 1) * rho * T / m * div + Q + cond + diss - cvadv) / (rho * cv)
    return drho, dv, dT


@pytest.mark.parametrize("mixture", [False, True])
@pytest.mark.parametrize("d", [1, 3])
def test_transformed_equations_match_ns1(d, mixture):
    P = _params(d, mixture)
    x = sp.symbols("x0:%d" % d, real=True)
    t = sp.Symbol("t", real=True)
    # arbitrary smooth primitive fields
    if d == 1:
        rho = sp.exp(0.3 * sp.sin(1.3 * x[0]) - 0.2 * x[0])
        v = [0.2 * sp.cos(0.7 * x[0]) + 0.1]
        T = 1.2 + 0.3 * sp.sin(0.9 * x[0] + 0.4)
    else:
        rho = sp.exp(0.3 * sp.sin(x[0]) + 0.2 * sp.cos(1.1 * x[1]) - 0.15 * x[2])
        v = [0.2 * sp.cos(x[1] + 0.3 * x[2]), -0.1 * sp.sin(x[0] * x[2] * 0.4), 0.15 * sp.cos(0.8 * x[0] - x[1])]
        T = 1.1 + 0.3 * sp.sin(0.5 * x[0] + 0.7 * x[1]) * sp.cos(0.6 * x[2])
    Q = ph.heating(list(x), t, P, sp)
    drho, dv, dT = _ns1_rates(rho, v, T, list(x), t, P, Q)
    sq = sp.sqrt(rho)
    rates = [drho / rho] + [sq * dv[i] + v[i] * drho / (2 * sq) for i in range(d)] + [sq * dT + T * drho / (2 * sq)]
    # the oracle's flux form
    u = [sp.log(rho)] + [sq * vi for vi in v] + [sq * T]
    q = [[sp.diff(uc, x[k]) for k in range(d)] for uc in u]
    F = ph.flux(u, q, P, sp, list(x))
    S = ph.source(u, q, list(x), t, P, sp)
    rhs = [-sum(sp.diff(F[c][k], x[k]) for k in range(d)) + S[c] for c in range(d + 2)]
    rng = np.random.default_rng(0)
    fa = sp.lambdify(list(x) + [t], rates, "numpy")
    fb = sp.lambdify(list(x) + [t], rhs, "numpy")
    for _ in range(6):
        if d == 1:
            pt = [rng.uniform(3.5, 5.0), 0.3]
        else:
            # a day-side point (cos chi > 0 for the sun near longitude 0.1)
            pt = list(np.array([4.0, 0.5, 0.3]) + rng.uniform(-0.4, 0.4, 3)) + [0.3]
        a = np.array(fa(*pt), dtype=float)
        b = np.array(fb(*pt), dtype=float)
        scale = np.max(np.abs(a)) + 1e-300
        assert np.max(np.abs(a - b)) / scale < 1e-12, (a, b)


def test_eddy_and_molecular_laws():
    """nondimensional transport: mu = sqrt(T m) + 200 rho, kappa = alpha0 T^0.69 + 10 rho c_p"""
    P = _params(1)
    P.update(nu_r=200.0, alpha_r=10.0, alpha0c=1.0)
    mu, kap = ph.transport(1.0, 1.0, P, np)
    assert abs(mu - 201.0) < 1e-13 and abs(kap - 11.0) < 1e-13
    mu, kap = ph.transport(np.exp(-10.0), 5.0, P, np)
    assert abs(mu - (np.sqrt(5.0) + 200 * np.exp(-10.0))) < 1e-13
    assert abs(kap - (5.0 ** 0.69 + 10 * np.exp(-10.0))) < 1e-13
