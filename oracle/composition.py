"""Chemically frozen mixture of N2, O2, O and He (section 2.1.1, with the conductivity law
of section 2.1.2 and the nondimensional form of section 2.5).

Test infrastructure only: the tests call it, the product path never does.

The mass fractions chi_s = rho_s / rho are known functions of the radius: for N2, O2 and
He a sum of two exponentials chi_s = sum_j a_j^s exp(b_j^s |r|) (fit coefficients are
inputs; the MSIS fits themselves are not available), and atomic oxygen closes the sum to
one. From them, in units of the oxygen mass m_O:
  * specific heat  c_v = sum_s chi_s c_v,s = sum_s chi_s / m_s  (every species with the
    same gamma, so c_v,s = 1 / m_s in units of c_v of oxygen);
  * mean molecular mass  m = 1 / sum_s (chi_s / m_s) = 1 / c_v;
  * mole fractions  x_s = n_s / sum_k n_k = m chi_s / m_s;
  * the molecular conductivity's species weighting sum_s x_s alpha_s, divided by
    alpha_O (the conductivity scale kappa_0 is that of atomic oxygen at T_0, as the mass
    scale is m_O);
  * grad c_v = (sum_s chi_s'(|r|) / m_s) r / |r|, the derivative of the fits.
Functions take a math namespace `xp` (numpy, or sympy for the symbolic checks).
"""
import numpy as np

SPECIES = ("N2", "O2", "O", "He")          # the order of Table A's cross sections
FITTED = ("N2", "O2", "He")                # the fitted fractions; O closes the sum
# molecular masses in units of m_O (standard atomic weights)
MASS = {"N2": 28.0134 / 15.9994, "O2": 31.9988 / 15.9994, "O": 1.0, "He": 4.002602 / 15.9994}
# conductivity coefficients alpha_s of section 2.1.2 (SI)
ALPHA = {"N2": 3.6e-4, "O2": 3.6e-4, "O": 5.6e-4, "He": 5.6e-4}


def enabled(P):
    return bool(P.get("composition", 0))


def _radius(x, xp):
    return xp.sqrt(sum(xk * xk for xk in x))


def fit_terms(P, s):
    """((a_1, b_1), (a_2, b_2)) of fitted species s; P["comp_a"], P["comp_b"] hold them
    in the order N2 (j = 1, 2), O2 (j = 1, 2), He (j = 1, 2)"""
    i = FITTED.index(s)
    return [(P["comp_a"][2 * i + j], P["comp_b"][2 * i + j]) for j in range(2)]


def mass_fractions(r, P, xp):
    """{species: chi_s} at radius r"""
    chi = {}
    for s in FITTED:
        chi[s] = sum(a * xp.exp(b * r) for a, b in fit_terms(P, s))
    chi["O"] = 1.0 - chi["N2"] - chi["O2"] - chi["He"]
    return chi


def mass_fraction_slopes(r, P, xp):
    """{species: d chi_s / d|r|}"""
    d = {}
    for s in FITTED:
        d[s] = sum(a * b * xp.exp(b * r) for a, b in fit_terms(P, s))
    d["O"] = -(d["N2"] + d["O2"] + d["He"])
    return d


def specific_heat(r, P, xp):
    """c_v(r) (units of c_v of oxygen)"""
    chi = mass_fractions(r, P, xp)
    return sum(chi[s] / MASS[s] for s in SPECIES)


def mean_mass(r, P, xp):
    """m(r) = [sum_s chi_s / m_s]^-1 (units of m_O)"""
    return 1.0 / specific_heat(r, P, xp)


def mole_fractions(r, P, xp):
    m = mean_mass(r, P, xp)
    chi = mass_fractions(r, P, xp)
    return {s: m * chi[s] / MASS[s] for s in SPECIES}


def conductivity_weight(r, P, xp):
    """sum_s x_s alpha_s / alpha_O"""
    x = mole_fractions(r, P, xp)
    return sum(x[s] * ALPHA[s] for s in SPECIES) / ALPHA["O"]


def grad_specific_heat(x, P, xp):
    """grad c_v at the point x (list of d coordinates)"""
    r = _radius(x, xp)
    d = mass_fraction_slopes(r, P, xp)
    dcv = sum(d[s] / MASS[s] for s in SPECIES)
    return [dcv * xk / r for xk in x]


def at(x, P, xp):
    """(m, conductivity weight) at x; the constant model (m = P["m"], weight 1) when the
    composition is off"""
    if not enabled(P):
        return P["m"], 1.0
    r = _radius(x, xp)
    return mean_mass(r, P, xp), conductivity_weight(r, P, xp)
