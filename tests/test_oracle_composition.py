"""Pins of the oracle's variable composition (section 2.1.1, the conductivity law of
section 2.1.2, the grad c_v term of eq. fluxSWNondimensional):
  * closed forms: a pure species, an equal-mass N2/O mixture worked by hand;
  * invariants: mole fractions sum to one and their mass-weighted sum is the mean mass;
    the synthetic fits are fractions in [0, 1] with a mean mass falling with height;
  * grad c_v against a central difference of c_v;
  * reductions: a composition that does not vary with height gives the residual of the
    constant-mass model with that mass (and the conductivity scaled by the weight), pure
    oxygen gives the default model, and the EUVAC heating of constant fractions equals
    the heating of the same mixture given by mole fractions.
The transformation with a variable c_v itself is pinned against eq. (NS1) in
test_oracle_physics."""
import numpy as np
import pytest

import synth
from oracle import composition as comp
from oracle import dg as odg
from oracle import euvac
from oracle import mesh as omesh

M_N2 = 28.0134 / 15.9994


def _pure(species):
    """fits of a constant composition of one species (b = 0)"""
    a = [0.0] * 6
    if species != "O":
        a[2 * ("N2", "O2", "He").index(species)] = 1.0
    return dict(composition=1, comp_a=a, comp_b=[0.0] * 6)


@pytest.mark.parametrize("species,m,w", [("N2", M_N2, 3.6 / 5.6), ("O2", 31.9988 / 15.9994, 3.6 / 5.6),
                                         ("He", 4.002602 / 15.9994, 1.0), ("O", 1.0, 1.0)])
def test_pure_species(species, m, w):
    P = _pure(species)
    r = np.array([600.0, 620.0])
    assert np.allclose(comp.mean_mass(r, P, np), m, rtol=1e-15)
    assert np.allclose(comp.specific_heat(r, P, np), 1.0 / m, rtol=1e-15)
    assert np.allclose(comp.conductivity_weight(r, P, np), w, rtol=1e-15)
    assert np.allclose(comp.mole_fractions(r, P, np)[species], 1.0, rtol=1e-15)


def test_equal_mass_nitrogen_and_oxygen():
    """chi_N2 = chi_O = 1/2: m = 2 / (1/m_N2 + 1) = 1.272966046, x_N2 = m / (2 m_N2) =
    0.363516977, weight (0.363517 * 3.6 + 0.636483 * 5.6) / 5.6 = 0.870172508"""
    P = dict(composition=1, comp_a=[0.5, 0, 0, 0, 0, 0], comp_b=[0.0] * 6)
    r = 610.0
    assert abs(comp.mean_mass(r, P, np) - 1.272966046) < 1e-9
    assert abs(comp.mole_fractions(r, P, np)["N2"] - 0.363516977) < 1e-9
    assert abs(comp.conductivity_weight(r, P, np) - 0.870172508) < 1e-9


def test_synthetic_fits_are_a_mixture():
    P = synth.composition_physics()
    r = np.linspace(synth.R_BOT, synth.R_TOP, 401)
    chi = comp.mass_fractions(r, P, np)
    for s in comp.SPECIES:
        assert np.all(chi[s] >= 0) and np.all(chi[s] <= 1), s
    m = comp.mean_mass(r, P, np)
    assert np.all(np.diff(m) < 0)
    assert 28.0 < m[0] * 15.9994 < 29.0 and 14.0 < m[-1] * 15.9994 < 15.0
    x = comp.mole_fractions(r, P, np)
    assert np.allclose(sum(x.values()), 1.0, rtol=0, atol=1e-14)
    assert np.allclose(sum(x[s] * comp.MASS[s] for s in comp.SPECIES), m, rtol=1e-14)
    # the input generator's rest state uses the same mixture
    assert np.allclose(synth.mixture_mass(P)(r), m, rtol=1e-14)


def test_grad_specific_heat_by_central_difference():
    P = synth.composition_physics()
    x = [np.array([350.0, -100.0]), np.array([200.0, 580.0]), np.array([400.0, 90.0])]
    g = comp.grad_specific_heat(x, P, np)
    h = 1e-4
    for k in range(3):
        xp_ = [xx.copy() for xx in x]
        xm_ = [xx.copy() for xx in x]
        xp_[k] += h
        xm_[k] -= h
        rp = np.sqrt(sum(xx * xx for xx in xp_))
        rm = np.sqrt(sum(xx * xx for xx in xm_))
        fd = (comp.specific_heat(rp, P, np) - comp.specific_heat(rm, P, np)) / (2 * h)
        assert np.allclose(g[k], fd, rtol=1e-6, atol=1e-12)


def _column(P, T_inf=900.0, mass=None):
    om = omesh.columns_mesh([5], 3, synth.R_BOT, synth.R_TOP, 1.1)
    u = np.moveaxis(synth.column_state(om.X[:, :, 0], T_inf, mass), 0, 1).copy()
    u[:, 1] += 0.01 * np.sin(om.X[:, :, 0])          # some motion, so every term is live
    return om, u


def test_constant_composition_reduces_to_constant_mass():
    base = synth.base_physics(1)
    base.update(synth.chapman_params(900.0, 200.0, 1.0))
    fits = dict(composition=1, comp_a=[0.3, 0.1, 0.05, 0.05, 0.01, 0.0], comp_b=[0.0] * 6)
    Pc = dict(base, **fits)
    r0 = 600.0
    m = comp.mean_mass(r0, Pc, np)
    w = comp.conductivity_weight(r0, Pc, np)
    Pm = dict(base, m=m, alpha0c=base["alpha0c"] * w)
    om, u = _column(Pc)
    R1 = odg.residual(om, Pc, u, 0.2)
    R2 = odg.residual(om, Pm, u, 0.2)
    assert np.max(np.abs(R1 - R2)) / np.max(np.abs(R2)) < 1e-13


def test_pure_oxygen_is_the_default_model():
    base = synth.base_physics(1)
    om, u = _column(base)
    R1 = odg.residual(om, dict(base, **_pure("O")), u, 0.0)
    R2 = odg.residual(om, base, u, 0.0)
    assert np.max(np.abs(R1 - R2)) / np.max(np.abs(R2)) < 1e-14


def test_variable_composition_changes_the_residual_where_it_should():
    """with the synthetic fits the continuity row is unchanged (it has no m) and the
    momentum and energy rows change"""
    base = synth.base_physics(1)
    Pc = dict(base, **synth.composition_physics())
    om, u = _column(Pc, mass=synth.mixture_mass(Pc))
    R1 = odg.residual(om, Pc, u, 0.0)
    R2 = odg.residual(om, base, u, 0.0)
    assert np.max(np.abs(R1[:, 0] - R2[:, 0])) == 0.0
    assert np.max(np.abs(R1[:, 1] - R2[:, 1])) > 1e-3 * np.max(np.abs(R2[:, 1]))
    assert np.max(np.abs(R1[:, 2] - R2[:, 2])) > 1e-3 * np.max(np.abs(R2[:, 2]))


def test_euvac_number_densities_of_constant_fractions():
    """constant mass fractions chi_s heat exactly as the constant-mass model with the
    mixture's m and the mole fractions x_s = m chi_s / m_s"""
    P = synth.base_physics(1)
    P.update(synth.euvac_physics(f107bar=120.0))
    P["heating_model"] = 1
    fits = dict(composition=1, comp_a=[0.4, 0.0, 0.1, 0.0, 0.02, 0.0], comp_b=[0.0] * 6)
    Pc = dict(P, **fits)
    r = np.linspace(synth.R_BOT, synth.R_TOP, 50)
    rho = np.exp(-(r - synth.R_BOT) / 2.0)
    T = 1.0 + 0.05 * (r - synth.R_BOT)
    m = comp.mean_mass(r[0], Pc, np)
    x = comp.mole_fractions(r[0], Pc, np)
    Pm = dict(P, m=m, euv_chi=[x[s] for s in comp.SPECIES])
    Q1 = euvac.heating([r], 0.0, rho, T, Pc)
    Q2 = euvac.heating([r], 0.0, rho, T, Pm)
    assert np.max(np.abs(Q1 - Q2)) / np.max(np.abs(Q2)) < 1e-13
    assert np.max(Q2) > 0
