"""EUVAC solar EUV heating (section 2.2, Table A of the appendix on EUV cross sections).

Test infrastructure only: the tests call it, the product path never does.

Q = eps sum_s n_s sum_j phi_s^j I^j hc/lambda_j, with I_0^j = F74113^j max(0.8, 1 + A_j
(F10.7bar - 80)) / d^2 the EUVAC flux and the attenuation exp(-tau^j) by the optical depth
along the path to the Sun, tau_s^j = N_s^j C(r~, chi) with N_s^j = n_s phi_s^j H, H = k T /
(m g), r~ = |r| / H, y = sqrt(r~/2) |cos chi| and the Smith-Smith form of the Chapman
function for an exponential (isothermal, constant-mixture) atmosphere:
  C = sqrt(pi r~/2) exp(y^2) erfc(y)                                  cos chi > 0
  C = sqrt(pi r~/2) [2 exp(r~ (1 - |sin chi|)) - exp(y^2) erfc(y)]   cos chi <= 0, |sin chi| > R0/|r|
  C = infinity (no flux)                                              otherwise (Earth's shadow).
The solar zenith angle comes from the declination (section 2.2's approximation from the
day of the year) and the local time; here the sub-solar point is a latitude (the
declination) and a longitude moving at the rotation rate, as for the prescribed heating.

Readings (the paper is silent or ambiguous):
  * composition: with the constant mean mass, constant mole fractions chi_s of N2, O2,
    O, He (P["euv_chi"]), n_s = chi_s n with n = rho / m-bar; with the variable
    composition (P["composition"], composition.py), the number densities of the fitted
    mass fractions, n_s = rho chi_s(r) / m_s, and H with the mixture's m(r);
  * one attenuation per bin by the total optical depth tau^j = sum_s tau_s^j (the
    formula's per-species index on I is read as the usual total column);
  * Table A's photon fluxes carry the exponent +13 (m^-2 s^-1), its cross sections
    1e-22 m^2; a wavelength range stands for its midpoint in hc/lambda;
  * exp(y^2) erfc(y) is evaluated as the scaled function erfcx(y).

Nondimensional form used by the model: with rho and T in units of rho0 and T0, lengths in
H0, H = T |r|^2 / (m r_ref^2) and
  Q = rho sum_j K_j exp(-kappa_j rho H C),
  K_j = eps (hc/lambda_j) I_0^j sigma_j (rho0 / (m m_O)) / Q_unit,
  kappa_j = sigma_j rho0 H0 / (m m_O),   sigma_j = sum_s chi_s phi_s^j.
P carries q_scale = rho0 / (m_O Q_unit) and col_scale = rho0 H0 / m_O. With the variable
composition sigma_j / m becomes sum_s (chi_s(r) / m_s) phi_s^j at every node.
"""
import numpy as np
from scipy.special import erfcx

from . import composition

H_PLANCK = 6.62607015e-34
C_LIGHT = 2.99792458e8

# Table A: bin, F74113 (1e13 m^-2 s^-1), A, cross sections of N2, O2, O, He (1e-22 m^2)
TABLE_A = [
    ("50-100", 1.200, 0.0100, 0.720, 1.316, 0.730, 0.144),
    ("100-150", 0.450, 0.0071, 2.261, 3.806, 1.839, 0.479),
    ("150-200", 4.800, 0.0134, 4.958, 7.509, 3.732, 1.157),
    ("200-250", 3.100, 0.0195, 8.392, 10.900, 5.202, 1.601),
    ("256.3", 0.460, 0.0028, 10.210, 13.370, 6.050, 2.121),
    ("284.15", 0.210, 0.1380, 10.900, 15.790, 7.080, 2.595),
    ("250-300", 1.679, 0.0265, 10.493, 14.387, 6.461, 2.321),
    ("303.31", 0.800, 0.0250, 11.670, 16.800, 7.680, 2.953),
    ("303.78", 6.900, 0.0033, 11.700, 16.810, 7.700, 2.962),
    ("300-350", 0.965, 0.0225, 13.857, 17.438, 8.693, 3.544),
    ("368.07", 0.650, 0.0066, 16.910, 18.320, 9.840, 4.268),
    ("350-400", 0.314, 0.0365, 16.395, 18.118, 9.687, 4.142),
    ("400-450", 0.383, 0.0074, 21.675, 20.310, 11.496, 5.447),
    ("465.22", 0.290, 0.0075, 23.160, 21.910, 11.930, 6.563),
    ("450-500", 0.285, 0.0202, 23.471, 23.101, 12.127, 7.208),
    ("500-550", 0.452, 0.0088, 24.501, 24.606, 12.059, 0.958),
    ("554.37", 0.720, 0.0033, 24.130, 26.040, 12.590, 0.0),
    ("584.33", 1.270, 0.0052, 22.400, 22.720, 13.090, 0.0),
    ("550-600", 0.357, 0.0037, 22.787, 26.610, 13.024, 0.0),
    ("609.76", 0.530, 0.0162, 22.790, 28.070, 13.400, 0.0),
    ("629.73", 1.590, 0.0033, 23.370, 32.060, 13.400, 0.0),
    ("600-650", 0.342, 0.0118, 23.339, 26.017, 13.365, 0.0),
    ("650-700", 0.230, 0.0043, 31.755, 21.919, 17.245, 0.0),
    ("703.31", 0.360, 0.0030, 26.540, 27.440, 11.460, 0.0),
    ("700-750", 0.141, 0.0047, 24.662, 28.535, 10.736, 0.0),
    ("765.15", 0.170, 0.0039, 120.490, 20.800, 4.000, 0.0),
    ("770.41", 0.260, 0.0128, 14.180, 18.910, 3.890, 0.0),
    ("789.36", 0.702, 0.0033, 16.487, 26.668, 3.749, 0.0),
    ("750-800", 0.758, 0.0048, 33.578, 22.145, 5.091, 0.0),
    ("800-850", 1.625, 0.0048, 16.992, 16.631, 3.498, 0.0),
    ("850-900", 3.537, 0.0057, 20.249, 8.562, 4.554, 0.0),
    ("900-950", 3.000, 0.0050, 9.680, 12.817, 1.315, 0.0),
    ("977.02", 4.400, 0.0039, 2.240, 18.730, 0.0, 0.0),
    ("950-1000", 1.475, 0.0044, 50.988, 21.108, 0.0, 0.0),
    ("1025.72", 3.500, 0.0052, 0.0, 1.630, 0.0, 0.0),
    ("1031.91", 2.100, 0.0053, 0.0, 1.050, 0.0, 0.0),
    ("1000-1050", 2.467, 0.0044, 0.0, 1.346, 0.0, 0.0),
]


def wavelength_m(label):
    """the bin's wavelength in m (a range by its midpoint)"""
    if "-" in label:
        a, b = label.split("-")
        return 0.5 * (float(a) + float(b)) * 1e-10
    return float(label) * 1e-10


def photon_flux(f107bar, sun_dist=1.0):
    """I_0^j (m^-2 s^-1) of every bin: the EUVAC scaling of F74113"""
    F = np.array([row[1] for row in TABLE_A]) * 1e13
    A = np.array([row[2] for row in TABLE_A])
    return F * np.maximum(0.8, 1.0 + A * (f107bar - 80.0)) / sun_dist ** 2


def photon_energy():
    """hc / lambda_j (J)"""
    return np.array([H_PLANCK * C_LIGHT / wavelength_m(row[0]) for row in TABLE_A])


def mixture_cross_section(chi):
    """sigma_j = sum_s chi_s phi_s^j (m^2), chi = mole fractions of N2, O2, O, He"""
    phi = np.array([row[3:7] for row in TABLE_A]) * 1e-22
    return phi @ np.asarray(chi, dtype=np.float64)


def declination(day):
    """north declination of the Sun (rad) on day of the year N_d (section 2.2)"""
    d0 = np.deg2rad(23.44)
    e = 0.0167
    w = 2.0 * np.pi / 365.24
    return np.arcsin(np.sin(-d0) * np.cos(w * (day + 9) + 2.0 * e * np.sin(w * (day - 3))))


def chapman(rt, cchi, r_over_R0):
    """C(r~, chi) of the three cases (np.inf in the Earth's shadow); complex r~ allowed
    (complex step), cos chi and |r|/R0 real"""
    cchi = np.asarray(cchi, dtype=np.float64)
    schi = np.sqrt(np.maximum(0.0, 1.0 - cchi * cchi))
    y = np.sqrt(rt / 2.0) * np.abs(cchi)
    base = np.sqrt(np.pi * rt / 2.0)
    ex = erfcx(y)
    day = base * ex
    lit = schi > 1.0 / np.asarray(r_over_R0, dtype=np.float64)
    # the night-side exponential only where it is used (it overflows deep in the shadow)
    arg = np.where((cchi <= 0) & lit, rt * (1.0 - schi), 0.0)
    night = base * (2.0 * np.exp(arg) - ex)
    return np.where(cchi > 0, day, np.where(lit, night, np.inf))


def bin_constants(P):
    """(K_j, kappa_j) of the nondimensional form"""
    sig = mixture_cross_section(P["euv_chi"])
    I0 = photon_flux(P["euv_f107"], P["euv_sun_dist"])
    E = photon_energy()
    K = P["euv_eps"] * E * I0 * sig * P["euv_q_scale"] / P["m"]
    kap = sig * P["euv_col_scale"] / P["m"]
    return K, kap


def sun_vector(t, P):
    """sub-solar unit vector at nondimensional time t: latitude = the declination of
    day euv_day (or sun_lat when euv_day is 0), longitude sun_lon0 - sun_rate t"""
    lat = declination(P["euv_day"]) if P.get("euv_day", 0) > 0 else P["sun_lat"]
    lon = P["sun_lon0"] - P["sun_rate"] * t
    return np.array([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)])


def heating(x, t, rho, T, P):
    """nondimensional EUVAC heating rate at nodes x (list of d coordinate arrays) for
    density rho and temperature T (nondimensional; complex allowed); 1D columns take
    cos chi from their site (P["site"], unit vector), or 1 without one"""
    d = P["d"]
    r2 = sum(np.asarray(x[k]) * np.asarray(x[k]) for k in range(d))
    r = np.sqrt(r2)
    if d == 3:
        sh = sun_vector(t, P)
        cchi = sum(np.asarray(x[k]) * sh[k] for k in range(3)) / r
    else:
        site = P.get("site")
        if site is None or not any(site):
            cchi = np.ones_like(r)
        else:
            sh = sun_vector(t, P)
            cchi = np.full_like(r, sum(site[k] * sh[k] for k in range(3)))
    if composition.enabled(P):
        m = composition.mean_mass(r, P, np)
        chi = composition.mass_fractions(r, P, np)
        phi = np.array([row[3:7] for row in TABLE_A]) * 1e-22           # [bin, N2 O2 O He]
        # sum_s n_s phi_s^j / rho, n_s = rho chi_s / m_s (m_O units)
        sig_n = sum(np.multiply.outer(phi[:, i], chi[s] / composition.MASS[s])
                    for i, s in enumerate(composition.SPECIES))          # [bin, nodes]
        flux = P["euv_eps"] * photon_energy() * photon_flux(P["euv_f107"], P["euv_sun_dist"])
        K = [flux[j] * P["euv_q_scale"] * sig_n[j] for j in range(len(TABLE_A))]
        kap = [P["euv_col_scale"] * sig_n[j] for j in range(len(TABLE_A))]
    else:
        m = P["m"]
        K, kap = bin_constants(P)
    H = T * r2 / (m * P["r_ref"] ** 2)
    C = chapman(r / H, cchi, r / P["r_ref"])
    Q = 0.0 * rho
    shade = np.isinf(np.real(C))
    Cs = np.where(shade, 0.0, C)
    col = rho * H * Cs
    for j in range(len(K)):
        Q = Q + K[j] * np.exp(-kap[j] * col)
    return np.where(shade, 0.0, rho * Q)
