// EUVAC heating constants (section 2.2, Table A of the appendix on EUV cross sections) and
// the host-side check of the variable composition (section 2.1.1).
//
// The heating rate in the model's units is Q = rho sum_j K_j exp(-kap_j rho H C) (rho, H in
// nondimensional units; C the Chapman factor evaluated on the device), with per bin j
//   sigma_j = sum_s chi_s phi_s^j                          (mixture cross section, m^2)
//   I_0^j   = F74113^j max(0.8, 1 + A_j (F10.7bar - 80)) / d^2
//   K_j     = eps (hc / lambda_j) I_0^j sigma_j q_scale / m
//   kap_j   = sigma_j col_scale / m
// for constant mole fractions chi_s and mean mass m. With the variable composition the
// number densities are rho chi_s(r) / m_s (chi_s mass fractions), so the device forms
// kap_j = sum_s chi_s phi'_sj with phi'_sj = col_scale phi_s^j / m_s, and K_j = A'_j kap_j with
// A'_j = eps (hc / lambda_j) I_0^j q_scale / col_scale. The table holds EUVT = 6 x 37 values:
// [K_j or A'_j, kap_j, phi'_N2, phi'_O2, phi'_O, phi'_He].
// Table A's photon fluxes are read with the exponent +13 (m^-2 s^-1), the cross sections
// in units of 1e-22 m^2; a wavelength range stands for its midpoint.
#include <cmath>
#include <vector>

#include "internal.h"

namespace dg {

namespace {

struct EuvBin {
  double lo, hi;          // wavelength range in Angstrom (lo == hi for a line)
  double f74113;          // 1e13 photons m^-2 s^-1
  double a;               // EUVAC scaling factor
  double phi[4];          // N2, O2, O, He cross sections, 1e-22 m^2
};

const EuvBin kTableA[37] = {
    {50, 100, 1.200, 0.0100, {0.720, 1.316, 0.730, 0.144}},
    {100, 150, 0.450, 0.0071, {2.261, 3.806, 1.839, 0.479}},
    {150, 200, 4.800, 0.0134, {4.958, 7.509, 3.732, 1.157}},
    {200, 250, 3.100, 0.0195, {8.392, 10.900, 5.202, 1.601}},
    {256.3, 256.3, 0.460, 0.0028, {10.210, 13.370, 6.050, 2.121}},
    {284.15, 284.15, 0.210, 0.1380, {10.900, 15.790, 7.080, 2.595}},
    {250, 300, 1.679, 0.0265, {10.493, 14.387, 6.461, 2.321}},
    {303.31, 303.31, 0.800, 0.0250, {11.670, 16.800, 7.680, 2.953}},
    {303.78, 303.78, 6.900, 0.0033, {11.700, 16.810, 7.700, 2.962}},
    {300, 350, 0.965, 0.0225, {13.857, 17.438, 8.693, 3.544}},
    {368.07, 368.07, 0.650, 0.0066, {16.910, 18.320, 9.840, 4.268}},
    {350, 400, 0.314, 0.0365, {16.395, 18.118, 9.687, 4.142}},
    {400, 450, 0.383, 0.0074, {21.675, 20.310, 11.496, 5.447}},
    {465.22, 465.22, 0.290, 0.0075, {23.160, 21.910, 11.930, 6.563}},
    {450, 500, 0.285, 0.0202, {23.471, 23.101, 12.127, 7.208}},
    {500, 550, 0.452, 0.0088, {24.501, 24.606, 12.059, 0.958}},
    {554.37, 554.37, 0.720, 0.0033, {24.130, 26.040, 12.590, 0}},
    {584.33, 584.33, 1.270, 0.0052, {22.400, 22.720, 13.090, 0}},
    {550, 600, 0.357, 0.0037, {22.787, 26.610, 13.024, 0}},
    {609.76, 609.76, 0.530, 0.0162, {22.790, 28.070, 13.400, 0}},
    {629.73, 629.73, 1.590, 0.0033, {23.370, 32.060, 13.400, 0}},
    {600, 650, 0.342, 0.0118, {23.339, 26.017, 13.365, 0}},
    {650, 700, 0.230, 0.0043, {31.755, 21.919, 17.245, 0}},
    {703.31, 703.31, 0.360, 0.0030, {26.540, 27.440, 11.460, 0}},
    {700, 750, 0.141, 0.0047, {24.662, 28.535, 10.736, 0}},
    {765.15, 765.15, 0.170, 0.0039, {120.490, 20.800, 4.000, 0}},
    {770.41, 770.41, 0.260, 0.0128, {14.180, 18.910, 3.890, 0}},
    {789.36, 789.36, 0.702, 0.0033, {16.487, 26.668, 3.749, 0}},
    {750, 800, 0.758, 0.0048, {33.578, 22.145, 5.091, 0}},
    {800, 850, 1.625, 0.0048, {16.992, 16.631, 3.498, 0}},
    {850, 900, 3.537, 0.0057, {20.249, 8.562, 4.554, 0}},
    {900, 950, 3.000, 0.0050, {9.680, 12.817, 1.315, 0}},
    {977.02, 977.02, 4.400, 0.0039, {2.240, 18.730, 0, 0}},
    {950, 1000, 1.475, 0.0044, {50.988, 21.108, 0, 0}},
    {1025.72, 1025.72, 3.500, 0.0052, {0, 1.630, 0, 0}},
    {1031.91, 1031.91, 2.100, 0.0053, {0, 1.050, 0, 0}},
    {1000, 1050, 2.467, 0.0044, {0, 1.346, 0, 0}},
};

}  // namespace

double euvac_declination(double day) {
  // section 2.2's approximation of the Sun's north declination on day N_d of the year
  const double kPi = 3.14159265358979323846;
  const double d0 = 23.44 * kPi / 180.0, e = 0.0167, w = 2.0 * kPi / 365.24;
  return std::asin(std::sin(-d0) * std::cos(w * (day + 9.0) + 2.0 * e * std::sin(w * (day - 3.0))));
}

void euvac_constants(const dg_physics_t& in, double* tab) {
  const double h = 6.62607015e-34, c = 2.99792458e8;
  const double inv_ms[4] = {kInvMassN2, kInvMassO2, 1.0, kInvMassHe};
  for (int j = 0; j < 37; ++j) {
    const EuvBin& b = kTableA[j];
    double sig = 0;
    for (int s = 0; s < 4; ++s) sig += in.euv_chi[s] * b.phi[s] * 1e-22;
    const double lam = 0.5 * (b.lo + b.hi) * 1e-10;
    const double scale = 1.0 + b.a * (in.euv_f107 - 80.0);
    const double I0 = b.f74113 * 1e13 * (scale > 0.8 ? scale : 0.8) / (in.euv_sun_dist * in.euv_sun_dist);
    if (in.composition) {
      tab[j] = in.euv_eps * (h * c / lam) * I0 * in.euv_q_scale / in.euv_col_scale;
      tab[37 + j] = 0.0;
    } else {
      tab[j] = in.euv_eps * (h * c / lam) * I0 * sig * in.euv_q_scale / in.m;
      tab[37 + j] = sig * in.euv_col_scale / in.m;
    }
    for (int s = 0; s < 4; ++s) tab[74 + 37 * s + j] = in.euv_col_scale * b.phi[s] * 1e-22 * inv_ms[s];
  }
}

bool composition_valid(const dg_physics_t& ph, double r_lo, double r_hi) {
  if (!ph.composition) return true;
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(ph.comp_a[i]) || !std::isfinite(ph.comp_b[i])) return false;
  const int n = 1024;
  for (int i = 0; i <= n; ++i) {
    const double r = r_lo + (r_hi - r_lo) * i / n;
    double sum = 0;
    for (int s = 0; s < 3; ++s) {
      const double chi = ph.comp_a[2 * s] * std::exp(ph.comp_b[2 * s] * r) +
                         ph.comp_a[2 * s + 1] * std::exp(ph.comp_b[2 * s + 1] * r);
      if (!(chi >= 0.0 && chi <= 1.0)) return false;
      sum += chi;
    }
    if (!(sum <= 1.0)) return false;
  }
  return true;
}

void col_params(const dg_physics_t& ph, int n_col, std::vector<double>& cpar) {
  cpar.assign((size_t)CPAR * n_col, 0.0);
  for (int c = 0; c < n_col; ++c) {
    double* p = &cpar[(size_t)CPAR * c];
    p[0] = ph.col_heat_amp ? ph.col_heat_amp[c] : ph.heat_amp;
    p[1] = ph.col_heat_qm ? ph.col_heat_qm[c] : ph.heat_qm;
    p[2] = ph.col_heat_rm ? ph.col_heat_rm[c] : ph.heat_rm;
    p[3] = 1.0 / (ph.col_heat_H ? ph.col_heat_H[c] : ph.heat_H);
    p[4] = ph.col_lam ? ph.col_lam[c] : ph.lam;
    p[5] = ph.col_alpha0c ? ph.col_alpha0c[c] : ph.alpha0c;
    for (int k = 0; k < 3; ++k) p[6 + k] = ph.col_site ? ph.col_site[3 * c + k] : 0.0;
  }
}

void col_euv_tables(const dg_physics_t& ph, int n_col, std::vector<double>& tab) {
  tab.assign((size_t)EUVT * n_col, 0.0);
  dg_physics_t q = ph;
  for (int c = 0; c < n_col; ++c) {
    if (ph.col_euv_eps) q.euv_eps = ph.col_euv_eps[c];
    if (ph.col_euv_f107) q.euv_f107 = ph.col_euv_f107[c];
    euvac_constants(q, &tab[(size_t)EUVT * c]);
  }
}

}  // namespace dg
