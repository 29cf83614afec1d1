// Shared device-side definitions of the DG thermosphere library: scalar types
// (double, float and their dual numbers for exact J(u)v), the nondimensional
// physics constants, and the pointwise flux/source of the transformed model
// (eq. fluxSWNondimensional with the acceleration of section 2.5 and the
// transport laws of section 2.1.2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace dg {

// ---------------------------------------------------------------- dual numbers
// Forward-mode AD: value and one directional derivative. J(u)v is the derivative
// of R along v, computed exactly (no finite-difference step).
template <class T>
struct Dual {
  T v, d;
  __host__ __device__ Dual() {}
  __host__ __device__ constexpr Dual(T a) : v(a), d(T(0)) {}
  __host__ __device__ constexpr Dual(T a, T b) : v(a), d(b) {}
};

template <class S> struct Base { typedef S type; };
template <class T> struct Base<Dual<T>> { typedef T type; };

// Workgroup barrier that orders LDS only. __syncthreads also fences global memory at
// workgroup scope, which makes every wave wait for all of its outstanding global stores
// (and loads) before the barrier; where a barrier only hands LDS data between the lanes of a
// block, this one waits for the LDS operations alone. Global stores issued before it stay in
// flight across it.
__device__ __attribute__((always_inline)) inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// 1/x for the nonzero normal divisors of the model (every one is positive: e^{-varrho/2},
// T, radii, Jacobians, cos chi on the day side). FP64: the hardware reciprocal estimate
// refined by two Newton steps, within about an ulp in five instructions where the IEEE
// division takes about twelve. FP32: the division.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline float recip(float x) { return 1.0f / x; }

template <class T> __device__ inline Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> __device__ inline Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> __device__ inline Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <class T> __device__ inline Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class T> __device__ inline Dual<T> operator/(Dual<T> a, Dual<T> b) {
  T inv = recip(b.v);
  T q = a.v * inv;
  return {q, (a.d - q * b.d) * inv};
}
template <class T> __device__ inline Dual<T> operator+(Dual<T> a, T b) { return {a.v + b, a.d}; }
template <class T> __device__ inline Dual<T> operator+(T b, Dual<T> a) { return {a.v + b, a.d}; }
template <class T> __device__ inline Dual<T> operator-(Dual<T> a, T b) { return {a.v - b, a.d}; }
template <class T> __device__ inline Dual<T> operator-(T b, Dual<T> a) { return {b - a.v, -a.d}; }
template <class T> __device__ inline Dual<T> operator*(Dual<T> a, T b) { return {a.v * b, a.d * b}; }
template <class T> __device__ inline Dual<T> operator*(T b, Dual<T> a) { return {a.v * b, a.d * b}; }
template <class T> __device__ inline Dual<T> operator/(Dual<T> a, T b) { T inv = recip(b); return {a.v * inv, a.d * inv}; }
template <class T> __device__ inline Dual<T> operator/(T a, Dual<T> b) {
  T inv = recip(b.v);
  T q = a * inv;
  return {q, -q * b.d * inv};
}
template <class T> __device__ inline Dual<T>& operator+=(Dual<T>& a, Dual<T> b) { a.v += b.v; a.d += b.d; return a; }
template <class T> __device__ inline Dual<T>& operator-=(Dual<T>& a, Dual<T> b) { a.v -= b.v; a.d -= b.d; return a; }

// FP64 exp and log for the model's arguments (trace and node states, the heating profile,
// the mixture fits), written from the textbook methods. exp: Cody-Waite reduction
// x = n ln2 + r with |r| <= ln2/2 (ln2 split in two doubles, fused multiply-adds), then the
// Taylor polynomial of e^r to degree 13 (remainder below 5e-18) and a scaling by 2^n.
// log: x = 2^e m with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(z) with z = (m - 1)/(m + 1),
// |z| <= 0.172, by the series 2 z sum_k z^2k/(2k + 1) to k = 11 (remainder below 1e-18),
// plus e ln2. Both are within a few ulp and take about half the instructions of the general
// library routines. NaN propagates; exp saturates to 0 below -746 and to inf above 710; log
// of a negative number is NaN, of zero -inf, of +inf +inf.
constexpr double kLn2Hi = 0.6931471805599453, kLn2Lo = 2.3190468138462996e-17;
__device__ inline double fexp(double x) {
  x = x < -746.0 ? -746.0 : (x > 710.0 ? 710.0 : x);
  const double nf = rint(x * 1.4426950408889634);
  double r = fma(-nf, kLn2Hi, x);
  r = fma(-nf, kLn2Lo, r);
  double p = 1.0 / 6227020800.0;           // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)nf);
}
__device__ inline double flog(double x) {
  int e;
  double m = frexp(x, &e);                 // x = m 2^e, m in [1/2, 1)
  const bool low = m < 0.7071067811865476;
  m = low ? 2.0 * m : m;
  e = low ? e - 1 : e;
  const double z = (m - 1.0) * recip(m + 1.0);
  const double z2 = z * z;
  double p = 1.0 / 23.0;
  p = fma(p, z2, 1.0 / 21.0);
  p = fma(p, z2, 1.0 / 19.0);
  p = fma(p, z2, 1.0 / 17.0);
  p = fma(p, z2, 1.0 / 15.0);
  p = fma(p, z2, 1.0 / 13.0);
  p = fma(p, z2, 1.0 / 11.0);
  p = fma(p, z2, 1.0 / 9.0);
  p = fma(p, z2, 1.0 / 7.0);
  p = fma(p, z2, 1.0 / 5.0);
  p = fma(p, z2, 1.0 / 3.0);
  p = fma(p, z2, 1.0);
  const double ef = (double)e;
  const double res = fma(ef, kLn2Hi, fma(ef, kLn2Lo, 2.0 * z * p));
  if (x > 0.0 && x < __builtin_inf()) return res;
  return x == 0.0 ? -__builtin_inf() : (x > 0.0 ? x : __builtin_nan(""));
}

__device__ inline double xexp(double a) { return fexp(a); }
__device__ inline float xexp(float a) { return expf(a); }
__device__ inline double xlog(double a) { return flog(a); }
__device__ inline float xlog(float a) { return logf(a); }
__device__ inline double xsqrt(double a) { return sqrt(a); }
__device__ inline float xsqrt(float a) { return sqrtf(a); }
template <class T> __device__ inline Dual<T> xexp(Dual<T> a) { T e = xexp(a.v); return {e, e * a.d}; }
template <class T> __device__ inline Dual<T> xlog(Dual<T> a) { return {xlog(a.v), a.d * recip(a.v)}; }
template <class T> __device__ inline Dual<T> xsqrt(Dual<T> a) { T s = xsqrt(a.v); return {s, a.d * (T(0.5) * recip(s))}; }
template <class T> __device__ inline Dual<T> recip(Dual<T> a) {
  const T i = recip(a.v);
  return {i, -a.d * i * i};
}
__device__ inline double xerfcx(double a) { return erfcx(a); }
__device__ inline float xerfcx(float a) { return erfcxf(a); }
// d/dy erfcx(y) = 2 y erfcx(y) - 2 / sqrt(pi)
template <class T> __device__ inline Dual<T> xerfcx(Dual<T> a) {
  const T e = xerfcx(a.v);
  return {e, (T(2) * a.v * e - T(1.1283791670955126)) * a.d};
}
// x^c for x > 0
__device__ inline double xpow(double a, double c) { return fexp(c * flog(a)); }
__device__ inline float xpow(float a, float c) { return expf(c * logf(a)); }
template <class T> __device__ inline Dual<T> xpow(Dual<T> a, T c) {
  T p = xpow(a.v, c);
  return {p, c * p * recip(a.v) * a.d};
}

template <class S> __device__ inline typename Base<S>::type val(S a) { return a; }
template <class T> __device__ inline T val(Dual<T> a) { return a.v; }

// loads and stores for the scalar types: a dual reads its value from the state and
// its derivative from the tangent array (both stored in T)
template <class S> struct Io;
template <> struct Io<double> {
  template <class P> __device__ static double ld(const double* u, const P*, int64_t i) { return u[i]; }
  __device__ static void st(double* r, void*, int64_t i, double x) { r[i] = x; }
};
template <> struct Io<float> {
  template <class P> __device__ static float ld(const float* u, const P*, int64_t i) { return u[i]; }
  __device__ static void st(float* r, void*, int64_t i, float x) { r[i] = x; }
};
template <class T> struct Io<Dual<T>> {
  template <class U> __device__ static Dual<T> ld(const U* u, const T* v, int64_t i) { return {T(u[i]), v[i]}; }
};

// ---------------------------------------------------------------- constants
// Nondimensional parameters (section 2.5), flattened for kernel arguments.
struct PhysC {
  double gamma, inv_gm, c_visc, c_cond, c_diss, m, inv_m;
  double nu_r, alpha_r, alpha0c, kexp;
  double lam, T_bot, r_ref2;
  double om[3], cent, cor;           // rotation vector, Fr^2/gamma, 2 Fr/sqrt(gamma)
  double heat_amp, heat_qm, heat_rm, heat_inv_H;
  double sun_lat, sun_lon0, sun_rate;
  double sun_dir[3];                 // sub-solar unit vector at the evaluation time (set per launch)
  int bc_mode;
  double bc_state[5];
  int euv;                           // 1: EUVAC heating (state dependent)
  const double* euv_tab;             // device [K_0..K_36, kap_0..kap_36]: Q = rho sum_j K_j exp(-kap_j rho H C)
  double euv_hfac, r_ref;            // H = T r^2 euv_hfac; the lower-boundary radius R0
  double site[3];                    // 1D: unit vector of the column's site (0: the Sun overhead)
  int comp;                          // 1: variable composition (mixture below), 0: constant m
  double comp_a[6], comp_b[6];       // chi_s = a_1 e^{b_1 |r|} + a_2 e^{b_2 |r|} of N2, O2, He
  // which extended-physics instantiation a mesh runs (template flag XP below)
  __host__ __device__ int xp_mode() const;
};

// Extended physics of an instantiation (template flag XP, a bit mask): kXpEuv contains the
// EUVAC heating, kXpComp the variable composition. The kernels without a bit keep their
// register budget; a mesh with the composition runs kXpEuv | kXpComp (EUVAC then checked
// at run time), one with EUVAC only kXpEuv, otherwise 0.
constexpr int kXpEuv = 1, kXpComp = 2;
__host__ __device__ inline int PhysC::xp_mode() const { return comp ? (kXpEuv | kXpComp) : (euv ? kXpEuv : 0); }

// ---------------------------------------------------------------- mixture
// Chemically frozen mixture (section 2.1.1): mass fractions of N2, O2 and He from their
// fits, atomic oxygen the balance. In units of m_O and of oxygen's c_v (all species with
// the same gamma): c_v = sum_s chi_s / m_s = 1 / m. Mole fractions x_s = m chi_s / m_s
// weight the species conductivities (section 2.1.2; alpha_N2 = alpha_O2 = 3.6e-4,
// alpha_O = alpha_He = 5.6e-4), taken relative to alpha_O.
constexpr double kInvMassN2 = 15.9994 / 28.0134, kInvMassO2 = 15.9994 / 31.9988, kInvMassHe = 15.9994 / 4.002602;
constexpr double kAlphaMol = 3.6 / 5.6;    // alpha_N2 / alpha_O = alpha_O2 / alpha_O

struct Mix {
  double m, inv_m, inv_gm;   // mean molecular mass, c_v = 1/m, 1/(gamma m)
  double kw;                 // conductivity weight sum_s x_s alpha_s / alpha_O
  double dlnm;               // d ln m / d|r| (the grad c_v term: grad c_v / c_v = -grad ln m)
  double chi[4];             // mass fractions of N2, O2, O, He (Table A's order)
};

// the mixture at radius r: the constants of the mesh unless XP has kXpComp and the
// composition is on
template <int XP>
__device__ inline Mix mixture(const PhysC& P, double r) {
  Mix x;
  if (!(XP & kXpComp) || !P.comp) {
    x.m = P.m;
    x.inv_m = P.inv_m;
    x.inv_gm = P.inv_gm;
    x.kw = 1.0;
    x.dlnm = 0.0;
    for (int s = 0; s < 4; ++s) x.chi[s] = 0.0;
    return x;
  }
  double c[3], dc[3];
  for (int s = 0; s < 3; ++s) {
    const double e0 = P.comp_a[2 * s] * fexp(P.comp_b[2 * s] * r);
    const double e1 = P.comp_a[2 * s + 1] * fexp(P.comp_b[2 * s + 1] * r);
    c[s] = e0 + e1;
    dc[s] = P.comp_b[2 * s] * e0 + P.comp_b[2 * s + 1] * e1;
  }
  const double cO = 1.0 - c[0] - c[1] - c[2];
  const double nN2 = c[0] * kInvMassN2, nO2 = c[1] * kInvMassO2, nHe = c[2] * kInvMassHe;  // chi_s / m_s
  x.inv_m = nN2 + nO2 + nHe + cO;
  x.m = 1.0 / x.inv_m;
  x.inv_gm = x.inv_m / P.gamma;
  x.kw = x.m * ((nN2 + nO2) * kAlphaMol + nHe + cO);
  // d c_v / d|r| with d chi_O = -(d chi_N2 + d chi_O2 + d chi_He)
  const double dcv = dc[0] * (kInvMassN2 - 1.0) + dc[1] * (kInvMassO2 - 1.0) + dc[2] * (kInvMassHe - 1.0);
  x.dlnm = -dcv * x.m;
  x.chi[0] = c[0];
  x.chi[1] = c[1];
  x.chi[2] = cO;
  x.chi[3] = c[2];
  return x;
}

// ---------------------------------------------------------------- pointwise physics
// cosine of the solar zenith angle at x: the shell from the node's direction, a column
// from its site's direction (the Sun overhead when no site is set); P.sun_dir holds the
// sub-solar direction at the evaluation time
template <int D>
__device__ inline double cos_zenith(const PhysC& P, const double* x) {
  if constexpr (D == 3) {
    const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    return (x[0] * P.sun_dir[0] + x[1] * P.sun_dir[1] + x[2] * P.sun_dir[2]) * recip(r);
  } else {
    if (P.site[0] == 0.0 && P.site[1] == 0.0 && P.site[2] == 0.0) return 1.0;
    return P.site[0] * P.sun_dir[0] + P.site[1] * P.sun_dir[1] + P.site[2] * P.sun_dir[2];
  }
}

// EUVAC heating (section 2.2) at position x for density rho and temperature Tm
// (nondimensional): Q = rho sum_j K_j exp(-kap_j rho H C), H = Tm r^2 hfac the scale
// height, C the Smith-Smith Chapman factor of r~ = r / H and the zenith angle (cos chi = 1 in
// 1D), zero in the Earth's shadow (R0 = r_ref). tab (EUVT entries) = [K_j, kap_j, phi'_sj]: with
// a constant composition K_j and kap_j are the bin constants; with the variable one
// (comp) kap_j = sum_s chi_s phi'_sj (phi' = col_scale phi_s^j / m_s, chi the local mass
// fractions: the species number densities rho chi_s / m_s) and K_j = tab[j] kap_j; only the
// COMP instantiation contains that branch. Terms whose optical depth exceeds what the
// type's exp resolves are dropped (their flux is below 1e-30 of the unattenuated one). Only
// the kernels instantiated with kXpEuv (flux_source) contain it: the element passes without
// it keep their register budget.
constexpr int EUVT = 6 * 37;
template <int D, class S, bool COMP>
__device__ inline S heating_euvac(const double* __restrict__ tab, double hfac, double r_ref, double cchi, double r,
                                  S rho, S Tm, bool comp, const double (&chi)[4]) {
  typedef typename Base<S>::type T;
  constexpr T kTauMax = sizeof(T) == 8 ? T(700) : T(80);
  const double r2 = r * r;
  const double schi = sqrt(fmax(0.0, 1.0 - cchi * cchi));
  const bool day = cchi > 0.0;
  if (!day && !(schi > r_ref / r)) return S(T(0));
  const S H = Tm * T(r2 * hfac);
  const S rt = T(r) / H;
  const S ex = xerfcx(xsqrt(T(0.5) * rt) * T(fabs(cchi)));
  const S base = xsqrt(T(1.5707963267948966) * rt);
  S C;
  if (day) {
    C = base * ex;
  } else {
    const S arg = rt * T(1.0 - schi);
    if (!(val(arg) < kTauMax)) return S(T(0));
    C = base * (T(2) * xexp(arg) - ex);
  }
  const S col = rho * H * C;
  S Q = S(T(0));
  if (COMP && comp) {
    for (int j = 0; j < 37; ++j) {
      const double kap = chi[0] * tab[74 + j] + chi[1] * tab[111 + j] + chi[2] * tab[148 + j] + chi[3] * tab[185 + j];
      const S tau = T(kap) * col;
      if (val(tau) < kTauMax) Q = Q + T(tab[j] * kap) * xexp(-tau);
    }
  } else {
    for (int j = 0; j < 37; ++j) {
      const S tau = T(tab[37 + j]) * col;
      if (val(tau) < kTauMax) Q = Q + T(tab[j]) * xexp(-tau);
    }
  }
  return rho * Q;
}

// Flux F[c][k] and source Sr[c] at one node of a D-dimensional problem (f = D + 2
// fields: varrho, sqrt(rho) v, sqrt(rho) T). x: node position; Q: heating rate there.
// XP: kXpEuv adds the EUVAC heating (heat && P.euv), kXpComp the variable composition
// (P.comp: m, c_v and the conductivity weight at |x|, and the energy source
// -(1/c_v) F_Theta . grad c_v = F_Theta . grad ln m of eq. fluxSWNondimensional).
template <int D, class S, int XP = 0>
__device__ inline void flux_source(const PhysC& P, const S* u, const S (*q)[D], const double* x, double Q,
                                   S (*F)[D], S* Sr, bool heat = true) {
  typedef typename Base<S>::type T;
  // (the radius is formed here only where the mixture needs it: the other instantiations
  // keep it out of the registers live across the flux)
  double rx = 0;
  if constexpr ((XP & kXpComp) != 0) {
    for (int k = 0; k < D; ++k) rx += x[k] * x[k];
    rx = sqrt(rx);
  }
  const Mix mx = mixture<XP>(P, rx);
  const S lr = u[0];
  const S s = xexp(T(-0.5) * lr);
  const S sq = recip(s);
  const S rho = sq * sq;
  S U[D], v[D];
  for (int i = 0; i < D; ++i) { U[i] = u[1 + i]; v[i] = s * U[i]; }
  const S Th = u[D + 1];
  const S Tm = s * Th;
  const S mu = xsqrt(Tm * T(mx.m)) + T(P.nu_r) * rho;
  const S kap = T(P.alpha0c * mx.kw) * xpow(Tm, T(P.kexp)) + T(P.alpha_r * mx.inv_m) * rho;
  S gl[D], gT[D], gv[D][D];
  for (int k = 0; k < D; ++k) gl[k] = q[0][k];
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k) gv[i][k] = s * (q[1 + i][k] - T(0.5) * U[i] * gl[k]);
  for (int k = 0; k < D; ++k) gT[k] = s * (q[D + 1][k] - T(0.5) * Th * gl[k]);
  S div = gv[0][0];
  for (int i = 1; i < D; ++i) div = div + gv[i][i];
  S eps[D][D];
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k) eps[i][k] = gv[i][k] + gv[k][i] - (i == k ? T(2.0 / 3.0) * div : S(T(0)));
  const S mus = T(P.c_visc) * mu * s;                 // mu / (sqrt(rho) sqrt(gamma Gr))
  const S kas = T(P.c_cond * mx.m) * kap * s;         // kappa / (Pr sqrt(rho) c_v) sqrt(gamma/Gr)
  for (int k = 0; k < D; ++k) F[0][k] = lr * v[k];
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k) {
      S f = U[i] * v[k] - mus * eps[i][k];
      if (i == k) f = f + T(mx.inv_gm) * Th;
      F[1 + i][k] = f;
    }
  for (int k = 0; k < D; ++k) F[D + 1][k] = Th * v[k] - kas * gT[k];
  // sources
  Sr[0] = (lr - T(1)) * div;
  double r2 = 0;
  for (int k = 0; k < D; ++k) r2 += x[k] * x[k];
  const double r = sqrt(r2);
  const double gfac = -P.r_ref2 * recip(r2 * r * P.gamma);   // g_k / gamma = gfac x_k
  double cen[3] = {0, 0, 0};
  if (D == 3) {
    const double wr = P.om[0] * x[0] + P.om[1] * x[1] + P.om[2] * x[2];
    const double ww = P.om[0] * P.om[0] + P.om[1] * P.om[1] + P.om[2] * P.om[2];
    for (int k = 0; k < 3; ++k) cen[k] = -P.cent * (P.om[k] * wr - ww * x[k]);
  }
  for (int i = 0; i < D; ++i) {
    S eg = eps[i][0] * gl[0];
    for (int k = 1; k < D; ++k) eg = eg + eps[i][k] * gl[k];
    S a = sq * T(gfac * x[i] + cen[i]) + T(0.5) * div * U[i] - T(0.5 * mx.inv_gm) * Th * gl[i] + T(0.5) * mus * eg;
    if (D == 3) {
      const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
      // - 2 Fr/sqrt(gamma) (w x U)_i
      a = a - T(P.cor) * (T(P.om[i1]) * U[i2 % D] - T(P.om[i2]) * U[i1 % D]);
    }
    Sr[1 + i] = a;
  }
  S Tg = gT[0] * gl[0];
  for (int k = 1; k < D; ++k) Tg = Tg + gT[k] * gl[k];
  S ed = eps[0][0] * gv[0][0];
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k)
      if (i + k > 0) ed = ed + eps[i][k] * gv[i][k];
  Sr[D + 1] = T(Q * mx.m) * s + T(1.5 - P.gamma) * Th * div + T(0.5) * kas * Tg + T(P.c_diss * mx.m) * mu * s * ed;
  constexpr bool kComp = (XP & kXpComp) != 0;
  if constexpr ((XP & kXpEuv) != 0) {
    if (heat && P.euv)
      Sr[D + 1] = Sr[D + 1] + T(mx.m) * s *
                                heating_euvac<D, S, kComp>(P.euv_tab, kComp && P.comp ? mx.inv_m / P.r_ref2 : P.euv_hfac,
                                                           P.r_ref, cos_zenith<D>(P, x), r, rho, Tm, P.comp != 0,
                                                           mx.chi);
  }
  if constexpr (kComp) {
    if (P.comp) {
      S Fx = F[D + 1][0] * T(x[0]);
      for (int k = 1; k < D; ++k) Fx = Fx + F[D + 1][k] * T(x[k]);
      Sr[D + 1] = Sr[D + 1] + T(mx.dlnm / r) * Fx;
    }
  }
}

// inviscid part of the flux only (upper boundary) at radius r
template <int D, class S, int XP = 0>
__device__ inline void flux_inviscid(const PhysC& P, const S* u, S (*F)[D], double r) {
  typedef typename Base<S>::type T;
  const double inv_gm = mixture<XP>(P, r).inv_gm;
  const S lr = u[0];
  const S s = xexp(T(-0.5) * lr);
  S v[D];
  for (int i = 0; i < D; ++i) v[i] = s * u[1 + i];
  for (int k = 0; k < D; ++k) F[0][k] = lr * v[k];
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k) {
      S f = u[1 + i] * v[k];
      if (i == k) f = f + T(inv_gm) * u[D + 1];
      F[1 + i][k] = f;
    }
  for (int k = 0; k < D; ++k) F[D + 1][k] = u[D + 1] * v[k];
}

// stabilisation sigma (eq. LDG2) at a trace state at radius r: lam + diag(0, mu s c_visc,
// kappa s m c_cond)
template <int D, class S, int XP = 0>
__device__ inline void sigma(const PhysC& P, const S* uh, S& sig_m, S& sig_e, double r) {
  typedef typename Base<S>::type T;
  const Mix mx = mixture<XP>(P, r);
  const S s = xexp(T(-0.5) * uh[0]);
  const S rho = recip(s * s);
  const S Tm = s * uh[D + 1];
  const S mu = xsqrt(Tm * T(mx.m)) + T(P.nu_r) * rho;
  const S kap = T(P.alpha0c * mx.kw) * xpow(Tm, T(P.kexp)) + T(P.alpha_r * mx.inv_m) * rho;
  sig_m = T(P.lam) + T(P.c_visc) * mu * s;
  sig_e = T(P.lam) + T(P.c_cond * mx.m) * kap * s;
}

// boundary state u_b for the lower boundary (or the Dirichlet state in bc_mode 1)
template <int D, class S>
__device__ inline void boundary_state(const PhysC& P, const S* u, S* ub) {
  typedef typename Base<S>::type T;
  if (P.bc_mode == 1) {
    for (int c = 0; c < D + 2; ++c) ub[c] = S(T(P.bc_state[c]));
    return;
  }
  ub[0] = u[0];
  for (int i = 0; i < D; ++i) ub[1 + i] = S(T(0));
  ub[D + 1] = T(P.T_bot) * xexp(T(0.5) * u[0]);
}

// Chapman-shaped day-side heating at position x, time t (depends on x and t only)
// P.sun_dir must hold the sub-solar direction at time t (sun_direction below)
template <int D>
__device__ inline double heating(const PhysC& P, const double* x, double t) {
  if (P.heat_amp == 0.0) return 0.0;
  double r2 = 0;
  for (int k = 0; k < D; ++k) r2 += x[k] * x[k];
  const double r = sqrt(r2);
  double cchi = 1.0;
  if constexpr (D == 3)
    cchi = (x[0] * P.sun_dir[0] + x[1] * P.sun_dir[1] + x[D - 1] * P.sun_dir[2]) * recip(r);
  else
    cchi = cos_zenith<1>(P, x);
  (void)t;
  if (!(cchi > 0.0)) return 0.0;
  const double z = (r - P.heat_rm) * P.heat_inv_H;
  return P.heat_amp * P.heat_qm * fexp(1.0 - z - fexp(-z) * recip(cchi));
}

// the same on the device (kernels that advance time themselves)
__device__ inline void sun_direction_dev(PhysC& P, double t) {
  const double lon = P.sun_lon0 - P.sun_rate * t;
  const double cl = cos(P.sun_lat);
  P.sun_dir[0] = cl * cos(lon);
  P.sun_dir[1] = cl * sin(lon);
  P.sun_dir[2] = sin(P.sun_lat);
}

// the sub-solar direction at time t: longitude sun_lon0 - sun_rate t, latitude sun_lat
inline void sun_direction(PhysC& P, double t) {
  const double lon = P.sun_lon0 - P.sun_rate * t;
  const double cl = std::cos(P.sun_lat);
  P.sun_dir[0] = cl * std::cos(lon);
  P.sun_dir[1] = cl * std::sin(lon);
  P.sun_dir[2] = std::sin(P.sun_lat);
}

}  // namespace dg
