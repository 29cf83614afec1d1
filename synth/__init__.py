"""Seeded synthetic workloads for the thermosphere DG solver.

This module is shared by the tests, the benchmark and the smoke run. It holds
the *inputs* only: physical constants and reference scales (paper section 2.5),
the random draws of each workload, the Bates temperature profile with its
hydrostatic log-density (the stand-in for the MSIS initial state of section 2.3),
seeded smooth perturbations and tangent vectors. It performs none of the DG
arithmetic (no basis, no mesh, no flux, no residual): states are produced as
callables of node coordinates, and each side evaluates them at its own nodes.

Everything is nondimensional in the scalings of section 2.5: lengths by H0,
speeds by a0, time by H0/a0, density by rho0, temperature by T0 = T(100 km).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# physical constants (SI)
KB = 1.380649e-23           # Boltzmann constant
AMU = 1.66053906660e-27     # atomic mass unit
M_O = 16.0 * AMU            # atomic oxygen, the reference molecular mass
R_EARTH = 6.371e6
GM = 3.986004418e14
OMEGA0 = 7.2921159e-5       # Earth rotation rate
GAMMA = 5.0 / 3.0
Z_BOT = 100e3
Z_TOP = 600e3
T_REF = 200.0               # T0: temperature at the lower boundary
RHO_REF = 5.0e-7            # rho0: order of magnitude at 100 km (assumed)
MU_REF = 4.03e-5            # mu0: molecular viscosity at T0 (reading of the viscosity law)
ALPHA_O = 5.6e-4            # conductivity coefficient of atomic oxygen
Q_COLUMN = 1.223e-3         # W/m^2, column EUV heating (0.25 x 4.89 mW/m^2 at F10.7 = 150)

R0_SI = R_EARTH + Z_BOT
G0 = GM / R0_SI ** 2
H0 = KB * T_REF / (M_O * G0)
A0 = math.sqrt(GAMMA * KB * T_REF / M_O)
T_UNIT = H0 / A0
KAPPA_REF = ALPHA_O * T_REF ** 0.69
CP_O = GAMMA / (GAMMA - 1.0) * KB / M_O
CV_O = CP_O / GAMMA
GR = G0 * H0 ** 3 / (MU_REF / RHO_REF) ** 2
PR = MU_REF * CP_O / KAPPA_REF
FR = math.sqrt(OMEGA0 ** 2 * H0 / G0)
Q_UNIT = RHO_REF * CV_O * T_REF * A0 / H0   # W/m^3 per unit nondimensional heating

R_BOT = R0_SI / H0
R_TOP = (R_EARTH + Z_TOP) / H0


def seconds_to_nondim(dt_s: float) -> float:
    return dt_s / T_UNIT


def z_km(r):
    """altitude in km from nondimensional radius"""
    return np.asarray(r) * H0 / 1e3 - R_EARTH / 1e3


# --------------------------------------------------------------------------
# physics parameter set: plain numbers consumed by both the oracle and the library
def base_physics(d: int) -> dict:
    return dict(
        d=d, gamma=GAMMA, Gr=GR, Pr=PR, Fr=FR, m=1.0,
        nu_r=200.0, alpha_r=10.0, alpha0c=1.0,
        lam=1.0, T_bot=1.0, r_ref=R_BOT,
        omega=[0.0, 0.0, 1.0] if d == 3 else [0.0, 0.0, 0.0],
        heat_amp=0.0, heat_qm=0.0, heat_rm=R_BOT, heat_H=1.0,
        sun_lat=0.0, sun_lon0=0.0, sun_rate=FR / math.sqrt(GAMMA),
        bc_mode=0, bc_state=[0.0] * 5,
        heating_model=0,
    )


# EUVAC heating inputs (section 2.2): efficiency, F10.7bar, distance to the Sun (AU), the
# day of the year (0: keep sun_lat), constant mole fractions of N2, O2, O, He (synthetic:
# the composition fits are not available), and the two dimensional scales that turn
# number columns and heating rates into the model's units
def euvac_physics(f107bar: float = 150.0, day: float = 0.0) -> dict:
    return dict(euv_eps=0.25, euv_f107=f107bar, euv_sun_dist=1.0, euv_day=day,
                euv_chi=[0.15, 0.01, 0.80, 0.04],
                euv_q_scale=RHO_REF / (M_O * Q_UNIT), euv_col_scale=RHO_REF * H0 / M_O)


# Variable composition (section 2.1.1): two-exponential fits in |r| of the mass fractions of
# N2, O2 and He, atomic oxygen closing the sum. The empirical model's averages are not
# available, so these are synthetic, shaped like them between 100 and 600 km (N2 and O2
# falling off, He growing, O the balance: mean mass about 28.5 amu at 100 km and 14.3 amu
# at 600 km). Each term is (value at 100 km, e-folding length in km; negative: growing).
COMPOSITION_FITS = (
    ("N2", ((0.90, 180.0), (-0.145, 40.0))),
    ("O2", ((0.26, 110.0), (-0.03, 30.0))),
    ("He", ((1.0e-4, -85.0), (1.0e-5, -70.0))),
)
SPECIES_MASS = {"N2": 28.0134 / 15.9994, "O2": 31.9988 / 15.9994, "O": 1.0, "He": 4.002602 / 15.9994}


def composition_physics() -> dict:
    """the fit coefficients a_j^s, b_j^s of chi_s = sum_j a_j^s exp(b_j^s |r|) in the
    model's units (|r| in H0), ordered N2 (j = 1, 2), O2, He"""
    a, b = [], []
    for _, terms in COMPOSITION_FITS:
        for c, L in terms:
            bj = -H0 / (L * 1e3)
            a.append(c * math.exp(-bj * R_BOT))
            b.append(bj)
    return dict(composition=1, comp_a=a, comp_b=b)


def mixture_mass(phys):
    """the rest state's mean molecular mass m(r) (a callable) for a physics set with the
    variable composition, else None (m = 1). It shapes the generated input state only."""
    if not phys.get("composition", 0):
        return None
    a, b = phys["comp_a"], phys["comp_b"]

    def m(r):
        r = np.asarray(r, dtype=np.float64)
        chi = [a[2 * i] * np.exp(b[2 * i] * r) + a[2 * i + 1] * np.exp(b[2 * i + 1] * r) for i in range(3)]
        inv = sum(chi[i] / SPECIES_MASS[s] for i, (s, _) in enumerate(COMPOSITION_FITS))
        return 1.0 / (inv + (1.0 - chi[0] - chi[1] - chi[2]) / SPECIES_MASS["O"])
    return m


# --------------------------------------------------------------------------
# Bates temperature profile and its hydrostatic log-density
def bates_T(r, T_inf):
    """nondimensional temperature T/T0 of the Bates profile at nondim radius r"""
    z = z_km(r)
    T = T_inf - (T_inf - T_REF) * np.exp(-0.02 * (z - Z_BOT / 1e3))
    return T / T_REF


_GL_X, _GL_W = np.polynomial.legendre.leggauss(24)


def hydrostatic_logrho(r, T_inf, r_ref=R_BOT, mass=None):
    """log(rho/rho0) of the hydrostatic rest state with temperature bates_T, gravity
    g = -(r_ref/r)^2 and mean mass m(r) (`mass`, a callable; None: m = 1):
    d(rho T / m)/dr = -rho (r_ref/r)^2, rho(r_ref) = 1, so that
    log rho = log(m / m(r_ref)) - log T - int m / T (r_ref/x)^2 dx.
    Integrated with composite 24-point Gauss-Legendre between sorted radii (every gap
    split into equal panels no longer than 0.5 in H0 units)."""
    r = np.asarray(r, dtype=np.float64)
    flat = r.ravel()
    uniq, inv = np.unique(flat, return_inverse=True)
    pts = np.concatenate([[r_ref], uniq])
    a, b = pts[:-1], pts[1:]
    nsub = max(1, int(np.ceil(np.max(np.abs(b - a)) / 0.5)))
    frac = np.arange(nsub + 1) / nsub
    edges = a[:, None] + (b - a)[:, None] * frac[None, :]
    lo, hi = edges[:, :-1], edges[:, 1:]
    x = 0.5 * (hi + lo)[..., None] + 0.5 * (hi - lo)[..., None] * _GL_X
    f = (r_ref / x) ** 2 / bates_T(x, T_inf)
    if mass is not None:
        f = f * mass(x)
    integ = np.sum(0.5 * (hi - lo) * (f @ _GL_W), axis=1)
    cum = np.cumsum(integ)
    lr = -np.log(bates_T(uniq, T_inf)) - cum
    if mass is not None:
        lr = lr + np.log(mass(uniq) / mass(r_ref))
    return lr[inv].reshape(r.shape)


def chapman_params(T_inf, z_peak_km, amp):
    """heating peak radius, width (local scale height at the peak) and peak rate
    so that the column integral e*qm*H equals Q_COLUMN (nondimensional)."""
    r_m = (R_EARTH + z_peak_km * 1e3) / H0
    g_m = (R_BOT / r_m) ** 2
    H_q = float(bates_T(r_m, T_inf)) / g_m
    q_m_si = Q_COLUMN / (math.e * H_q * H0)
    return dict(heat_amp=float(amp), heat_qm=q_m_si / Q_UNIT, heat_rm=r_m, heat_H=H_q)


def sound_speed_max(T_inf, mass=None):
    """max over the rest state of |v| + sqrt(T/m): the top of the Bates profile (m = 1),
    or the maximum over radii with the mean mass m(r)"""
    if mass is None:
        return float(math.sqrt(np.max(bates_T(np.array([R_BOT, R_TOP]), T_inf))))
    r = np.linspace(R_BOT, R_TOP, 513)
    return float(math.sqrt(np.max(bates_T(r, T_inf) / mass(r))))


# --------------------------------------------------------------------------
# state generators (callables of node coordinates)
def column_state(r, T_inf, mass=None):
    """(logrho, sqrt(rho) v_r, sqrt(rho) T) of the hydrostatic rest column"""
    lr = hydrostatic_logrho(r, T_inf, mass=mass)
    T = bates_T(r, T_inf)
    return np.stack([lr, np.zeros_like(lr), np.exp(0.5 * lr) * T])


def _real_sph_harm(l, m, theta, phi):
    """real orthonormal spherical harmonic; theta = colatitude"""
    from scipy.special import lpmv
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    P = lpmv(am, l, np.cos(theta)) * (-1) ** am   # remove Condon-Shortley phase
    if m == 0:
        return norm * P
    if m > 0:
        return math.sqrt(2) * norm * P * np.cos(am * phi)
    return math.sqrt(2) * norm * P * np.sin(am * phi)


@dataclass
class ShellPerturbation:
    coef: np.ndarray          # [5, 80]
    amp: float = 1e-3
    lmax: int = 8

    def angular(self, unit):
        """sum_lm c_lm Y_lm at unit vectors [..., 3] -> [5, ...]"""
        theta = np.arccos(np.clip(unit[..., 2], -1, 1))
        phi = np.arctan2(unit[..., 1], unit[..., 0])
        Y = []
        for l in range(1, self.lmax + 1):
            for m in range(-l, l + 1):
                Y.append(_real_sph_harm(l, m, theta, phi))
        Y = np.stack(Y, axis=-1)                  # [..., 80]
        return np.einsum("...j,kj->k...", Y, self.coef)

    def radial(self, r):
        return self.amp * np.sin(math.pi * (np.asarray(r) - R_BOT) / (R_TOP - R_BOT))

    def __call__(self, xyz):
        r = np.linalg.norm(xyz, axis=-1)
        return self.angular(xyz / r[..., None]) * self.radial(r)


def shell_state_fn(T_inf, pert: ShellPerturbation | None, mass=None):
    """hydrostatic Bates rest state on the shell plus smooth perturbations:
    logrho += d1, T *= (1 + d2), v += (d3, d4, d5) (so U = sqrt(rho) v)."""
    def fn(xyz):
        xyz = np.asarray(xyz, dtype=np.float64)
        r = np.linalg.norm(xyz, axis=-1)
        lr = hydrostatic_logrho(r, T_inf, mass=mass)
        T = bates_T(r, T_inf)
        v = np.zeros(xyz.shape[:-1] + (3,))
        if pert is not None:
            dd = pert(xyz)
            lr = lr + dd[0]
            T = T * (1.0 + dd[1])
            v = np.moveaxis(dd[2:5], 0, -1)
        sq = np.exp(0.5 * lr)
        U = sq[..., None] * v
        return np.stack([lr, U[..., 0], U[..., 1], U[..., 2], sq * T])
    return fn


def shell_state_at(w, X):
    """the workload's state at shell nodes X [E, N, 3] ordered element e = cell * n_rad +
    layer, node j = cz * n^2 + angular node: the angular directions are shared by every
    layer and radial node of a cell, so the separable generator runs on (cell, angular
    node) x (layer, cz); returns [E, 5, N]"""
    n = w.p + 1
    N2 = n * n
    A = 6 * w.n_ang ** 2
    Xg = np.asarray(X, dtype=np.float64).reshape(A, w.n_rad, n, N2, 3)
    unit = Xg[:, 0, 0] / np.linalg.norm(Xg[:, 0, 0], axis=-1, keepdims=True)      # [A, N2, 3]
    radii = np.linalg.norm(Xg[0, :, :, 0], axis=-1)                               # [n_rad, n]
    u = shell_state_product(w.T_inf, w.pert, unit.reshape(-1, 3), radii.ravel(),
                            mixture_mass(w.phys))                                 # [5, A*N2, n_rad*n]
    u = u.reshape(5, A, N2, w.n_rad, n)
    return np.ascontiguousarray(np.transpose(u, (1, 3, 0, 4, 2))).reshape(A * w.n_rad, 5, n * N2)


def shell_state_product(T_inf, pert, unit, radii, mass=None):
    """the same state as shell_state_fn on the product of M angular directions
    (unit [M, 3]) and K radii ([K]): returns [5, M, K]. The perturbation is separable
    (angular harmonics times a radial sine), so it is evaluated once per direction."""
    unit = np.asarray(unit, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)
    lr = hydrostatic_logrho(radii, T_inf, mass=mass)[None, :]
    T = bates_T(radii, T_inf)[None, :]
    if pert is not None:
        ang = pert.angular(unit)                    # [5, M]
        rad = pert.radial(radii)                    # [K]
        dd = ang[:, :, None] * rad[None, None, :]   # [5, M, K]
        lr = lr + dd[0]
        T = T * (1.0 + dd[1])
        v = dd[2:5]
    else:
        lr = np.broadcast_to(lr, (len(unit), len(radii)))
        T = np.broadcast_to(T, lr.shape)
        v = np.zeros((3,) + lr.shape)
    sq = np.exp(0.5 * lr)
    return np.stack([lr, sq * v[0], sq * v[1], sq * v[2], sq * T])


# --------------------------------------------------------------------------
# workloads
@dataclass
class ColumnWorkload:
    name: str
    nelem: np.ndarray          # [n_col] elements per column
    p: np.ndarray              # [n_col] degree per column
    T_inf: np.ndarray          # [n_col]
    phys: dict                 # shared physics
    col_phys: dict             # per-column arrays: heat_amp, heat_qm, heat_rm, heat_H, lam
    stretch: float | np.ndarray = 1.0    # one growth ratio, or one per column
    r_bot: float = R_BOT
    r_top: float = R_TOP
    dt: float = seconds_to_nondim(10.0)
    n_steps: int = 200

    def state(self, col, r):
        return column_state(r, self.T_inf[col], mixture_mass(self.phys))


@dataclass
class ShellWorkload:
    name: str
    p: int
    n_ang: int
    n_rad: int
    stretch: float
    T_inf: float
    phys: dict
    pert: ShellPerturbation | None
    r_bot: float = R_BOT
    r_top: float = R_TOP
    dt: float = seconds_to_nondim(60.0)
    n_steps: int = 5
    extra: dict = field(default_factory=dict)

    def state_fn(self):
        return shell_state_fn(self.T_inf, self.pert, mixture_mass(self.phys))

    @property
    def n_elem(self):
        return 6 * self.n_ang * self.n_ang * self.n_rad

    @property
    def n_dof(self):
        return self.n_elem * (self.p + 1) ** 3 * 5


def _column_phys(T_inf, z_pk, amp):
    c = chapman_params(T_inf, z_pk, amp)
    c["lam"] = sound_speed_max(T_inf)
    return c


def column_workload(seed=0, n_elem=64, p=2, n_col=1, stretch=1.0, name="column") -> ColumnWorkload:
    """A column (or several identical-shape columns) of the 1D radial model,
    100-600 km: T_inf ~ U(700, 1300) K, heating peak z_m ~ U(150, 250) km."""
    rng = np.random.default_rng(seed)
    T_inf = rng.uniform(700.0, 1300.0, n_col)
    z_pk = rng.uniform(150.0, 250.0, n_col)
    amp = np.ones(n_col)
    return _columns(name, np.full(n_col, n_elem), np.full(n_col, p), T_inf, z_pk, amp, stretch)


def graded_stretch(n_elem, first_km=2.5, length_km=500.0):
    """growth ratio that gives a first element of first_km on a column of n_elem
    elements (the 1D mesh of section 4.1.3 grows geometrically from 2.5 km); 1 when
    uniform elements are already that thin. Bisection on the (decreasing) first
    element length L (s - 1)/(s^n - 1)."""
    if length_km / n_elem <= first_km:
        return 1.0
    first = lambda s: length_km * (s - 1.0) / (s ** n_elem - 1.0)
    lo, hi = 1.0 + 1e-12, 2.0
    while first(hi) > first_km:
        hi = 1.0 + 2.0 * (hi - 1.0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if first(mid) > first_km:
            lo = mid
        else:
            hi = mid
    return float(0.5 * (lo + hi))


# --------------------------------------------------------------------------
# the parametric study of the 1D model (section 4.3): EUV efficiency x conductivity
# multiplier grids, three solar-activity cases and three sites
SWEEP_EPS = [0.2, 0.225, 0.25, 0.275, 0.3]
SWEEP_ALPHA0 = [0.5, 0.625, 0.75, 0.875, 1.0]
SWEEP_SITES = {"Millstone Hill": (42.6347, -71.4883), "Quito": (-0.1859, -78.4663),
               "Santiago": (-33.3458, -70.6786)}
# case: (day of the year of the first date, F10.7, its 81-day mean, top altitude km, elements)
SWEEP_CASES = {1: (79, 150.0, 150.0, 600.0, 28), 2: (80, 70.0, 70.0, 500.0, 26), 3: (166, 150.0, 120.0, 600.0, 28)}


def site_vector(lat_deg, lon_deg):
    """Earth-fixed unit vector of a site"""
    la, lo = math.radians(lat_deg), math.radians(lon_deg)
    return [math.cos(la) * math.cos(lo), math.cos(la) * math.sin(lo), math.sin(la)]


def sweep_case(case: int) -> ColumnWorkload:
    """the 75 columns of one case: every (efficiency, conductivity multiplier) pair at each
    site, p = 2, the case's element count on a geometric mesh with a 2.5 km first element,
    DIRK(2,2) steps of 30 s from 00 UTC of the case's first day (sub-solar longitude 180
    degrees at t = 0), EUVAC heating at the case's F10.7bar. The initial state is a
    hydrostatic Bates column with T_inf = 500 K + 3 K x F10.7bar (synthetic: the paper starts
    from empirical profiles that are not available)."""
    day, f107, f81, top_km, n_elem = SWEEP_CASES[case]
    fbar = 0.5 * (f107 + f81)
    T_inf = 500.0 + 3.0 * fbar
    combos = [(site, e, a) for site in SWEEP_SITES for e in SWEEP_EPS for a in SWEEP_ALPHA0]
    n_col = len(combos)
    r_top = (R_EARTH + top_km * 1e3) / H0
    phys = base_physics(1)
    phys.update(euvac_physics(f107bar=fbar, day=float(day)))
    phys["heating_model"] = 1
    phys["sun_lon0"] = math.pi
    cp = _column_phys(T_inf, 200.0, 0.0)
    phys.update(cp)
    col_phys = {k: np.full(n_col, float(v)) for k, v in cp.items()}
    col_phys["euv_eps"] = np.array([e for _, e, _ in combos])
    col_phys["alpha0c"] = np.array([a for _, _, a in combos])
    col_phys["site"] = np.array([site_vector(*SWEEP_SITES[s]) for s, _, _ in combos])
    w = ColumnWorkload(name="sweep-case%d" % case, nelem=np.full(n_col, n_elem, np.int32),
                       p=np.full(n_col, 2, np.int32), T_inf=np.full(n_col, T_inf), phys=phys, col_phys=col_phys,
                       stretch=graded_stretch(n_elem, 2.5, top_km - 100.0), r_top=r_top,
                       dt=seconds_to_nondim(30.0), n_steps=8640)
    w.extra = {"combos": combos, "fbar": fbar, "day": day, "r400": (R_EARTH + 400e3) / H0}
    return w


def column_batch_workload(seed=0, n_col=4096, name="column-batch") -> ColumnWorkload:
    """The parametric sweep: n_col columns, elements ~ U{32..256}, p ~ U{2,3,4},
    T_inf ~ U(600, 1500) K, heating multiplier ~ U(0.5, 3), z_m ~ U(150, 250) km.
    Every column is graded geometrically from a 2.5 km first element."""
    rng = np.random.default_rng(seed)
    nelem = rng.integers(32, 257, n_col)
    p = rng.integers(2, 5, n_col)
    T_inf = rng.uniform(600.0, 1500.0, n_col)
    amp = rng.uniform(0.5, 3.0, n_col)
    z_pk = rng.uniform(150.0, 250.0, n_col)
    w = _columns(name, nelem, p, T_inf, z_pk, amp, 1.0)
    w.stretch = np.array([graded_stretch(int(e)) for e in nelem])
    w.n_steps = 100
    return w


def _columns(name, nelem, p, T_inf, z_pk, amp, stretch):
    cp = [_column_phys(T_inf[i], z_pk[i], amp[i]) for i in range(len(nelem))]
    col_phys = {k: np.array([c[k] for c in cp]) for k in cp[0]}
    phys = base_physics(1)
    for k in col_phys:
        phys[k] = float(col_phys[k][0])
    return ColumnWorkload(name=name, nelem=np.asarray(nelem, np.int32), p=np.asarray(p, np.int32),
                          T_inf=np.asarray(T_inf, np.float64), phys=phys, col_phys=col_phys,
                          stretch=stretch)


def shell_workload(seed=0, p=3, n_ang=16, n_rad=16, stretch=1.15, name="shell",
                   perturb=True, heating=True, rotation=True) -> ShellWorkload:
    """3D shell 100-600 km: Bates hydrostatic state (T_inf ~ U(700, 1300) K) plus
    spherical-harmonic perturbations up to l = 8 of amplitude 1e-3, rotation about z,
    day-side Chapman heating with the sub-solar point at (0, 0) at t = 0."""
    rng = np.random.default_rng(seed)
    T_inf = float(rng.uniform(700.0, 1300.0))
    z_pk = float(rng.uniform(150.0, 250.0))
    coef = rng.standard_normal((5, 80)) / math.sqrt(80.0)
    phys = base_physics(3)
    phys.update(chapman_params(T_inf, z_pk, 1.0 if heating else 0.0))
    phys["lam"] = sound_speed_max(T_inf) + (0.01 if perturb else 0.0)
    if not rotation:
        phys["omega"] = [0.0, 0.0, 0.0]
    pert = ShellPerturbation(coef) if perturb else None
    return ShellWorkload(name=name, p=p, n_ang=n_ang, n_rad=n_rad, stretch=stretch,
                         T_inf=T_inf, phys=phys, pert=pert)


def with_composition(w):
    """the workload with the variable composition of section 2.1.1: the synthetic fits,
    the rest state in hydrostatic balance with m(r) (the state generators follow the
    physics set), and lambda_max = max sqrt(T/m) over the rest state"""
    import dataclasses
    phys = dict(w.phys)
    phys.update(composition_physics())
    mass = mixture_mass(phys)
    if isinstance(w, ShellWorkload):
        phys["lam"] = sound_speed_max(w.T_inf, mass) + (0.01 if w.pert is not None else 0.0)
        return dataclasses.replace(w, phys=phys, name=w.name + "-mixture")
    col_phys = dict(w.col_phys)
    col_phys["lam"] = np.array([sound_speed_max(float(T), mass) for T in w.T_inf])
    phys["lam"] = float(col_phys["lam"][0])
    return dataclasses.replace(w, phys=phys, col_phys=col_phys, name=w.name + "-mixture")


def config_column(seed=0):
    """1D column, 64 uniform elements, p = 2, 200 DIRK(3,3) steps of 10 s"""
    return column_workload(seed=seed, n_elem=64, p=2, name="column-64e-p2")


def config_shell_p3(seed=0):
    """cubed sphere 6x16x16 x 16 layers, stretch 1.15, p = 3 (7,864,320 DOF)"""
    return shell_workload(seed=seed, p=3, n_ang=16, n_rad=16, stretch=1.15, name="shell-6x16x16x16-p3")


def config_shell_p4(seed=0):
    """cubed sphere 6x32x32 x 24 layers, stretch 1.15, p = 4 (92,160,000 DOF)"""
    return shell_workload(seed=seed, p=4, n_ang=32, n_rad=24, stretch=1.15, name="shell-6x32x32x24-p4")


def fullsize_workload(name):
    """the benchmark shells of the full-size parity fixtures: the 7.9M-DOF p = 3 and the
    92M-DOF p = 4 shells, and the p = 3 shell with the variable composition and EUVAC
    heating (June solstice, F10.7bar 150) in place of the prescribed profile"""
    import dataclasses
    if name == "shell-p3":
        return config_shell_p3(0)
    if name == "shell-p4":
        return config_shell_p4(0)
    if name == "shell-p3-mixture-euvac":
        w = with_composition(config_shell_p3(0))
        phys = dict(w.phys)
        phys.update(euvac_physics(f107bar=150.0, day=172.0))
        phys["heating_model"] = 1
        phys["heat_amp"] = 0.0
        return dataclasses.replace(w, phys=phys, name=w.name + "-euvac")
    raise ValueError("unknown full-size workload " + name)


def tangent(shape, seed=1):
    """unit-norm Gaussian tangent vector"""
    v = np.random.default_rng(seed).standard_normal(shape)
    return v / np.linalg.norm(v)


def uniform_state(d, rho_log=-0.3, U=(0.05, -0.02, 0.03), Theta=1.1):
    """a constant state (free-stream tests)"""
    return np.array([rho_log, *U[:d], Theta])
