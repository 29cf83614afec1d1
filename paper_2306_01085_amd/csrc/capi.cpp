// C-ABI entry points of libdgthermo: argument validation, ownership of device
// buffers, error reporting. Every device computation is delegated to the HIP
// kernels of shell.hip, column.hip and solver.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

namespace dg {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

// ---------------------------------------------------------------- allocation-free residual
// dg_residual_noalloc keeps the face traces of its R(u) evaluation in this file-scope device
// array instead of the mesh's trace buffer. Every GPU the library runs on holds its own
// copy for the life of the process; host code never names the array itself (its name is a
// host-side stand-in there) but the per-device address that hipGetSymbolAddress returns.
constexpr int64_t kScratchDoubles = DG_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// the current device's address of the scratch array, looked up once per device
static dg_status_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_error(std::string("scratch: ") + hipGetErrorString(e));
    return DG_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("scratch: device index out of range");
    return DG_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("scratch: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
      return DG_ERR_HIP;
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return DG_OK;
}

dg_status_t build_shell(dg_mesh_s* m, const dg_mesh_desc_t& d);
dg_status_t build_columns(dg_mesh_s* m, const dg_mesh_desc_t& d, const dg_physics_t& ph);

void fill_phys(PhysC& P, const dg_physics_t& in) {
  P.gamma = in.gamma;
  P.inv_gm = 1.0 / (in.gamma * in.m);
  P.c_visc = 1.0 / std::sqrt(in.gamma * in.Gr);
  P.c_cond = (1.0 / in.Pr) * std::sqrt(in.gamma / in.Gr);
  P.c_diss = (in.gamma - 1.0) * std::sqrt(in.gamma / in.Gr);
  P.m = in.m;
  P.inv_m = 1.0 / in.m;
  P.nu_r = in.nu_r;
  P.alpha_r = in.alpha_r;
  P.alpha0c = in.alpha0c;
  P.kexp = 0.69;
  P.lam = in.lam;
  P.T_bot = in.T_bot;
  P.r_ref2 = in.r_ref * in.r_ref;
  for (int k = 0; k < 3; ++k) P.om[k] = in.omega[k];
  P.cent = in.Fr * in.Fr / in.gamma;
  P.cor = 2.0 * in.Fr / std::sqrt(in.gamma);
  P.heat_amp = in.heat_amp;
  P.heat_qm = in.heat_qm;
  P.heat_rm = in.heat_rm;
  P.heat_inv_H = 1.0 / in.heat_H;
  P.sun_lat = in.sun_lat;
  P.sun_lon0 = in.sun_lon0;
  P.sun_rate = in.sun_rate;
  P.euv = in.heating_model == 1 ? 1 : 0;
  P.euv_tab = nullptr;
  P.r_ref = in.r_ref;
  P.euv_hfac = 1.0 / (in.m * in.r_ref * in.r_ref);
  if (P.euv && in.euv_day > 0) P.sun_lat = euvac_declination(in.euv_day);
  P.bc_mode = in.bc_mode;
  for (int c = 0; c < 5; ++c) P.bc_state[c] = in.bc_state[c];
  P.comp = in.composition ? 1 : 0;
  for (int i = 0; i < 6; ++i) {
    P.comp_a[i] = in.composition ? in.comp_a[i] : 0.0;
    P.comp_b[i] = in.composition ? in.comp_b[i] : 0.0;
  }
}

// radial extent of a mesh
static void radial_range(const dg_mesh_s* m, double& lo, double& hi) {
  if (m->kind == DG_MESH_SHELL) {
    lo = m->h_edges.front();
    hi = m->h_edges.back();
    return;
  }
  lo = m->h_geo[0];
  hi = m->h_geo[0] + m->h_geo[1];
  for (size_t e = 0; 2 * e < m->h_geo.size(); ++e) {
    lo = std::min(lo, m->h_geo[2 * e]);
    hi = std::max(hi, m->h_geo[2 * e] + m->h_geo[2 * e + 1]);
  }
}

// the physics of a mesh, with the EUVAC bin constants in a mesh-owned device table
static dg_status_t set_phys(dg_mesh_s* m, const dg_physics_t& in) {
  double lo, hi;
  radial_range(m, lo, hi);
  if (!composition_valid(in, lo, hi)) {
    set_error("dg_mesh: the composition's mass fractions leave [0, 1] over the mesh");
    return DG_ERR_ARG;
  }
  fill_phys(m->phys, in);
  if (!m->phys.euv) return DG_OK;
  if (m->kind == DG_MESH_COLUMNS) {
    std::vector<double> tab;
    col_euv_tables(in, m->n_col, tab);
    if (!m->d_euv_cols && hipMalloc(&m->d_euv_cols, tab.size() * sizeof(double)) != hipSuccess) {
      set_error("dg_mesh: device allocation of the column EUVAC tables failed");
      return DG_ERR_ALLOC;
    }
    DG_HIP_CHECK(hipDeviceSynchronize());
    DG_HIP_CHECK(hipMemcpy(m->d_euv_cols, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  double tab[EUVT];
  euvac_constants(in, tab);
  if (!m->d_euv && hipMalloc(&m->d_euv, sizeof(tab)) != hipSuccess) {
    set_error("dg_mesh: device allocation of the EUVAC table failed");
    return DG_ERR_ALLOC;
  }
  DG_HIP_CHECK(hipDeviceSynchronize());
  DG_HIP_CHECK(hipMemcpy(m->d_euv, tab, sizeof(tab), hipMemcpyHostToDevice));
  m->phys.euv_tab = m->d_euv;
  return DG_OK;
}

static bool phys_ok(const dg_physics_t& p) {
  const bool euv_ok = p.heating_model == 0 ||
                      (p.heating_model == 1 && p.euv_eps >= 0 && p.euv_sun_dist > 0 && p.euv_q_scale > 0 &&
                       p.euv_col_scale > 0 && p.euv_chi[0] >= 0 && p.euv_chi[1] >= 0 && p.euv_chi[2] >= 0 &&
                       p.euv_chi[3] >= 0 && std::isfinite(p.euv_f107) && p.r_ref > 0);
  return p.gamma > 1.0 && p.Gr > 0 && p.Pr > 0 && p.m > 0 && p.heat_H > 0 && std::isfinite(p.lam) &&
         (p.bc_mode == 0 || p.bc_mode == 1) && euv_ok;
}

static void free_mesh(dg_mesh_s* m) {
  void* ptrs[] = {m->d_ang,  m->d_edges,  m->d_cnbr,  m->d_cface,     m->d_cmap,      m->d_off,
                  m->d_prev, m->d_next,   m->d_geo,   m->d_col,       m->d_cpar,      m->d_fn64,
                  m->d_fn32, m->d_plist[0], m->d_plist[1], m->d_plist[2], m->d_bstate, m->d_coloff,
                  m->d_cols_ws, m->ws_norm, m->ws_X, m->ws_Y, m->d_bf16op, m->d_euv, m->d_euv_cols,
                  m->d_fd, m->d_quad};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  free_workspace(m);
  delete m;
}

}  // namespace dg

using namespace dg;

extern "C" {

const char* dg_last_error(void) { return dg::g_err.c_str(); }
int32_t dg_version(void) { return 1; }

dg_status_t dg_profile_enable(dg_mesh_t m, int32_t on) {
  if (!m) {
    set_error("dg_profile_enable: null mesh");
    return DG_ERR_ARG;
  }
  m->prof = on != 0;
  return DG_OK;
}

dg_status_t dg_profile_read(dg_mesh_t m, double* ms, int64_t* counts, int32_t n, int32_t reset) {
  if (!m || !ms || !counts || n < 1) {
    set_error("dg_profile_read: invalid argument");
    return DG_ERR_ARG;
  }
  for (auto& ev : m->prof_events) {
    float el = 0.f;
    DG_HIP_CHECK(hipEventSynchronize(ev.b));
    DG_HIP_CHECK(hipEventElapsedTime(&el, ev.a, ev.b));
    if (ev.id >= 0 && ev.id < DG_PROF_SLOTS) {
      m->prof_ms[ev.id] += el;
      m->prof_cnt[ev.id] += 1;
    }
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  m->prof_events.clear();
  for (int i = 0; i < n; ++i) {
    ms[i] = i < DG_PROF_SLOTS ? m->prof_ms[i] : 0.0;
    counts[i] = i < DG_PROF_SLOTS ? m->prof_cnt[i] : 0;
  }
  if (reset)
    for (int i = 0; i < DG_PROF_SLOTS; ++i) {
      m->prof_ms[i] = 0;
      m->prof_cnt[i] = 0;
    }
  return DG_OK;
}

dg_status_t dg_set_option(dg_mesh_t m, const char* name, int64_t value) {
  if (!m || !name) {
    set_error("dg_set_option: null argument");
    return DG_ERR_ARG;
  }
  if (std::strcmp(name, "shell_pass1_config") == 0 && value >= 0 && value <= 5) {
    m->tune_p1 = (int)value;
    return DG_OK;
  }
  if (std::strcmp(name, "columns_grid") == 0 && value >= 1 && value <= 65536) {
    m->tune_cols_grid = (int)value;
    return DG_OK;
  }
  if (std::strcmp(name, "line_pc_every") == 0 && value >= 1 && value <= 1000000) {
    m->line_pc_every = (int)value;
    return DG_OK;
  }
  if (std::strcmp(name, "line_solve_config") == 0 && value >= -1 && value <= 5) {
    m->tune_lsolve = (int)value;
    return DG_OK;
  }
  if (std::strcmp(name, "column_quadrature") == 0 && (value == 0 || value == 1) && m->kind == DG_MESH_COLUMNS) {
    m->col_quad = (int)value;
    return DG_OK;
  }
  if (std::strcmp(name, "columns_jac_every") == 0 && value >= 1 && value <= 1000000) {
    m->cols_jac_every = (int)value;
    return DG_OK;
  }
  if (std::strcmp(name, "columns_jac_slow_pct") == 0 && value >= 1 && value <= 100) {
    m->cols_jac_slow_pct = (int)value;
    return DG_OK;
  }
  if (std::strcmp(name, "columns_jac_stale_its") == 0 && value >= 1 && value <= 1000) {
    m->cols_jac_stale = (int)value;
    return DG_OK;
  }
  if (std::strcmp(name, "line_pc_precision") == 0 && (value == 64 || value == 32 || value == 16)) {
    m->line_pc_prec = (int)value;
    return DG_OK;
  }
  set_error(std::string("dg_set_option: unknown option or value: ") + name);
  return DG_ERR_ARG;
}

dg_status_t dg_mesh_create(const dg_mesh_desc_t* desc, const dg_physics_t* phys, void* stream, dg_mesh_t* out) {
  if (!desc || !phys || !out) {
    set_error("dg_mesh_create: null argument");
    return DG_ERR_ARG;
  }
  *out = nullptr;
  if (!phys_ok(*phys)) {
    set_error("dg_mesh_create: invalid physics parameters");
    return DG_ERR_ARG;
  }
  dg_mesh_s* m = new (std::nothrow) dg_mesh_s();
  if (!m) {
    set_error("dg_mesh_create: out of host memory");
    return DG_ERR_ALLOC;
  }
  m->kind = desc->kind;
  dg_status_t st;
  if (desc->kind == DG_MESH_SHELL)
    st = build_shell(m, *desc);
  else if (desc->kind == DG_MESH_COLUMNS)
    st = build_columns(m, *desc, *phys);
  else {
    set_error("dg_mesh_create: unknown mesh kind");
    st = DG_ERR_ARG;
  }
  if (st != DG_OK) {
    free_mesh(m);
    return st;
  }
  st = set_phys(m, *phys);
  if (st != DG_OK) {
    free_mesh(m);
    return st;
  }
  hipError_t e1 = hipMalloc(&m->d_fn64, m->fn_len * sizeof(double));
  hipError_t e2 = hipMalloc(&m->d_fn32, m->fn_len * sizeof(float));
  // the finite-difference J v's two state-sized buffers and norm partials: allocated here so
  // that no later call allocates
  hipError_t e4 = hipMalloc(&m->d_fd, fd_buffer_len(m->n_dof) * sizeof(double));
  if (e1 != hipSuccess || e2 != hipSuccess || e4 != hipSuccess) {
    set_error("dg_mesh_create: device allocation of the face traces or finite-difference buffers failed");
    free_mesh(m);
    return DG_ERR_ALLOC;
  }
  if (m->kind == DG_MESH_SHELL && (m->p == 3 || m->p == 4)) {
    const std::vector<uint16_t> ops = bf16_operators(m->p);
    if (hipMalloc(&m->d_bf16op, ops.size() * sizeof(uint16_t)) != hipSuccess ||
        hipMemcpy(m->d_bf16op, ops.data(), ops.size() * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("dg_mesh_create: device allocation of the bf16 operators failed");
      free_mesh(m);
      return DG_ERR_ALLOC;
    }
  }
  hipError_t e3 = hipStreamSynchronize((hipStream_t)stream);
  if (e3 != hipSuccess) {
    set_error(std::string("dg_mesh_create: ") + hipGetErrorString(e3));
    free_mesh(m);
    return DG_ERR_HIP;
  }
  // set-up of the allocation-free residual: the scratch array's address on this device
  double* scr = nullptr;
  st = scratch_address(&scr);
  if (st != DG_OK) {
    free_mesh(m);
    return st;
  }
  *out = m;
  return DG_OK;
}

dg_status_t dg_mesh_destroy(dg_mesh_t m) {
  if (!m) return DG_OK;
  (void)hipDeviceSynchronize();
  free_mesh(m);
  return DG_OK;
}

dg_status_t dg_mesh_set_physics(dg_mesh_t m, const dg_physics_t* phys) {
  if (!m || !phys || !phys_ok(*phys)) {
    set_error("dg_mesh_set_physics: invalid argument");
    return DG_ERR_ARG;
  }
  const dg_status_t st = set_phys(m, *phys);
  if (st != DG_OK) return st;
  if (m->kind == DG_MESH_COLUMNS) {
    std::vector<double> cpar;
    col_params(*phys, m->n_col, cpar);
    DG_HIP_CHECK(hipDeviceSynchronize());
    DG_HIP_CHECK(hipMemcpy(m->d_cpar, cpar.data(), cpar.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  return DG_OK;
}

dg_status_t dg_mesh_info(dg_mesh_t m, int64_t* n_dof, int64_t* n_elem, int32_t* n_fields, int32_t* dim) {
  if (!m) {
    set_error("dg_mesh_info: null mesh");
    return DG_ERR_ARG;
  }
  if (n_dof) *n_dof = m->n_dof;
  if (n_elem) *n_elem = m->n_elem;
  if (n_fields) *n_fields = m->nf;
  if (dim) *dim = m->dim;
  return DG_OK;
}

dg_status_t dg_mesh_nodes(dg_mesh_t m, double* xyz, int64_t n_values) {
  if (!m || !xyz) {
    set_error("dg_mesh_nodes: null argument");
    return DG_ERR_ARG;
  }
  const int64_t nodes = m->n_dof / m->nf;
  if (n_values != nodes * m->dim) {
    set_error("dg_mesh_nodes: n_values must be n_nodes * dim");
    return DG_ERR_ARG;
  }
  if (m->kind == DG_MESH_SHELL) {
    Gll g = make_gll(m->p);
    const int n = m->n, N2 = m->N2, N = m->N;
    for (int64_t e = 0; e < m->n_elem; ++e) {
      const int cell = (int)(e / m->n_rad), k = (int)(e % m->n_rad);
      const double rk = m->h_edges[k], hk = m->h_edges[k + 1] - rk;
      const double* ang = &m->h_ang[(size_t)cell * 13 * N2];
      for (int j = 0; j < N; ++j) {
        const int ja = j % N2, cz = j / N2;
        const double r = rk + 0.5 * (g.x[cz] + 1.0) * hk;
        for (int d = 0; d < 3; ++d) xyz[(e * N + j) * 3 + d] = r * ang[(10 + d) * N2 + ja];
      }
      (void)n;
    }
  } else {
    int64_t i = 0;
    for (int64_t e = 0; e < m->n_elem; ++e) {
      Gll g = make_gll(m->elem_p[e]);
      for (int j = 0; j < g.n; ++j) xyz[i++] = m->h_geo[2 * e] + 0.5 * (g.x[j] + 1.0) * m->h_geo[2 * e + 1];
    }
  }
  return DG_OK;
}

dg_status_t dg_mesh_col_offsets(dg_mesh_t m, int64_t* off, int64_t n) {
  if (!m || !off || m->kind != DG_MESH_COLUMNS || n != m->n_col + 1) {
    set_error("dg_mesh_col_offsets: needs a column mesh and n = n_col + 1");
    return DG_ERR_ARG;
  }
  for (int64_t i = 0; i <= m->n_col; ++i) off[i] = m->col_off[i];
  return DG_OK;
}

dg_status_t dg_residual(dg_mesh_t m, double t, const double* u, double* r, int64_t n_dof, void* stream) {
  if (!m || !u || !r || n_dof != m->n_dof || u == r) {
    set_error("dg_residual: null pointer, aliasing or n_dof mismatch");
    return DG_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  return m->kind == DG_MESH_SHELL ? shell_residual(m, t, u, r, s) : col_residual(m, t, u, r, s);
}

dg_status_t dg_residual_noalloc(dg_mesh_t m, double t, const double* u, double* r, int64_t n_dof, void* stream) {
  if (!m || !u || !r || n_dof != m->n_dof || u == r) {
    set_error("dg_residual_noalloc: null pointer, aliasing or n_dof mismatch");
    return DG_ERR_ARG;
  }
  if (m->fn_len > kScratchDoubles) {
    set_error("dg_residual_noalloc: the mesh's face traces (" + std::to_string(m->fn_len * 8) +
              " bytes) exceed the scratch array (" + std::to_string((long long)DG_NOALLOC_SCRATCH_BYTES) +
              " bytes); use dg_residual");
    return DG_ERR_ARG;
  }
  double* scr = nullptr;
  const dg_status_t st = scratch_address(&scr);
  if (st != DG_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  return m->kind == DG_MESH_SHELL ? shell_residual_traces(m, t, u, r, scr, s) : col_residual_traces(m, t, u, r, scr, s);
}

dg_status_t dg_jvp(dg_mesh_t m, double t, const double* u, const void* v, void* jv, int64_t n_dof, dg_prec_t prec,
                   void* stream) {
  if (!m || !u || !v || !jv || n_dof != m->n_dof || jv == v || (const void*)u == jv) {
    set_error("dg_jvp: null pointer, aliasing or n_dof mismatch");
    return DG_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  if (prec == DG_F64)
    return m->kind == DG_MESH_SHELL ? shell_jvp64(m, t, u, (const double*)v, (double*)jv, s)
                                    : col_jvp64(m, t, u, (const double*)v, (double*)jv, s);
  if (prec == DG_F32)
    return m->kind == DG_MESH_SHELL ? shell_jvp32(m, t, u, (const float*)v, (float*)jv, s)
                                    : col_jvp32(m, t, u, (const float*)v, (float*)jv, s);
  if (prec == DG_BF16 && m->kind == DG_MESH_SHELL) return shell_jvp_bf16(m, t, u, (const float*)v, (float*)jv, s);
  if (prec == DG_F64_FD) return jvp_fd(m, t, u, (const double*)v, (double*)jv, s);
  set_error("dg_jvp: precision not available");
  return DG_ERR_UNSUPPORTED;
}

dg_status_t dg_implicit_step(dg_mesh_t m, double t, double dt, double* u, int64_t n_dof,
                             const dg_solver_opts_t* opts, dg_step_stats_t* stats, void* stream) {
  if (!m || !u || !opts || n_dof != m->n_dof || !(dt > 0) || !std::isfinite(t)) {
    set_error("dg_implicit_step: invalid argument");
    return DG_ERR_ARG;
  }
  if ((opts->scheme != 33 && opts->scheme != 22) || opts->gmres_m < 1 || opts->gmres_m > 32 ||
      opts->max_newton < 1 || opts->max_restarts < 1 || !(opts->newton_rtol > 0) || !(opts->gmres_rtol > 0) ||
      (opts->jvp_prec != DG_F64 && opts->jvp_prec != DG_F32 && opts->jvp_prec != DG_BF16 &&
       opts->jvp_prec != DG_F64_FD) || opts->precond < 0 ||
      opts->precond > 2 ||
      opts->guess < 0 || opts->guess > 1 || opts->forcing < 0 || opts->forcing > 1 || !(opts->filter_rate >= 0) ||
      !std::isfinite(opts->filter_rate) || opts->n_rb < 0 || opts->n_rb > 8) {
    set_error("dg_implicit_step: invalid solver options");
    return DG_ERR_ARG;
  }
  return implicit_step(m, t, dt, u, *opts, stats, (hipStream_t)stream);
}

dg_status_t dg_columns_integrate(dg_mesh_t m, double t0, double dt, int32_t n_steps, double* u, int64_t n_dof,
                                 const dg_solver_opts_t* opts, int32_t* newton_host, int32_t* status_host,
                                 void* stream) {
  if (!m || !u || !opts || m->kind != DG_MESH_COLUMNS || n_dof != m->n_dof || !(dt > 0) || n_steps < 0 ||
      (opts->scheme != 33 && opts->scheme != 22) || opts->max_newton < 1 || !(opts->newton_rtol > 0) ||
      !(opts->filter_rate >= 0) || !std::isfinite(opts->filter_rate)) {
    set_error("dg_columns_integrate: invalid argument (needs a column mesh)");
    return DG_ERR_ARG;
  }
  if (n_steps == 0) return DG_OK;
  return columns_integrate(m, t0, dt, n_steps, u, *opts, newton_host, status_host, (hipStream_t)stream);
}

}  // extern "C"
