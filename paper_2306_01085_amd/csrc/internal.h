// Host-side definition of a mesh handle and helpers shared by the library's
// translation units.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/dgthermo.h"
#include "dg_common.h"

#define DG_PROF_SLOTS 16

namespace dg {

void set_error(const std::string& msg);

#define DG_HIP_CHECK(call)                                                                 \
  do {                                                                                     \
    hipError_t err_ = (call);                                                              \
    if (err_ != hipSuccess) {                                                              \
      ::dg::set_error(std::string(#call) + ": " + hipGetErrorString(err_));                \
      return DG_ERR_HIP;                                                                   \
    }                                                                                      \
  } while (0)

// GLL nodes, weights and differentiation matrix D[i][j] = l_j'(x_i) for degree p
struct Gll {
  int p, n;
  std::vector<double> x, w, D;
};
Gll make_gll(int p);

// the same tables flattened for kernel arguments (D[i*n + j])
struct GllC {
  double D[25], x[5], w[5];
};
GllC make_gllc(int p);

// Gauss quadrature of the over-integrated 1D residual: nq = p + 2 Gauss-Legendre points x, w
// on [-1, 1], the nodal (GLL) basis there, V[g][j] = l_j(x_g), its derivative Dg[g][j] =
// l_j'(x_g), and the inverse Mi of the exact reference mass matrix sum_g w_g l_i l_j
struct QuadC {
  int nq;
  double x[6], w[6];
  double V[30], Dg[30];   // [g * n + j]
  double Mi[25];          // [i * n + j]
};
QuadC make_quadc(int p);

// per-column parameters of a column mesh, CPAR per column: heat_amp, heat_qm, heat_rm,
// 1 / heat_H, lam, alpha0c, site unit vector (3; zero: the Sun overhead)
constexpr int CPAR = 9;
void col_params(const dg_physics_t& ph, int n_col, std::vector<double>& cpar);
// per-column EUVAC bin constants [n_col][EUVT] (efficiency and F10.7bar per column)
void col_euv_tables(const dg_physics_t& ph, int n_col, std::vector<double>& tab);
// EUVAC heating constants of the 37 bins (EUVT values, the layout heating_euvac reads) and
// the declination of day N_d (euvac.cpp)
void euvac_constants(const dg_physics_t& in, double* tab);
double euvac_declination(double day);
// true unless the composition is on and a fitted mass fraction leaves [0, 1] (or their sum
// exceeds 1) somewhere in [r_lo, r_hi]
bool composition_valid(const dg_physics_t& ph, double r_lo, double r_hi);
// modal filter of degree p on the GLL nodes: F = I - (1 - sigma) P_p(x_a) c_p(i), where
// c_p(i) = w_i P_p(x_i) / sum_j w_j P_p(x_j)^2 extracts the coefficient of the Legendre
// polynomial P_p (GLL quadrature is exact for P_k P_p with k < p, so the lower modes
// are untouched); F[a*n + i]
struct FiltC {
  double F[25];
};
FiltC make_filter(int p, double sigma);

// device view of the shell geometry and connectivity (kernel argument)
struct ShellDev {
  int n_ang, n_rad, E;
  const double* ang;     // [A][13][n2]: A1 (3), A2 (3), A3 (3), Jang, unit position (3)
  const double* edges;   // [n_rad + 1] layer interfaces
  const int* cnbr;       // [A][4] neighbour cell across angular faces 0..3
  const int* cface;      // [A][4] the neighbour's face index
  const int* cmap;       // [A][4][n] along-edge index s -> neighbour's along-edge index
};

// device view of a batch of columns (kernel argument)
struct ColDev {
  int E;                 // total elements
  const int64_t* off;    // [E] DOF offset of the element
  const int* prev;       // [E] element below (-1: lower boundary)
  const int* next;       // [E] element above (-1: upper boundary)
  const double* geo;     // [E][2] bottom radius, thickness
  const int* col;        // [E] column of the element
  const double* cpar;    // [n_col][CPAR] per-column parameters (col_params)
  const double* euv;     // [n_col][EUVT] per-column EUVAC bin constants, or null (the mesh's table)
};

struct Workspace;   // implicit-step buffers (solver.hip)

}  // namespace dg

struct dg_mesh_s {
  int kind = 0;
  int dim = 3, nf = 5;
  int64_t n_dof = 0, n_elem = 0;
  dg::PhysC phys{};
  // shell
  int p = 0, n = 0, N = 0, N2 = 0, n_ang = 0, n_rad = 0, A = 0;
  double* d_ang = nullptr;
  double* d_edges = nullptr;
  int* d_cnbr = nullptr;
  int* d_cface = nullptr;
  int* d_cmap = nullptr;
  std::vector<double> h_ang, h_edges;
  // columns
  int n_col = 0;
  std::vector<int> col_nelem, col_p;
  std::vector<int64_t> col_off;          // [n_col + 1]
  std::vector<int> elem_p;               // [E]
  std::vector<double> h_geo;             // [E][2]
  int64_t* d_off = nullptr;
  int* d_prev = nullptr;
  int* d_next = nullptr;
  double* d_geo = nullptr;
  int* d_col = nullptr;
  double* d_cpar = nullptr;
  double* d_euv_cols = nullptr;   // per-column EUVAC bin constants (heating model 1 on columns)
  int* d_plist[3] = {nullptr, nullptr, nullptr};   // element ids of degree 2, 3, 4
  int plist_n[3] = {0, 0, 0};
  // face-flux traces (one buffer per precision)
  double* d_fn64 = nullptr;
  float* d_fn32 = nullptr;
  uint16_t* d_bf16op = nullptr;   // dense bf16 reference operators of the BF16 J v (p = 3 shells)
  double* d_euv = nullptr;        // EUVAC bin constants [EUVT] (heating model 1)
  bool krylov_bf16 = false;       // the implicit step in progress takes the BF16 J v
  bool krylov_fd = false;         // the implicit step in progress takes the finite-difference J v
  double* d_fd = nullptr;         // finite-difference J v: [2][n_dof] states and the norm partials
  int line_pc_every = 1;          // rebuild the radial-line preconditioner every this many steps
  int line_pc_prec = 32;          // storage precision of its factors: 64, 32 or 16 (bf16)
  int tune_lsolve = -1;           // launch configuration of its substitution (0..5, -1 automatic)
  int64_t fn_len = 0;
  dg::Workspace* ws = nullptr;
  // batched-column solver state (dg_columns_integrate)
  int* d_bstate = nullptr;               // [8][n_col] ints: E, p, first element, order, stats, counter
  int64_t* d_coloff = nullptr;
  dg::QuadC* d_quad = nullptr;    // columns: Gauss tables of degrees 2, 3, 4 (over-integration)
  int col_quad = 0;               // columns: 0 GLL collocation, 1 over-integrated (option "column_quadrature")
  double* d_cols_ws = nullptr;
  int64_t cols_ws_len = 0;
  int col_max_dof = 0;
  int tune_cols_grid = 2048;             // persistent wavefronts (dg_set_option "columns_grid")
  int cols_jac_every = 32;               // chord Jacobian of the column batch rebuilt every this many steps,
  int cols_jac_slow_pct = 75;            // within a stage when an iteration leaves |G| above this percentage
  int cols_jac_stale = 5;                // and after a step with a stage of more than this many iterations
  int tune_p1 = 2;
  // learned warm start (dg_warmstart_set / dg_warmstart_record)
  struct dg_mlp_s* ws_mlp = nullptr;
  float* ws_norm = nullptr;              // device: x_mean [n_in], x_scale [n_in], y_mean [n_out], y_scale [n_out]
  float* ws_X = nullptr;                 // device features [E][n_in]
  float* ws_Y = nullptr;                 // device outputs [E][n_out]
  float* rec_x = nullptr;
  float* rec_y = nullptr;
  int64_t rec_cap = 0, rec_count = 0;
  int rec_every = 1;
  int64_t rec_phase = 0;                       // pass-1 launch configuration (dg_set_option)
  // per-kernel event timing (dg_profile_enable / dg_profile_read)
  bool prof = false;
  struct ProfEv { int id; hipEvent_t a, b; };
  std::vector<ProfEv> prof_events;
  double prof_ms[DG_PROF_SLOTS] = {};
  int64_t prof_cnt[DG_PROF_SLOTS] = {};

  dg::ShellDev shell() const {
    return dg::ShellDev{n_ang, n_rad, (int)n_elem, d_ang, d_edges, d_cnbr, d_cface, d_cmap};
  }
  dg::ColDev cols() const {
    return dg::ColDev{(int)n_elem, d_off, d_prev, d_next, d_geo, d_col, d_cpar, d_euv_cols};
  }
};

namespace dg {
// records a pair of events around the enclosed launches when profiling is on
struct ProfScope {
  dg_mesh_s* m;
  int id;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(dg_mesh_s* m_, int id_, hipStream_t s_) : m(m_), id(id_), s(s_) {
    if (m->prof && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    hipEvent_t b = nullptr;
    if (m->prof && a && hipEventCreate(&b) == hipSuccess) {
      (void)hipEventRecord(b, s);
      m->prof_events.push_back({id, a, b});
    }
  }
};
// Launch kernel k(args) on s. With the mesh's profiling on, the dispatch itself records the
// start and stop events (hipExtLaunchKernel), so the interval is the kernel's execution
// alone, as a kernel trace reports it, without the gap to the previous dispatch that
// events recorded around the launch include. The arguments are converted to the kernel's
// parameter types first.
template <typename... Prm, typename... Arg>
inline void launch_timed(dg_mesh_s* m, int id, void (*k)(Prm...), dim3 grid, dim3 block, hipStream_t s,
                         Arg&&... a) {
  std::tuple<Prm...> args{std::forward<Arg>(a)...};
  void* ptrs[sizeof...(Prm)];
  std::apply([&](auto&... x) {
    int i = 0;
    ((ptrs[i++] = (void*)&x), ...);
  }, args);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (m->prof && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    (void)hipExtLaunchKernel((const void*)k, grid, block, ptrs, 0, s, e0, e1, 0);
    m->prof_events.push_back({id, e0, e1});
    return;
  }
  if (e0) (void)hipEventDestroy(e0);
  (void)hipExtLaunchKernel((const void*)k, grid, block, ptrs, 0, s, nullptr, nullptr, 0);
}
// kernels (shell.hip, column.hip)
dg_status_t shell_residual(dg_mesh_s* m, double t, const double* u, double* r, hipStream_t s);
// the same with the face traces in a caller-chosen device buffer of m->fn_len doubles
dg_status_t shell_residual_traces(dg_mesh_s* m, double t, const double* u, double* r, double* fn, hipStream_t s);
// the element pass of the FP64 residual (shell_r64.hip); m->p in {2, 3, 4}; profiled
// launches record into slot pid
void shell_pass1_f64(dg_mesh_s* m, const ShellDev& M, const PhysC& ph, const GllC& gc, double t, const double* u,
                     double* out, double* fn, hipStream_t s, int pid);
dg_status_t shell_jvp64(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s);
dg_status_t shell_jvp32(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s);
dg_status_t col_residual(dg_mesh_s* m, double t, const double* u, double* r, hipStream_t s);
dg_status_t col_residual_traces(dg_mesh_s* m, double t, const double* u, double* r, double* fn, hipStream_t s);
dg_status_t col_jvp64(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s);
dg_status_t col_jvp32(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s);
dg_status_t shell_jvp_bf16(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s);
// the finite-difference J v of section 3.2 (solver.hip): two residuals, the step on the device
dg_status_t jvp_fd(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s);
// doubles of the buffer jvp_fd uses (allocated with the mesh)
int64_t fd_buffer_len(int64_t n_dof);
std::vector<uint16_t> bf16_operators(int p);
// radial-line linearisation J_rad v (FP64) and the radial-line block-Jacobi preconditioner
dg_status_t shell_jvp_radial(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s);
int64_t line_pc_doubles(const dg_mesh_s* m);
dg_status_t shell_jvp_radial32(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s);
int64_t line_pc_packed(const dg_mesh_s* m);   // entries of the packed factor array
dg_status_t line_pc_build(dg_mesh_s* m, double t, const double* u, double dta, double* Lo, double* Di, double* Up,
                          double* v, void* jr, bool f32, int prec, void* P, hipStream_t s);
dg_status_t line_pc_apply(dg_mesh_s* m, int prec, const void* P, const double* r, double* z, hipStream_t s);
dg_status_t line_pc_apply(dg_mesh_s* m, int prec, const void* P, const float* r, float* z, hipStream_t s);
// modal filter (highest Legendre mode x sigma per direction), in place on u
dg_status_t shell_filter_apply(dg_mesh_s* m, double sigma, double* u, hipStream_t s);
dg_status_t col_filter_apply(dg_mesh_s* m, double sigma, double* u, hipStream_t s);
dg_status_t shell_bjac_build(dg_mesh_s* m, double t, const double* u, double dta, double* Binv, hipStream_t s);
dg_status_t shell_bjac_apply64(dg_mesh_s* m, const double* B, const double* v, double* z, hipStream_t s);
dg_status_t shell_bjac_apply32(dg_mesh_s* m, const double* B, const float* v, float* z, hipStream_t s);
dg_status_t columns_integrate(dg_mesh_s* m, double t0, double dt, int n_steps, double* u, const dg_solver_opts_t& o,
                              int32_t* newton_host, int32_t* status_host, hipStream_t s);
dg_status_t mlp_forward(struct dg_mlp_s* m, const float* X, int64_t n, float* Y, hipStream_t s, bool keep);
int mlp_n_in(const struct dg_mlp_s* m);
int mlp_n_out(const struct dg_mlp_s* m);
void fill_phys(PhysC& P, const dg_physics_t& in);
dg_status_t implicit_step(dg_mesh_s* m, double t, double dt, double* u, const dg_solver_opts_t& o,
                          dg_step_stats_t* st, hipStream_t s);
void free_workspace(dg_mesh_s* m);
}  // namespace dg
