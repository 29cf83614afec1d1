/*
 * dgthermo -- matrix-free high-order DG residual R(u), Jacobian-vector product
 * J(u)v and implicit DIRK/Newton-GMRES steps of the physics-based thermosphere
 * model of Vila-Perez, Nguyen and Peraire (arXiv 2306.01085), on AMD MI355X.
 *
 * C ABI. Every pointer argument is either a HOST pointer (descriptors, stats,
 * per-column parameter arrays, node-coordinate outputs) or a DEVICE pointer
 * (states u, residuals r, tangents v, products jv), as stated per argument.
 * Device arrays are allocated by the caller (e.g. torch tensors on the GPU),
 * must be 16-byte aligned, and must not alias each other unless stated.
 * `stream` is a hipStream_t (NULL selects the default stream). Calls that only
 * enqueue work return before it completes; dg_implicit_step and
 * dg_columns_integrate synchronise the stream because they report stats.
 *
 * Errors: every function returns a dg_status_t; no C++ exception crosses the
 * ABI. dg_last_error() returns a thread-local message describing the last
 * failure of the calling thread. A mesh may be used by one stream at a time.
 *
 * Units: everything is nondimensional in the scalings of section 2.5 of the
 * paper (lengths / H0, speeds / a0, time / (H0/a0), density / rho0, T / T0).
 *
 * State layout (section 2.4 variables, m = d + 2 fields per node:
 * varrho = log(rho/rho0), sqrt(rho) v (d components), sqrt(rho) T):
 *   shell  : u[e][c][j], e = ((panel*n_ang + j_ang)*n_ang + i_ang)*n_rad + k
 *            (radial layer fastest), c = field, j = a + n*b + n*n*cz node of the
 *            tensor-product GLL element (n = p+1; a along the panel's alpha
 *            direction, b along beta, cz along the radius)
 *   columns: columns concatenated, each column's elements bottom to top, each
 *            element u[c][i] with i = 0..p (bottom to top); column offsets from
 *            dg_mesh_col_offsets.
 * DOF = nodes x fields (the paper's convention in its convergence table).
 */
#ifndef DGTHERMO_H
#define DGTHERMO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_mesh_s* dg_mesh_t;

typedef enum {
  DG_OK = 0,
  DG_ERR_ARG = 1,          /* invalid argument (null pointer, size mismatch, unsupported degree) */
  DG_ERR_ALLOC = 2,        /* device or host allocation failed */
  DG_ERR_HIP = 3,          /* a HIP runtime call failed; message in dg_last_error() */
  DG_ERR_NOCONV = 4,       /* Newton did not reach the tolerance; the state is left unchanged */
  DG_ERR_NAN = 5,          /* a non-finite norm was met; the state is left unchanged */
  DG_ERR_UNSUPPORTED = 6   /* the requested precision / mode is not available */
} dg_status_t;

/* DG_F64_FD: FP64, the finite difference of R that section 3.2 describes (a check mode; see dg_jvp) */
typedef enum { DG_F64 = 0, DG_F32 = 1, DG_BF16 = 2, DG_F64_FD = 3 } dg_prec_t;

typedef enum { DG_MESH_COLUMNS = 0, DG_MESH_SHELL = 1 } dg_mesh_kind_t;

/* Geometry (section 3.3): host memory, copied by dg_mesh_create. */
typedef struct {
  int32_t kind;            /* dg_mesh_kind_t */
  int32_t p;               /* shell: polynomial degree per direction, 2..4 */
  int32_t n_ang;           /* shell: elements per panel edge (6*n_ang^2 angular cells) */
  int32_t n_rad;           /* shell: radial layers */
  double r_bot, r_top;     /* radii of the lower and upper boundary (nondimensional) */
  double stretch;          /* geometric growth ratio of the layer (element) thickness; 1 = uniform */
  int32_t n_col;           /* columns: number of independent radial columns */
  const int32_t* col_nelem;/* columns: host [n_col] elements per column (>= 1) */
  const int32_t* col_p;    /* columns: host [n_col] degree per column, 2..4 */
  const double* col_stretch; /* columns: optional host [n_col] growth ratio per column (NULL: stretch) */
} dg_mesh_desc_t;

/* Nondimensional physics (eq. fluxSWNondimensional, section 2.5). */
typedef struct {
  double gamma;            /* ratio of specific heats (5/3) */
  double Gr, Pr, Fr;       /* Grasshoff, Prandtl, Froude numbers */
  double m;                /* mean molecular mass / m_O (constant) */
  double nu_r, alpha_r;    /* eddy viscosity and diffusivity ratios nu_eddy/nu0, alpha_eddy/alpha0 */
  double alpha0c;          /* multiplier of the molecular conductivity */
  double lam;              /* global Lax-Friedrichs speed lambda_max (eq. LDG2) */
  double T_bot;            /* temperature imposed at the lower boundary */
  double r_ref;            /* radius where |g| = 1: g = -(r_ref/|r|)^2 r_hat */
  double omega[3];         /* rotation vector (shell only) */
  double heat_amp, heat_qm, heat_rm, heat_H; /* Chapman heating amp*qm*exp(1-z-e^{-z}/cos chi), z=(r-rm)/H */
  double sun_lat, sun_lon0, sun_rate;        /* sub-solar latitude, longitude at t = 0, longitude rate (shell) */
  int32_t bc_mode;         /* 0: lower boundary no-slip isothermal, upper boundary adiabatic stress-free;
                              1: every boundary is the constant Dirichlet state bc_state (test problems) */
  double bc_state[5];
  /* columns: optional host arrays [n_col] overriding the shared value per column, or NULL */
  const double* col_heat_amp;
  const double* col_heat_qm;
  const double* col_heat_rm;
  const double* col_heat_H;
  const double* col_lam;
  /* heating model: 0 the prescribed Chapman-shaped profile above (heat_*); 1 EUVAC (section 2.2,
     Table A): Q = eps sum_j (hc/lambda_j) I_0^j e^{-tau_j} sum_s n_s phi_s^j over the 37 bins, I_0^j the
     EUVAC flux at F10.7bar, tau_j the total optical depth n sigma_j H C with the Smith-Smith Chapman
     function C of the exponential atmosphere (scale height H = k T / (m g)), zero in the Earth's
     shadow; the composition is the constant mole fractions euv_chi, n = rho / m. State-dependent: it
     enters R and J v. The shell takes the zenith angle from the sub-solar point (latitude: the
     declination of day euv_day when euv_day > 0, else sun_lat), columns take cos chi = 1. */
  int32_t heating_model;
  double euv_eps;          /* heating efficiency (0.25) */
  double euv_f107;         /* F10.7bar = (F10.7 + its 81-day mean) / 2 */
  double euv_sun_dist;     /* distance to the Sun (AU) */
  double euv_day;          /* day of the year (1 = January 1st), or 0 */
  double euv_chi[4];       /* mole fractions of N2, O2, O, He */
  double euv_q_scale;      /* rho0 / (m_O Q_unit): m^-3 per W m^-3 of the model's heating unit */
  double euv_col_scale;    /* rho0 H0 / m_O: m^-2 per unit nondimensional density x length */
  /* columns: more optional host arrays [n_col] (or NULL for the shared value) */
  const double* col_alpha0c;   /* multiplier of the molecular conductivity (alpha0 of section 4.3) */
  const double* col_site;      /* [n_col][3] Earth-fixed unit vector of the column's site: cos chi =
                                  site . sub-solar direction at time t; NULL: the Sun overhead */
  const double* col_euv_eps;   /* EUVAC efficiency (heating model 1) */
  const double* col_euv_f107;  /* EUVAC F10.7bar (heating model 1) */
  /* composition 1: the chemically frozen mixture of section 2.1.1 replaces the constant m. The
     mass fractions of N2, O2 and He are chi_s = a_1^s exp(b_1^s |r|) + a_2^s exp(b_2^s |r|) (|r|
     nondimensional), O closes the sum to one; m = [sum_s chi_s / m_s]^-1 (masses over m_O:
     N2 28.0134, O2 31.9988, He 4.002602 over 15.9994), c_v = c_p = 1/m, the molecular
     conductivity takes the mole-fraction weight sum_s x_s alpha_s / alpha_O (section 2.1.2:
     alpha = 3.6e-4 for N2 and O2, 5.6e-4 for O and He) as a factor of alpha0c, the energy
     equation carries the grad c_v term of eq. (fluxSWNondimensional), and EUVAC (heating model 1)
     takes the species number densities rho chi_s / m_s (euv_chi unused) and H with m(r). The
     fractions must lie in [0, 1] over the mesh: dg_mesh_create and dg_mesh_set_physics check
     them at the mesh's nodes and return DG_ERR_ARG otherwise. */
  int32_t composition;
  double comp_a[6];        /* a_1, a_2 of N2, then of O2, then of He */
  double comp_b[6];        /* b_1, b_2 in the same order (per unit nondimensional radius) */
} dg_physics_t;

/* Create a mesh: builds GLL tables, the factored curved geometry (invariant curl
 * form metric terms), the connectivity, and uploads them. `out` receives the
 * handle, owned by the caller until dg_mesh_destroy. All later device work of the
 * mesh goes to the stream passed to each call. */
dg_status_t dg_mesh_create(const dg_mesh_desc_t* desc, const dg_physics_t* phys, void* stream, dg_mesh_t* out);
dg_status_t dg_mesh_destroy(dg_mesh_t mesh);
/* Replace the physics parameters (host struct, copied). With heating_model 1 it waits for the
 * device to be idle, then uploads the EUVAC bin constants to the mesh's table. An invalid
 * parameter set (including mass fractions outside [0, 1] at the mesh's nodes) returns
 * DG_ERR_ARG and leaves the mesh's physics unchanged. */
dg_status_t dg_mesh_set_physics(dg_mesh_t mesh, const dg_physics_t* phys);

/* Sizes: total DOF, elements, fields per node, dimension. Any output may be NULL. */
dg_status_t dg_mesh_info(dg_mesh_t mesh, int64_t* n_dof, int64_t* n_elem, int32_t* n_fields, int32_t* dim);
/* Node coordinates in DOF-node order: host output [n_nodes*dim] with n_nodes = n_dof/n_fields
 * (shell: [e][j][3]; columns: radius of every node in storage order). */
dg_status_t dg_mesh_nodes(dg_mesh_t mesh, double* xyz_host, int64_t n_values);
/* Columns: DOF offset of every column, host output [n_col + 1]. */
dg_status_t dg_mesh_col_offsets(dg_mesh_t mesh, int64_t* offsets_host, int64_t n);

/* R(u) = du/dt of the semi-discrete LDG system eq. (DGformulation) with the
 * traces and fluxes of eq. (LDG2), at time t. u: device [n_dof] double (input);
 * r: device [n_dof] double (output, must not alias u). Enqueue only. */
dg_status_t dg_residual(dg_mesh_t mesh, double t, const double* u, double* r, int64_t n_dof, void* stream);

/* For callers that cannot allocate device memory during a call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): R(u) exactly as
 * dg_residual computes it (the same kernels, bitwise the same result), with the face traces
 * held in a library-owned device array of DG_NOALLOC_SCRATCH_BYTES per GPU instead of the
 * mesh's trace buffer. Every GPU the library runs on holds that array until the process
 * ends; its address is looked up when a mesh is created on the GPU. Nothing is allocated
 * and nothing needs clearing: every trace slot the evaluation reads is written by the same
 * evaluation. All calls on one GPU share the array, so calls that overlap in time on one
 * GPU (different streams, or other host threads) race and give wrong results: serialise
 * them. A mesh whose traces exceed the array (shell: n_elem * 30 * (p+1)^2 * 8 bytes; at
 * p = 3 at most 26,214 elements) gets DG_ERR_ARG with a message naming both sizes.
 * Arguments and other errors as dg_residual. Enqueue only. */
#define DG_NOALLOC_SCRATCH_BYTES (96ll << 20)
dg_status_t dg_residual_noalloc(dg_mesh_t mesh, double t, const double* u, double* r, int64_t n_dof, void* stream);

/* J(u) v, the exact directional derivative of R at u along v (section 3.2 uses a
 * finite difference of R; dual-number arithmetic gives the same product without the
 * step error). u: device double [n_dof]; v and jv: device arrays [n_dof] of the
 * precision `prec` (DG_F64: double, DG_F32: float); jv must not alias v or u.
 * The arithmetic runs in that precision. DG_BF16 (shells of degree 3 and 4 only, else
 * DG_ERR_UNSUPPORTED): v and jv are float; the tangent's gradient and the divergence
 * of the linearised flux are bf16 MFMA products (operands rounded to bf16, FP32
 * accumulation) of the dense reference derivative operators, the rest as DG_F32.
 * DG_F64_FD (v, jv double): the paper's matrix-free product, the one-sided difference
 * jv = (R(u + h v) - R(u)) / h with h = sqrt(eps_64) (1 + |u|_2) / |v|_2 (the paper gives no
 * step), jv = 0 for v = 0; two R evaluations, its error is O(h) plus rounding of order
 * eps_64 / h. The norms and h stay on the device, in two state-sized buffers that
 * dg_mesh_create allocates with the mesh (no call of dg_jvp allocates). Enqueue only. */
dg_status_t dg_jvp(dg_mesh_t mesh, double t, const double* u, const void* v, void* jv, int64_t n_dof,
                   dg_prec_t prec, void* stream);

/* ---- implicit time stepping (section 3.1 DIRK, section 3.2 Newton-GMRES) ---- */
typedef struct {
  int32_t scheme;          /* 33: DIRK(3,3); 22: DIRK(2,2) */
  int32_t gmres_m;         /* Krylov dimension per restart (30; 1..32) */
  int32_t max_newton;      /* Newton iterations per stage */
  int32_t max_restarts;    /* GMRES restarts per Newton iteration */
  double newton_rtol;      /* stop when |G(U)| <= newton_rtol |G(u_n)| (1e-8) */
  double gmres_rtol;       /* inexact Newton: relative GMRES tolerance (1e-3) */
  int32_t jvp_prec;        /* dg_prec_t of J v inside GMRES (DG_F32 and DG_BF16 keep FP32 Krylov vectors;
                              DG_BF16 needs a shell of degree 3 or 4; DG_F64_FD: FP64 vectors, the
                              finite-difference product of dg_jvp) */
  int32_t precond;         /* shell meshes: 0 none; 1 node 5x5 block Jacobi (q held fixed, rebuilt every
                              Newton iteration); 2 radial-line block Jacobi: I - dt a_ii J_rad with J_rad
                              the linearisation that drops the tangent's coupling between different
                              angular nodes (exact along each radial line), block tridiagonal per line,
                              built at u_n by 15 (p+1) dual probes (every step, or every
                              "line_pc_every" steps), factored by block LU */
  int32_t guess;           /* 0: previous state (first step) / extrapolation, 1: learned warm start */
  int32_t forcing;         /* GMRES tolerance per Newton iteration: 0 fixed gmres_rtol; 1 Eisenstat-Walker:
                              eta_0 = 0.1, eta_k = min(0.1, 0.9 (|G_k|/|G_k-1|)^2) (kept >= 0.9 eta_k-1^2
                              when that exceeds 0.1), and >= 0.5 newton_rtol |G(u_n)| / |G_k| so the last
                              iteration does not solve past the Newton tolerance */
  double filter_rate;      /* >= 0. After every step the highest Legendre mode of each element is
                              multiplied by exp(-filter_rate dt) in every direction (tensor-product
                              modal filter, applied to u_{n+1}); 0 leaves the DIRK step unfiltered.
                              Not part of the paper's method: it damps the intra-element mode that
                              the collocated (under-integrated) products let grow. */
  int32_t n_rb;            /* 0..8, reduced basis of section 3.2 (0: off). The n_rb most recent Newton
                              updates d_j (kept across stages and steps; emptied when dt a_ii changes or
                              a step does not continue the previous one) and z_j = A d_j (A = I - dt a_ii J
                              at the iterate where d_j was solved, one J v each) give GMRES the initial
                              guess W c(rhs) and the preconditioner v -> W c(v) + P^-1 (v - Z c(v)),
                              c(v) = (Z^T Z)^+ Z^T v, P the preconditioner chosen by precond. Changes the
                              GMRES path, not the converged step. */
} dg_solver_opts_t;

typedef struct {
  int32_t newton_its[3];   /* per stage */
  int32_t gmres_its[3];    /* per stage, summed over Newton iterations */
  int32_t fallback[3];     /* 1 if the learned guess was rejected for the plain one */
  double res0[3];          /* |G(guess)| per stage */
  double res[3];           /* final |G| per stage */
  double ref[3];           /* |G(u_n)| per stage (the reference norm) */
  double guess_scale[3];   /* learned guess: the factor applied to the network's correction */
  double seconds;          /* wall time of the call */
} dg_step_stats_t;

/* One DIRK step u(t) -> u(t + dt) in place. u: device double [n_dof]. stats: host
 * output (may be NULL). Synchronises `stream`. On DG_ERR_NOCONV or DG_ERR_NAN
 * u is left unchanged. Workspace is allocated on the first call and kept by the
 * mesh. */
dg_status_t dg_implicit_step(dg_mesh_t mesh, double t, double dt, double* u, int64_t n_dof,
                             const dg_solver_opts_t* opts, dg_step_stats_t* stats, void* stream);

/* Batched columns (the radial 1D model, section 4.1.3, used for parametric sweeps in
 * section 4.2): advance EVERY column of a column mesh by n_steps DIRK steps
 * (opts->scheme) from t0 in ONE persistent launch. Each wavefront takes columns from
 * an atomic queue ordered by decreasing cost and runs the whole time loop of a
 * column: Newton on every stage with the exact block-tridiagonal Jacobian of the 1D
 * residual (assembled by 3-colour probing with dual numbers, factored by block LU,
 * reused across the stages of a step). Stops a column at |G| <= newton_rtol |G(u_n)|
 * per stage; opts->max_newton bounds the iterations per stage (gmres_*, jvp_prec,
 * precond and guess are not used). u: device double [n_dof], in/out.
 * newton_host / status_host: optional host [n_col] outputs (Newton iterations of the
 * call; 0 ok, 4 no convergence, 5 non-finite). A failed column keeps its input state.
 * Synchronises `stream`. Returns DG_ERR_NOCONV / DG_ERR_NAN if any column failed. */
dg_status_t dg_columns_integrate(dg_mesh_t mesh, double t0, double dt, int32_t n_steps, double* u, int64_t n_dof,
                                 const dg_solver_opts_t* opts, int32_t* newton_host, int32_t* status_host,
                                 void* stream);

/* ---- learned Newton warm start (the per-element network and its use) ----
 * A network maps per-element features to a correction of the plain extrapolated
 * stage guess: n_in -> 128 -> 128 -> n_out, ReLU hidden layers. Precision contract:
 * weights, the input and the hidden activations are rounded to bfloat16 where they
 * enter a matrix product (bf16 MFMA); biases and accumulation are FP32; training
 * keeps FP32 master weights (Adam) and treats the roundings as the identity in the
 * backward pass. Parameters are packed as W1 [128][n_in], b1 [128], W2 [128][128],
 * b2 [128], W3 [n_out][128], b3 [n_out] (row-major, FP32 on the host). */
typedef struct dg_mlp_s* dg_mlp_t;
/* n_in a multiple of 8, n_hidden = 128, n_out a multiple of 32; params_host: packed FP32 */
dg_status_t dg_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, const float* params_host, dg_mlp_t* out);
dg_status_t dg_mlp_destroy(dg_mlp_t mlp);
int64_t dg_mlp_param_count(dg_mlp_t mlp);
/* FP32 master parameters to a host array of dg_mlp_param_count entries (synchronises) */
dg_status_t dg_mlp_get_params(dg_mlp_t mlp, float* params_host, int64_t len);
/* y = net(x): x device FP32 [n][n_in] (16-byte aligned), y device FP32 [n][n_out]. Enqueue only. */
dg_status_t dg_mlp_forward(dg_mlp_t mlp, const float* x, int64_t n, float* y, void* stream);
/* mean-squared-error loss against t (device FP32 [n][n_out]; x as for dg_mlp_forward) and its gradient, kept in
 * the handle for dg_mlp_adam_step; loss_host / grad_host (packed) are optional host
 * outputs (either one synchronises the stream). */
dg_status_t dg_mlp_grad(dg_mlp_t mlp, const float* x, const float* t, int64_t n, double* loss_host, float* grad_host,
                        void* stream);
/* one Adam update of the master parameters with the last gradient (bias-corrected). */
dg_status_t dg_mlp_adam_step(dg_mlp_t mlp, float lr, float beta1, float beta2, float eps, void* stream);

/* x[r][k] = (x[r][k] - mean[k]) / scale[k] for a device FP32 [n][width] array in place
 * (standardisation of recorded training rows); mean / scale: device FP32 [width], read by
 * the kernel (they must stay valid until it has run). Enqueue only; allocates nothing. */
dg_status_t dg_affine_rows(float* x, int64_t n, int32_t width, const float* mean, const float* scale,
                           void* stream);

/* Attach a trained network to a shell mesh for opts->guess = 1 (NULL detaches). The
 * features of element e at stage i are [U_a, U_a - U_b, b_i - U_a] (U_a, U_b the two
 * latest stage solutions, b_i the stage right-hand side; 3 x 5 x N values, node-major
 * per field as in the state layout), standardised with x_mean / x_scale (host [n_in]);
 * the output de-standardised with y_mean / y_scale (host [n_out], n_out = 5 N) is the
 * correction D of the plain guess U_p. The guess is U_p + alpha D with alpha in [0, 2]
 * minimising the linearised stage residual |G(U_p) + alpha (I - dt a_ii J(U_p)) D|
 * (one FP64 J v; reported in dg_step_stats_t.guess_scale); it is kept only if its |G|
 * is below |G(U_p)| (otherwise U_p: dg_step_stats_t.fallback). The network is not
 * owned. */
dg_status_t dg_warmstart_set(dg_mesh_t mesh, dg_mlp_t mlp, const float* x_mean_host, const float* x_scale_host,
                             const float* y_mean_host, const float* y_scale_host);
/* Record training pairs during later dg_implicit_step calls on a shell mesh: for one
 * element in `every` (deterministic), after each stage converges, the raw features
 * (as above, unstandardised) go to x_dev [capacity][n_in] and the raw target
 * U_i - U_plain to y_dev [capacity][n_out] (device FP32, caller-owned) until capacity
 * rows are written. capacity = 0 stops recording. dg_warmstart_recorded returns the
 * number of rows written so far. */
dg_status_t dg_warmstart_record(dg_mesh_t mesh, float* x_dev, float* y_dev, int64_t capacity, int32_t every);
dg_status_t dg_warmstart_recorded(dg_mesh_t mesh, int64_t* count_host);

/* ---- event timing of the library's own launches (tracing subsystem) ----
 * When enabled, every launch group is bracketed by hipEvents on the stream it runs on.
 * dg_profile_read synchronises those events and returns, per slot, the accumulated
 * milliseconds and launch counts (host arrays of n entries; reset != 0 clears them).
 * Slots: 0 shell pass 1 (R), 1 shell pass 2 (R), 2 / 3 shell passes of J v FP64,
 * 4 / 5 shell passes of J v FP32, 6 columns R, 7 columns J v FP64, 8 columns J v FP32,
 * 9 GMRES Arnoldi (orthogonalisation), 10 / 11 preconditioner build / apply (node or
 * radial-line block-Jacobi),
 * 12 vector updates, 13 batched columns, 14 / 15 shell passes of J v BF16. */
dg_status_t dg_profile_enable(dg_mesh_t mesh, int32_t on);
dg_status_t dg_profile_read(dg_mesh_t mesh, double* ms_host, int64_t* counts_host, int32_t n, int32_t reset);

/* Tuning knobs (host values):
 *   "shell_pass1_config" 0..5: elements per block and register budget of the shell's
 *   element pass (0: 256-thread blocks; 1/2: one/two elements per block; 3/4: one/two
 *   elements with a register budget for 3 waves per SIMD; 5: one element, 4 waves).
 *   No effect on results.
 *   "columns_grid" >= 1: number of persistent wavefronts of dg_columns_integrate.
 *   No effect on results.
 *   "line_solve_config" -1..5: launch configuration of the radial-line preconditioner's
 *   substitution (0/2: one wavefront per block, 1/3: four, 4/5: the (p + 1)^2 lines of
 *   one angular cell per block; 0/1/5: loads one matrix ahead, 2/3/4: three ahead;
 *   default -1: 5 for FP64 Krylov vectors, 3 for FP32). No effect on results.
 *   "line_pc_every" >= 1 (default 1): dg_implicit_step with precond 2 rebuilds the
 *   radial-line preconditioner from the current state only every this many steps (and
 *   whenever dt a_ii or the J v precision changes or a step does not start where the
 *   previous one ended), reusing it in between. It changes the
 *   GMRES iteration counts, not what Newton converges to (within newton_rtol).
 *   "line_pc_precision" 64, 32 (default) or 16: storage precision of the radial-line
 *   preconditioner's factors (double, float, bfloat16) read by its substitution, whatever
 *   the J v precision; the substitution computes in the precision of the Krylov vectors.
 *   Like line_pc_every it changes iteration counts, not the converged step.
 *   "columns_jac_every" >= 1 (default 32): dg_columns_integrate factors each column's chord
 *   Jacobian I - dt a_ii J (shared by the SDIRK stages) at the start of every this many
 *   steps instead of every step, and sooner after a step whose stages needed more than
 *   "columns_jac_stale_its" (default 5) iterations or within a stage whose iteration left |G|
 *   above "columns_jac_slow_pct" percent (1..100, default 75) of its previous value. All three
 *   change iteration counts, not what each stage converges to (within newton_rtol).
 *   "column_quadrature" 0 (default) or 1, column meshes only: 0 evaluates eq. (DGformulation)
 *   with the collocated GLL rule (diagonal mass); 1 integrates the volume terms of both LDG
 *   equations with p + 2 Gauss points and the exact mass matrix (over-integration; the traces,
 *   numerical fluxes and boundary treatment unchanged). It changes R, J v, dg_implicit_step and
 *   dg_columns_integrate of the mesh; the linearised operator of the collocated residual has
 *   growing intra-element modes that the over-integrated one does not have.
 * Returns DG_ERR_ARG for an unknown name or value. */
dg_status_t dg_set_option(dg_mesh_t mesh, const char* name, int64_t value);

const char* dg_last_error(void);
int32_t dg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DGTHERMO_H */
