// Implicit DIRK stages solved by Newton-GMRES.
//
// DIRK(3,3) / DIRK(2,2): Alexander's stiffly accurate, L-stable singly diagonal
// schemes (cited in section 3.1; their tableaux are restated from the order
// conditions). Stage i solves
//   G_i(U) = U - dt a_ii R(U, t + c_i dt) - b_i = 0,  b_i = u_n + dt sum_{j<i} a_ij R(U_j)
// by Newton (eq. NewtonSolve); every Newton correction solves
//   (I - dt a_ii J(U)) delta = -G_i(U)
// with right-preconditioned restarted GMRES(m) (section 3.2): classical Gram-Schmidt
// applied twice with fused multi-vector dot products (one read of the new vector and
// of the basis per pass, block reductions in LDS, a deterministic second stage),
// Givens rotations on the host (one device-to-host copy per Krylov iteration).
// J(U) v is the exact product of the residual kernels, in FP64 or FP32 (the Krylov
// basis is then stored in FP32 too; dot products accumulate in FP64).
// Convergence: |G_i(U)| <= rtol |G_i(u_n)| -- the reference norm does not depend on
// the initial guess.
#include <chrono>
#include <cmath>
#include <type_traits>
#include <vector>

#include "internal.h"

namespace dg {

constexpr int RED_BLOCKS = 2048;
constexpr int RED_THREADS = 256;
constexpr int KMAX = 66;

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

// block-level sum of K accumulators; thread 0 ends with the totals in red[0..K)
template <int K>
__device__ inline void block_sum(double (&acc)[K], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[wid * K + k] = s;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0;
    for (int w = 0; w < RED_THREADS / 64; ++w) s += red[w * K + threadIdx.x];
    red[threadIdx.x] = s;
  }
  __syncthreads();
}

// part[b*K + k] = sum over this block's indices of V_k[i] * w[i]  (K <= 33 vectors)
template <int K, class T>
__global__ __launch_bounds__(RED_THREADS) void k_mdot(int64_t n, const T* __restrict__ V, int64_t ldv,
                                                      const T* __restrict__ w, double* __restrict__ part) {
  __shared__ double red[(RED_THREADS / 64) * K + K];
  double acc[K];
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = (double)w[i];
    for (int k = 0; k < K; ++k) acc[k] += (double)V[k * ldv + i] * wi;
  }
  block_sum<K>(acc, red);
  if (threadIdx.x < K) part[blockIdx.x * K + threadIdx.x] = red[threadIdx.x];
}

// out[k] = sum_b part[b*K + k]; block i takes k = i, i + gridDim.x, ... (launched with one
// block per k; every k is summed in the same order whatever the grid)
__global__ __launch_bounds__(RED_THREADS) void k_reduce(const double* __restrict__ part, int nb, int K,
                                                        double* __restrict__ out) {
  __shared__ double red[RED_THREADS / 64];
  for (int k = blockIdx.x; k < K; k += gridDim.x) {
    double s = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b * K + k];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int w = 0; w < RED_THREADS / 64; ++w) t += red[w];
      out[k] = t;
    }
    __syncthreads();
  }
}

// the middle sweep of CGS2: w -= sum_k h[k] V_k, and in the same pass the K dot products
// V_k . w of the updated (stored) w for the second orthogonalisation
template <int K, class T>
__global__ __launch_bounds__(RED_THREADS) void k_orth_mdot(int64_t n, const T* __restrict__ V, int64_t ldv,
                                                           const double* __restrict__ h, T* __restrict__ w,
                                                           double* __restrict__ part) {
  __shared__ double red[(RED_THREADS / 64) * K + K];
  double hk[K], acc[K];
  for (int k = 0; k < K; ++k) {
    hk[k] = h[k];
    acc[k] = 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v[K];
    double x = (double)w[i];
    for (int k = 0; k < K; ++k) {
      v[k] = (double)V[k * ldv + i];
      x -= hk[k] * v[k];
    }
    const T xt = (T)x;
    w[i] = xt;
    for (int k = 0; k < K; ++k) acc[k] += v[k] * (double)xt;
  }
  block_sum<K>(acc, red);
  if (threadIdx.x < K) part[blockIdx.x * K + threadIdx.x] = red[threadIdx.x];
}

// w -= sum_k h[k] V_k ; part = partial sums of w^2 (for the norm). K is a template argument
// like the dot-product sweeps': with K known the loads of the K basis vectors are issued
// together (with K read at run time each load was waited for before the next, the sweep ran
// at a quarter of the HBM rate); the subtraction order is the same.
template <int K, class T>
__global__ __launch_bounds__(RED_THREADS) void k_orth_update(int64_t n, const T* __restrict__ V, int64_t ldv,
                                                             const double* __restrict__ h, T* __restrict__ w,
                                                             double* __restrict__ part) {
  __shared__ double red[(RED_THREADS / 64) + 1];
  double hk[K];
  for (int k = 0; k < K; ++k) hk[k] = h[k];
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double x = (double)w[i];
    for (int k = 0; k < K; ++k) x -= hk[k] * (double)V[k * ldv + i];
    const T xt = (T)x;
    w[i] = xt;
    acc[0] += (double)xt * (double)xt;
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// y = x * (1/sqrt(nrm2[0]))
template <class T>
__global__ void k_normalize(int64_t n, const T* __restrict__ x, const double* __restrict__ nrm2, T* __restrict__ y) {
  const double s = 1.0 / sqrt(nrm2[0]);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (T)((double)x[i] * s);
}

// y = a*x + b*y (double) and optional partial sums of y^2
__global__ __launch_bounds__(RED_THREADS) void k_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                                                       double* __restrict__ y, double* __restrict__ part) {
  __shared__ double red[(RED_THREADS / 64) + 1];
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = a * x[i] + b * y[i];
    y[i] = v;
    acc[0] += v * v;
  }
  if (part) {
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
  }
}

// G = U - c R - B, with partial sums of G^2
__global__ __launch_bounds__(RED_THREADS) void k_stage_residual(int64_t n, const double* __restrict__ U,
                                                                const double* __restrict__ R, double c,
                                                                const double* __restrict__ B, double* __restrict__ G,
                                                                double* __restrict__ part) {
  __shared__ double red[(RED_THREADS / 64) + 1];
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double g = U[i] - c * R[i] - B[i];
    G[i] = g;
    acc[0] += g * g;
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// partial sums of a.b and b.b (two accumulators per block)
__global__ __launch_bounds__(RED_THREADS) void k_dot2(int64_t n, const double* __restrict__ a,
                                                      const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double red[(RED_THREADS / 64) * 2 + 2];
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    acc[0] += a[i] * b[i];
    acc[1] += b[i] * b[i];
  }
  block_sum<2>(acc, red);
  if (threadIdx.x < 2) part[blockIdx.x * 2 + threadIdx.x] = red[threadIdx.x];
}

// r = s * x (T <- double): start vector of a GMRES cycle
template <class T>
__global__ void k_scale_to(int64_t n, double s, const double* __restrict__ x, T* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (T)(s * x[i]);
}

// w = z - c * jz  (the stage operator applied to z)
template <class T>
__global__ void k_stage_op(int64_t n, const T* __restrict__ z, double c, T* __restrict__ jz) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    jz[i] = (T)((double)z[i] - c * (double)jz[i]);
}

// s = sum_k y[k] V_k (T), with y on the device (K a template argument, as in k_orth_update)
template <int K, class T>
__global__ void k_combine(int64_t n, const T* __restrict__ V, int64_t ldv, const double* __restrict__ y,
                          T* __restrict__ s) {
  double yk[K];
  for (int k = 0; k < K; ++k) yk[k] = y[k];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double a = 0;
    for (int k = 0; k < K; ++k) a += yk[k] * (double)V[k * ldv + i];
    s[i] = (T)a;
  }
}

template <class T>
__global__ void k_zero(int64_t n, T* __restrict__ s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s[i] = T(0);
}

template <class T, int K = 1>
static void launch_combine(int kk, int nb, hipStream_t st, int64_t n, const T* V, int64_t ldv, const double* y,
                           T* s) {
  if (K == 1 && kk < 1) {   // (an empty basis: s = 0)
    k_zero<T><<<nb, RED_THREADS, 0, st>>>(n, s);
    return;
  }
  if constexpr (K > 33) {
    (void)kk; (void)nb; (void)st; (void)n; (void)V; (void)ldv; (void)y; (void)s;
  } else {
    if (kk == K) {
      k_combine<K, T><<<nb, RED_THREADS, 0, st>>>(n, V, ldv, y, s);
      return;
    }
    launch_combine<T, K + 1>(kk, nb, st, n, V, ldv, y, s);
  }
}

// V0 = rhs - w with partial sums of V0^2
template <class T>
__global__ __launch_bounds__(RED_THREADS) void k_restart_vector(int64_t n, const double* __restrict__ rhs,
                                                                const T* __restrict__ w, T* __restrict__ v0,
                                                                double* __restrict__ part) {
  __shared__ double red[(RED_THREADS / 64) + 1];
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T x = (T)(rhs[i] - (double)w[i]);
    v0[i] = x;
    acc[0] += (double)x * (double)x;
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

template <class T>
__global__ void k_add_to(int64_t n, const T* __restrict__ z, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += (double)z[i];
}

template <class T>
__global__ void k_copy_cast(int64_t n, const double* __restrict__ x, T* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (T)x[i];
}

// linear extrapolation through (ta, A) and (tb, B) to time t: out = A + (t - ta)/(ta - tb) (A - B)
__global__ void k_extrapolate(int64_t n, const double* __restrict__ A, const double* __restrict__ B, double f,
                              double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = A[i] + f * (A[i] - B[i]);
}

// ---------------------------------------------------------------- reduced basis (section 3.2)
constexpr int RB_MAX = 8;

// c = Gp d (k x k, row-major), one block
__global__ void k_rb_coef(int k, const double* __restrict__ Gp, const double* __restrict__ d, double* __restrict__ c) {
  const int i = threadIdx.x;
  if (i >= k) return;
  double a = 0;
  for (int j = 0; j < k; ++j) a += Gp[i * k + j] * d[j];
  c[i] = a;
}

// r = v - sum_j c_j Z_j and x = sum_j c_j W_j; with r == x (no base preconditioner) the
// sum r + x is written instead
template <class T>
__global__ void k_rb_split(int64_t n, int k, const T* __restrict__ Z, const T* __restrict__ W,
                           const double* __restrict__ c, const T* __restrict__ v, T* r, T* x) {
  double cc[RB_MAX];
  for (int j = 0; j < k; ++j) cc[j] = c[j];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double a = (double)v[i], b = 0;
    for (int j = 0; j < k; ++j) {
      a -= cc[j] * (double)Z[j * n + i];
      b += cc[j] * (double)W[j * n + i];
    }
    if (r == x) {
      r[i] = (T)(a + b);
    } else {
      r[i] = (T)a;
      x[i] = (T)b;
    }
  }
}

// X = sum_j c_j W_j (the GMRES initial guess, double)
template <class T>
__global__ void k_rb_guess(int64_t n, int k, const T* __restrict__ W, const double* __restrict__ c,
                           double* __restrict__ X) {
  double cc[RB_MAX];
  for (int j = 0; j < k; ++j) cc[j] = c[j];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double b = 0;
    for (int j = 0; j < k; ++j) b += cc[j] * (double)W[j * n + i];
    X[i] = b;
  }
}

template <class T>
__global__ void k_add_T(int64_t n, const T* __restrict__ x, T* __restrict__ z) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = (T)((double)z[i] + (double)x[i]);
}

// ---------------------------------------------------------------- learned warm start
// features of element e: [U_a, U_a - U_b, b - U_a] per field and node (3 x 5 x N), standardised
__global__ void k_ws_features(int64_t E, int N, const double* __restrict__ Ua, const double* __restrict__ Ub,
                              const double* __restrict__ Bv, const float* __restrict__ mean,
                              const float* __restrict__ scale, float* __restrict__ X) {
  const int64_t nin = 15 * (int64_t)N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * nin) return;
  const int64_t e = idx / nin;
  const int k = (int)(idx % nin);
  const int grp = k / (5 * N), cj = k % (5 * N);
  const int64_t g = e * 5 * N + cj;
  double x;
  if (grp == 0)
    x = Ua[g];
  else if (grp == 1)
    x = Ua[g] - Ub[g];
  else
    x = Bv[g] - Ua[g];
  X[idx] = mean ? (float)((x - (double)mean[k]) / (double)scale[k]) : (float)x;
}

// U = Up + y * y_scale + y_mean
__global__ void k_ws_apply(int64_t n, const double* __restrict__ Up, const float* __restrict__ Y,
                           const float* __restrict__ ym, const float* __restrict__ ys, int nout, double* __restrict__ U) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = (int)(i % nout);
  U[i] = Up[i] + (double)Y[i] * (double)ys[k] + (double)ym[k];
}

// training pairs of the selected elements e = phase + every * r: raw features and
// target U - Up, written at rows row0 + r (r < nrows)
__global__ void k_ws_record(int64_t nrows, int64_t phase, int every, int N, const double* __restrict__ Ua,
                            const double* __restrict__ Ub, const double* __restrict__ Bv,
                            const double* __restrict__ U, const double* __restrict__ Up, float* __restrict__ rx,
                            float* __restrict__ ry, int64_t row0) {
  const int64_t nin = 15 * (int64_t)N, nout = 5 * (int64_t)N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nrows * (nin + nout)) return;
  const int64_t r = idx / (nin + nout);
  const int k = (int)(idx % (nin + nout));
  const int64_t e = phase + (int64_t)every * r;
  if (k < nin) {
    const int grp = k / (5 * N), cj = k % (5 * N);
    const int64_t g = e * 5 * N + cj;
    const double x = grp == 0 ? Ua[g] : (grp == 1 ? Ua[g] - Ub[g] : Bv[g] - Ua[g]);
    rx[(row0 + r) * nin + k] = (float)x;
  } else {
    const int kk = k - (int)nin;
    const int64_t g = e * nout + kk;
    ry[(row0 + r) * nout + kk] = (float)(U[g] - Up[g]);
  }
}

// ---------------------------------------------------------------- workspace
struct Workspace {
  int64_t n = 0;
  int m = 0;
  bool f32 = false;
  double *un = nullptr, *U = nullptr, *G = nullptr, *B = nullptr, *X = nullptr, *Rc = nullptr, *Up = nullptr;
  double* Rs[3] = {nullptr, nullptr, nullptr};
  double* hist[2] = {nullptr, nullptr};   // the two most recent stage solutions
  double hist_t[2] = {0, 0};
  int hist_n = 0;
  double t_end = NAN;                     // end time of the last step (history continuity)
  double* Binv = nullptr;
  double *lineLo = nullptr, *lineDi = nullptr, *lineUp = nullptr;   // radial-line preconditioner factors
  void* lineP = nullptr;  // the packed factors used by the substitution
  int lineP_prec = 0;     // their storage precision (64, 32, 16)
  int line_age = -1;      // steps since the line preconditioner was built (-1: not built)
  double line_dta = 0;    // dt a_ii it was built for
  bool line_f32 = false;  // it was built from the FP32 linearisation
  // reduced basis: W (updates) and Z = A W, rb_cap vectors each in the Krylov precision, a ring
  // of rb_count valid slots; G = Z^T Z on the host, its pseudo-inverse on the device
  void* rbW = nullptr;
  void* rbZ = nullptr;
  void* rbT = nullptr;                    // one scratch vector
  int rb_cap = 0, rb_count = 0, rb_head = 0, rb_n = 0;
  double rb_dta = 0;
  double rb_G[RB_MAX * RB_MAX] = {};
  double* rb_dev = nullptr;               // Gp [RB_MAX^2], d [RB_MAX], c [RB_MAX]
  double* rb_host = nullptr;              // pinned staging of Gp
  void* V = nullptr;                      // (m+1) basis vectors, double or float
  void* w = nullptr;
  void* z = nullptr;
  void* s = nullptr;
  double* part = nullptr;
  double* dev_small = nullptr;            // h1 [KMAX], h2 [KMAX], nrm [1], y [KMAX]
  double* host_small = nullptr;           // pinned mirror
};

void free_workspace(dg_mesh_s* m) {
  Workspace* w = m->ws;
  if (!w) return;
  void* ptrs[] = {w->un, w->U, w->G, w->B, w->X, w->Rc, w->Rs[0], w->Rs[1], w->Rs[2], w->hist[0], w->hist[1],
                  w->Binv, w->V, w->w, w->z, w->s, w->part, w->dev_small, w->Up, w->lineLo, w->lineDi, w->lineUp,
                  w->lineP, w->rbW, w->rbZ, w->rbT, w->rb_dev};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (w->host_small) (void)hipHostFree(w->host_small);
  if (w->rb_host) (void)hipHostFree(w->rb_host);
  delete w;
  m->ws = nullptr;
}

// the Krylov part of the workspace (basis, work vectors, reduced-basis window): stored in
// the J v precision, so re-allocated when the precision or the basis size changes
static void free_krylov(Workspace* w) {
  for (void* p : {w->V, w->w, w->z, w->s, w->rbW, w->rbZ, w->rbT})
    if (p) (void)hipFree(p);
  w->V = w->w = w->z = w->s = w->rbW = w->rbZ = w->rbT = nullptr;
  w->rb_cap = w->rb_count = w->rb_head = 0;
}

static dg_status_t ensure_workspace(dg_mesh_s* m, int mk, bool f32) {
  Workspace* w = m->ws;
  if (w && w->m == mk && w->f32 == f32) return DG_OK;
  const int64_t n = m->n_dof;
  const size_t vb = f32 ? sizeof(float) : sizeof(double);
  if (w) {
    // a change of J v precision or basis size: the FP64 stage vectors, the guess history and
    // the preconditioner stay; only the Krylov part is re-allocated
    free_krylov(w);
    w->m = mk;
    w->f32 = f32;
  } else {
    w = new Workspace();
    m->ws = w;
    w->n = n;
    w->m = mk;
    w->f32 = f32;
    double** dbl[] = {&w->un, &w->U, &w->G, &w->B, &w->X, &w->Rc, &w->Rs[0], &w->Rs[1], &w->Rs[2], &w->hist[0],
                      &w->hist[1], &w->Up};
    for (double** p : dbl)
      if (hipMalloc(p, n * sizeof(double)) != hipSuccess) goto fail;
    if (m->kind == DG_MESH_SHELL && hipMalloc(&w->Binv, n * 5 * sizeof(double)) != hipSuccess) goto fail;
    if (hipMalloc(&w->part, (size_t)RED_BLOCKS * KMAX * sizeof(double)) != hipSuccess) goto fail;
    if (hipMalloc(&w->dev_small, 4 * KMAX * sizeof(double)) != hipSuccess) goto fail;
    if (hipHostMalloc(&w->host_small, 4 * KMAX * sizeof(double)) != hipSuccess) goto fail;
  }
  if (hipMalloc(&w->V, (size_t)(mk + 1) * n * vb) != hipSuccess) goto fail;
  if (hipMalloc(&w->w, n * vb) != hipSuccess || hipMalloc(&w->z, n * vb) != hipSuccess ||
      hipMalloc(&w->s, n * vb) != hipSuccess)
    goto fail;
  return DG_OK;
fail:
  free_workspace(m);
  set_error("dg_implicit_step: workspace allocation failed");
  return DG_ERR_ALLOC;
}

// ---------------------------------------------------------------- operators
static dg_status_t residual(dg_mesh_s* m, double t, const double* u, double* r, hipStream_t s) {
  return m->kind == DG_MESH_SHELL ? shell_residual(m, t, u, r, s) : col_residual(m, t, u, r, s);
}

// ---------------------------------------------------------------- finite-difference J v
// Section 3.2 forms J v as a finite difference of R. One-sided, with the usual
// Jacobian-free Newton-Krylov step (the paper gives none) h = sqrt(eps) (1 + |u|) / |v|
// (2-norms). sums[0] = |u|^2, sums[1] = |v|^2 are reduced on the device.
__device__ inline double fd_step(const double* __restrict__ sums) {
  const double nv = sqrt(sums[1]);
  if (!(nv > 0.0)) return 0.0;
  return 1.4901161193847656e-08 * (1.0 + sqrt(sums[0])) / nv;   // 2^-26 = sqrt(eps_64)
}

// partial sums of a.a and b.b (two accumulators per block)
__global__ __launch_bounds__(RED_THREADS) void k_sumsq2(int64_t n, const double* __restrict__ a,
                                                        const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double red[(RED_THREADS / 64) * 2 + 2];
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    acc[0] += a[i] * a[i];
    acc[1] += b[i] * b[i];
  }
  block_sum<2>(acc, red);
  if (threadIdx.x < 2) part[blockIdx.x * 2 + threadIdx.x] = red[threadIdx.x];
}

// w = u + h v
__global__ void k_fd_perturb(int64_t n, const double* __restrict__ u, const double* __restrict__ v,
                             const double* __restrict__ sums, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  w[i] = u[i] + fd_step(sums) * v[i];
}

// jv = (R(u + h v) - R(u)) / h, held in jv and r0 on entry; 0 when h = 0
__global__ void k_fd_finish(int64_t n, const double* __restrict__ r0, const double* __restrict__ sums,
                            double* __restrict__ jv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double h = fd_step(sums);
  jv[i] = h > 0.0 ? (jv[i] - r0[i]) / h : 0.0;
}

// doubles of the mesh-owned finite-difference buffer: [w (n) | r0 (n) | partials (2 RED_BLOCKS) | sums (2)]
int64_t fd_buffer_len(int64_t n_dof) { return 2 * n_dof + 2 * RED_BLOCKS + 2; }

dg_status_t jvp_fd(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s) {
  const int64_t n = m->n_dof;
  if (!m->d_fd) {
    set_error("dg_jvp: the mesh has no finite-difference buffers");
    return DG_ERR_ALLOC;
  }
  double* w = m->d_fd;
  double* r0 = w + n;
  double* part = r0 + n;
  double* sums = part + 2 * RED_BLOCKS;
  const int nb = (int)std::min<int64_t>((n + RED_THREADS - 1) / RED_THREADS, RED_BLOCKS);
  k_sumsq2<<<nb, RED_THREADS, 0, s>>>(n, u, v, part);
  k_reduce<<<2, RED_THREADS, 0, s>>>(part, nb, 2, sums);
  const unsigned g = (unsigned)((n + 255) / 256);
  k_fd_perturb<<<g, 256, 0, s>>>(n, u, v, sums, w);
  dg_status_t st = residual(m, t, w, jv, s);
  if (st != DG_OK) return st;
  st = residual(m, t, u, r0, s);
  if (st != DG_OK) return st;
  k_fd_finish<<<g, 256, 0, s>>>(n, r0, sums, jv);
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

static dg_status_t jvp(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s) {
  if (m->krylov_fd) return jvp_fd(m, t, u, v, jv, s);
  return m->kind == DG_MESH_SHELL ? shell_jvp64(m, t, u, v, jv, s) : col_jvp64(m, t, u, v, jv, s);
}
static dg_status_t jvp(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s) {
  if (m->kind == DG_MESH_SHELL) return m->krylov_bf16 ? shell_jvp_bf16(m, t, u, v, jv, s) : shell_jvp32(m, t, u, v, jv, s);
  return col_jvp32(m, t, u, v, jv, s);
}
// z = M^-1 v: mode 0 identity, 1 node block-Jacobi, 2 radial-line block-Jacobi
static dg_status_t precond(dg_mesh_s* m, const Workspace* ws, int mode, const double* v, double* z, hipStream_t s) {
  if (mode == 1) return shell_bjac_apply64(m, ws->Binv, v, z, s);
  if (mode == 2) return line_pc_apply(m, ws->lineP_prec, ws->lineP, v, z, s);
  DG_HIP_CHECK(hipMemcpyAsync(z, v, m->n_dof * sizeof(double), hipMemcpyDeviceToDevice, s));
  return DG_OK;
}
static dg_status_t precond(dg_mesh_s* m, const Workspace* ws, int mode, const float* v, float* z, hipStream_t s) {
  if (mode == 1) return shell_bjac_apply32(m, ws->Binv, v, z, s);
  if (mode == 2) return line_pc_apply(m, ws->lineP_prec, ws->lineP, v, z, s);
  DG_HIP_CHECK(hipMemcpyAsync(z, v, m->n_dof * sizeof(float), hipMemcpyDeviceToDevice, s));
  return DG_OK;
}

static inline int grid_for(int64_t n) {
  int64_t b = (n + RED_THREADS - 1) / RED_THREADS;
  return (int)std::min<int64_t>(b, RED_BLOCKS);
}

// squared norm of the partial sums held in ws->part (RED_BLOCKS entries) -> host (synchronises)
static dg_status_t finish_norm2(Workspace* w, int nb, hipStream_t s, double* out) {
  k_reduce<<<1, RED_THREADS, 0, s>>>(w->part, nb, 1, w->dev_small);
  DG_HIP_CHECK(hipMemcpyAsync(w->host_small, w->dev_small, sizeof(double), hipMemcpyDeviceToHost, s));
  DG_HIP_CHECK(hipStreamSynchronize(s));
  *out = w->host_small[0];
  return DG_OK;
}

// blocks of RED_THREADS of kernel f resident on the device at once (at most RED_BLOCKS). The
// grid of a grid-stride sweep is capped there: with more registers than 64 per lane the full
// RED_BLOCKS no longer fit in one round, and the blocks of a second round would run on a
// nearly empty chip. The cap depends only on the kernel, so each kernel's partition of the
// sum, and with it the summation order, stays fixed.
static int resident_grid(const void* f) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, RED_THREADS, 0) != hipSuccess || per < 1 || cus < 1)
    return RED_BLOCKS;
  return std::min(RED_BLOCKS, per * cus);
}

// the launches below return the grid they used: the caller's k_reduce sums that many parts
template <int K, class T>
static int launch_mdot_k(int64_t n, const T* V, int64_t ldv, const T* w, double* part, int nb, hipStream_t s) {
  static const int cap = resident_grid(reinterpret_cast<const void*>(&k_mdot<K, T>));
  nb = std::min(nb, cap);
  k_mdot<K, T><<<nb, RED_THREADS, 0, s>>>(n, V, ldv, w, part);
  return nb;
}

template <int K, class T>
static int launch_orth_mdot_k(int64_t n, const T* V, int64_t ldv, const double* h, T* w, double* part, int nb,
                              hipStream_t s) {
  static const int cap = resident_grid(reinterpret_cast<const void*>(&k_orth_mdot<K, T>));
  nb = std::min(nb, cap);
  k_orth_mdot<K, T><<<nb, RED_THREADS, 0, s>>>(n, V, ldv, h, w, part);
  return nb;
}

template <int K, class T>
static int launch_orth_update_k(int64_t n, const T* V, int64_t ldv, const double* h, T* w, double* part, int nb,
                                hipStream_t s) {
  static const int cap = resident_grid(reinterpret_cast<const void*>(&k_orth_update<K, T>));
  nb = std::min(nb, cap);
  k_orth_update<K, T><<<nb, RED_THREADS, 0, s>>>(n, V, ldv, h, w, part);
  return nb;
}

template <class T, int K = 1>
static int launch_orth_update(int kk, int64_t n, const T* V, int64_t ldv, const double* h, T* w, double* part, int nb,
                              hipStream_t s) {
  if constexpr (K > 33) {
    (void)kk; (void)n; (void)V; (void)ldv; (void)h; (void)w; (void)part; (void)s;
    return nb;
  } else {
    if (kk == K) return launch_orth_update_k<K, T>(n, V, ldv, h, w, part, nb, s);
    return launch_orth_update<T, K + 1>(kk, n, V, ldv, h, w, part, nb, s);
  }
}

template <class T, int K = 1>
static int launch_orth_mdot(int kk, int64_t n, const T* V, int64_t ldv, const double* h, T* w, double* part, int nb,
                            hipStream_t s) {
  if constexpr (K > 33) {
    (void)kk; (void)n; (void)V; (void)ldv; (void)h; (void)w; (void)part; (void)s;
    return nb;
  } else {
    if (kk == K) return launch_orth_mdot_k<K, T>(n, V, ldv, h, w, part, nb, s);
    return launch_orth_mdot<T, K + 1>(kk, n, V, ldv, h, w, part, nb, s);
  }
}

template <class T, int K = 1>
static int launch_mdot(int kk, int64_t n, const T* V, int64_t ldv, const T* w, double* part, int nb, hipStream_t s) {
  if constexpr (K > 33) {
    (void)kk; (void)n; (void)V; (void)ldv; (void)w; (void)part; (void)s;
    return nb;
  } else {
    if (kk == K) return launch_mdot_k<K, T>(n, V, ldv, w, part, nb, s);
    return launch_mdot<T, K + 1>(kk, n, V, ldv, w, part, nb, s);
  }
}

// ---- reduced basis: the pseudo-inverse of the Gram matrix (cyclic Jacobi, k <= RB_MAX)
static void rb_pinv(const double* G, int k, double rcond, double* Gp) {
  double a[RB_MAX][RB_MAX], v[RB_MAX][RB_MAX];
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      a[i][j] = G[i * RB_MAX + j];
      v[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j) off += a[i][j] * a[i][j];
    if (off == 0) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        if (a[p][q] == 0) continue;
        const double th = (a[q][q] - a[p][p]) / (2 * a[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        const double c = 1 / std::sqrt(t * t + 1), sn = t * c;
        for (int r = 0; r < k; ++r) {   // columns p, q
          const double ap = a[r][p], aq = a[r][q];
          a[r][p] = c * ap - sn * aq;
          a[r][q] = sn * ap + c * aq;
        }
        for (int r = 0; r < k; ++r) {   // rows p, q
          const double ap = a[p][r], aq = a[q][r];
          a[p][r] = c * ap - sn * aq;
          a[q][r] = sn * ap + c * aq;
        }
        for (int r = 0; r < k; ++r) {
          const double vp = v[r][p], vq = v[r][q];
          v[r][p] = c * vp - sn * vq;
          v[r][q] = sn * vp + c * vq;
        }
      }
  }
  double lmax = 0;
  for (int i = 0; i < k; ++i) lmax = std::max(lmax, a[i][i]);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double g = 0;
      for (int l = 0; l < k; ++l)
        if (a[l][l] > rcond * lmax && a[l][l] > 0) g += v[i][l] * v[j][l] / a[l][l];
      Gp[i * k + j] = g;
    }
}

// c = (Z^T Z)^+ Z^T v on the device (rb_dev: Gp, d, c)
template <class T>
static void rb_coefficients(dg_mesh_s* m, Workspace* ws, const T* v, hipStream_t s) {
  const int64_t n = m->n_dof;
  const int nb = grid_for(n);
  const int k = ws->rb_count;
  double* d = ws->rb_dev + RB_MAX * RB_MAX;
  const int nbd = launch_mdot<T>(k, n, (const T*)ws->rbZ, n, v, ws->part, nb, s);
  k_reduce<<<k, RED_THREADS, 0, s>>>(ws->part, nbd, k, d);
  k_rb_coef<<<1, 64, 0, s>>>(k, ws->rb_dev, d, d + RB_MAX);
}

// z = W c(v) + P^-1 (v - Z c(v)); scratch: a free vector of the Krylov precision
template <class T>
static dg_status_t precond_rb(dg_mesh_s* m, Workspace* ws, int pc, const T* v, T* z, T* scratch, hipStream_t s) {
  const int k = ws->rb_count;
  if (k == 0) return precond(m, ws, pc, v, z, s);
  const int64_t n = m->n_dof;
  const int nb = grid_for(n);
  rb_coefficients<T>(m, ws, v, s);
  const double* c = ws->rb_dev + RB_MAX * RB_MAX + RB_MAX;
  const T* Z = (const T*)ws->rbZ;
  const T* W = (const T*)ws->rbW;
  if (pc == 0) {
    k_rb_split<T><<<nb, RED_THREADS, 0, s>>>(n, k, Z, W, c, v, z, z);
    return DG_OK;
  }
  T* x = (T*)ws->rbT;
  k_rb_split<T><<<nb, RED_THREADS, 0, s>>>(n, k, Z, W, c, v, scratch, x);
  dg_status_t st = precond(m, ws, pc, scratch, z, s);
  if (st != DG_OK) return st;
  k_add_T<T><<<nb, RED_THREADS, 0, s>>>(n, x, z);
  return DG_OK;
}

// X = W c(rhs): the GMRES initial guess from the reduced basis
template <class T>
static void rb_initial_guess(dg_mesh_s* m, Workspace* ws, const double* rhs, double* X, hipStream_t s) {
  const int64_t n = m->n_dof;
  const int nb = grid_for(n);
  k_copy_cast<T><<<nb, RED_THREADS, 0, s>>>(n, rhs, (T*)ws->rbT);
  rb_coefficients<T>(m, ws, (const T*)ws->rbT, s);
  k_rb_guess<T><<<nb, RED_THREADS, 0, s>>>(n, ws->rb_count, (const T*)ws->rbW,
                                           ws->rb_dev + RB_MAX * RB_MAX + RB_MAX, X);
}

// the Newton update X joins the window with z = (I - c J(U)) X; the Gram matrix and its
// pseudo-inverse are updated (synchronises)
template <class T>
static dg_status_t rb_push(dg_mesh_s* m, Workspace* ws, int n_rb, double t, double c, const double* U,
                           const double* X, hipStream_t s) {
  const int64_t n = m->n_dof;
  const int nb = grid_for(n);
  const int slot = ws->rb_head;
  T* Wd = (T*)ws->rbW + (size_t)slot * n;
  T* Zd = (T*)ws->rbZ + (size_t)slot * n;
  k_copy_cast<T><<<nb, RED_THREADS, 0, s>>>(n, X, Wd);
  dg_status_t st = jvp(m, t, U, Wd, Zd, s);
  if (st != DG_OK) return st;
  k_stage_op<T><<<nb, RED_THREADS, 0, s>>>(n, Wd, c, Zd);
  ws->rb_head = (slot + 1) % n_rb;
  ws->rb_count = std::min(ws->rb_count + 1, n_rb);
  const int k = ws->rb_count;
  double* d = ws->rb_dev + RB_MAX * RB_MAX;
  const int nbd = launch_mdot<T>(k, n, (const T*)ws->rbZ, n, Zd, ws->part, nb, s);
  k_reduce<<<k, RED_THREADS, 0, s>>>(ws->part, nbd, k, d);
  DG_HIP_CHECK(hipMemcpyAsync(ws->host_small, d, k * sizeof(double), hipMemcpyDeviceToHost, s));
  DG_HIP_CHECK(hipStreamSynchronize(s));
  for (int j = 0; j < k; ++j) {
    if (!std::isfinite(ws->host_small[j])) {
      set_error("dg_implicit_step: non-finite value in the reduced basis");
      return DG_ERR_NAN;
    }
    ws->rb_G[slot * RB_MAX + j] = ws->rb_G[j * RB_MAX + slot] = ws->host_small[j];
  }
  const double rcond = std::is_same<T, float>::value ? 1e-7 : 1e-10;
  rb_pinv(ws->rb_G, k, rcond, ws->rb_host);
  DG_HIP_CHECK(hipMemcpyAsync(ws->rb_dev, ws->rb_host, (size_t)k * k * sizeof(double), hipMemcpyHostToDevice, s));
  return DG_OK;
}

// GMRES(m) for (I - c J(U)) x = rhs (rhs = -G, double), x returned in ws->X; with x0 set,
// ws->X holds the initial guess on entry. The preconditioner is P (pc) wrapped by the
// reduced basis when the window holds vectors.
template <class T>
static dg_status_t gmres(dg_mesh_s* m, Workspace* ws, double t, double c, const double* U, const double* rhs,
                         double rhs_norm, int pc, int mk, int max_restarts, double rtol, bool x0, int* iters,
                         hipStream_t s) {
  const int64_t n = m->n_dof;
  const int nb = grid_for(n);
  T* V = (T*)ws->V;
  T* w = (T*)ws->w;
  T* z = (T*)ws->z;
  T* sv = (T*)ws->s;
  double* X = ws->X;
  double* h1 = ws->dev_small;
  double* h2 = ws->dev_small + KMAX;
  double* nr = ws->dev_small + 2 * KMAX;
  double* yv = ws->dev_small + 3 * KMAX;
  double* host = ws->host_small;
  if (!x0) DG_HIP_CHECK(hipMemsetAsync(X, 0, n * sizeof(double), s));
  std::vector<double> H((size_t)(mk + 1) * mk), g(mk + 1), cs(mk), sn(mk), y(mk);
  const double target = rtol * rhs_norm;
  int total = 0;
  for (int cycle = 0; cycle < max_restarts; ++cycle) {
    double beta;
    if (cycle == 0 && !x0) {
      beta = rhs_norm;
      k_scale_to<T><<<nb, RED_THREADS, 0, s>>>(n, 1.0 / beta, rhs, V);
    } else {
      // true residual of the current iterate: V0 = rhs - A x (A applied in the Krylov precision)
      k_copy_cast<T><<<nb, RED_THREADS, 0, s>>>(n, X, z);
      dg_status_t st = jvp(m, t, U, z, w, s);
      if (st != DG_OK) return st;
      k_stage_op<T><<<nb, RED_THREADS, 0, s>>>(n, z, c, w);
      k_restart_vector<T><<<nb, RED_THREADS, 0, s>>>(n, rhs, w, V, ws->part);
      k_reduce<<<1, RED_THREADS, 0, s>>>(ws->part, nb, 1, nr);
      DG_HIP_CHECK(hipMemcpyAsync(host, nr, sizeof(double), hipMemcpyDeviceToHost, s));
      DG_HIP_CHECK(hipStreamSynchronize(s));
      beta = std::sqrt(host[0]);
      if (!std::isfinite(beta)) {
        set_error("dg_implicit_step: non-finite value in GMRES");
        return DG_ERR_NAN;
      }
      if (beta <= target) break;
      k_normalize<T><<<nb, RED_THREADS, 0, s>>>(n, V, nr, V);
    }
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int kused = 0;
    bool done = false;
    for (int j = 0; j < mk; ++j) {
      T* vj = V + (size_t)j * n;
      dg_status_t st = precond_rb(m, ws, pc, vj, z, w, s);
      if (st != DG_OK) return st;
      st = jvp(m, t, U, z, w, s);
      if (st != DG_OK) return st;
      k_stage_op<T><<<nb, RED_THREADS, 0, s>>>(n, z, c, w);
      // classical Gram-Schmidt, twice
      {
        ProfScope ps(m, 9, s);
        const int nb1 = launch_mdot<T>(j + 1, n, V, n, w, ws->part, nb, s);
        k_reduce<<<j + 1, RED_THREADS, 0, s>>>(ws->part, nb1, j + 1, h1);
        const int nb2 = launch_orth_mdot<T>(j + 1, n, V, n, h1, w, ws->part, nb, s);
        k_reduce<<<j + 1, RED_THREADS, 0, s>>>(ws->part, nb2, j + 1, h2);
        const int nb3 = launch_orth_update<T>(j + 1, n, V, n, h2, w, ws->part, nb, s);
        k_reduce<<<1, RED_THREADS, 0, s>>>(ws->part, nb3, 1, nr);
        k_normalize<T><<<nb, RED_THREADS, 0, s>>>(n, w, nr, V + (size_t)(j + 1) * n);
      }
      DG_HIP_CHECK(hipMemcpyAsync(host, ws->dev_small, (2 * KMAX + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      DG_HIP_CHECK(hipStreamSynchronize(s));
      ++total;
      double* col = &H[(size_t)j * (mk + 1)];
      for (int i = 0; i <= j; ++i) col[i] = host[i] + host[KMAX + i];
      const double hn = std::sqrt(host[2 * KMAX]);
      col[j + 1] = hn;
      if (!std::isfinite(hn)) {
        set_error("dg_implicit_step: non-finite value in GMRES");
        return DG_ERR_NAN;
      }
      for (int i = 0; i < j; ++i) {
        const double a = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = a;
      }
      const double den = std::hypot(col[j], col[j + 1]);
      cs[j] = den > 0 ? col[j] / den : 1.0;
      sn[j] = den > 0 ? col[j + 1] / den : 0.0;
      col[j] = den;
      col[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      kused = j + 1;
      if (std::fabs(g[j + 1]) <= target || hn == 0.0) {
        done = true;
        break;
      }
    }
    // back substitution  H(0:k,0:k) y = g(0:k)
    for (int i = kused - 1; i >= 0; --i) {
      double a = g[i];
      for (int k2 = i + 1; k2 < kused; ++k2) a -= H[(size_t)k2 * (mk + 1) + i] * y[k2];
      y[i] = a / H[(size_t)i * (mk + 1) + i];
    }
    for (int i = 0; i < kused; ++i) host[3 * KMAX + i] = y[i];
    DG_HIP_CHECK(hipMemcpyAsync(yv, host + 3 * KMAX, kused * sizeof(double), hipMemcpyHostToDevice, s));
    launch_combine<T>(kused, nb, s, n, V, n, yv, sv);
    dg_status_t st = precond_rb(m, ws, pc, sv, z, w, s);
    if (st != DG_OK) return st;
    k_add_to<T><<<nb, RED_THREADS, 0, s>>>(n, z, X);
    if (done) break;
  }
  *iters = total;
  return DG_OK;
}

static void dirk_tableau(int scheme, double A[3][3], double c[3], int& ns) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = 0;
  if (scheme == 22) {
    const double g = 1.0 - 1.0 / std::sqrt(2.0);
    A[0][0] = g;
    A[1][0] = 1.0 - g;
    A[1][1] = g;
    c[0] = g;
    c[1] = 1.0;
    ns = 2;
    return;
  }
  // g: root in (1/6, 1/2) of g^3 - 3 g^2 + 3/2 g - 1/6 (Newton from 0.4)
  double g = 0.4;
  for (int it = 0; it < 60; ++it) {
    const double f = ((g - 3.0) * g + 1.5) * g - 1.0 / 6.0;
    const double df = (3.0 * g - 6.0) * g + 1.5;
    g -= f / df;
  }
  A[0][0] = g;
  A[1][0] = 0.5 * (1.0 - g);
  A[1][1] = g;
  A[2][0] = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0;
  A[2][1] = (6.0 * g * g - 20.0 * g + 5.0) / 4.0;
  A[2][2] = g;
  c[0] = g;
  c[1] = 0.5 * (1.0 + g);
  c[2] = 1.0;
  ns = 3;
}

template <class T>
static dg_status_t step_impl(dg_mesh_s* m, double t, double dt, double* u, const dg_solver_opts_t& o,
                             dg_step_stats_t* st, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  dg_status_t rc = ensure_workspace(m, o.gmres_m, std::is_same<T, float>::value);
  if (rc != DG_OK) return rc;
  Workspace* ws = m->ws;
  const int64_t n = m->n_dof;
  const int nb = grid_for(n);
  const int pc = (m->kind == DG_MESH_SHELL) ? o.precond : 0;
  const bool f32 = std::is_same<T, float>::value;
  if (pc == 2 && (!ws->lineLo || ws->lineP_prec != m->line_pc_prec)) {
    const size_t cnt = (size_t)line_pc_doubles(m);
    const int prec = m->line_pc_prec;
    bool ok = true;
    if (!ws->lineLo)
      ok = hipMalloc(&ws->lineLo, cnt * sizeof(double)) == hipSuccess &&
           hipMalloc(&ws->lineDi, cnt * sizeof(double)) == hipSuccess &&
           hipMalloc(&ws->lineUp, cnt * sizeof(double)) == hipSuccess;
    if (ws->lineP) (void)hipFree(ws->lineP);
    ws->lineP = nullptr;
    ws->lineP_prec = 0;
    ws->line_age = -1;
    if (ok) ok = hipMalloc(&ws->lineP, (size_t)line_pc_packed(m) * (prec / 8)) == hipSuccess;
    if (!ok) {
      set_error("dg_implicit_step: allocation of the line preconditioner failed");
      return DG_ERR_ALLOC;
    }
    ws->lineP_prec = prec;
  }
  if (o.n_rb > ws->rb_cap) {
    for (void* p : {ws->rbW, ws->rbZ, ws->rbT, (void*)ws->rb_dev})
      if (p) (void)hipFree(p);
    if (ws->rb_host) (void)hipHostFree(ws->rb_host);
    ws->rbW = ws->rbZ = ws->rbT = nullptr;
    ws->rb_dev = ws->rb_host = nullptr;
    ws->rb_cap = ws->rb_count = ws->rb_head = 0;
    const size_t vb = f32 ? sizeof(float) : sizeof(double);
    const bool ok = hipMalloc(&ws->rbW, (size_t)o.n_rb * n * vb) == hipSuccess &&
                    hipMalloc(&ws->rbZ, (size_t)o.n_rb * n * vb) == hipSuccess &&
                    hipMalloc(&ws->rbT, (size_t)n * vb) == hipSuccess &&
                    hipMalloc(&ws->rb_dev, (RB_MAX * RB_MAX + 2 * RB_MAX) * sizeof(double)) == hipSuccess &&
                    hipHostMalloc(&ws->rb_host, RB_MAX * RB_MAX * sizeof(double)) == hipSuccess;
    if (!ok) {
      set_error("dg_implicit_step: allocation of the reduced basis failed");
      return DG_ERR_ALLOC;
    }
    ws->rb_cap = o.n_rb;
  }
  double A[3][3], c[3];
  int ns;
  dirk_tableau(o.scheme, A, c, ns);
  dg_step_stats_t stats{};
  // a step that does not continue the previous one starts a new guess history
  if (!(std::fabs(ws->t_end - t) <= 1e-12 * std::max(1.0, std::fabs(t)))) {
    ws->hist_n = 0;
    ws->line_age = -1;   // and a new radial-line preconditioner
  }
  // the reduced basis lives as long as the stage operator's dt a_ii, the window size and
  // the history do
  if (o.n_rb == 0 || ws->hist_n == 0 || ws->rb_dta != dt * A[0][0] || ws->rb_n != o.n_rb) {
    ws->rb_count = ws->rb_head = 0;
    ws->rb_dta = dt * A[0][0];
    ws->rb_n = o.n_rb;
  }
  DG_HIP_CHECK(hipMemcpyAsync(ws->un, u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  // radial-line preconditioner: built at (t + c_1 dt, u_n) and kept for line_pc_every steps;
  // a_ii is the same for every stage of the singly-diagonal schemes
  if (pc == 2) {
    const bool stale = ws->line_age < 0 || ws->line_age + 1 >= m->line_pc_every || ws->line_f32 != f32 ||
                       ws->line_dta != dt * A[0][0];
    if (stale) {
      rc = line_pc_build(m, t + c[0] * dt, ws->un, dt * A[0][0], ws->lineLo, ws->lineDi, ws->lineUp, ws->X, ws->Rc,
                         f32, ws->lineP_prec, ws->lineP, s);
      if (rc != DG_OK) return rc;
      ws->line_age = 0;
      ws->line_f32 = f32;
      ws->line_dta = dt * A[0][0];
    } else {
      ++ws->line_age;
    }
  }
  for (int i = 0; i < ns; ++i) {
    const double ti = t + c[i] * dt;
    const double ca = dt * A[i][i];
    // b_i = u_n + dt sum_{j<i} a_ij R_j
    DG_HIP_CHECK(hipMemcpyAsync(ws->B, ws->un, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    for (int j = 0; j < i; ++j) k_axpby<<<nb, RED_THREADS, 0, s>>>(n, dt * A[i][j], ws->Rs[j], 1.0, ws->B, nullptr);
    // reference norm |G(u_n)|
    rc = residual(m, ti, ws->un, ws->Rc, s);
    if (rc != DG_OK) return rc;
    k_stage_residual<<<nb, RED_THREADS, 0, s>>>(n, ws->un, ws->Rc, ca, ws->B, ws->G, ws->part);
    double ref2;
    rc = finish_norm2(ws, nb, s, &ref2);
    if (rc != DG_OK) return rc;
    const double ref = std::sqrt(ref2);
    // plain initial guess: extrapolation through the two latest stage solutions
    const bool have_hist = ws->hist_n >= 2 && ws->hist_t[0] != ws->hist_t[1];
    if (have_hist) {
      const double f = (ti - ws->hist_t[0]) / (ws->hist_t[0] - ws->hist_t[1]);
      k_extrapolate<<<nb, RED_THREADS, 0, s>>>(n, ws->hist[0], ws->hist[1], f, ws->U);
    } else {
      DG_HIP_CHECK(hipMemcpyAsync(ws->U, ws->un, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    DG_HIP_CHECK(hipMemcpyAsync(ws->Up, ws->U, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    // learned guess: the network's correction of the plain guess, kept only if it lowers |G|
    bool have_G = false;
    double g2_guess = 0;
    if (o.guess == 1 && m->ws_mlp && have_hist) {
      const int N = m->N, nin = 15 * N, nout = 5 * N;
      const int64_t E = m->n_elem;
      k_ws_features<<<(unsigned)((E * nin + 255) / 256), 256, 0, s>>>(E, N, ws->hist[0], ws->hist[1], ws->B,
                                                                       m->ws_norm, m->ws_norm + nin, m->ws_X);
      rc = mlp_forward(m->ws_mlp, m->ws_X, E, m->ws_Y, s, false);
      if (rc != DG_OK) return rc;
      k_ws_apply<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, ws->Up, m->ws_Y, m->ws_norm + 2 * nin,
                                                             m->ws_norm + 2 * nin + nout, nout, ws->U);
      // the network's correction D = U - U_p, scaled by the alpha that minimises the
      // linearised stage residual |G(U_p) + alpha (I - dt a_ii J(U_p)) D|
      k_axpby<<<nb, RED_THREADS, 0, s>>>(n, 1.0, ws->U, 0.0, ws->X, nullptr);
      k_axpby<<<nb, RED_THREADS, 0, s>>>(n, -1.0, ws->Up, 1.0, ws->X, nullptr);
      double gl2, gp2;
      rc = residual(m, ti, ws->Up, ws->Rc, s);
      if (rc != DG_OK) return rc;
      k_stage_residual<<<nb, RED_THREADS, 0, s>>>(n, ws->Up, ws->Rc, ca, ws->B, ws->G, ws->part);
      rc = finish_norm2(ws, nb, s, &gp2);
      if (rc != DG_OK) return rc;
      rc = jvp(m, ti, ws->Up, ws->X, ws->Rc, s);
      if (rc != DG_OK) return rc;
      k_stage_op<double><<<nb, RED_THREADS, 0, s>>>(n, ws->X, ca, ws->Rc);
      k_dot2<<<nb, RED_THREADS, 0, s>>>(n, ws->G, ws->Rc, ws->part);
      k_reduce<<<2, RED_THREADS, 0, s>>>(ws->part, nb, 2, ws->dev_small);
      DG_HIP_CHECK(hipMemcpyAsync(ws->host_small, ws->dev_small, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      DG_HIP_CHECK(hipStreamSynchronize(s));
      const double gd = ws->host_small[0], dd = ws->host_small[1];
      double alpha = (dd > 0 && std::isfinite(gd)) ? -gd / dd : 0.0;
      alpha = std::min(std::max(alpha, 0.0), 2.0);
      stats.guess_scale[i] = alpha;
      k_axpby<<<nb, RED_THREADS, 0, s>>>(n, 1.0, ws->Up, 0.0, ws->U, nullptr);
      k_axpby<<<nb, RED_THREADS, 0, s>>>(n, alpha, ws->X, 1.0, ws->U, nullptr);
      rc = residual(m, ti, ws->U, ws->Rc, s);
      if (rc != DG_OK) return rc;
      k_stage_residual<<<nb, RED_THREADS, 0, s>>>(n, ws->U, ws->Rc, ca, ws->B, ws->G, ws->part);
      rc = finish_norm2(ws, nb, s, &gl2);
      if (rc != DG_OK) return rc;
      if (!(gl2 < gp2)) {
        DG_HIP_CHECK(hipMemcpyAsync(ws->U, ws->Up, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        stats.fallback[i] = 1;
      } else {
        have_G = true;     // G and R of the accepted guess are in ws->G and ws->Rc
        g2_guess = gl2;
      }
    }
    int newton = 0, gm_total = 0, halvings = 0;
    double nG = 0, prev = 0, alpha = 1.0, eta = 0.1;
    for (;;) {
      double g2;
      if (newton == 0 && have_G) {
        g2 = g2_guess;
      } else {
        rc = residual(m, ti, ws->U, ws->Rc, s);
        if (rc != DG_OK) return rc;
        k_stage_residual<<<nb, RED_THREADS, 0, s>>>(n, ws->U, ws->Rc, ca, ws->B, ws->G, ws->part);
        rc = finish_norm2(ws, nb, s, &g2);
        if (rc != DG_OK) return rc;
      }
      nG = std::sqrt(g2);
      if (newton == 0) stats.res0[i] = nG;
      // backtracking: a Newton update that leaves a non-finite or larger residual is halved
      if (newton > 0 && !(nG <= prev) && halvings < 6) {
        alpha *= 0.5;
        k_axpby<<<nb, RED_THREADS, 0, s>>>(n, -alpha, ws->X, 1.0, ws->U, nullptr);
        ++halvings;
        continue;
      }
      if (!std::isfinite(nG)) {
        DG_HIP_CHECK(hipMemcpyAsync(u, ws->un, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        set_error("dg_implicit_step: non-finite stage residual");
        return DG_ERR_NAN;
      }
      if (nG <= o.newton_rtol * ref || newton >= o.max_newton) break;
      if (pc == 1) {
        rc = shell_bjac_build(m, ti, ws->U, ca, ws->Binv, s);
        if (rc != DG_OK) return rc;
      }
      // rhs = -G
      k_axpby<<<nb, RED_THREADS, 0, s>>>(n, 0.0, ws->G, -1.0, ws->G, nullptr);
      int its = 0;
      double rtol = o.gmres_rtol;
      if (o.forcing == 1) {
        if (newton > 0) {
          const double r = nG / prev;
          double e2 = 0.9 * r * r;
          const double safe = 0.9 * eta * eta;
          if (safe > 0.1) e2 = std::max(e2, safe);
          eta = std::min(0.1, e2);
        }
        rtol = std::max(eta, 0.5 * o.newton_rtol * ref / nG);
        rtol = std::min(rtol, 0.1);
      }
      const bool x0 = o.n_rb > 0 && ws->rb_count > 0;
      if (x0) rb_initial_guess<T>(m, ws, ws->G, ws->X, s);
      rc = gmres<T>(m, ws, ti, ca, ws->U, ws->G, nG, pc, o.gmres_m, o.max_restarts, rtol, x0, &its, s);
      if (rc == DG_OK && o.n_rb > 0) rc = rb_push<T>(m, ws, o.n_rb, ti, ca, ws->U, ws->X, s);
      if (rc != DG_OK) {
        (void)hipMemcpyAsync(u, ws->un, n * sizeof(double), hipMemcpyDeviceToDevice, s);
        return rc;
      }
      gm_total += its;
      k_axpby<<<nb, RED_THREADS, 0, s>>>(n, 1.0, ws->X, 1.0, ws->U, nullptr);
      ++newton;
      prev = nG;
      alpha = 1.0;
      halvings = 0;
    }
    stats.newton_its[i] = newton;
    stats.gmres_its[i] = gm_total;
    stats.res[i] = nG;
    stats.ref[i] = ref;
    if (!(nG <= o.newton_rtol * ref)) {
      DG_HIP_CHECK(hipMemcpyAsync(u, ws->un, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      DG_HIP_CHECK(hipStreamSynchronize(s));
      if (st) {
        stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *st = stats;
      }
      ws->hist_n = 0;
      set_error("dg_implicit_step: Newton did not reach the tolerance");
      return DG_ERR_NOCONV;
    }
    DG_HIP_CHECK(hipMemcpyAsync(ws->Rs[i], ws->Rc, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    // training pairs for the warm-start network (before the history moves on)
    if (m->rec_cap > m->rec_count && have_hist && m->kind == DG_MESH_SHELL) {
      const int every = m->rec_every;
      const int64_t phase = m->rec_phase % every;
      const int64_t sel = (m->n_elem - phase + every - 1) / every;
      const int64_t rows = std::min(sel, m->rec_cap - m->rec_count);
      const int64_t tot = rows * 20 * (int64_t)m->N;
      if (rows > 0)
        k_ws_record<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(rows, phase, every, m->N, ws->hist[0], ws->hist[1],
                                                                  ws->B, ws->U, ws->Up, m->rec_x, m->rec_y,
                                                                  m->rec_count);
      m->rec_count += rows;
      m->rec_phase += 1;
    }
    // history: newest first
    std::swap(ws->hist[0], ws->hist[1]);
    ws->hist_t[1] = ws->hist_t[0];
    DG_HIP_CHECK(hipMemcpyAsync(ws->hist[0], ws->U, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    ws->hist_t[0] = ti;
    ws->hist_n = std::min(ws->hist_n + 1, 2);
  }
  // stiffly accurate: u_{n+1} = U_last, then the optional modal filter
  DG_HIP_CHECK(hipMemcpyAsync(u, ws->U, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (o.filter_rate > 0) {
    const double sigma = std::exp(-o.filter_rate * dt);
    rc = (m->kind == DG_MESH_SHELL) ? shell_filter_apply(m, sigma, u, s) : col_filter_apply(m, sigma, u, s);
    if (rc != DG_OK) return rc;
  }
  DG_HIP_CHECK(hipStreamSynchronize(s));
  ws->t_end = t + dt;
  stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = stats;
  return DG_OK;
}

dg_status_t implicit_step(dg_mesh_s* m, double t, double dt, double* u, const dg_solver_opts_t& o,
                          dg_step_stats_t* st, hipStream_t s) {
  if (o.guess == 1 && !m->ws_mlp) {
    set_error("dg_implicit_step: the learned guess needs a warm-start network (dg_warmstart_set)");
    return DG_ERR_UNSUPPORTED;
  }
  if (o.jvp_prec == DG_BF16 && !(m->kind == DG_MESH_SHELL && m->d_bf16op)) {
    set_error("dg_implicit_step: the BF16 J v is available for shells of degree 3 and 4");
    return DG_ERR_UNSUPPORTED;
  }
  m->krylov_bf16 = (o.jvp_prec == DG_BF16);
  m->krylov_fd = (o.jvp_prec == DG_F64_FD);
  const dg_status_t rc = (o.jvp_prec == DG_F32 || o.jvp_prec == DG_BF16) ? step_impl<float>(m, t, dt, u, o, st, s)
                                                                         : step_impl<double>(m, t, dt, u, o, st, s);
  if (rc != DG_OK && m->ws) {
    // a failed step leaves u unchanged: the next one starts a new guess history and
    // reduced-basis window (nothing from the failed attempt is reused)
    m->ws->hist_n = 0;
    m->ws->rb_count = m->ws->rb_head = 0;
    m->ws->t_end = NAN;
  }
  return rc;
}

}  // namespace dg
