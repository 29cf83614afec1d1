// Radial-line block-Jacobi preconditioner for the shell's stage matrix I - dta J(u).
//
// A line is the column of nodes above one angular node: (angular cell, a + n b), its
// n_rad (p + 1) nodes and 5 fields. The preconditioner is I - dta J_rad with J_rad the
// radial-line linearisation (shell_jvp_radial: the tangent's coupling between different
// angular nodes dropped, the radial coupling exact), block diagonal in the lines and,
// along each line, block tridiagonal across the radial layers with blocks of
// b = 5 (p + 1) unknowns (index field * (p + 1) + radial node).
//  * build: 3 b probes v = e_(field, radial node) on every layer of one colour (layer
//    mod 3) give every block column (the response of a layer comes from its own and its
//    two neighbours' probes only);
//  * factor: block LU per line, one wavefront per line (Schur complements inverted by
//    Gauss-Jordan with partial pivoting, W = D^-1 U kept for the back substitution);
//  * apply: forward and back substitution, several lines per wavefront.
// Blocks are stored column-major (entry (r, c) at c b + r): the probes fill columns, and
// the lanes of the substitution (one row each) read consecutive addresses.
// The radial direction carries the stiffness of the thin layers (vertical acoustics and
// conduction), so these blocks catch most of it at the cost of a few R-sized sweeps.
#include "internal.h"

namespace dg {

struct LineDev {
  int n, b, bb, n_rad, E, N, N2;
  double* Lo;   // [lines][n_rad][b x b column-major]
  double* Di;
  double* Up;
};

// v = 1 at (field pc, radial node pcz) of every node on layers k = kap (mod 3), else 0
__global__ void k_line_probe(int64_t n_dof, int N, int N2, int n, int n_rad, int pc, int pcz, int kap,
                             double* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_dof) return;
  const int j = (int)(i % N);
  const int64_t ec = i / N;
  const int c = (int)(ec % 5);
  const int64_t e = ec / 5;
  const int k = (int)(e % n_rad);
  v[i] = (c == pc && j / N2 == pcz && k % 3 == kap) ? 1.0 : 0.0;
}

// the response jr of probe (pc, pcz, kap) into block column l = pc * n + pcz. One thread
// per (line, layer, row): consecutive threads write consecutive rows of the column-major
// blocks (entry (r, c) of a block at c b + r).
template <class R>
__global__ void k_line_scatter(LineDev L, int pc, int pcz, int kap, double dta, const R* __restrict__ jr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)L.E * 5 * L.N) return;
  const int r = (int)(t % L.b);
  const int kp = (int)((t / L.b) % L.n_rad);
  const int64_t line = t / ((int64_t)L.b * L.n_rad);
  const int64_t cell = line / L.N2;
  const int ab = (int)(line % L.N2);
  // the source layer of this probe colour next to kp (at most one)
  int ks = -1;
  for (int d = -1; d <= 1; ++d) {
    const int kk = kp + d;
    if (kk >= 0 && kk < L.n_rad && kk % 3 == kap) ks = kk;
  }
  if (ks < 0) return;
  const int c = r / L.n, cz = r % L.n;
  const int64_t e = cell * L.n_rad + kp;
  const int l = pc * L.n + pcz;
  double* blk = (ks == kp - 1) ? L.Lo : (ks == kp ? L.Di : L.Up);
  const double val = ((ks == kp && r == l) ? 1.0 : 0.0) - dta * (double)jr[(e * 5 + c) * L.N + ab + L.N2 * cz];
  blk[(line * L.n_rad + kp) * L.bb + (int64_t)l * L.b + r] = val;
}

// index of the largest |v| over the wavefront (lowest lane on ties); lanes pass -1 to abstain
__device__ inline int wave_argmax(double v) {
  int idx = threadIdx.x & 63;
  for (int off = 32; off > 0; off >>= 1) {
    const double v2 = __shfl_xor(v, off, 64);
    const int i2 = __shfl_xor(idx, off, 64);
    if (v2 > v || (v2 == v && i2 < idx)) {
      v = v2;
      idx = i2;
    }
  }
  return idx;
}

// Gauss-Jordan inverse in LDS: M = [A | I] (row-major, b x 2b) -> [I | A^-1]; one wavefront
template <int b>
__device__ void line_gj(double (*M)[2 * b], double* fac) {
  const int lane = threadIdx.x;
  for (int k = 0; k < b; ++k) {
    const int piv = wave_argmax((lane >= k && lane < b) ? fabs(M[lane][k]) : -1.0);
    if (piv != k)
      for (int c = lane; c < 2 * b; c += 64) {
        const double tmp = M[k][c];
        M[k][c] = M[piv][c];
        M[piv][c] = tmp;
      }
    __syncthreads();
    const double inv = 1.0 / M[k][k];
    __syncthreads();
    for (int c = lane; c < 2 * b; c += 64) M[k][c] *= inv;
    __syncthreads();
    if (lane < b) fac[lane] = M[lane][k];
    __syncthreads();
    for (int idx = lane; idx < b * 2 * b; idx += 64) {
      const int r = idx / (2 * b), c = idx % (2 * b);
      if (r != k) M[r][c] -= fac[r] * M[k][c];
    }
    __syncthreads();
  }
}

// block LU of every line (grid: one 64-thread block per line), column-major blocks.
// After it: Di = inverses of the Schur complements, Up = W = Di Up, Lo unchanged.
template <int b>
__global__ __launch_bounds__(64) void k_line_factor(LineDev L) {
  constexpr int bb = b * b;
  __shared__ double M[b][2 * b];
  __shared__ double fac[b];
  __shared__ double Ls[bb], Ws[bb], Us[bb];
  const int64_t line = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t base = line * L.n_rad * bb;
  for (int k = 0; k < L.n_rad; ++k) {
    const int64_t off = base + (int64_t)k * bb;
    // M <- [D_k - L_k W_{k-1} | I]
    if (k > 0)
      for (int idx = lane; idx < bb; idx += 64) Ls[idx] = L.Lo[off + idx];
    __syncthreads();
    for (int idx = lane; idx < b * 2 * b; idx += 64) {
      const int r = idx / (2 * b), c = idx % (2 * b);
      double val;
      if (c < b) {
        val = L.Di[off + (int64_t)c * b + r];
        if (k > 0) {
          double s = 0;
          for (int q = 0; q < b; ++q) s += Ls[q * b + r] * Ws[c * b + q];
          val -= s;
        }
      } else {
        val = (c - b == r) ? 1.0 : 0.0;
      }
      M[r][c] = val;
    }
    __syncthreads();
    line_gj<b>(M, fac);
    for (int idx = lane; idx < bb; idx += 64) {
      const int c = idx / b, r = idx % b;
      L.Di[off + idx] = M[r][b + c];
    }
    if (k < L.n_rad - 1) {
      for (int idx = lane; idx < bb; idx += 64) Us[idx] = L.Up[off + idx];
      __syncthreads();
      // W_k = Dinv_k U_k, kept in LDS for the next layer
      for (int idx = lane; idx < bb; idx += 64) {
        const int c = idx / b, r = idx % b;
        double s = 0;
        for (int q = 0; q < b; ++q) s += M[r][b + q] * Us[c * b + q];
        Ws[idx] = s;
        L.Up[off + idx] = s;
      }
    }
    __syncthreads();
  }
}

// z = M^-1 r for every line; LPB lines per 64-thread block, lane = line slot * b + row.
// T: vector type, F: factor type.
template <int b, class T, class F>
__global__ __launch_bounds__(64) void k_line_solve(LineDev L, int64_t n_lines, const F* __restrict__ fLo,
                                                   const F* __restrict__ fDi, const F* __restrict__ fUp,
                                                   const T* __restrict__ rin, T* __restrict__ z) {
  constexpr int bb = b * b;
  constexpr int LPB = 64 / b;
  extern __shared__ double x[];   // [LPB][n_rad][b]
  __shared__ double y[LPB * b];
  const int lane = threadIdx.x;
  const int ls = lane / b, r = lane % b;
  const int64_t line = (int64_t)blockIdx.x * LPB + ls;
  const bool act = ls < LPB && line < n_lines;
  const int nb = L.n_rad * b;
  const int64_t line0 = (int64_t)blockIdx.x * LPB;
  // gather: unknown (k, c * n + cz) of line slot q <- r[e = cell n_rad + k][c][ab + N2 cz]
  for (int idx = lane; idx < LPB * nb; idx += 64) {
    const int q = idx / nb, w = idx % nb;
    const int64_t ln = line0 + q;
    if (ln >= n_lines) continue;
    const int k = w / b, rr = w % b, c = rr / L.n, cz = rr % L.n;
    const int64_t e = (ln / L.N2) * L.n_rad + k;
    x[idx] = (double)rin[(e * 5 + c) * L.N + (ln % L.N2) + L.N2 * cz];
  }
  __syncthreads();
  double* xl = x + ls * nb;
  const int64_t base = line * L.n_rad * bb;
  // forward: x_k <- Dinv_k (x_k - L_k x_{k-1})
  for (int k = 0; k < L.n_rad; ++k) {
    double* xk = xl + k * b;
    if (act && k > 0) {
      const F* Lc = fLo + base + (int64_t)k * bb;
      const double* xp = xl + (k - 1) * b;
      double s = 0;
      for (int q = 0; q < b; ++q) s += (double)Lc[q * b + r] * xp[q];
      xk[r] -= s;
    }
    __syncthreads();
    if (act) {
      const F* Dc = fDi + base + (int64_t)k * bb;
      double s = 0;
      for (int q = 0; q < b; ++q) s += (double)Dc[q * b + r] * xk[q];
      y[lane] = s;
    }
    __syncthreads();
    if (act) xk[r] = y[lane];
    __syncthreads();
  }
  // back: x_k <- x_k - W_k x_{k+1}
  for (int k = L.n_rad - 2; k >= 0; --k) {
    if (act) {
      const F* Wc = fUp + base + (int64_t)k * bb;
      const double* xn = xl + (k + 1) * b;
      double s = 0;
      for (int q = 0; q < b; ++q) s += (double)Wc[q * b + r] * xn[q];
      y[lane] = s;
    }
    __syncthreads();
    if (act) xl[k * b + r] -= y[lane];
    __syncthreads();
  }
  for (int idx = lane; idx < LPB * nb; idx += 64) {
    const int q = idx / nb, w = idx % nb;
    const int64_t ln = line0 + q;
    if (ln >= n_lines) continue;
    const int k = w / b, rr = w % b, c = rr / L.n, cz = rr % L.n;
    const int64_t e = (ln / L.N2) * L.n_rad + k;
    z[(e * 5 + c) * L.N + (ln % L.N2) + L.N2 * cz] = (T)x[idx];
  }
}

static LineDev line_dev(dg_mesh_s* m, double* Lo, double* Di, double* Up) {
  LineDev L;
  L.n = m->p + 1;
  L.b = 5 * L.n;
  L.bb = L.b * L.b;
  L.n_rad = m->n_rad;
  L.E = (int)m->n_elem;
  L.N = m->N;
  L.N2 = L.n * L.n;
  L.Lo = Lo;
  L.Di = Di;
  L.Up = Up;
  return L;
}

int64_t line_pc_doubles(const dg_mesh_s* m) {
  const int64_t n = m->p + 1, b = 5 * n;
  const int64_t lines = (m->n_elem / m->n_rad) * n * n;
  return lines * m->n_rad * b * b;
}

__global__ void k_to_float(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// build and factor at (t, u) for the stage matrix I - dta J; v, jr: scratch [n_dof]
// (jr: double, or float when f32 is set). With f32 the probes use the FP32 dual-number
// linearisation and the factors are also written as float to Lo32 / Di32 / Up32.
dg_status_t line_pc_build(dg_mesh_s* m, double t, const double* u, double dta, double* Lo, double* Di, double* Up,
                          double* v, void* jr, bool f32, float* Lo32, float* Di32, float* Up32, hipStream_t s) {
  ProfScope ps(m, 10, s);
  const LineDev L = line_dev(m, Lo, Di, Up);
  const int64_t nd = m->n_dof;
  const unsigned blocks = (unsigned)((nd + 255) / 256);
  const int64_t nblk = line_pc_doubles(m);
  // blocks of layers with no neighbour (Lo of layer 0, Up of the top layer) stay zero
  DG_HIP_CHECK(hipMemsetAsync(Lo, 0, nblk * sizeof(double), s));
  DG_HIP_CHECK(hipMemsetAsync(Up, 0, nblk * sizeof(double), s));
  for (int kap = 0; kap < 3; ++kap)
    for (int pc = 0; pc < 5; ++pc)
      for (int pcz = 0; pcz < L.n; ++pcz) {
        k_line_probe<<<blocks, 256, 0, s>>>(nd, L.N, L.N2, L.n, L.n_rad, pc, pcz, kap, v);
        if (f32) {
          k_to_float<<<blocks, 256, 0, s>>>(nd, v, (float*)jr + nd);
          dg_status_t rc = shell_jvp_radial32(m, t, u, (const float*)jr + nd, (float*)jr, s);
          if (rc != DG_OK) return rc;
          k_line_scatter<float><<<blocks, 256, 0, s>>>(L, pc, pcz, kap, dta, (const float*)jr);
        } else {
          dg_status_t rc = shell_jvp_radial(m, t, u, v, (double*)jr, s);
          if (rc != DG_OK) return rc;
          k_line_scatter<double><<<blocks, 256, 0, s>>>(L, pc, pcz, kap, dta, (const double*)jr);
        }
      }
  const unsigned lines = (unsigned)(m->n_elem / m->n_rad * L.N2);
  switch (m->p) {
    case 2: k_line_factor<15><<<lines, 64, 0, s>>>(L); break;
    case 3: k_line_factor<20><<<lines, 64, 0, s>>>(L); break;
    default: k_line_factor<25><<<lines, 64, 0, s>>>(L); break;
  }
  if (f32) {
    const unsigned g = 4096;
    k_to_float<<<g, 256, 0, s>>>(nblk, Lo, Lo32);
    k_to_float<<<g, 256, 0, s>>>(nblk, Di, Di32);
    k_to_float<<<g, 256, 0, s>>>(nblk, Up, Up32);
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

template <class T, class F>
static dg_status_t line_pc_apply_t(dg_mesh_s* m, const F* Lo, const F* Di, const F* Up, const T* r, T* z,
                                   hipStream_t s) {
  ProfScope ps(m, 11, s);
  const LineDev L = line_dev(m, nullptr, nullptr, nullptr);
  const int64_t lines = m->n_elem / m->n_rad * L.N2;
  const int lpb = 64 / L.b;
  const unsigned grid = (unsigned)((lines + lpb - 1) / lpb);
  const size_t shm = (size_t)lpb * L.n_rad * L.b * sizeof(double);
  switch (m->p) {
    case 2: k_line_solve<15, T, F><<<grid, 64, shm, s>>>(L, lines, Lo, Di, Up, r, z); break;
    case 3: k_line_solve<20, T, F><<<grid, 64, shm, s>>>(L, lines, Lo, Di, Up, r, z); break;
    default: k_line_solve<25, T, F><<<grid, 64, shm, s>>>(L, lines, Lo, Di, Up, r, z); break;
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

dg_status_t line_pc_apply(dg_mesh_s* m, const double* Lo, const double* Di, const double* Up, const double* r,
                          double* z, hipStream_t s) {
  return line_pc_apply_t<double, double>(m, Lo, Di, Up, r, z, s);
}
dg_status_t line_pc_apply(dg_mesh_s* m, const float* Lo, const float* Di, const float* Up, const float* r, float* z,
                          hipStream_t s) {
  return line_pc_apply_t<float, float>(m, Lo, Di, Up, r, z, s);
}

}  // namespace dg
