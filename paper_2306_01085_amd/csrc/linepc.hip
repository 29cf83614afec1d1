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
//  * apply: forward and back substitution, several lines per wavefront, from a packed
//    row-major copy of the factors in a selectable storage precision (double, float,
//    bf16) that the lanes (one row each) read with wide loads.
// The blocks of the build are column-major (entry (r, c) at c b + r): the probes fill
// columns with consecutive writes.
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
template <class V>
__global__ void k_line_probe(int64_t n_dof, int N, int N2, int n, int n_rad, int pc, int pcz, int kap,
                             V* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_dof) return;
  const int j = (int)(i % N);
  const int64_t ec = i / N;
  const int c = (int)(ec % 5);
  const int64_t e = ec / 5;
  const int k = (int)(e % n_rad);
  v[i] = (c == pc && j / N2 == pcz && k % 3 == kap) ? (V)1 : (V)0;
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

// Packed factors for the substitution, one array of the storage type F (double, float or
// bf16 bits): per line and layer k the three matrices L_k, Dinv_k, W_k, each row-major
// with the row stride RS = b rounded up to a multiple of 4 (zero padding), so that a
// lane reads its whole row with 16- or 8-byte loads.
__host__ __device__ constexpr int line_rs(int b) { return (b + 3) & ~3; }


template <class F> __device__ inline F line_st(double v);
template <> __device__ inline double line_st<double>(double v) { return v; }
template <> __device__ inline float line_st<float>(double v) { return (float)v; }
template <> __device__ inline unsigned short line_st<unsigned short>(double v) {
  // bf16 by round to nearest even of the float value
  const unsigned u = __float_as_uint((float)v);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// P <- the packed copy of (Lo, Di, Up): one thread per packed entry
template <class F>
__global__ void k_line_pack(LineDev L, int64_t n_lines, F* __restrict__ P) {
  const int RS = line_rs(L.b), MS = L.b * RS;
  const int64_t total = n_lines * L.n_rad * 3 * (int64_t)MS;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(t % RS);
    const int r = (int)((t / RS) % L.b);
    const int64_t lkm = t / MS;
    const int mat = (int)(lkm % 3);
    const int64_t lk = lkm / 3;
    double v = 0;
    if (q < L.b) {
      const double* src = mat == 0 ? L.Lo : (mat == 1 ? L.Di : L.Up);
      v = src[lk * L.bb + (int64_t)q * L.b + r];
    }
    P[t] = line_st<F>(v);
  }
}

// A row of a packed matrix held as the 32-bit words it was loaded as (RS entries of F,
// RS * sizeof(F) a multiple of 8, src aligned to it); entries are widened where they are used
// (line_at). BF16 rows take two entries per register, as the compiler already kept them.
template <int RS, class F>
struct LineRow {
  static constexpr int W = RS * (int)sizeof(F) / 4;
  uint32_t w[W];
};
template <int RS, class F>
__device__ inline void line_row(LineRow<RS, F>& dst, const F* __restrict__ src) {
  constexpr int bytes = RS * (int)sizeof(F);
  if constexpr (bytes % 16 == 0) {
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
#pragma unroll
    for (int i = 0; i < bytes / 16; ++i) {
      const uint4 v = s4[i];
      dst.w[4 * i] = v.x;
      dst.w[4 * i + 1] = v.y;
      dst.w[4 * i + 2] = v.z;
      dst.w[4 * i + 3] = v.w;
    }
  } else {
    static_assert(bytes % 8 == 0, "row size");
    const uint2* s2 = reinterpret_cast<const uint2*>(src);
#pragma unroll
    for (int i = 0; i < bytes / 8; ++i) {
      const uint2 v = s2[i];
      dst.w[2 * i] = v.x;
      dst.w[2 * i + 1] = v.y;
    }
  }
}
// entry q of a row, widened (bf16 -> float exactly, float and double as they are)
template <int RS>
__device__ inline float line_at(const LineRow<RS, unsigned short>& r, int q) {
  const uint32_t w = r.w[q >> 1];
  return __uint_as_float((q & 1) ? (w & 0xffff0000u) : (w << 16));
}
template <int RS>
__device__ inline float line_at(const LineRow<RS, float>& r, int q) { return __uint_as_float(r.w[q]); }
template <int RS>
__device__ inline double line_at(const LineRow<RS, double>& r, int q) {
  return __hiloint2double((int)r.w[2 * q + 1], (int)r.w[2 * q]);
}

// a loaded value required at this point (an empty instruction that reads and writes the
// register): the load is not sunk past it into the branch that stores the value, so the loads
// before a group of pins are issued together
__device__ inline void line_pin(double& x) { __asm__ __volatile__("" : "+v"(x)); }
__device__ inline void line_pin(float& x) { __asm__ __volatile__("" : "+v"(x)); }

// ordering of LDS accesses among the lanes of one wavefront (LDS operations of a
// wavefront complete in issue order; this only keeps the compiler from moving them)
__device__ inline void line_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// z = M^-1 r for every line. WPB wavefronts per block, 64 / b whole lines per wavefront
// (lane = line slot * b + row), so that the substitution needs no block barrier.
// T: vector (and arithmetic) type, F: storage type of the packed factors. D register rows
// form a ring: the loads of the next D - 1 matrices are in flight while one is applied.
template <int b, int WPB, int D, int LPB, class T, class F>
__global__ __launch_bounds__(64 * WPB) void k_line_solve(LineDev L, int64_t n_lines, const F* __restrict__ P,
                                                         const T* __restrict__ rin, T* __restrict__ z) {
  constexpr int RS = line_rs(b), MS = b * RS;
  constexpr int LPW = 64 / b;
  static_assert(LPB <= LPW * WPB, "lines per block");
  extern __shared__ unsigned char line_smem[];
  T* x = reinterpret_cast<T*>(line_smem);   // [LPB][n_rad][b]
  const int lane = threadIdx.x & 63;
  const int ls = lane / b, r = lane % b;
  const int slot = (threadIdx.x >> 6) * LPW + ls;
  const int64_t line0 = (int64_t)blockIdx.x * LPB;
  const int64_t line = line0 + slot;
  const bool act = ls < LPW && slot < LPB && line < n_lines;
  const int nr = L.n_rad;
  const int nb = nr * b;
  // gather: unknown w = (k, c n + cz) of line slot q <- r[e = cell n_rad + k][c][ab + N2 cz],
  // taken in the order idx = w LPB + q (consecutive lanes read consecutive lines: the same
  // node of consecutive (a, b) columns, adjacent in memory), GK loads per thread issued before
  // any is stored (a load-store loop waits for memory once per round); lanes past the end read
  // the last in-range entry and store nothing
  constexpr int n = b / 5, N2 = n * n, N = N2 * n, GK = 8, NT = 64 * WPB;
  const int tot = LPB * nb;
  auto rin_index = [&](int idx) -> int64_t {
    const int q = idx % LPB, w = idx / LPB;
    const int64_t ln = min(line0 + q, n_lines - 1);
    const int k = w / b, rr = w % b, c = rr / n, cz = rr % n;
    const int64_t e = (ln / N2) * nr + k;
    return (e * 5 + c) * N + (ln % N2) + N2 * cz;
  };
  for (int i0 = threadIdx.x; i0 < tot; i0 += GK * NT) {
    T g[GK];
#pragma unroll
    for (int u = 0; u < GK; ++u) g[u] = rin[rin_index(min(i0 + u * NT, tot - 1))];
#pragma unroll
    for (int u = 0; u < GK; ++u) line_pin(g[u]);
#pragma unroll
    for (int u = 0; u < GK; ++u) {
      const int idx = i0 + u * NT;
      if (idx < tot) x[(idx % LPB) * nb + idx / LPB] = g[u];
    }
  }
  __syncthreads();
  T* xl = x + (act ? slot : 0) * nb;
  // The substitution is a stream of nm = 3 nr - 2 matrix applications:
  //   j = 2k (k < nr):          x_k <- Dinv_k x_k
  //   j = 2k - 1 (0 < k < nr):  x_k <- x_k - L_k x_{k-1}
  //   j = 2 nr - 1 + i:         x_k <- x_k - W_k x_{k+1},  k = nr - 2 - i
  // Row r of the matrix of step j sits at Pl + (layer * 3 + mat) * MS.
  const F* Pl = P + (act ? line : 0) * (int64_t)nr * 3 * MS + r * RS;
  const int nm = 3 * nr - 2;
  auto row_of = [&](int j) -> const F* {
    j = min(j, nm - 1);   // loads past the end re-read the last matrix
    if (j < 2 * nr - 1) return Pl + ((int64_t)((j + 1) / 2) * 3 + ((j & 1) ? 0 : 1)) * MS;
    return Pl + ((int64_t)(nr - 2 - (j - (2 * nr - 1))) * 3 + 2) * MS;
  };
  auto step = [&](int j, const LineRow<RS, F>& R) {
    if (j < 2 * nr - 1 && !(j & 1)) {
      T* xk = xl + (j / 2) * b;
      T sum = 0;
#pragma unroll
      for (int q = 0; q < b; ++q) sum += (T)line_at(R, q) * xk[q];
      line_wave_sync();
      if (act) xk[r] = sum;
    } else {
      const int k = j < 2 * nr - 1 ? (j + 1) / 2 : nr - 2 - (j - (2 * nr - 1));
      const T* xo = xl + (j < 2 * nr - 1 ? k - 1 : k + 1) * b;
      T sum = 0;
#pragma unroll
      for (int q = 0; q < b; ++q) sum += (T)line_at(R, q) * xo[q];
      if (act) xl[k * b + r] -= sum;
    }
    line_wave_sync();
  };
  // loads are issued on every lane and every pass (idle lanes read line 0) so that the
  // wait for one row never covers the younger ones
  LineRow<RS, F> R[D];
#pragma unroll
  for (int d = 0; d < D; ++d) line_row<RS>(R[d], row_of(d));
  for (int j = 0; j < nm; j += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (j + d < nm) step(j + d, R[d]);
      line_row<RS>(R[d], row_of(j + d + D));
    }
  }
  __syncthreads();
  // scatter, in the gather's order
  for (int idx = threadIdx.x; idx < tot; idx += NT)
    if (line0 + idx % LPB < n_lines) z[rin_index(idx)] = x[(idx % LPB) * nb + idx / LPB];
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

int64_t line_pc_packed(const dg_mesh_s* m) {
  const int64_t n = m->p + 1, b = 5 * n;
  const int64_t lines = (m->n_elem / m->n_rad) * n * n;
  return lines * m->n_rad * 3 * b * line_rs((int)b);
}

// build and factor at (t, u) for the stage matrix I - dta J, then pack the factors into P
// with storage precision prec (64 double, 32 float, 16 bf16); v, jr: scratch [n_dof]
// (jr: double, or float when f32 is set). With f32 the probes use the FP32 dual-number
// linearisation.
dg_status_t line_pc_build(dg_mesh_s* m, double t, const double* u, double dta, double* Lo, double* Di, double* Up,
                          double* v, void* jr, bool f32, int prec, void* P, hipStream_t s) {
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
        if (f32) {
          float* vf = (float*)jr + nd;
          k_line_probe<float><<<blocks, 256, 0, s>>>(nd, L.N, L.N2, L.n, L.n_rad, pc, pcz, kap, vf);
          dg_status_t rc = shell_jvp_radial32(m, t, u, vf, (float*)jr, s);
          if (rc != DG_OK) return rc;
          k_line_scatter<float><<<blocks, 256, 0, s>>>(L, pc, pcz, kap, dta, (const float*)jr);
        } else {
          k_line_probe<double><<<blocks, 256, 0, s>>>(nd, L.N, L.N2, L.n, L.n_rad, pc, pcz, kap, v);
          dg_status_t rc = shell_jvp_radial(m, t, u, v, (double*)jr, s);
          if (rc != DG_OK) return rc;
          k_line_scatter<double><<<blocks, 256, 0, s>>>(L, pc, pcz, kap, dta, (const double*)jr);
        }
      }
  const int64_t n_lines = m->n_elem / m->n_rad * L.N2;
  switch (m->p) {
    case 2: k_line_factor<15><<<(unsigned)n_lines, 64, 0, s>>>(L); break;
    case 3: k_line_factor<20><<<(unsigned)n_lines, 64, 0, s>>>(L); break;
    default: k_line_factor<25><<<(unsigned)n_lines, 64, 0, s>>>(L); break;
  }
  const unsigned g = 8192;
  if (prec == 64) k_line_pack<double><<<g, 256, 0, s>>>(L, n_lines, (double*)P);
  else if (prec == 32) k_line_pack<float><<<g, 256, 0, s>>>(L, n_lines, (float*)P);
  else k_line_pack<unsigned short><<<g, 256, 0, s>>>(L, n_lines, (unsigned short*)P);
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

constexpr size_t LINE_MAX_LDS = 65536;   // dynamic LDS of one block of the substitution

template <int b, int WPB, int D, int LPB, class T>
static void line_solve_launch(const LineDev& L, int64_t lines, int prec, const void* P, const T* r, T* z,
                              hipStream_t s) {
  const size_t shm = (size_t)LPB * L.n_rad * b * sizeof(T);
  if (shm > LINE_MAX_LDS) {
    // tall lines: one wavefront's lines per block (line_pc_apply checks that these fit)
    if constexpr (WPB > 1) line_solve_launch<b, 1, 2, 64 / b, T>(L, lines, prec, P, r, z, s);
    return;
  }
  const unsigned grid = (unsigned)((lines + LPB - 1) / LPB);
  const unsigned th = 64 * WPB;
  if (prec == 64)
    k_line_solve<b, WPB, D, LPB, T, double><<<grid, th, shm, s>>>(L, lines, (const double*)P, r, z);
  else if (prec == 32)
    k_line_solve<b, WPB, D, LPB, T, float><<<grid, th, shm, s>>>(L, lines, (const float*)P, r, z);
  else
    k_line_solve<b, WPB, D, LPB, T, unsigned short><<<grid, th, shm, s>>>(L, lines, (const unsigned short*)P, r, z);
}

// launch configurations of the substitution (the "line_solve_config" option):
// 0: 1 wavefront per block, 2-deep ring; 1: 4 wavefronts, 2-deep; 2: 1 wavefront, 4-deep;
// 3: 4 wavefronts, 4-deep; 4 / 5: the (p + 1)^2 lines of one angular cell per block (its
// vector entries are whole cache lines), 4-deep / 2-deep (at p = 4, whose cell would take
// 13 wavefronts, the same as 3 / 1). Eight-deep rings measured the same as four-deep ones
// (within 1% at p = 3 and p = 4): the substitution streams its factors near the HBM rate.
template <int b, class T>
static void line_solve_cfg(int cfg, const LineDev& L, int64_t lines, int prec, const void* P, const T* r, T* z,
                           hipStream_t s) {
  constexpr int LPW = 64 / b, n = b / 5, N2 = n * n;
  constexpr int WC = (N2 + LPW - 1) / LPW;   // wavefronts for one cell's lines
  switch (cfg) {
    case 1: line_solve_launch<b, 4, 2, 4 * LPW, T>(L, lines, prec, P, r, z, s); break;
    case 2: line_solve_launch<b, 1, 4, LPW, T>(L, lines, prec, P, r, z, s); break;
    case 3: line_solve_launch<b, 4, 4, 4 * LPW, T>(L, lines, prec, P, r, z, s); break;
    case 4:
      if constexpr (WC <= 8) line_solve_launch<b, WC, 4, N2, T>(L, lines, prec, P, r, z, s);
      else line_solve_launch<b, 4, 4, 4 * LPW, T>(L, lines, prec, P, r, z, s);
      break;
    case 5:
      if constexpr (WC <= 8) line_solve_launch<b, WC, 2, N2, T>(L, lines, prec, P, r, z, s);
      else line_solve_launch<b, 4, 2, 4 * LPW, T>(L, lines, prec, P, r, z, s);
      break;
    default: line_solve_launch<b, 1, 2, LPW, T>(L, lines, prec, P, r, z, s); break;
  }
}

template <class T>
static dg_status_t line_pc_apply_t(dg_mesh_s* m, int prec, const void* P, const T* r, T* z, hipStream_t s) {
  ProfScope ps(m, 11, s);
  const LineDev L = line_dev(m, nullptr, nullptr, nullptr);
  const int64_t lines = m->n_elem / m->n_rad * L.N2;
  if ((size_t)(64 / L.b) * L.n_rad * L.b * sizeof(T) > LINE_MAX_LDS) {
    set_error("radial-line preconditioner: too many radial layers for the substitution's LDS");
    return DG_ERR_ARG;
  }
  // automatic choice (implicit steps on the 7.9M-DOF p = 3 shell at the sustained clock): cell
  // blocks with a 2-deep ring for double vectors, 4 wavefronts with a 4-deep ring for float
  const int cfg = m->tune_lsolve >= 0 ? m->tune_lsolve : (sizeof(T) == 8 ? 5 : 3);
  switch (m->p) {
    case 2: line_solve_cfg<15, T>(cfg, L, lines, prec, P, r, z, s); break;
    case 3: line_solve_cfg<20, T>(cfg, L, lines, prec, P, r, z, s); break;
    default: line_solve_cfg<25, T>(cfg, L, lines, prec, P, r, z, s); break;
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

dg_status_t line_pc_apply(dg_mesh_s* m, int prec, const void* P, const double* r, double* z, hipStream_t s) {
  return line_pc_apply_t<double>(m, prec, P, r, z, s);
}
dg_status_t line_pc_apply(dg_mesh_s* m, int prec, const void* P, const float* r, float* z, hipStream_t s) {
  return line_pc_apply_t<float>(m, prec, P, r, z, s);
}

}  // namespace dg
