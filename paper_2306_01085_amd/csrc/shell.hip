// Residual R(u) and J(u)v on the cubed-sphere shell.
//
// The LDG weak form eq. (DGformulation) with GLL collocation is evaluated in its
// algebraically identical strong form (summation by parts of the GLL rule):
//   q  = (1/J) sum_a D_a(J a^a u) + sum_faces Sn (u_hat - u) / (w_end J)
//   R  = -(1/J) sum_a D_a(J a^a . F(u, q)) + s(u, q) + sum_faces ((F - F_hat).Sn) / (w_end J)
// with Sn = side * J a^a the scaled outward normal of a face node and the traces of
// eq. (LDG2): u_hat = (u + u^-)/2, F_hat.n = (F + F^-).n/2 + sigma(u_hat)(u - u_hat).
//
// Two kernels per evaluation:
//  pass 1 (one element per 32/64/128 threads, one thread per node): loads the
//    element's state and the neighbours' face values, computes q in registers
//    (never stored), the pointwise flux and source, the contravariant fluxes in
//    LDS, the volume divergence, the own half of every interior face term and the
//    complete boundary-face terms; writes the partial R.
//    The interior-face stabilisation -|Sn| sigma(u_hat)(u - u_hat) is done here too
//    (pass 1 already holds u^- for the gradient), and every F(u, q).Sn is written
//    into the neighbour's incoming slot for the matching face node.
//  pass 2 (same layout): adds half of the incoming traces, a coalesced stream.
// With S = Dual<T> the same code yields J(u)v (the derivative part), exactly.
#include <type_traits>

#include "internal.h"
#include "shell_pass1.h"
#include "mfma_bf16.h"

namespace dg {

// pass 2: R += (F^-.(-Sn))/(2 w_end J) on every interior face node, reading the
// traces that the neighbours' pass 1 wrote into this element's incoming slots. The
// element's 6 x 5 x (p+1)^2 slots are one contiguous block: its lanes copy it into LDS with
// coalesced 8-byte loads (each slot read once), then every face node sums the slots of the
// faces it lies on (the faces in order, those it is not on adding zero as before) and
// updates its R. Slots of boundary faces are never written and may hold any bits: they
// are copied but never added.
template <int P, class OT>
__global__ __launch_bounds__(256) void shell_pass2(ShellDev M, GllC gc, const OT* __restrict__ Fin,
                                                   OT* __restrict__ R) {
  typedef Shape<P> Sh;
  constexpr int n = Sh::n, N = Sh::N, N2 = Sh::N2, TPE = Sh::TPE, EPB = Sh::EPB;
  constexpr int L = 30 * N2;                                    // trace slots of one element
  constexpr int W = L * (int)sizeof(OT) / 8;                    // as 8-byte words
  static_assert((L * sizeof(OT)) % 8 == 0, "trace block must be whole 8-byte words");
  constexpr bool kWide = (W % 2) == 0;                          // the block is whole 16-byte words
  // (each element's block padded to whole rounds of TPE copies: every lane stores each round)
  constexpr int WP = kWide ? 2 * TPE * ((W / 2 + TPE - 1) / TPE) : TPE * ((W + TPE - 1) / TPE);
  __shared__ __align__(16) uint64_t s_tw[EPB][WP];
  const int le = threadIdx.x / TPE;
  const int j = threadIdx.x % TPE;
  const int e = xcd_block_reversed(blockIdx.x, gridDim.x) * EPB + le;
  const bool live = e < M.E;
  const int a = j % n, b = (j / n) % n, cz = j / N2;
  const int k = live ? e % M.n_rad : 0;
  const bool on[6] = {a == 0, a == n - 1, b == 0, b == n - 1, cz == 0 && k > 0, cz == n - 1 && k < M.n_rad - 1};
  const bool upd = live && j < N && (on[0] || on[1] || on[2] || on[3] || on[4] || on[5]);
  // Every load of the pass is issued in one branch-free stretch, before any is used, so that a
  // wavefront waits for memory once: the lanes without work (past the last element, past the
  // element's nodes, interior nodes) read in-range addresses of element min(e, E - 1) and node
  // min(j, N - 1) and store nothing.
  const int ec = live ? e : M.E - 1;
  const int jc = j < N ? j : N - 1;
  const int64_t base = (int64_t)ec * 5 * N;
  OT r[5];
  for (int c = 0; c < 5; ++c) r[c] = R[base + c * N + jc];
  const int ja = (jc % n) + n * ((jc / n) % n);
  const int kc = ec % M.n_rad;
  const double jang = M.ang[((int64_t)(ec / M.n_rad) * 13 + 9) * N2 + ja];
  const double e0 = M.edges[kc], e1 = M.edges[kc + 1];
  double xz = gc.x[0];   // the node's GLL point
  for (int q = 1; q < n; ++q) xz = (cz == q) ? gc.x[q] : xz;
  // the element's incoming trace block (it starts at e * L * sizeof(OT) bytes, a multiple of 8,
  // of 16 where the block is made of 16-byte words), copied to LDS
  if constexpr (kWide) {
    constexpr int NW = W / 2, NI = (NW + TPE - 1) / TPE;
    const uint4* src = reinterpret_cast<const uint4*>(Fin + (int64_t)ec * L);
    uint4* dst = reinterpret_cast<uint4*>(&s_tw[le][0]);
    uint4 tw[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) tw[i] = src[min(j + i * TPE, NW - 1)];
#pragma unroll
    for (int i = 0; i < NI; ++i) dst[j + i * TPE] = tw[i];
  } else {
    constexpr int NI = (W + TPE - 1) / TPE;
    const uint64_t* src = reinterpret_cast<const uint64_t*>(Fin + (int64_t)ec * L);
    uint64_t tw[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) tw[i] = src[min(j + i * TPE, W - 1)];
#pragma unroll
    for (int i = 0; i < NI; ++i) s_tw[le][j + i * TPE] = tw[i];
  }
  // (the compiler turns the GLL point's selection into a load from the argument block and
  // would sink it past the barrier, into the updating lanes' branch: its value is required here)
  __asm__ __volatile__("" : "+v"(xz));
  lds_barrier();
  if (!upd) return;
  const OT* Fe = reinterpret_cast<const OT*>(&s_tw[le][0]);
  const double hk = e1 - e0;
  const double rc = e0 + 0.5 * (xz + 1.0) * hk;
  const double Jac = rc * rc * (0.5 * hk) * jang;
  const OT hl = OT(0.5 / (gc.w[0] * Jac));
  OT acc[5] = {OT(0), OT(0), OT(0), OT(0), OT(0)};
  for (int f = 0; f < 6; ++f) {
    if (!on[f]) continue;
    const int m = face_slot<P>(f, a, b, cz);
    for (int c = 0; c < 5; ++c) acc[c] += Fe[(f * 5 + c) * N2 + m];
  }
  for (int c = 0; c < 5; ++c) R[base + c * N + j] = r[c] + hl * acc[c];
}


template <class S, class SU, class TV, class OT>
static dg_status_t launch(dg_mesh_s* m, double t, const SU* u, const TV* v, OT* out, OT* fn, hipStream_t s,
                          int prof_base) {
  ShellDev M = m->shell();
  const int E = M.E;
  if ((int64_t)E * 30 * (m->p + 1) * (m->p + 1) >= INT32_MAX) {
    set_error("shell mesh too large for 32-bit trace-slot indices");
    return DG_ERR_UNSUPPORTED;
  }
  const GllC gc = make_gllc(m->p);
  PhysC ph = m->phys;
  sun_direction(ph, t);
#define DG_LAUNCH(P_)                                                                                     \
  {                                                                                                        \
    {                                                                                                      \
      if constexpr (std::is_same<S, double>::value)                                                        \
        shell_pass1_f64(m, M, ph, gc, t, u, out, fn, s, prof_base);                                         \
      else                                                                                                 \
        dispatch_p1<P_, S>(m, M, ph, gc, t, u, v, out, fn, s, prof_base);                                  \
    }                                                                                                      \
    {                                                                                                      \
      const int blocks = (E + Shape<P_>::EPB - 1) / Shape<P_>::EPB;                                        \
      if (m->prof)                                                                                         \
        launch_timed(m, prof_base + 1, &shell_pass2<P_, OT>, dim3(blocks), dim3(256), s, M, gc, fn, out);   \
      else                                                                                                 \
        shell_pass2<P_, OT><<<blocks, 256, 0, s>>>(M, gc, fn, out);                                       \
    }                                                                                                      \
  }
  switch (m->p) {
    case 2: DG_LAUNCH(2); break;
    case 3: DG_LAUNCH(3); break;
    case 4: DG_LAUNCH(4); break;
    default: set_error("unsupported degree"); return DG_ERR_ARG;
  }
#undef DG_LAUNCH
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

// J_rad(u) v: the radial-line linearisation (RAD above), FP64
dg_status_t shell_jvp_radial(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s) {
  ShellDev M = m->shell();
  const GllC gc = make_gllc(m->p);
  PhysC ph = m->phys;
  sun_direction(ph, t);
  const int E = M.E;
#define DG_RAD(P_)                                                                                          \
  if (ph.xp_mode())                                                                                        \
    shell_pass1<P_, 1, 1, Dual<double>, double, double, double, true, kXpEuv | kXpComp><<<E, Shape<P_>::TPE, 0, s>>>(       \
        M, ph, gc, t, u, v, jv, m->d_fn64);                                                                \
  else                                                                                                     \
    shell_pass1<P_, 1, 2, Dual<double>, double, double, double, true><<<E, Shape<P_>::TPE, 0, s>>>(M, ph, gc, t, u, \
                                                                                                 v, jv, m->d_fn64); \
  shell_pass2<P_, double><<<(E + Shape<P_>::EPB - 1) / Shape<P_>::EPB, 256, 0, s>>>(M, gc, m->d_fn64, jv);
  switch (m->p) {
    case 2: DG_RAD(2); break;
    case 3: DG_RAD(3); break;
    default: DG_RAD(4); break;
  }
#undef DG_RAD
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

// the same radial-line linearisation with FP32 dual numbers (preconditioner of FP32 runs)
dg_status_t shell_jvp_radial32(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s) {
  ShellDev M = m->shell();
  const GllC gc = make_gllc(m->p);
  PhysC ph = m->phys;
  sun_direction(ph, t);
  const int E = M.E;
#define DG_RAD32(P_)                                                                                        \
  if (ph.xp_mode())                                                                                        \
    shell_pass1<P_, 1, 1, Dual<float>, double, float, float, true, kXpEuv | kXpComp><<<E, Shape<P_>::TPE, 0, s>>>(           \
        M, ph, gc, t, u, v, jv, m->d_fn32);                                                                \
  else                                                                                                     \
    shell_pass1<P_, 1, 1, Dual<float>, double, float, float, true><<<E, Shape<P_>::TPE, 0, s>>>(M, ph, gc, t, u, v, \
                                                                                              jv, m->d_fn32); \
  shell_pass2<P_, float><<<(E + Shape<P_>::EPB - 1) / Shape<P_>::EPB, 256, 0, s>>>(M, gc, m->d_fn32, jv);
  switch (m->p) {
    case 2: DG_RAD32(2); break;
    case 3: DG_RAD32(3); break;
    default: DG_RAD32(4); break;
  }
#undef DG_RAD32
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

dg_status_t shell_residual(dg_mesh_s* m, double t, const double* u, double* r, hipStream_t s) {
  return launch<double, double, double, double>(m, t, u, (const double*)nullptr, r, m->d_fn64, s, 0);
}
dg_status_t shell_residual_traces(dg_mesh_s* m, double t, const double* u, double* r, double* fn, hipStream_t s) {
  return launch<double, double, double, double>(m, t, u, (const double*)nullptr, r, fn, s, 0);
}
dg_status_t shell_jvp64(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s) {
  return launch<Dual<double>, double, double, double>(m, t, u, v, jv, m->d_fn64, s, 2);
}
dg_status_t shell_jvp32(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s) {
  return launch<Dual<float>, double, float, float>(m, t, u, v, jv, m->d_fn32, s, 4);
}

// ================================================================ BF16-MFMA J(u)v
// J(u)v with the tangent's tensor-product contractions on bf16 MFMA, FP32 accumulation:
// the gradient of the tangent, sum_a D_a(J a^a v), and the divergence of the linearised
// contravariant flux, sum_a D_a dG^a, are products of the dense reference operators
// D1 = D x I x I, D2 = I x D x I, D3 = I x I x D (64 x 64 at p = 3, bf16 in global
// memory) with the tangent-derived operands rounded to bf16 in LDS. The state's gradient,
// the pointwise linearisation (FP32 dual numbers) and the face terms are those of the
// FP32 J v. Degrees 3 and 4, two elements per block; the node dimension is padded to
// NP = the element's thread count (64 at p = 3, 128 at p = 4 with 125 nodes), so that
// each wavefront computes one 32-node row tile of both elements' columns.
constexpr int BF_EPB = 2;
template <int P> struct BfShape {
  static constexpr int NP = Shape<P>::TPE;                       // padded node count
  static constexpr int THREADS = BF_EPB * Shape<P>::TPE;
  // operand space: gradient B1 [32][2NP] and B3 [32][NP] (bf16), outputs C1 [NP][30] and
  // C3 [NP][10] (f32); the divergence's Bd [32][3NP] (bf16) and Cd [NP][10] reuse it
  static constexpr int MM_BYTES = 32 * 2 * NP * 2 + 32 * NP * 2 + NP * 30 * 4 + NP * 10 * 4;
};

// XP: kXpEuv, or kXpEuv | kXpComp for a mesh with the variable composition
template <int P, int XP>
__global__ __launch_bounds__(BfShape<P>::THREADS) void shell_pass1_bf16(ShellDev M, PhysC ph, GllC gc, double t,
                                                                       const double* __restrict__ u,
                                                                       const float* __restrict__ v,
                                                                       const uint16_t* __restrict__ ops,
                                                                       float* __restrict__ R, float* __restrict__ Fn) {
  typedef Dual<float> S;
  typedef float T;
  constexpr int n = Shape<P>::n, N = Shape<P>::N, N2 = Shape<P>::N2, TPE = Shape<P>::TPE, EPB = BF_EPB;
  constexpr int NP = BfShape<P>::NP, BF_MM_BYTES = BfShape<P>::MM_BYTES;
  __shared__ double s_ang[EPB][13][N2];
  __shared__ S s_u[EPB][5][N];
  __shared__ S s_f[EPB][6][5][N2];
  __shared__ S s_z[EPB][5][5][N2];
  __shared__ int s_nb[EPB][6][N2];
  __shared__ double D[n * n];
  __shared__ __align__(16) unsigned char s_mm[BF_MM_BYTES];
  uint16_t* B1 = (uint16_t*)s_mm;
  uint16_t* B3 = B1 + 32 * 2 * NP;
  float* C1 = (float*)(B3 + 32 * NP);
  float* C3 = C1 + NP * 30;
  uint16_t* Bd = (uint16_t*)s_mm;
  float* Cd = (float*)(Bd + 32 * 3 * NP);
  const uint16_t* opG1 = ops;                      // [NP][2NP] = [D1 | D2]
  const uint16_t* opG3 = ops + NP * 2 * NP;        // [NP][NP]  = D3
  const uint16_t* opDv = opG3 + NP * NP;           // [NP][3NP] = [D1 D2 D3]
  const int wave = threadIdx.x >> 6;
  const int le = threadIdx.x / TPE;
  const int j = threadIdx.x % TPE;
  const int e = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
  const bool live = e < M.E;
  const bool active = live && j < N;
  const int cell = live ? e / M.n_rad : 0;
  const int k = live ? e % M.n_rad : 0;
  if (threadIdx.x < n * n) D[threadIdx.x] = gc.D[threadIdx.x];
  const double w_end = gc.w[0];
  if (live)
    for (int idx = j; idx < 13 * N2; idx += TPE) s_ang[le][idx / N2][idx % N2] = M.ang[(int64_t)cell * 13 * N2 + idx];
  S uu[5];
  const int64_t base = (int64_t)e * 5 * N;
  if (active)
    for (int c = 0; c < 5; ++c) {
      uu[c] = load_state<S>(u, v, base + c * N + j);
      s_u[le][c][j] = uu[c];
    }
  const double rk = live ? M.edges[k] : 0.0;
  const double hk = live ? M.edges[k + 1] - rk : 1.0;
  int own = 0;
  if (live) {
    for (int f = 0; f < 4; ++f)
      if (M.cnbr[cell * 4 + f] * M.n_rad + k > e) own |= 1 << f;
    if (k < M.n_rad - 1) own |= 1 << 5;
  }
  const int n_own = __popc(own);
  __syncthreads();

  // ---- face-node tasks (owned faces first): u_hat - u, neighbour slots, Z
  if (live)
    for (int tsk = j; tsk < 6 * N2; tsk += TPE) {
      const int r = tsk / N2, m = tsk % N2;
      const int f = (r < n_own) ? nth_bit(own, r) : nth_bit(~own & 63, r - n_own);
      int fa, fb, fcz;
      slot_node<P>(f, m, fa, fb, fcz);
      const int jo = fa + n * fb + N2 * fcz;
      S uo[5], du[5];
      for (int c = 0; c < 5; ++c) uo[c] = s_u[le][c][jo];
      int jn, fn, mn;
      const int en = face_neighbour<P>(M, cell, k, f, fa, fb, fcz, jn, fn, mn);
      if (en >= 0) {
        for (int c = 0; c < 5; ++c) du[c] = T(0.5) * (load_state<S>(u, v, (int64_t)en * 5 * N + c * N + jn) - uo[c]);
        s_nb[le][f][m] = (en * 6 + fn) * 5 * N2 + mn;
        if (r < n_own) {
          const int dd = f >> 1;
          const int ja = fa + n * fb;
          const double rc = rk + 0.5 * (gc.x[fcz] + 1.0) * hk;
          const double fac = (dd < 2) ? rc * 0.5 * hk : rc * rc;
          const double A0 = s_ang[le][3 * dd][ja], A1 = s_ang[le][3 * dd + 1][ja], A2 = s_ang[le][3 * dd + 2][ja];
          const double Smag = fac * sqrt(A0 * A0 + A1 * A1 + A2 * A2);
          S uh[5];
          for (int c = 0; c < 5; ++c) uh[c] = uo[c] + du[c];
          S sm, se;
          sigma<3, S, XP & kXpComp>(ph, uh, sm, se, rc);
          for (int c = 0; c < 5; ++c) {
            const S sg = (c == 0) ? S(T(ph.lam)) : (c == 4 ? se : sm);
            s_z[le][r][c][m] = T(Smag) * sg * du[c];
          }
        }
      } else if (ph.bc_mode == 1 || f == 4) {
        S ub[5];
        boundary_state<3, S>(ph, uo, ub);
        for (int c = 0; c < 5; ++c) du[c] = ub[c] - uo[c];
      } else {
        for (int c = 0; c < 5; ++c) du[c] = S(T(0));
      }
      for (int c = 0; c < 5; ++c) s_f[le][f][c][m] = du[c];
    }
  // tangent operands of the gradient products: B1[col][k] = A1_d(k) v(k) (k < NP) and
  // A2_d(k - NP) v(k - NP); B3[col][k] = r_k^2 v(k); col = d * 10 + field * 2 + element.
  // The padding nodes N <= k < NP get zeros (the operators' padding columns are zero, and
  // stale LDS could hold non-finite bits).
  const int a = j % n, b = (j / n) % n, cz = j / N2;
  if (active) {
    const int ja = a + n * b;
    const double rj = rk + 0.5 * (gc.x[cz] + 1.0) * hk;
    for (int c = 0; c < 5; ++c) {
      const float vd = s_u[le][c][j].d;
      for (int d = 0; d < 3; ++d) {
        B1[(d * 10 + c * 2 + le) * 2 * NP + j] = f2bf((float)s_ang[le][d][ja] * vd);
        B1[(d * 10 + c * 2 + le) * 2 * NP + NP + j] = f2bf((float)s_ang[le][3 + d][ja] * vd);
      }
      B3[(c * 2 + le) * NP + j] = f2bf((float)(rj * rj) * vd);
    }
  } else if (j >= N) {
    for (int c = 0; c < 5; ++c) {
      for (int d = 0; d < 3; ++d) {
        B1[(d * 10 + c * 2 + le) * 2 * NP + j] = 0;
        B1[(d * 10 + c * 2 + le) * 2 * NP + NP + j] = 0;
      }
      B3[(c * 2 + le) * NP + j] = 0;
    }
  }
  __syncthreads();
  {
    v16f acc1, acc3;
    for (int i = 0; i < 16; ++i) acc1[i] = acc3[i] = 0.f;
    mfma_tile_lds_global(acc1, opG1 + 32 * wave * 2 * NP, 2 * NP, B1, 2 * NP, 2 * NP);
    mfma_tile_lds_global(acc3, opG3 + 32 * wave * NP, NP, B3, NP, NP);
    const int col = threadIdx.x & 31;
    for (int a2 = 0; a2 < 16; ++a2) {
      const int row = 32 * wave + mfma_out_row(a2);
      if (col < 30) C1[row * 30 + col] = acc1[a2];
      if (col < 10) C3[row * 10 + col] = acc3[a2];
    }
  }
  __syncthreads();

  // ---- node threads: gradient (state part on the VALU, tangent part from the products),
  // lift, pointwise flux and source, boundary faces, contravariant fluxes
  NodeGeo g;
  S Sr[5], G[5][3];
  if (active) {
    g = node_geo<P>(M, gc, s_ang[le], k, j);
    const double rrp = g.rc * g.rp, rc2 = g.rc * g.rc;
    const double invJ = recip(g.Jac);
    const double lfac = invJ * recip(w_end);
    const double Ja[3][3] = {{rrp * g.A1[0], rrp * g.A1[1], rrp * g.A1[2]},
                             {rrp * g.A2[0], rrp * g.A2[1], rrp * g.A2[2]},
                             {rc2 * g.A3[0], rc2 * g.A3[1], rc2 * g.A3[2]}};
    float c1[n][3], c2[n][3], c3[n];
    for (int i = 0; i < n; ++i) {
      const double ri = rk + 0.5 * (gc.x[i] + 1.0) * hk;
      c3[i] = (float)(D[cz * n + i] * ri * ri);
      for (int d = 0; d < 3; ++d) {
        c1[i][d] = (float)(D[a * n + i] * rrp * s_ang[le][d][i + n * b]);
        c2[i][d] = (float)(D[b * n + i] * rrp * s_ang[le][3 + d][a + n * i]);
      }
    }
    S q[5][3];
    for (int c = 0; c < 5; ++c) {
      float g1[3] = {0.f, 0.f, 0.f}, d3 = 0.f;
      for (int i = 0; i < n; ++i) {
        const float u1 = s_u[le][c][i + n * b + N2 * cz].v;
        const float u2 = s_u[le][c][a + n * i + N2 * cz].v;
        const float u3 = s_u[le][c][g.ja + N2 * i].v;
        for (int d = 0; d < 3; ++d) g1[d] += u1 * c1[i][d] + u2 * c2[i][d];
        d3 += u3 * c3[i];
      }
      const float d3t = C3[j * 10 + c * 2 + le];
      for (int d = 0; d < 3; ++d) {
        const float g1t = (float)rrp * C1[j * 30 + d * 10 + c * 2 + le];
        q[c][d].v = (g1[d] + (float)g.A3[d] * d3) * (float)invJ;
        q[c][d].d = (g1t + (float)g.A3[d] * d3t) * (float)invJ;
      }
    }
    const bool on[6] = {a == 0, a == n - 1, b == 0, b == n - 1, cz == 0, cz == n - 1};
    for (int f = 0; f < 6; ++f) {
      if (!on[f]) continue;
      const int m = face_slot<P>(f, a, b, cz);
      const double sd = ((f & 1) ? 1.0 : -1.0) * lfac;
      const int dd = f >> 1;
      for (int c = 0; c < 5; ++c) {
        const S du = s_f[le][f][c][m];
        for (int d = 0; d < 3; ++d) q[c][d] = q[c][d] + du * T(sd * Ja[dd][d]);
      }
    }
    const bool bot = (k == 0 && cz == 0);
    const bool top = (k == M.n_rad - 1 && cz == n - 1);
    const bool dir = bot || (top && ph.bc_mode == 1);
    const double bside = bot ? -rc2 : rc2;
    S Bc[5];
    if (dir) {
      double Sn[3];
      for (int d = 0; d < 3; ++d) Sn[d] = bside * g.A3[d];
      const double Smag = sqrt(Sn[0] * Sn[0] + Sn[1] * Sn[1] + Sn[2] * Sn[2]);
      S ub[5], Fb[5][3], Sb[5];
      boundary_state<3, S>(ph, uu, ub);
      flux_source<3, S, XP & kXpComp>(ph, ub, q, g.x, 0.0, Fb, Sb, false);
      S sm, se;
      sigma<3, S, XP & kXpComp>(ph, ub, sm, se, g.rc);
      for (int c = 0; c < 5; ++c) {
        const S sg = (c == 0) ? S(T(ph.lam)) : (c == 4 ? se : sm);
        Bc[c] = -(Fb[c][0] * T(Sn[0]) + Fb[c][1] * T(Sn[1]) + Fb[c][2] * T(Sn[2])) - T(Smag) * sg * (uu[c] - ub[c]);
      }
    }
    const double Q = heating<3>(ph, g.x, t);
    S F[5][3];
    flux_source<3, S, XP>(ph, uu, q, g.x, Q, F, Sr);
    __asm__ __volatile__("" ::: "memory");
    const double (*ang)[N2] = s_ang[le];
    if (dir || top) {
      double Sn[3];
      for (int d = 0; d < 3; ++d) Sn[d] = bside * ang[6 + d][g.ja];
      if (dir) {
        for (int c = 0; c < 5; ++c)
          Sr[c] = Sr[c] + (F[c][0] * T(Sn[0]) + F[c][1] * T(Sn[1]) + F[c][2] * T(Sn[2]) + Bc[c]) * T(lfac);
      } else {
        S Fi[5][3];
        flux_inviscid<3, S, XP & kXpComp>(ph, uu, Fi, g.rc);
        const double Smag = sqrt(Sn[0] * Sn[0] + Sn[1] * Sn[1] + Sn[2] * Sn[2]);
        const S Un = (uu[1] * T(Sn[0]) + uu[2] * T(Sn[1]) + uu[3] * T(Sn[2])) * T(ph.lam / Smag);
        for (int c = 0; c < 5; ++c) {
          S fd = (F[c][0] - Fi[c][0]) * T(Sn[0]) + (F[c][1] - Fi[c][1]) * T(Sn[1]) +
                 (F[c][2] - Fi[c][2]) * T(Sn[2]);
          if (c >= 1 && c <= 3) fd = fd - Un * T(Sn[c - 1]);
          Sr[c] = Sr[c] + fd * T(lfac);
        }
      }
    }
    for (int dd = 0; dd < 3; ++dd) {
      const double fac = (dd < 2) ? rrp : rc2;
      const double J0 = fac * ang[3 * dd][g.ja], J1 = fac * ang[3 * dd + 1][g.ja], J2 = fac * ang[3 * dd + 2][g.ja];
      for (int c = 0; c < 5; ++c) G[c][dd] = F[c][0] * T(J0) + F[c][1] * T(J1) + F[c][2] * T(J2);
    }
  }
  __syncthreads();   // every node has read C1 and C3: the operand space takes the divergence
  // divergence operands Bd[col][a * NP + node] = dG^a (col = field * 2 + element), zeros
  // at the padding nodes
  if (active) {
    for (int c = 0; c < 5; ++c)
      for (int dd = 0; dd < 3; ++dd) Bd[(c * 2 + le) * 3 * NP + dd * NP + j] = f2bf(G[c][dd].d);
  } else if (j >= N) {
    for (int c = 0; c < 5; ++c)
      for (int dd = 0; dd < 3; ++dd) Bd[(c * 2 + le) * 3 * NP + dd * NP + j] = 0;
  }
  __syncthreads();
  {
    v16f accd;
    for (int i = 0; i < 16; ++i) accd[i] = 0.f;
    mfma_tile_lds_global(accd, opDv + 32 * wave * 3 * NP, 3 * NP, Bd, 3 * NP, 3 * NP);
    const int col = threadIdx.x & 31;
    for (int a2 = 0; a2 < 16; ++a2) {
      const int row = 32 * wave + mfma_out_row(a2);
      if (col < 10) Cd[row * 10 + col] = accd[a2];
    }
  }
  __syncthreads();

  // ---- node threads: interior-face terms, sent traces, output
  if (active) {
    const double invJ = recip(g.Jac);
    const double lfac = invJ * recip(w_end);
    const bool on[6] = {a == 0, a == n - 1, b == 0, b == n - 1, cz == 0 && k > 0, cz == n - 1 && k < M.n_rad - 1};
    for (int f = 0; f < 6; ++f) {
      if (!on[f]) continue;
      const int m = face_slot<P>(f, a, b, cz);
      const int dd = f >> 1;
      const T side = (f & 1) ? T(1) : T(-1);
      const int nb = s_nb[le][f][m];
      const bool mine = (own >> f) & 1;
      const int r = __popc(own & ((1 << f) - 1));
      for (int c = 0; c < 5; ++c) {
        const S Fs = side * G[c][dd];
        const S z = mine ? s_z[le][r][c][m] : S(T(0));
        Sr[c] = Sr[c] + (T(0.5) * Fs + z) * T(lfac);
        Fn[(int64_t)nb + c * N2] = (Fs - T(2) * z).d;
      }
    }
    for (int c = 0; c < 5; ++c) R[base + c * N + j] = Sr[c].d - Cd[j * 10 + c * 2 + le] * (float)invJ;
  }
}

dg_status_t shell_jvp_bf16(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s) {
  if ((m->p != 3 && m->p != 4) || !m->d_bf16op) {
    set_error("dg_jvp: the BF16 J v is available for shells of degree 3 and 4");
    return DG_ERR_UNSUPPORTED;
  }
  ShellDev M = m->shell();
  const GllC gc = make_gllc(m->p);
  PhysC ph = m->phys;
  sun_direction(ph, t);
  const unsigned blocks = (unsigned)((M.E + BF_EPB - 1) / BF_EPB);
  {
    ProfScope ps(m, 14, s);
    constexpr int X1 = kXpEuv, X3 = kXpEuv | kXpComp;
    const bool comp = ph.comp != 0;
    if (m->p == 3 && comp)
      shell_pass1_bf16<3, X3><<<blocks, BfShape<3>::THREADS, 0, s>>>(M, ph, gc, t, u, v, m->d_bf16op, jv, m->d_fn32);
    else if (m->p == 3)
      shell_pass1_bf16<3, X1><<<blocks, BfShape<3>::THREADS, 0, s>>>(M, ph, gc, t, u, v, m->d_bf16op, jv, m->d_fn32);
    else if (comp)
      shell_pass1_bf16<4, X3><<<blocks, BfShape<4>::THREADS, 0, s>>>(M, ph, gc, t, u, v, m->d_bf16op, jv, m->d_fn32);
    else
      shell_pass1_bf16<4, X1><<<blocks, BfShape<4>::THREADS, 0, s>>>(M, ph, gc, t, u, v, m->d_bf16op, jv, m->d_fn32);
  }
  {
    ProfScope ps(m, 15, s);
    if (m->p == 3)
      shell_pass2<3, float><<<(M.E + Shape<3>::EPB - 1) / Shape<3>::EPB, 256, 0, s>>>(M, gc, m->d_fn32, jv);
    else
      shell_pass2<4, float><<<(M.E + Shape<4>::EPB - 1) / Shape<4>::EPB, 256, 0, s>>>(M, gc, m->d_fn32, jv);
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

// the dense bf16 reference operators of the BF16 J v (degrees 3 and 4), zero-padded to NP
// nodes (64 at p = 3, 128 at p = 4): [D1 | D2] (NP x 2NP), D3 (NP x NP), [D1 D2 D3] (NP x 3NP),
// row-major, D1 = D x I x I etc. on the element's node order j = a + n b + n^2 c
std::vector<uint16_t> bf16_operators(int p) {
  const Gll g = make_gll(p);
  const int n = p + 1, N = n * n * n;
  const int NP = (p == 3) ? BfShape<3>::NP : BfShape<4>::NP;
  auto Dk = [&](int dir, int j, int k2) -> double {
    if (j >= N || k2 >= N) return 0.0;
    const int a = j % n, b = (j / n) % n, c = j / (n * n);
    const int a2 = k2 % n, b2 = (k2 / n) % n, c2 = k2 / (n * n);
    if (dir == 0) return (b == b2 && c == c2) ? g.D[a * n + a2] : 0.0;
    if (dir == 1) return (a == a2 && c == c2) ? g.D[b * n + b2] : 0.0;
    return (a == a2 && b == b2) ? g.D[c * n + c2] : 0.0;
  };
  std::vector<uint16_t> out((size_t)NP * 2 * NP + (size_t)NP * NP + (size_t)NP * 3 * NP);
  uint16_t* g1 = out.data();
  uint16_t* g3 = g1 + (size_t)NP * 2 * NP;
  uint16_t* dv = g3 + (size_t)NP * NP;
  for (int j = 0; j < NP; ++j)
    for (int k2 = 0; k2 < NP; ++k2) {
      g1[j * 2 * NP + k2] = f2bf((float)Dk(0, j, k2));
      g1[j * 2 * NP + NP + k2] = f2bf((float)Dk(1, j, k2));
      g3[j * NP + k2] = f2bf((float)Dk(2, j, k2));
      for (int dd = 0; dd < 3; ++dd) dv[j * 3 * NP + dd * NP + k2] = f2bf((float)Dk(dd, j, k2));
    }
  return out;
}

// tensor-product modal filter of every element: the 1D filter F applied along the three
// directions in turn (LDS-staged), in place on u [E][5][N]
template <int P>
__global__ __launch_bounds__(256) void shell_filter(int E, FiltC f, double* __restrict__ u) {
  typedef Shape<P> Sh;
  constexpr int n = Sh::n, N = Sh::N, N2 = Sh::N2, TPE = Sh::TPE, EPB = Sh::EPB;
  __shared__ double s_x[EPB][N];
  __shared__ double F[n * n];
  const int le = threadIdx.x / TPE;
  const int j = threadIdx.x % TPE;
  const int e = blockIdx.x * EPB + le;
  const bool active = e < E && j < N;
  if (threadIdx.x < n * n) F[threadIdx.x] = f.F[threadIdx.x];
  const int a = j % n, b = (j / n) % n, cz = j / N2;
  const int64_t base = (int64_t)e * 5 * N;
  for (int c = 0; c < 5; ++c) {
    double x = active ? u[base + c * N + j] : 0.0;
    if (active) s_x[le][j] = x;
    __syncthreads();
    if (active) {
      x = 0.0;
      for (int i = 0; i < n; ++i) x += F[a * n + i] * s_x[le][i + n * b + N2 * cz];
    }
    __syncthreads();
    if (active) s_x[le][j] = x;
    __syncthreads();
    if (active) {
      x = 0.0;
      for (int i = 0; i < n; ++i) x += F[b * n + i] * s_x[le][a + n * i + N2 * cz];
    }
    __syncthreads();
    if (active) s_x[le][j] = x;
    __syncthreads();
    if (active) {
      x = 0.0;
      for (int i = 0; i < n; ++i) x += F[cz * n + i] * s_x[le][a + n * b + N2 * i];
      u[base + c * N + j] = x;
    }
    __syncthreads();
  }
}

dg_status_t shell_filter_apply(dg_mesh_s* m, double sigma, double* u, hipStream_t s) {
  const int E = (int)m->n_elem;
  const FiltC f = make_filter(m->p, sigma);
  switch (m->p) {
    case 2: shell_filter<2><<<(E + Shape<2>::EPB - 1) / Shape<2>::EPB, 256, 0, s>>>(E, f, u); break;
    case 3: shell_filter<3><<<(E + Shape<3>::EPB - 1) / Shape<3>::EPB, 256, 0, s>>>(E, f, u); break;
    default: shell_filter<4><<<(E + Shape<4>::EPB - 1) / Shape<4>::EPB, 256, 0, s>>>(E, f, u); break;
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

// Node block-Jacobi blocks of the stage matrix I - dta J(u): for every node, the 5x5
// derivative of R at the node with respect to the node's own state through its
// pointwise flux and source (the gradient q held fixed), the diagonal entries of the
// volume derivative operators and the own-face terms with their stabilisation.
// Stored inverted, entry (r, c) of node j of element e at Binv[(e*25 + r*5 + c)*N + j].
template <int P>
__global__ __launch_bounds__(256) void shell_bjac(ShellDev M, PhysC ph, GllC gc, double t,
                                                  const double* __restrict__ u, double dta,
                                                  double* __restrict__ Binv) {
  typedef Shape<P> Sh;
  typedef Dual<double> DD;
  constexpr int n = Sh::n, N = Sh::N, N2 = Sh::N2, TPE = Sh::TPE, EPB = Sh::EPB;
  __shared__ double s_ang[EPB][13][N2];
  __shared__ double s_u[EPB][5][N];
  __shared__ double D[n * n];
  const int le = threadIdx.x / TPE;
  const int j = threadIdx.x % TPE;
  const int e = blockIdx.x * EPB + le;
  const bool live = e < M.E;
  const bool active = live && (j < N);
  const int cell = live ? e / M.n_rad : 0;
  const int k = live ? e % M.n_rad : 0;
  if (threadIdx.x < n * n) D[threadIdx.x] = gc.D[threadIdx.x];
  const double w_end = gc.w[0];
  if (live)
    for (int idx = j; idx < 13 * N2; idx += TPE) s_ang[le][idx / N2][idx % N2] = M.ang[(int64_t)cell * 13 * N2 + idx];
  double uu[5];
  const int64_t base = (int64_t)e * 5 * N;
  if (active)
    for (int c = 0; c < 5; ++c) {
      uu[c] = u[base + c * N + j];
      s_u[le][c][j] = uu[c];
    }
  __syncthreads();
  if (!active) return;
  const NodeGeo g = node_geo<P>(M, gc, s_ang[le], k, j);
  double q[5][3];
  node_gradient<P, double>(M, ph, D, gc.x, w_end, s_ang[le], s_u[le], u, (const double*)nullptr, cell, k, g, uu, q);
  const double Q = heating<3>(ph, g.x, t);
  const double invJ = 1.0 / g.Jac, lfac = 1.0 / (w_end * g.Jac);
  const int idx3[3] = {g.a, g.b, g.cz};
  const double fac3[3] = {g.rc * g.rp, g.rc * g.rp, g.rc * g.rc};
  const double* Am3[3] = {g.A1, g.A2, g.A3};
  const bool on[6] = {g.a == 0, g.a == n - 1, g.b == 0, g.b == n - 1, g.cz == 0, g.cz == n - 1};
  double sm, se;
  sigma<3, double, kXpComp>(ph, uu, sm, se, g.rc);
  double blk[5][10];
  for (int c = 0; c < 5; ++c) {
    DD ud[5], qd[5][3], Fd[5][3], Sd[5];
    for (int r = 0; r < 5; ++r) {
      ud[r] = DD(uu[r], r == c ? 1.0 : 0.0);
      for (int d = 0; d < 3; ++d) qd[r][d] = DD(q[r][d], 0.0);
    }
    flux_source<3, DD, kXpEuv | kXpComp>(ph, ud, qd, g.x, Q, Fd, Sd);
    for (int r = 0; r < 5; ++r) {
      double col = Sd[r].d;
      double gd[3];
      for (int dd = 0; dd < 3; ++dd) {
        gd[dd] = fac3[dd] * (Am3[dd][0] * Fd[r][0].d + Am3[dd][1] * Fd[r][1].d + Am3[dd][2] * Fd[r][2].d);
        col -= D[idx3[dd] * n + idx3[dd]] * gd[dd] * invJ;
      }
      for (int f = 0; f < 6; ++f) {
        if (!on[f]) continue;
        const int dd = f >> 1;
        const double side = (f & 1) ? 1.0 : -1.0;
        const bool bnd = (f == 4 && k == 0) || (f == 5 && k == M.n_rad - 1);
        double Sn2 = 0;
        for (int d = 0; d < 3; ++d) Sn2 += fac3[dd] * Am3[dd][d] * fac3[dd] * Am3[dd][d];
        const double sg = (r == 0) ? ph.lam : (r == 4 ? se : sm);
        if (!bnd) {
          col += 0.5 * lfac * side * gd[dd];
          if (r == c) col -= 0.5 * lfac * sqrt(Sn2) * sg;
        } else if (f == 4 || ph.bc_mode == 1) {
          if (r == c && r > 0) col -= lfac * sqrt(Sn2) * sg;
        } else if (r >= 1 && r <= 3 && c >= 1 && c <= 3) {
          // upper face: lambda (U.Sn) Sn / |Sn|
          col -= lfac * ph.lam * fac3[dd] * Am3[dd][r - 1] * fac3[dd] * Am3[dd][c - 1] / sqrt(Sn2);
        }
      }
      blk[r][c] = (r == c ? 1.0 : 0.0) - dta * col;
    }
  }
  // invert by Gauss-Jordan elimination with partial pivoting on [blk | I]
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) blk[r][5 + c] = (r == c) ? 1.0 : 0.0;
  for (int c = 0; c < 5; ++c) {
    int piv = c;
    for (int r = c + 1; r < 5; ++r)
      if (fabs(blk[r][c]) > fabs(blk[piv][c])) piv = r;
    if (piv != c)
      for (int q2 = 0; q2 < 10; ++q2) {
        const double tmp = blk[c][q2];
        blk[c][q2] = blk[piv][q2];
        blk[piv][q2] = tmp;
      }
    const double inv = 1.0 / blk[c][c];
    for (int q2 = 0; q2 < 10; ++q2) blk[c][q2] *= inv;
    for (int r = 0; r < 5; ++r) {
      if (r == c) continue;
      const double f = blk[r][c];
      for (int q2 = 0; q2 < 10; ++q2) blk[r][q2] -= f * blk[c][q2];
    }
  }
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) Binv[((int64_t)e * 25 + r * 5 + c) * N + j] = blk[r][5 + c];
}

template <int N_, class T>
__global__ __launch_bounds__(256) void shell_bjac_apply(int64_t nnodes, const double* __restrict__ Binv,
                                                        const T* __restrict__ v, T* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnodes) return;
  const int64_t e = i / N_;
  const int j = (int)(i % N_);
  T vv[5];
  for (int c = 0; c < 5; ++c) vv[c] = v[(e * 5 + c) * N_ + j];
  for (int r = 0; r < 5; ++r) {
    double acc = 0;
    for (int c = 0; c < 5; ++c) acc += Binv[(e * 25 + r * 5 + c) * N_ + j] * (double)vv[c];
    z[(e * 5 + r) * N_ + j] = (T)acc;
  }
}

dg_status_t shell_bjac_build(dg_mesh_s* m, double t, const double* u, double dta, double* Binv, hipStream_t s) {
  ShellDev M = m->shell();
  const GllC gc = make_gllc(m->p);
  PhysC ph = m->phys;
  sun_direction(ph, t);
  ProfScope ps(m, 10, s);
  switch (m->p) {
    case 2: shell_bjac<2><<<(M.E + Shape<2>::EPB - 1) / Shape<2>::EPB, 256, 0, s>>>(M, ph, gc, t, u, dta, Binv); break;
    case 3: shell_bjac<3><<<(M.E + Shape<3>::EPB - 1) / Shape<3>::EPB, 256, 0, s>>>(M, ph, gc, t, u, dta, Binv); break;
    default: shell_bjac<4><<<(M.E + Shape<4>::EPB - 1) / Shape<4>::EPB, 256, 0, s>>>(M, ph, gc, t, u, dta, Binv); break;
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

template <class T>
dg_status_t shell_bjac_apply_t(dg_mesh_s* m, const double* Binv, const T* v, T* z, hipStream_t s) {
  const int64_t nn = m->n_elem * m->N;
  const int blocks = (int)((nn + 255) / 256);
  ProfScope ps(m, 11, s);
  switch (m->p) {
    case 2: shell_bjac_apply<27, T><<<blocks, 256, 0, s>>>(nn, Binv, v, z); break;
    case 3: shell_bjac_apply<64, T><<<blocks, 256, 0, s>>>(nn, Binv, v, z); break;
    default: shell_bjac_apply<125, T><<<blocks, 256, 0, s>>>(nn, Binv, v, z); break;
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}
dg_status_t shell_bjac_apply64(dg_mesh_s* m, const double* B, const double* v, double* z, hipStream_t s) {
  return shell_bjac_apply_t<double>(m, B, v, z, s);
}
dg_status_t shell_bjac_apply32(dg_mesh_s* m, const double* B, const float* v, float* z, hipStream_t s) {
  return shell_bjac_apply_t<float>(m, B, v, z, s);
}

}  // namespace dg
