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
//    complete boundary-face terms; writes the partial R and the face trace
//    F(u, q).Sn of every face node.
//  pass 2 (same layout): for the interior faces adds half the neighbour's trace
//    and the stabilisation -|Sn| sigma(u_hat)(u - u_hat).
// With S = Dual<T> the same code yields J(u)v (the derivative part), exactly.
#include "internal.h"

namespace dg {

template <int P> struct Shape {
  static constexpr int n = P + 1, N = n * n * n, N2 = n * n;
  static constexpr int TPE = (P == 2) ? 32 : (P == 3 ? 64 : 128);
  static constexpr int EPB = 256 / TPE;
};

// output part of a scalar: the value, or the derivative of a dual
__device__ inline double outp(double x) { return x; }
__device__ inline float outp(float x) { return x; }
template <class T> __device__ inline T outp(Dual<T> x) { return x.d; }

template <class S, class SU, class TV>
__device__ inline S load_state(const SU* u, const TV* v, int64_t i) {
  return Io<S>::ld(u, v, i);
}

// neighbour of a face node: returns the neighbour element (or -1 on a boundary),
// the neighbour's local node and the neighbour's face index / face-node index
template <int P>
__device__ inline int face_neighbour(const ShellDev& M, int cell, int k, int f, int a, int b, int cz,
                                     int& jn, int& fn, int& mn) {
  constexpr int n = P + 1, N2 = n * n;
  if (f >= 4) {
    if (f == 4) {
      if (k == 0) return -1;
      jn = a + n * b + N2 * (n - 1);
      fn = 5;
      mn = a + n * b;
      return cell * M.n_rad + k - 1;
    }
    if (k == M.n_rad - 1) return -1;
    jn = a + n * b;
    fn = 4;
    mn = a + n * b;
    return cell * M.n_rad + k + 1;
  }
  const int s = (f < 2) ? b : a;
  const int c2 = M.cnbr[cell * 4 + f];
  fn = M.cface[cell * 4 + f];
  const int s2 = M.cmap[(cell * 4 + f) * n + s];
  int a2, b2;
  switch (fn) {
    case 0: a2 = 0; b2 = s2; break;
    case 1: a2 = n - 1; b2 = s2; break;
    case 2: a2 = s2; b2 = 0; break;
    default: a2 = s2; b2 = n - 1; break;
  }
  jn = a2 + n * b2 + N2 * cz;
  mn = s2 + n * cz;
  return c2 * M.n_rad + k;
}

// face-node index of node (a, b, cz) within face f
template <int P>
__device__ inline int face_slot(int f, int a, int b, int cz) {
  constexpr int n = P + 1;
  if (f < 2) return b + n * cz;
  if (f < 4) return a + n * cz;
  return a + n * b;
}

template <int P, class S, class SU, class TV, class OT>
__global__ __launch_bounds__(256) void shell_pass1(ShellDev M, PhysC ph, GllC gc, double t, const SU* __restrict__ u,
                                                   const TV* __restrict__ v, OT* __restrict__ R,
                                                   OT* __restrict__ Fn) {
  typedef Shape<P> Sh;
  typedef typename Base<S>::type T;
  constexpr int n = Sh::n, N = Sh::N, N2 = Sh::N2, TPE = Sh::TPE, EPB = Sh::EPB;
  __shared__ double s_ang[EPB][13][N2];
  __shared__ S s_u[EPB][5][N];
  __shared__ S s_G[EPB][3][5][N];
  __shared__ double D[n * n];
  const int le = threadIdx.x / TPE;
  const int j = threadIdx.x % TPE;
  const int e = blockIdx.x * EPB + le;
  const bool live = e < M.E;
  const bool active = live && (j < N);
  const int cell = live ? e / M.n_rad : 0;
  const int k = live ? e % M.n_rad : 0;
  if (threadIdx.x < n * n) D[threadIdx.x] = gc.D[threadIdx.x];
  const double* xg = gc.x;
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
  __syncthreads();

  const int a = j % n, b = (j / n) % n, cz = j / N2;
  const int ja = a + n * b;
  double rk = 0, hk = 1, rc = 1, rp = 1, Jac = 1, x[3] = {0, 0, 0};
  double A1[3], A2[3], A3[3];
  S F[5][3], Sr[5];
  if (active) {
    rk = M.edges[k];
    hk = M.edges[k + 1] - rk;
    rp = 0.5 * hk;
    rc = rk + 0.5 * (xg[cz] + 1.0) * hk;
    for (int d = 0; d < 3; ++d) {
      A1[d] = s_ang[le][d][ja];
      A2[d] = s_ang[le][3 + d][ja];
      A3[d] = s_ang[le][6 + d][ja];
      x[d] = rc * s_ang[le][10 + d][ja];
    }
    Jac = rc * rc * rp * s_ang[le][9][ja];
    const double rrp = rc * rp;
    double r2[n];
    for (int i = 0; i < n; ++i) {
      double ri = rk + 0.5 * (xg[i] + 1.0) * hk;
      r2[i] = ri * ri;
    }
    // ---- auxiliary gradient q (conservative form of the weak gradient)
    S q[5][3];
    const double invJ = 1.0 / Jac;
    for (int c = 0; c < 5; ++c) {
      S d1[3], d2[3], d3;
      for (int d = 0; d < 3; ++d) { d1[d] = S(T(0)); d2[d] = S(T(0)); }
      d3 = S(T(0));
      for (int i = 0; i < n; ++i) {
        const S u1 = s_u[le][c][i + n * b + N2 * cz];
        const S u2 = s_u[le][c][a + n * i + N2 * cz];
        const S u3 = s_u[le][c][ja + N2 * i];
        const double Da = D[a * n + i], Db = D[b * n + i], Dc = D[cz * n + i] * r2[i];
        for (int d = 0; d < 3; ++d) {
          d1[d] = d1[d] + u1 * T(Da * s_ang[le][d][i + n * b]);
          d2[d] = d2[d] + u2 * T(Db * s_ang[le][3 + d][a + n * i]);
        }
        d3 = d3 + u3 * T(Dc);
      }
      for (int d = 0; d < 3; ++d) q[c][d] = (T(rrp) * (d1[d] + d2[d]) + T(A3[d]) * d3) * T(invJ);
    }
    // lift of (u_hat - u) on the faces through this node
    const double lfac = 1.0 / (w_end * Jac);
    for (int f = 0; f < 6; ++f) {
      const bool on = (f == 0 && a == 0) || (f == 1 && a == n - 1) || (f == 2 && b == 0) || (f == 3 && b == n - 1) ||
                      (f == 4 && cz == 0) || (f == 5 && cz == n - 1);
      if (!on) continue;
      const double side = (f & 1) ? 1.0 : -1.0;
      double Sn[3];
      for (int d = 0; d < 3; ++d) Sn[d] = side * (f < 2 ? rrp * A1[d] : (f < 4 ? rrp * A2[d] : rc * rc * A3[d]));
      int jn, fn, mn;
      const int en = face_neighbour<P>(M, cell, k, f, a, b, cz, jn, fn, mn);
      S du[5];
      if (en >= 0) {
        for (int c = 0; c < 5; ++c) du[c] = T(0.5) * (load_state<S>(u, v, (int64_t)en * 5 * N + c * N + jn) - uu[c]);
      } else if (ph.bc_mode == 1 || f == 4) {
        S ub[5];
        boundary_state<3, S>(ph, uu, ub);
        for (int c = 0; c < 5; ++c) du[c] = ub[c] - uu[c];
      } else {
        continue;   // upper boundary: u_hat = u
      }
      for (int c = 0; c < 5; ++c)
        for (int d = 0; d < 3; ++d) q[c][d] = q[c][d] + du[c] * T(Sn[d] * lfac);
    }
    // ---- pointwise flux and source
    const double Q = heating<3>(ph, x, t);
    flux_source<3, S>(ph, uu, q, x, Q, F, Sr);
    for (int c = 0; c < 5; ++c) {
      for (int dd = 0; dd < 3; ++dd) {
        const double* Am = (dd == 0) ? A1 : (dd == 1 ? A2 : A3);
        const double fac = (dd < 2) ? rrp : rc * rc;
        S g = F[c][0] * T(fac * Am[0]) + F[c][1] * T(fac * Am[1]) + F[c][2] * T(fac * Am[2]);
        s_G[le][dd][c][j] = g;
      }
    }
    // boundary faces need the flux at the boundary state with the interior gradient;
    // keep q around through F (recomputed below only on boundary nodes)
    if (k == 0 && cz == 0) {
      // lower boundary (or Dirichlet state)
      S ub[5], Fb[5][3], Sb[5];
      boundary_state<3, S>(ph, uu, ub);
      flux_source<3, S>(ph, ub, q, x, 0.0, Fb, Sb);
      S sm, se;
      sigma<3, S>(ph, ub, sm, se);
      double Sn[3];
      for (int d = 0; d < 3; ++d) Sn[d] = -rc * rc * A3[d];
      const double Smag = sqrt(Sn[0] * Sn[0] + Sn[1] * Sn[1] + Sn[2] * Sn[2]);
      for (int c = 0; c < 5; ++c) {
        S fd = (F[c][0] - Fb[c][0]) * T(Sn[0]) + (F[c][1] - Fb[c][1]) * T(Sn[1]) + (F[c][2] - Fb[c][2]) * T(Sn[2]);
        const S sg = (c == 0) ? S(T(ph.lam)) : (c == 4 ? se : sm);
        Sr[c] = Sr[c] + (fd - T(Smag) * sg * (uu[c] - ub[c])) * T(lfac);
      }
    }
    if (k == M.n_rad - 1 && cz == n - 1) {
      double Sn[3];
      for (int d = 0; d < 3; ++d) Sn[d] = rc * rc * A3[d];
      if (ph.bc_mode == 1) {
        S ub[5], Fb[5][3], Sb[5];
        boundary_state<3, S>(ph, uu, ub);
        flux_source<3, S>(ph, ub, q, x, 0.0, Fb, Sb);
        S sm, se;
        sigma<3, S>(ph, ub, sm, se);
        const double Smag = sqrt(Sn[0] * Sn[0] + Sn[1] * Sn[1] + Sn[2] * Sn[2]);
        for (int c = 0; c < 5; ++c) {
          S fd = (F[c][0] - Fb[c][0]) * T(Sn[0]) + (F[c][1] - Fb[c][1]) * T(Sn[1]) + (F[c][2] - Fb[c][2]) * T(Sn[2]);
          const S sg = (c == 0) ? S(T(ph.lam)) : (c == 4 ? se : sm);
          Sr[c] = Sr[c] + (fd - T(Smag) * sg * (uu[c] - ub[c])) * T(lfac);
        }
      } else {
        // adiabatic, zero normal stress: F_hat.n = F_inviscid.n, so (F - F_hat).n = F_viscous.n
        S Fi[5][3];
        flux_inviscid<3, S>(ph, uu, Fi);
        for (int c = 0; c < 5; ++c) {
          S fd = (F[c][0] - Fi[c][0]) * T(Sn[0]) + (F[c][1] - Fi[c][1]) * T(Sn[1]) + (F[c][2] - Fi[c][2]) * T(Sn[2]);
          Sr[c] = Sr[c] + fd * T(lfac);
        }
      }
    }
  }
  __syncthreads();
  if (!active) return;
  // ---- volume divergence and own half of interior faces
  const double invJ = 1.0 / Jac;
  const double lfac = 1.0 / (w_end * Jac);
  for (int c = 0; c < 5; ++c) {
    S dv = S(T(0));
    for (int i = 0; i < n; ++i) {
      dv = dv + s_G[le][0][c][i + n * b + N2 * cz] * T(D[a * n + i]);
      dv = dv + s_G[le][1][c][a + n * i + N2 * cz] * T(D[b * n + i]);
      dv = dv + s_G[le][2][c][ja + N2 * i] * T(D[cz * n + i]);
    }
    Sr[c] = Sr[c] - dv * T(invJ);
  }
  for (int f = 0; f < 6; ++f) {
    const bool on = (f == 0 && a == 0) || (f == 1 && a == n - 1) || (f == 2 && b == 0) || (f == 3 && b == n - 1) ||
                    (f == 4 && cz == 0) || (f == 5 && cz == n - 1);
    if (!on) continue;
    if ((f == 4 && k == 0) || (f == 5 && k == M.n_rad - 1)) continue;   // done above
    const double side = (f & 1) ? 1.0 : -1.0;
    const int m = face_slot<P>(f, a, b, cz);
    const int dd = f >> 1;
    for (int c = 0; c < 5; ++c) {
      const S fsn = T(side) * s_G[le][dd][c][j];
      Sr[c] = Sr[c] + T(0.5 * lfac) * fsn;
      Fn[(((int64_t)e * 6 + f) * 5 + c) * N2 + m] = outp(fsn);
    }
  }
  for (int c = 0; c < 5; ++c) R[base + c * N + j] = outp(Sr[c]);
}

template <int P, class S, class SU, class TV, class OT>
__global__ __launch_bounds__(256) void shell_pass2(ShellDev M, PhysC ph, GllC gc, const SU* __restrict__ u,
                                                   const TV* __restrict__ v, const OT* __restrict__ Fn,
                                                   OT* __restrict__ R) {
  typedef Shape<P> Sh;
  typedef typename Base<S>::type T;
  constexpr int n = Sh::n, N = Sh::N, N2 = Sh::N2, TPE = Sh::TPE, EPB = Sh::EPB;
  const int le = threadIdx.x / TPE;
  const int j = threadIdx.x % TPE;
  const int e = blockIdx.x * EPB + le;
  if (e >= M.E || j >= N) return;
  const int a = j % n, b = (j / n) % n, cz = j / N2;
  const bool on[6] = {a == 0, a == n - 1, b == 0, b == n - 1, cz == 0, cz == n - 1};
  const int cell = e / M.n_rad, k = e % M.n_rad;
  if (!(on[0] || on[1] || on[2] || on[3] || (on[4] && k > 0) || (on[5] && k < M.n_rad - 1))) return;
  const int ja = a + n * b;
  const double rk = M.edges[k], hk = M.edges[k + 1] - rk, rp = 0.5 * hk;
  const double rc = rk + 0.5 * (gc.x[cz] + 1.0) * hk;
  const double w_end = gc.w[0];
  const double* ang = M.ang + (int64_t)cell * 13 * N2;
  const double Jac = rc * rc * rp * ang[9 * N2 + ja];
  const double lfac = 1.0 / (w_end * Jac);
  const int64_t base = (int64_t)e * 5 * N;
  S uu[5];
  for (int c = 0; c < 5; ++c) uu[c] = load_state<S>(u, v, base + c * N + j);
  OT acc[5];
  for (int c = 0; c < 5; ++c) acc[c] = R[base + c * N + j];
  for (int f = 0; f < 6; ++f) {
    if (!on[f]) continue;
    int jn, fn, mn;
    const int en = face_neighbour<P>(M, cell, k, f, a, b, cz, jn, fn, mn);
    if (en < 0) continue;
    const int dd = f >> 1;
    const double fac = (dd < 2) ? rc * rp : rc * rc;
    double Sn2 = 0;
    for (int d = 0; d < 3; ++d) {
      const double s_ = fac * ang[(3 * dd + d) * N2 + ja];
      Sn2 += s_ * s_;
    }
    const double Smag = sqrt(Sn2);
    S um[5], uh[5];
    for (int c = 0; c < 5; ++c) {
      um[c] = load_state<S>(u, v, (int64_t)en * 5 * N + c * N + jn);
      uh[c] = T(0.5) * (uu[c] + um[c]);
    }
    S sm, se;
    sigma<3, S>(ph, uh, sm, se);
    for (int c = 0; c < 5; ++c) {
      const S sg = (c == 0) ? S(T(ph.lam)) : (c == 4 ? se : sm);
      const S stab = T(Smag) * sg * (uu[c] - uh[c]);
      const OT fnb = Fn[(((int64_t)en * 6 + fn) * 5 + c) * N2 + mn];
      acc[c] += OT(lfac) * (OT(0.5) * fnb - outp(stab));
    }
  }
  for (int c = 0; c < 5; ++c) R[base + c * N + j] = acc[c];
}

template <class S, class SU, class TV, class OT>
static dg_status_t launch(dg_mesh_s* m, double t, const SU* u, const TV* v, OT* out, OT* fn, hipStream_t s,
                          int prof_base) {
  ShellDev M = m->shell();
  const int E = M.E;
  const GllC gc = make_gllc(m->p);
#define DG_LAUNCH(P_)                                                                                     \
  {                                                                                                        \
    const int blocks = (E + Shape<P_>::EPB - 1) / Shape<P_>::EPB;                                          \
    {                                                                                                      \
      ProfScope ps(m, prof_base, s);                                                                       \
      shell_pass1<P_, S, SU, TV, OT><<<blocks, 256, 0, s>>>(M, m->phys, gc, t, u, v, out, fn);             \
    }                                                                                                      \
    {                                                                                                      \
      ProfScope ps(m, prof_base + 1, s);                                                                   \
      shell_pass2<P_, S, SU, TV, OT><<<blocks, 256, 0, s>>>(M, m->phys, gc, u, v, fn, out);                \
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

dg_status_t shell_residual(dg_mesh_s* m, double t, const double* u, double* r, hipStream_t s) {
  return launch<double, double, double, double>(m, t, u, (const double*)nullptr, r, m->d_fn64, s, 0);
}
dg_status_t shell_jvp64(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s) {
  return launch<Dual<double>, double, double, double>(m, t, u, v, jv, m->d_fn64, s, 2);
}
dg_status_t shell_jvp32(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s) {
  return launch<Dual<float>, double, float, float>(m, t, u, v, jv, m->d_fn32, s, 4);
}

}  // namespace dg
