// Residual R(u) and J(u)v for batches of independent 1D radial columns (the
// radial one-dimensional model of section 4.1.3): d = 1, fields (varrho,
// sqrt(rho) v_r, sqrt(rho) T), the same LDG weak form as the shell in its strong
// form. One thread per element; the same two-pass split as the shell kernels
// (pass 1: everything an element can do alone, writing its face traces F.n;
// pass 2: neighbour halves and the interior-face stabilisation).
#include "internal.h"

namespace dg {

__device__ inline double outc(double x) { return x; }
__device__ inline float outc(float x) { return x; }
template <class T> __device__ inline T outc(Dual<T> x) { return x.d; }

__device__ inline PhysC column_phys(const ColDev& C, const PhysC& ph, int col) {
  PhysC P = ph;
  const double* cp = C.cpar + 5 * col;
  P.heat_amp = cp[0];
  P.heat_qm = cp[1];
  P.heat_rm = cp[2];
  P.heat_inv_H = cp[3];
  P.lam = cp[4];
  return P;
}

template <int P, class S, class SU, class TV, class OT>
__global__ __launch_bounds__(128) void col_pass1(ColDev C, const int* __restrict__ elist, int ne, PhysC ph, GllC gc, double t,
                                                 const SU* __restrict__ u, const TV* __restrict__ v,
                                                 OT* __restrict__ R, OT* __restrict__ Fn) {
  typedef typename Base<S>::type T;
  constexpr int n = P + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ne) return;
  const int e = elist[idx];
  const PhysC Pc = column_phys(C, ph, C.col[e]);
  const double* D = gc.D;
  const double* xg = gc.x;
  const double w_end = gc.w[0];
  const int64_t off = C.off[e];
  const double r0 = C.geo[2 * e], h = C.geo[2 * e + 1];
  const double Jac = 0.5 * h, invJ = 1.0 / Jac, lfac = 1.0 / (w_end * Jac);
  const int ep = C.prev[e], en = C.next[e];
  S uu[3][n];
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) uu[c][i] = Io<S>::ld(u, v, off + c * n + i);
  S q[3][n][1];
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) {
      S s = S(T(0));
      for (int l = 0; l < n; ++l) s = s + uu[c][l] * T(D[i * n + l]);
      q[c][i][0] = s * T(invJ);
    }
  // lift of (u_hat - u): lower face (Sn = -1), upper face (Sn = +1)
  {
    S u0[3], ub[3];
    for (int c = 0; c < 3; ++c) u0[c] = uu[c][0];
    if (ep >= 0) {
      const int64_t o2 = C.off[ep];
      for (int c = 0; c < 3; ++c) ub[c] = T(0.5) * (Io<S>::ld(u, v, o2 + c * n + (n - 1)) + u0[c]);
    } else {
      boundary_state<1, S>(Pc, u0, ub);
    }
    for (int c = 0; c < 3; ++c) q[c][0][0] = q[c][0][0] - (ub[c] - u0[c]) * T(lfac);
    S ut[3];
    for (int c = 0; c < 3; ++c) ut[c] = uu[c][n - 1];
    bool have = true;
    if (en >= 0) {
      const int64_t o2 = C.off[en];
      for (int c = 0; c < 3; ++c) ub[c] = T(0.5) * (Io<S>::ld(u, v, o2 + c * n) + ut[c]);
    } else if (Pc.bc_mode == 1) {
      boundary_state<1, S>(Pc, ut, ub);
    } else {
      have = false;
    }
    if (have)
      for (int c = 0; c < 3; ++c) q[c][n - 1][0] = q[c][n - 1][0] + (ub[c] - ut[c]) * T(lfac);
  }
  S F[3][n][1], Sr[3][n];
  for (int i = 0; i < n; ++i) {
    S ui[3], qi[3][1], Fi[3][1], Si[3];
    for (int c = 0; c < 3; ++c) { ui[c] = uu[c][i]; qi[c][0] = q[c][i][0]; }
    const double x = r0 + 0.5 * (xg[i] + 1.0) * h;
    const double Q = heating<1>(Pc, &x, t);
    flux_source<1, S>(Pc, ui, qi, &x, Q, Fi, Si);
    for (int c = 0; c < 3; ++c) { F[c][i][0] = Fi[c][0]; Sr[c][i] = Si[c]; }
  }
  S Rl[3][n];
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) {
      S dv = S(T(0));
      for (int l = 0; l < n; ++l) dv = dv + F[c][l][0] * T(D[i * n + l]);
      Rl[c][i] = Sr[c][i] - dv * T(invJ);
    }
  // lower face
  if (ep >= 0) {
    for (int c = 0; c < 3; ++c) {
      const S fsn = -F[c][0][0];
      Rl[c][0] = Rl[c][0] + T(0.5 * lfac) * fsn;
      Fn[((int64_t)e * 2 + 0) * 3 + c] = outc(fsn);
    }
  } else {
    S u0[3], ub[3], qi[3][1], Fb[3][1], Sb[3], sm, se;
    for (int c = 0; c < 3; ++c) { u0[c] = uu[c][0]; qi[c][0] = q[c][0][0]; }
    boundary_state<1, S>(Pc, u0, ub);
    const double x = r0;
    flux_source<1, S>(Pc, ub, qi, &x, 0.0, Fb, Sb);
    sigma<1, S>(Pc, ub, sm, se);
    for (int c = 0; c < 3; ++c) {
      const S sg = (c == 0) ? S(T(Pc.lam)) : (c == 2 ? se : sm);
      const S fd = -(F[c][0][0] - Fb[c][0]);
      Rl[c][0] = Rl[c][0] + (fd - sg * (u0[c] - ub[c])) * T(lfac);
    }
  }
  // upper face
  if (en >= 0) {
    for (int c = 0; c < 3; ++c) {
      const S fsn = F[c][n - 1][0];
      Rl[c][n - 1] = Rl[c][n - 1] + T(0.5 * lfac) * fsn;
      Fn[((int64_t)e * 2 + 1) * 3 + c] = outc(fsn);
    }
  } else {
    S ut[3], qi[3][1];
    for (int c = 0; c < 3; ++c) { ut[c] = uu[c][n - 1]; qi[c][0] = q[c][n - 1][0]; }
    if (Pc.bc_mode == 1) {
      S ub[3], Fb[3][1], Sb[3], sm, se;
      boundary_state<1, S>(Pc, ut, ub);
      const double x = r0 + h;
      flux_source<1, S>(Pc, ub, qi, &x, 0.0, Fb, Sb);
      sigma<1, S>(Pc, ub, sm, se);
      for (int c = 0; c < 3; ++c) {
        const S sg = (c == 0) ? S(T(Pc.lam)) : (c == 2 ? se : sm);
        Rl[c][n - 1] = Rl[c][n - 1] + ((F[c][n - 1][0] - Fb[c][0]) - sg * (ut[c] - ub[c])) * T(lfac);
      }
    } else {
      S Fi[3][1];
      flux_inviscid<1, S>(Pc, ut, Fi);
      for (int c = 0; c < 3; ++c) Rl[c][n - 1] = Rl[c][n - 1] + (F[c][n - 1][0] - Fi[c][0]) * T(lfac);
    }
  }
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) R[off + c * n + i] = outc(Rl[c][i]);
}

template <int P, class S, class SU, class TV, class OT>
__global__ __launch_bounds__(128) void col_pass2(ColDev C, const int* __restrict__ elist, int ne, PhysC ph, GllC gc,
                                                 const SU* __restrict__ u, const TV* __restrict__ v,
                                                 const OT* __restrict__ Fn, OT* __restrict__ R) {
  typedef typename Base<S>::type T;
  constexpr int n = P + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ne) return;
  const int e = elist[idx];
  const PhysC Pc = column_phys(C, ph, C.col[e]);
  const double w_end = gc.w[0];
  const int64_t off = C.off[e];
  const double h = C.geo[2 * e + 1];
  const double lfac = 1.0 / (w_end * 0.5 * h);
  for (int side = 0; side < 2; ++side) {
    const int nb = side ? C.next[e] : C.prev[e];
    if (nb < 0) continue;
    const int i = side ? n - 1 : 0;
    const int inb = side ? 0 : n - 1;
    const int64_t o2 = C.off[nb];
    S ui[3], uh[3];
    for (int c = 0; c < 3; ++c) {
      ui[c] = Io<S>::ld(u, v, off + c * n + i);
      uh[c] = T(0.5) * (ui[c] + Io<S>::ld(u, v, o2 + c * n + inb));
    }
    S sm, se;
    sigma<1, S>(Pc, uh, sm, se);
    for (int c = 0; c < 3; ++c) {
      const S sg = (c == 0) ? S(T(Pc.lam)) : (c == 2 ? se : sm);
      const OT fnb = Fn[((int64_t)nb * 2 + (1 - side)) * 3 + c];
      R[off + c * n + i] += OT(lfac) * (OT(0.5) * fnb - outc(sg * (ui[c] - uh[c])));
    }
  }
}

template <class S, class SU, class TV, class OT>
static dg_status_t launch_cols(dg_mesh_s* m, double t, const SU* u, const TV* v, OT* out, OT* fn, hipStream_t s,
                               int prof_base) {
  ColDev C = m->cols();
  ProfScope ps(m, prof_base, s);
  const GllC gc[3] = {make_gllc(2), make_gllc(3), make_gllc(4)};
  PhysC ph = m->phys;
  sun_direction(ph, t);
  for (int pi = 0; pi < 3; ++pi) {
    const int ne = m->plist_n[pi];
    if (!ne) continue;
    const int blocks = (ne + 127) / 128;
    const int* el = m->d_plist[pi];
    switch (pi + 2) {
      case 2: col_pass1<2, S, SU, TV, OT><<<blocks, 128, 0, s>>>(C, el, ne, ph, gc[0], t, u, v, out, fn); break;
      case 3: col_pass1<3, S, SU, TV, OT><<<blocks, 128, 0, s>>>(C, el, ne, ph, gc[1], t, u, v, out, fn); break;
      default: col_pass1<4, S, SU, TV, OT><<<blocks, 128, 0, s>>>(C, el, ne, ph, gc[2], t, u, v, out, fn); break;
    }
  }
  for (int pi = 0; pi < 3; ++pi) {
    const int ne = m->plist_n[pi];
    if (!ne) continue;
    const int blocks = (ne + 127) / 128;
    const int* el = m->d_plist[pi];
    switch (pi + 2) {
      case 2: col_pass2<2, S, SU, TV, OT><<<blocks, 128, 0, s>>>(C, el, ne, ph, gc[0], u, v, fn, out); break;
      case 3: col_pass2<3, S, SU, TV, OT><<<blocks, 128, 0, s>>>(C, el, ne, ph, gc[1], u, v, fn, out); break;
      default: col_pass2<4, S, SU, TV, OT><<<blocks, 128, 0, s>>>(C, el, ne, ph, gc[2], u, v, fn, out); break;
    }
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

dg_status_t col_residual(dg_mesh_s* m, double t, const double* u, double* r, hipStream_t s) {
  return launch_cols<double, double, double, double>(m, t, u, (const double*)nullptr, r, m->d_fn64, s, 6);
}
dg_status_t col_jvp64(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s) {
  return launch_cols<Dual<double>, double, double, double>(m, t, u, v, jv, m->d_fn64, s, 7);
}
dg_status_t col_jvp32(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s) {
  return launch_cols<Dual<float>, double, float, float>(m, t, u, v, jv, m->d_fn32, s, 8);
}

}  // namespace dg
