// Residual R(u) and J(u)v for batches of independent 1D radial columns (the
// radial one-dimensional model of section 4.1.3): d = 1, fields (varrho,
// sqrt(rho) v_r, sqrt(rho) T), the same LDG weak form as the shell in its strong
// form. One thread per element; the same two-pass split as the shell kernels
// (pass 1: everything an element can do alone, writing its face traces F.n;
// pass 2: neighbour halves and the interior-face stabilisation).
#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

namespace dg {

__device__ inline double outc(double x) { return x; }
__device__ inline float outc(float x) { return x; }
template <class T> __device__ inline T outc(Dual<T> x) { return x.d; }

// the physics of column col: its parameter block (CPAR values) and EUVAC table
__device__ inline void set_column_phys(PhysC& P, const double* __restrict__ cpar, const double* euv, int col) {
  const double* cp = cpar + CPAR * col;
  P.heat_amp = cp[0];
  P.heat_qm = cp[1];
  P.heat_rm = cp[2];
  P.heat_inv_H = cp[3];
  P.lam = cp[4];
  P.alpha0c = cp[5];
  P.site[0] = cp[6];
  P.site[1] = cp[7];
  P.site[2] = cp[8];
  if (euv) P.euv_tab = euv + EUVT * col;
}

__device__ inline PhysC column_phys(const ColDev& C, const PhysC& ph, int col) {
  PhysC P = ph;
  set_column_phys(P, C.cpar, C.euv, col);
  return P;
}

// one element of a column: DOF offsets of itself and of its neighbours (-1 on a
// boundary), its bottom radius and thickness, and its slot in the face-trace array
struct ColElem {
  int64_t off, off_prev, off_next;
  double r0, h;
  int64_t fslot, fslot_prev, fslot_next;   // Fn[(fslot*2 + side)*3 + c]
};

// XP: the extended physics the instantiation contains (kXpEuv, kXpComp; PhysC::xp_mode)
template <int P, class S, int XP = 0, class SU, class TV, class OT>
__device__ __forceinline__ void col_elem_pass1(const ColElem& ce, const PhysC& Pc, const GllC& gc, double t,
                                      const SU* __restrict__ u, const TV* __restrict__ v, OT* __restrict__ R,
                                      OT* __restrict__ Fn) {
  typedef typename Base<S>::type T;
  constexpr int n = P + 1;
  const double* D = gc.D;
  const double* xg = gc.x;
  const double w_end = gc.w[0];
  const int64_t off = ce.off;
  const double r0 = ce.r0, h = ce.h;
  const double Jac = 0.5 * h, invJ = 1.0 / Jac, lfac = 1.0 / (w_end * Jac);
  const bool hp = ce.off_prev >= 0, hn = ce.off_next >= 0;
  const int64_t e = ce.fslot;
  S uu[3][n];
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) uu[c][i] = Io<S>::ld(u, v, off + c * n + i);
  // face traces u_hat - u at the two end nodes (lift of the gradient)
  S dlo[3], dhi[3];
  {
    S u0[3], ub[3];
    for (int c = 0; c < 3; ++c) u0[c] = uu[c][0];
    if (hp) {
      for (int c = 0; c < 3; ++c) dlo[c] = T(0.5) * (Io<S>::ld(u, v, ce.off_prev + c * n + (n - 1)) - u0[c]);
    } else {
      boundary_state<1, S>(Pc, u0, ub);
      for (int c = 0; c < 3; ++c) dlo[c] = ub[c] - u0[c];
    }
    for (int c = 0; c < 3; ++c) u0[c] = uu[c][n - 1];
    if (hn) {
      for (int c = 0; c < 3; ++c) dhi[c] = T(0.5) * (Io<S>::ld(u, v, ce.off_next + c * n) - u0[c]);
    } else if (Pc.bc_mode == 1) {
      boundary_state<1, S>(Pc, u0, ub);
      for (int c = 0; c < 3; ++c) dhi[c] = ub[c] - u0[c];
    } else {
      for (int c = 0; c < 3; ++c) dhi[c] = S(T(0));
    }
  }
  // node by node: q_i, flux and source, accumulated into the divergence of every node
  S Rl[3][n];
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) Rl[c][i] = S(T(0));
  S Flo[3], Fhi[3], qlo[3][1], qhi[3][1];
  for (int i = 0; i < n; ++i) {
    S ui[3], qi[3][1], Fi[3][1], Si[3];
    for (int c = 0; c < 3; ++c) {
      ui[c] = uu[c][i];
      S g = S(T(0));
      for (int l = 0; l < n; ++l) g = g + uu[c][l] * T(D[i * n + l]);
      g = g * T(invJ);
      if (i == 0) g = g - dlo[c] * T(lfac);
      if (i == n - 1) g = g + dhi[c] * T(lfac);
      qi[c][0] = g;
    }
    const double x = r0 + 0.5 * (xg[i] + 1.0) * h;
    const double Q = heating<1>(Pc, &x, t);
    flux_source<1, S, XP>(Pc, ui, qi, &x, Q, Fi, Si);
    for (int c = 0; c < 3; ++c) {
      Rl[c][i] = Rl[c][i] + Si[c];
      for (int r = 0; r < n; ++r) Rl[c][r] = Rl[c][r] - Fi[c][0] * T(D[r * n + i] * invJ);
      if (i == 0) { Flo[c] = Fi[c][0]; qlo[c][0] = qi[c][0]; }
      if (i == n - 1) { Fhi[c] = Fi[c][0]; qhi[c][0] = qi[c][0]; }
    }
  }
  // lower face
  if (hp) {
    for (int c = 0; c < 3; ++c) {
      const S fsn = -Flo[c];
      Rl[c][0] = Rl[c][0] + T(0.5 * lfac) * fsn;
      Fn[(e * 2 + 0) * 3 + c] = outc(fsn);
    }
  } else {
    S u0[3], ub[3], Fb[3][1], Sb[3], sm, se;
    for (int c = 0; c < 3; ++c) u0[c] = uu[c][0];
    boundary_state<1, S>(Pc, u0, ub);
    const double x = r0;
    flux_source<1, S, XP & kXpComp>(Pc, ub, qlo, &x, 0.0, Fb, Sb, false);
    sigma<1, S, XP & kXpComp>(Pc, ub, sm, se, x);
    for (int c = 0; c < 3; ++c) {
      const S sg = (c == 0) ? S(T(Pc.lam)) : (c == 2 ? se : sm);
      const S fd = -(Flo[c] - Fb[c][0]);
      Rl[c][0] = Rl[c][0] + (fd - sg * (u0[c] - ub[c])) * T(lfac);
    }
  }
  // upper face
  if (hn) {
    for (int c = 0; c < 3; ++c) {
      const S fsn = Fhi[c];
      Rl[c][n - 1] = Rl[c][n - 1] + T(0.5 * lfac) * fsn;
      Fn[(e * 2 + 1) * 3 + c] = outc(fsn);
    }
  } else {
    S ut[3];
    for (int c = 0; c < 3; ++c) ut[c] = uu[c][n - 1];
    if (Pc.bc_mode == 1) {
      S ub[3], Fb[3][1], Sb[3], sm, se;
      boundary_state<1, S>(Pc, ut, ub);
      const double x = r0 + h;
      flux_source<1, S, XP & kXpComp>(Pc, ub, qhi, &x, 0.0, Fb, Sb, false);
      sigma<1, S, XP & kXpComp>(Pc, ub, sm, se, x);
      for (int c = 0; c < 3; ++c) {
        const S sg = (c == 0) ? S(T(Pc.lam)) : (c == 2 ? se : sm);
        Rl[c][n - 1] = Rl[c][n - 1] + ((Fhi[c] - Fb[c][0]) - sg * (ut[c] - ub[c])) * T(lfac);
      }
    } else {
      // adiabatic, zero normal stress, open, with the penalty lambda U on the momentum
      S Fi[3][1];
      flux_inviscid<1, S, XP & kXpComp>(Pc, ut, Fi, r0 + h);
      for (int c = 0; c < 3; ++c) {
        S fd = Fhi[c] - Fi[c][0];
        if (c == 1) fd = fd - T(Pc.lam) * ut[1];
        Rl[c][n - 1] = Rl[c][n - 1] + fd * T(lfac);
      }
    }
  }
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) R[off + c * n + i] = outc(Rl[c][i]);
}

// The over-integrated variant of pass 1 (mesh option "column_quadrature" 1): the weak form of
// eq. (DGformulation) with the volume integrals taken by nq = p + 2 Gauss points and the exact
// mass matrix,
//   J M q = M D u + e_end (u_hat - u) n                      (u is polynomial: exact)
//   J M R = sum_g w_g [F(u_g, q_g) l'(x_g) + J s(u_g, q_g) l(x_g)] - e_end F_hat.n
// so every face term reaches all nodes through the columns of M^-1. The traces sent to the
// neighbours (F.n of this side at the end nodes) and the boundary fluxes are those of the
// collocated pass.
template <int P, class S, int XP = 0, class SU, class TV, class OT>
__device__ __forceinline__ void col_elem_pass1_oi(const ColElem& ce, const PhysC& Pc, const GllC& gc, const QuadC& qc,
                                                  double t, const SU* __restrict__ u, const TV* __restrict__ v,
                                                  OT* __restrict__ R, OT* __restrict__ Fn) {
  typedef typename Base<S>::type T;
  constexpr int n = P + 1, nq = P + 2;
  const double* D = gc.D;
  const int64_t off = ce.off;
  const double r0 = ce.r0, h = ce.h;
  const double Jac = 0.5 * h, invJ = 1.0 / Jac;
  const bool hp = ce.off_prev >= 0, hn = ce.off_next >= 0;
  const int64_t e = ce.fslot;
  S uu[3][n];
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) uu[c][i] = Io<S>::ld(u, v, off + c * n + i);
  S dlo[3], dhi[3];
  {
    S u0[3], ub[3];
    for (int c = 0; c < 3; ++c) u0[c] = uu[c][0];
    if (hp) {
      for (int c = 0; c < 3; ++c) dlo[c] = T(0.5) * (Io<S>::ld(u, v, ce.off_prev + c * n + (n - 1)) - u0[c]);
    } else {
      boundary_state<1, S>(Pc, u0, ub);
      for (int c = 0; c < 3; ++c) dlo[c] = ub[c] - u0[c];
    }
    for (int c = 0; c < 3; ++c) u0[c] = uu[c][n - 1];
    if (hn) {
      for (int c = 0; c < 3; ++c) dhi[c] = T(0.5) * (Io<S>::ld(u, v, ce.off_next + c * n) - u0[c]);
    } else if (Pc.bc_mode == 1) {
      boundary_state<1, S>(Pc, u0, ub);
      for (int c = 0; c < 3; ++c) dhi[c] = ub[c] - u0[c];
    } else {
      for (int c = 0; c < 3; ++c) dhi[c] = S(T(0));
    }
  }
  // gradient at the nodes: D u / J plus the lifts of both faces through M^-1
  S qq[3][n];
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) {
      S g = S(T(0));
      for (int l = 0; l < n; ++l) g = g + uu[c][l] * T(D[i * n + l]);
      g = g + dhi[c] * T(qc.Mi[i * n + (n - 1)]) - dlo[c] * T(qc.Mi[i * n]);
      qq[c][i] = g * T(invJ);
    }
  // volume and source integrals at the Gauss points
  S rr[3][n];
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) rr[c][i] = S(T(0));
  // the Gauss loop stays rolled: fully unrolled, the dual-number (FP64 J v) instantiation at
  // p = 3 returned non-finite values on gfx950 while the same source built for the host and the
  // p = 2 and p = 4 instantiations were exact; rolled it matches the oracle's complex step
#pragma unroll 1
  for (int gq = 0; gq < nq; ++gq) {
    S ug[3], qg[3][1], Fg[3][1], Sg[3];
    for (int c = 0; c < 3; ++c) {
      S a = S(T(0)), b = S(T(0));
      for (int j = 0; j < n; ++j) {
        a = a + uu[c][j] * T(qc.V[gq * n + j]);
        b = b + qq[c][j] * T(qc.V[gq * n + j]);
      }
      ug[c] = a;
      qg[c][0] = b;
    }
    const double x = r0 + 0.5 * (qc.x[gq] + 1.0) * h;
    const double Q = heating<1>(Pc, &x, t);
    flux_source<1, S, XP>(Pc, ug, qg, &x, Q, Fg, Sg);
    for (int c = 0; c < 3; ++c)
      for (int i = 0; i < n; ++i)
        rr[c][i] = rr[c][i] + Fg[c][0] * T(qc.w[gq] * qc.Dg[gq * n + i]) + Sg[c] * T(qc.w[gq] * Jac * qc.V[gq * n + i]);
  }
  // face terms: -F_hat.n at the end node of each face (projected below)
  S flo[3], fhi[3];
  {
    S u0[3], q0[3][1], F0[3][1];
    for (int c = 0; c < 3; ++c) {
      u0[c] = uu[c][0];
      q0[c][0] = qq[c][0];
    }
    const double x = r0;
    if (hp) {
      // own half of the central flux; the trace F.n (n = -1) goes to the neighbour
      S S0[3];
      flux_source<1, S, XP & kXpComp>(Pc, u0, q0, &x, 0.0, F0, S0, false);
      for (int c = 0; c < 3; ++c) {
        const S fsn = -F0[c][0];
        flo[c] = -T(0.5) * fsn;
        Fn[(e * 2 + 0) * 3 + c] = outc(fsn);
      }
    } else {
      S ub[3], Sb[3], sm, se;
      boundary_state<1, S>(Pc, u0, ub);
      flux_source<1, S, XP & kXpComp>(Pc, ub, q0, &x, 0.0, F0, Sb, false);
      sigma<1, S, XP & kXpComp>(Pc, ub, sm, se, x);
      for (int c = 0; c < 3; ++c) {
        const S sg = (c == 0) ? S(T(Pc.lam)) : (c == 2 ? se : sm);
        flo[c] = F0[c][0] - sg * (u0[c] - ub[c]);        // -F_hat.n, n = -1
      }
    }
    for (int c = 0; c < 3; ++c) {
      u0[c] = uu[c][n - 1];
      q0[c][0] = qq[c][n - 1];
    }
    const double x1 = r0 + h;
    if (hn) {
      S S0[3];
      flux_source<1, S, XP & kXpComp>(Pc, u0, q0, &x1, 0.0, F0, S0, false);
      for (int c = 0; c < 3; ++c) {
        const S fsn = F0[c][0];
        fhi[c] = -T(0.5) * fsn;
        Fn[(e * 2 + 1) * 3 + c] = outc(fsn);
      }
    } else if (Pc.bc_mode == 1) {
      S ub[3], Sb[3], sm, se;
      boundary_state<1, S>(Pc, u0, ub);
      flux_source<1, S, XP & kXpComp>(Pc, ub, q0, &x1, 0.0, F0, Sb, false);
      sigma<1, S, XP & kXpComp>(Pc, ub, sm, se, x1);
      for (int c = 0; c < 3; ++c) {
        const S sg = (c == 0) ? S(T(Pc.lam)) : (c == 2 ? se : sm);
        fhi[c] = -(F0[c][0] + sg * (u0[c] - ub[c]));
      }
    } else {
      // adiabatic, zero normal stress, open, with the penalty lambda U on the momentum
      flux_inviscid<1, S, XP & kXpComp>(Pc, u0, F0, x1);
      for (int c = 0; c < 3; ++c) fhi[c] = -F0[c][0];
      fhi[1] = fhi[1] - T(Pc.lam) * u0[1];
    }
  }
  for (int c = 0; c < 3; ++c) {
    rr[c][0] = rr[c][0] + flo[c];
    rr[c][n - 1] = rr[c][n - 1] + fhi[c];
  }
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < n; ++i) {
      S r = S(T(0));
      for (int j = 0; j < n; ++j) r = r + rr[c][j] * T(qc.Mi[i * n + j]);
      R[off + c * n + i] = outc(r * T(invJ));
    }
}

// OI: the face term reaches every node through the column of M^-1 of its end node (the
// over-integrated residual); otherwise the end node alone, with the collocated 1/(w_end J)
template <int P, class S, int XP, bool OI = false, class SU, class TV, class OT>
__device__ __forceinline__ void col_elem_pass2(const ColElem& ce, const PhysC& Pc, const GllC& gc, const QuadC& qc,
                                               const SU* __restrict__ u, const TV* __restrict__ v,
                                               const OT* __restrict__ Fn, OT* __restrict__ R) {
  typedef typename Base<S>::type T;
  constexpr int n = P + 1;
  const double w_end = gc.w[0];
  const int64_t off = ce.off;
  const double lfac = 1.0 / (w_end * 0.5 * ce.h);
  const double invJ = 1.0 / (0.5 * ce.h);
  for (int side = 0; side < 2; ++side) {
    const int64_t o2 = side ? ce.off_next : ce.off_prev;
    if (o2 < 0) continue;
    const int64_t nb = side ? ce.fslot_next : ce.fslot_prev;
    const int i = side ? n - 1 : 0;
    const int inb = side ? 0 : n - 1;
    S ui[3], uh[3];
    for (int c = 0; c < 3; ++c) {
      ui[c] = Io<S>::ld(u, v, off + c * n + i);
      uh[c] = T(0.5) * (ui[c] + Io<S>::ld(u, v, o2 + c * n + inb));
    }
    S sm, se;
    sigma<1, S, XP & kXpComp>(Pc, uh, sm, se, side ? ce.r0 + ce.h : ce.r0);
    for (int c = 0; c < 3; ++c) {
      const S sg = (c == 0) ? S(T(Pc.lam)) : (c == 2 ? se : sm);
      const OT fnb = Fn[(nb * 2 + (1 - side)) * 3 + c];
      const OT term = OT(0.5) * fnb - outc(sg * (ui[c] - uh[c]));
      if constexpr (OI) {
        for (int r = 0; r < n; ++r) R[off + c * n + r] += OT(qc.Mi[r * n + i] * invJ) * term;
      } else {
        R[off + c * n + i] += OT(lfac) * term;
      }
    }
  }
}

__device__ inline ColElem col_elem_of(const ColDev& C, int e) {
  ColElem ce;
  ce.off = C.off[e];
  const int ep = C.prev[e], en = C.next[e];
  ce.off_prev = ep >= 0 ? C.off[ep] : -1;
  ce.off_next = en >= 0 ? C.off[en] : -1;
  ce.r0 = C.geo[2 * e];
  ce.h = C.geo[2 * e + 1];
  ce.fslot = e;
  ce.fslot_prev = ep;
  ce.fslot_next = en;
  return ce;
}

template <int P, class S, class SU, class TV, class OT, int XP = 0, bool OI = false>
__global__ __launch_bounds__(128) void col_pass1(ColDev C, const int* __restrict__ elist, int ne, PhysC ph, GllC gc,
                                                 QuadC qc, double t, const SU* __restrict__ u,
                                                 const TV* __restrict__ v, OT* __restrict__ R, OT* __restrict__ Fn) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ne) return;
  const int e = elist[idx];
  if constexpr (OI)
    col_elem_pass1_oi<P, S, XP>(col_elem_of(C, e), column_phys(C, ph, C.col[e]), gc, qc, t, u, v, R, Fn);
  else
    col_elem_pass1<P, S, XP>(col_elem_of(C, e), column_phys(C, ph, C.col[e]), gc, t, u, v, R, Fn);
}

template <int P, class S, class SU, class TV, class OT, int XP = 0, bool OI = false>
__global__ __launch_bounds__(128) void col_pass2(ColDev C, const int* __restrict__ elist, int ne, PhysC ph, GllC gc,
                                                 QuadC qc, const SU* __restrict__ u, const TV* __restrict__ v,
                                                 const OT* __restrict__ Fn, OT* __restrict__ R) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ne) return;
  const int e = elist[idx];
  col_elem_pass2<P, S, XP, OI>(col_elem_of(C, e), column_phys(C, ph, C.col[e]), gc, qc, u, v, Fn, R);
}

template <class S, class SU, class TV, class OT>
static dg_status_t launch_cols(dg_mesh_s* m, double t, const SU* u, const TV* v, OT* out, OT* fn, hipStream_t s,
                               int prof_base) {
  ColDev C = m->cols();
  ProfScope ps(m, prof_base, s);
  const GllC gc[3] = {make_gllc(2), make_gllc(3), make_gllc(4)};
  const QuadC qc[3] = {make_quadc(2), make_quadc(3), make_quadc(4)};
  const bool oi = m->col_quad == 1;
  PhysC ph = m->phys;
  sun_direction(ph, t);
  for (int pi = 0; pi < 3; ++pi) {
    const int ne = m->plist_n[pi];
    if (!ne) continue;
    const int blocks = (ne + 127) / 128;
    const int* el = m->d_plist[pi];
#define DG_COL_P1(P_, G_, Q_)                                                                              \
  if (oi) {                                                                                               \
    if (ph.xp_mode() == (kXpEuv | kXpComp))                                                               \
      col_pass1<P_, S, SU, TV, OT, kXpEuv | kXpComp, true><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, t, u, v, out, fn); \
    else if (ph.xp_mode() == kXpEuv)                                                                      \
      col_pass1<P_, S, SU, TV, OT, kXpEuv, true><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, t, u, v, out, fn); \
    else                                                                                                  \
      col_pass1<P_, S, SU, TV, OT, 0, true><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, t, u, v, out, fn); \
  } else if (ph.xp_mode() == (kXpEuv | kXpComp))                                                          \
    col_pass1<P_, S, SU, TV, OT, kXpEuv | kXpComp><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, t, u, v, out, fn); \
  else if (ph.xp_mode() == kXpEuv)                                                                        \
    col_pass1<P_, S, SU, TV, OT, kXpEuv><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, t, u, v, out, fn);  \
  else                                                                                                    \
    col_pass1<P_, S, SU, TV, OT><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, t, u, v, out, fn);
    switch (pi + 2) {
      case 2: DG_COL_P1(2, gc[0], qc[0]); break;
      case 3: DG_COL_P1(3, gc[1], qc[1]); break;
      default: DG_COL_P1(4, gc[2], qc[2]); break;
    }
#undef DG_COL_P1
  }
  for (int pi = 0; pi < 3; ++pi) {
    const int ne = m->plist_n[pi];
    if (!ne) continue;
    const int blocks = (ne + 127) / 128;
    const int* el = m->d_plist[pi];
#define DG_COL_P2(P_, G_, Q_)                                                                              \
  if (oi) {                                                                                               \
    if (ph.comp)                                                                                          \
      col_pass2<P_, S, SU, TV, OT, kXpComp, true><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, u, v, fn, out); \
    else                                                                                                  \
      col_pass2<P_, S, SU, TV, OT, 0, true><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, u, v, fn, out);   \
  } else if (ph.comp)                                                                                     \
    col_pass2<P_, S, SU, TV, OT, kXpComp><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, u, v, fn, out);       \
  else                                                                                                    \
    col_pass2<P_, S, SU, TV, OT><<<blocks, 128, 0, s>>>(C, el, ne, ph, G_, Q_, u, v, fn, out);
    switch (pi + 2) {
      case 2: DG_COL_P2(2, gc[0], qc[0]); break;
      case 3: DG_COL_P2(3, gc[1], qc[1]); break;
      default: DG_COL_P2(4, gc[2], qc[2]); break;
    }
#undef DG_COL_P2
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

// modal filter of every column element (one thread per element and field), in place
template <int P>
__global__ __launch_bounds__(128) void col_filter(ColDev C, const int* __restrict__ elist, int ne, FiltC f,
                                                  double* __restrict__ u) {
  constexpr int n = P + 1;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * ne) return;
  const int e = elist[idx / 3];
  double* x = u + C.off[e] + (idx % 3) * n;
  double y[n];
  for (int a = 0; a < n; ++a) {
    y[a] = 0.0;
    for (int i = 0; i < n; ++i) y[a] += f.F[a * n + i] * x[i];
  }
  for (int a = 0; a < n; ++a) x[a] = y[a];
}

dg_status_t col_filter_apply(dg_mesh_s* m, double sigma, double* u, hipStream_t s) {
  ColDev C = m->cols();
  for (int pi = 0; pi < 3; ++pi) {
    const int ne = m->plist_n[pi];
    if (!ne) continue;
    const int blocks = (3 * ne + 127) / 128;
    const int* el = m->d_plist[pi];
    const FiltC f = make_filter(pi + 2, sigma);
    switch (pi + 2) {
      case 2: col_filter<2><<<blocks, 128, 0, s>>>(C, el, ne, f, u); break;
      case 3: col_filter<3><<<blocks, 128, 0, s>>>(C, el, ne, f, u); break;
      default: col_filter<4><<<blocks, 128, 0, s>>>(C, el, ne, f, u); break;
    }
  }
  DG_HIP_CHECK(hipGetLastError());
  return DG_OK;
}

dg_status_t col_residual(dg_mesh_s* m, double t, const double* u, double* r, hipStream_t s) {
  return launch_cols<double, double, double, double>(m, t, u, (const double*)nullptr, r, m->d_fn64, s, 6);
}
dg_status_t col_residual_traces(dg_mesh_s* m, double t, const double* u, double* r, double* fn, hipStream_t s) {
  return launch_cols<double, double, double, double>(m, t, u, (const double*)nullptr, r, fn, s, 6);
}
dg_status_t col_jvp64(dg_mesh_s* m, double t, const double* u, const double* v, double* jv, hipStream_t s) {
  return launch_cols<Dual<double>, double, double, double>(m, t, u, v, jv, m->d_fn64, s, 7);
}
dg_status_t col_jvp32(dg_mesh_s* m, double t, const double* u, const float* v, float* jv, hipStream_t s) {
  return launch_cols<Dual<float>, double, float, float>(m, t, u, v, jv, m->d_fn32, s, 8);
}


// ======================================================================== batched columns
// Many independent columns advanced by n_steps DIRK steps in ONE persistent launch.
// Every 64-thread workgroup (one wavefront) pops column ids from an atomic queue
// ordered by decreasing cost and runs the whole time loop of that column:
//  * stage equations G_i(U) = U - dt a_ii R(U) - b_i = 0 solved by Newton;
//  * the Jacobian of R is block tridiagonal in 1D (the LDG lift is collocated at
//    the face node, so R of an element depends on its own and its two neighbours'
//    states only); it is assembled exactly by 3-colour probing with dual numbers
//    (3 * 3(p+1) directional derivatives), then I - dt a_ii J is factored by block
//    LU (Gauss-Jordan inverses of the diagonal blocks, partial pivoting);
//  * a_ii is the same for every stage (singly diagonal), so one factorization per
//    step serves the chord-Newton iterations of all stages; it is refreshed at the
//    current iterate when a stage stalls.
// The converged stage solutions are those of the implicit step; only the iteration
// path differs from GMRES.
namespace {

struct ColBatch {
  int n_col;
  const int* order;
  int* counter;
  const int* col_E;
  const int* col_p;
  const int64_t* col_off;
  const int* col_e0;
  const double* geo;
  const double* cpar;
  const double* euv;
  double* u;
  double t0, dt;
  int n_steps, n_stages;
  double A[3][3], c[3];
  int max_newton;
  double rtol;
  double* ws;
  int64_t ws_stride;
  int max_dof;
  int* newton_total;
  int* status;
  int* jac_builds;
  int filter;          // 1: modal filter after every step
  FiltC filt[3];       // for p = 2, 3, 4
  int jac_every;       // the chord Jacobian is rebuilt at the start of every jac_every-th step
  double jac_slow;     // ... within a stage when an iteration reduces |G| by less than this factor
  int jac_stale;       // ... at the next step when a stage needed more than this many iterations
  const QuadC* quad;   // Gauss tables of degrees 2, 3, 4 (over-integrated residual)
};

// The lane index for the batched-column functions, opaque to the optimiser. Everything a
// function derives from it (element offsets, shuffle addresses) is then formed where it is
// used; derived from threadIdx.x directly, those values are hoisted to the kernel's entry,
// live across the residual passes and spilled (the persistent kernel runs at its register
// limit), and every reload from scratch inside a chain of small steps waits for all
// outstanding memory operations.
__device__ __forceinline__ int wlane() {
  int l = threadIdx.x;
  __asm__ __volatile__("" : "+v"(l));
  return l;
}
// x from lane (lane ^ off) of the wavefront
__device__ __forceinline__ double wshfl_xor(double x, int lane, int off) {
  const int idx = (lane ^ off) << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(idx, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(idx, __double2hiint(x));
  return __hiloint2double(hi, lo);
}
__device__ inline double wave_allsum(double x) {
  const int lane = wlane();
  for (int off = 32; off > 0; off >>= 1) x += wshfl_xor(x, lane, off);
  return x;
}

// (not inlined, as the Jacobian build below and the substitution: each gets a register
// allocation of its own; inlined, the kernel's one allocation spilled across all of them)
template <int P, class S, class TV, class OT, int XP, bool OI>
__device__ __attribute__((noinline)) void colw_residual(const ColBatch& B, int E, int e0, const PhysC& Pc, const GllC& gc, double t,
                              const double* u, const TV* v, OT* out, OT* fn) {
  constexpr int b = 3 * (P + 1);
  const int lane = wlane();
  const QuadC& qc = B.quad[P - 2];
  for (int el = lane; el < E; el += 64) {
    ColElem ce;
    ce.off = (int64_t)el * b;
    ce.off_prev = el > 0 ? (int64_t)(el - 1) * b : -1;
    ce.off_next = el < E - 1 ? (int64_t)(el + 1) * b : -1;
    ce.r0 = B.geo[2 * (e0 + el)];
    ce.h = B.geo[2 * (e0 + el) + 1];
    ce.fslot = el;
    ce.fslot_prev = el - 1;
    ce.fslot_next = el + 1;
    if constexpr (OI)
      col_elem_pass1_oi<P, S, XP>(ce, Pc, gc, qc, t, u, v, out, fn);
    else
      col_elem_pass1<P, S, XP>(ce, Pc, gc, t, u, v, out, fn);
  }
  __syncthreads();
  for (int el = lane; el < E; el += 64) {
    ColElem ce;
    ce.off = (int64_t)el * b;
    ce.off_prev = el > 0 ? (int64_t)(el - 1) * b : -1;
    ce.off_next = el < E - 1 ? (int64_t)(el + 1) * b : -1;
    ce.r0 = B.geo[2 * (e0 + el)];
    ce.h = B.geo[2 * (e0 + el) + 1];
    ce.fslot = el;
    ce.fslot_prev = el - 1;
    ce.fslot_next = el + 1;
    col_elem_pass2<P, S, XP, OI>(ce, Pc, gc, qc, u, v, fn, out);
  }
  __syncthreads();
}

// The whole-column vector steps below take kVec entries per lane at a time and form all of
// them (every load issued) before storing any, so the loads' latencies overlap; one entry at a
// time, each store waits on its own loads and a 3840-entry column costs 60 such round trips
// per step. Indices past nd are clamped to nd - 1 and their values dropped.
constexpr int kVec = 4;

// Y[i] = f(i) for i < nd. Y may be an array that f reads at index i: every entry a lane
// stores is one it alone reads, before the store (a clamped read of entry nd - 1 by another
// lane is dropped).
template <class F>
__device__ __forceinline__ void colw_map(int nd, double* Y, F f) {
  for (int i0 = wlane(); i0 < nd; i0 += 64 * kVec) {
    double v[kVec];
#pragma unroll
    for (int k = 0; k < kVec; ++k) v[k] = f(min(i0 + 64 * k, nd - 1));
    // keeps the loads ahead of the stores' branches (otherwise each is sunk into its own)
#pragma unroll
    for (int k = 0; k < kVec; ++k) __asm__("" : "+v"(v[k]));
#pragma unroll
    for (int k = 0; k < kVec; ++k)
      if (i0 + 64 * k < nd) Y[i0 + 64 * k] = v[k];
  }
}

// G = U - ca R - Bv, stored negated (-G is the right-hand side of the Newton correction);
// returns |G|^2 (all lanes; each lane sums its entries in index order)
__device__ inline double colw_stage_residual(int nd, const double* U, const double* R, double ca, const double* Bv,
                                             double* mG) {
  double acc = 0;
  for (int i0 = wlane(); i0 < nd; i0 += 64 * kVec) {
    double g[kVec];
#pragma unroll
    for (int k = 0; k < kVec; ++k) {
      const int i = min(i0 + 64 * k, nd - 1);
      g[k] = U[i] - ca * R[i] - Bv[i];
    }
#pragma unroll
    for (int k = 0; k < kVec; ++k) __asm__("" : "+v"(g[k]));
#pragma unroll
    for (int k = 0; k < kVec; ++k)
      if (i0 + 64 * k < nd) {
        mG[i0 + 64 * k] = -g[k];
        acc += g[k] * g[k];
      }
  }
  __syncthreads();
  return wave_allsum(acc);
}

// in-place inverse of a b x b block (row-major) by Gauss-Jordan with partial pivoting
template <int b>
__device__ __forceinline__ void colw_invert(double* blk, double (*M)[2 * b], double* fac, int* piv_s) {
  const int lane = wlane();
  for (int idx = lane; idx < b * 2 * b; idx += 64) {
    const int r = idx / (2 * b), c = idx % (2 * b);
    M[r][c] = c < b ? blk[r * b + c] : (c - b == r ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    if (lane == 0) {
      int piv = k;
      double best = fabs(M[k][k]);
      for (int r = k + 1; r < b; ++r)
        if (fabs(M[r][k]) > best) {
          best = fabs(M[r][k]);
          piv = r;
        }
      *piv_s = piv;
    }
    __syncthreads();
    const int piv = *piv_s;
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
    if (lane < b) fac[lane] = M[lane][k];
    __syncthreads();
    for (int idx = lane; idx < b * 2 * b; idx += 64) {
      const int r = idx / (2 * b), c = idx % (2 * b);
      if (r != k) M[r][c] -= fac[r] * M[k][c];
    }
    __syncthreads();
  }
  for (int idx = lane; idx < b * b; idx += 64) blk[idx] = M[idx / b][b + idx % b];
  __syncthreads();
}

// Probing: elements of one colour are perturbed together. The collocated residual of an
// element depends on its own and its two neighbours' states (3 colours separate them; the
// Jacobian is block tridiagonal); the over-integrated one also on the states two elements
// away (its neighbours' gradients take their far faces' traces through M^-1), so 5 colours
// keep every response apart and the Jacobian is block pentadiagonal (Lo2, Up2 hold the blocks
// two elements away).
// Block LU, A = L (I + W), without pivoting between blocks (partial pivoting inside each
// diagonal block's inverse): per element e, in order,
//   L2_e = A_{e,e-2},  L1_e = A_{e,e-1} - L2_e W1_{e-2},
//   S_e = A_ee - L1_e W1_{e-1} - L2_e W2_{e-2},
//   W1_e = S_e^-1 (A_{e,e+1} - L1_e W2_{e-1}),  W2_e = S_e^-1 A_{e,e+2};
// in place: Lo = L1, Di = S^-1, Up = W1, Lo2 = L2, Up2 = W2. Without the far blocks
// (collocated) the same recurrence is the block-tridiagonal LU.
template <int P, int XP, bool OI>
__device__ __attribute__((noinline)) void colw_build_and_factor(const ColBatch& B, int E, int e0, const PhysC& Pc, const GllC& gc, double t,
                                      double ca, const double* U, double* V, double* Jv, double* fnT, double* Lo,
                                      double* Di, double* Up, double* Lo2, double* Up2) {
  constexpr int b = 3 * (P + 1);
  constexpr int bb = b * b;
  const int lane = wlane();
  const int nd = E * b;
  __shared__ double M[b][2 * b];
  __shared__ double fac[b];
  __shared__ double tmp[bb];
  __shared__ int piv_s;
  constexpr int NCOL = OI ? 5 : 3;
  constexpr int BW = OI ? 2 : 1;   // block bandwidth
  for (int kap = 0; kap < NCOL; ++kap)
    for (int l = 0; l < b; ++l) {
      for (int i = lane; i < nd; i += 64) V[i] = (((i / b) % NCOL == kap) && (i % b == l)) ? 1.0 : 0.0;
      __syncthreads();
      colw_residual<P, Dual<double>, double, double, XP, OI>(B, E, e0, Pc, gc, t, U, V, Jv, fnT);
      for (int idx = lane; idx < E * b; idx += 64) {
        const int ep = idx / b, r = idx % b;
        for (int d = -BW; d <= BW; ++d) {
          const int e = ep + d;
          if (e < 0 || e >= E || e % NCOL != kap) continue;
          double* blk = (d == -2) ? Lo2 : (d == -1) ? Lo : (d == 0) ? Di : (d == 1) ? Up : Up2;
          blk[(int64_t)ep * bb + r * b + l] = (d == 0 && r == l ? 1.0 : 0.0) - ca * Jv[ep * b + r];
        }
      }
      __syncthreads();
    }
  // Dst -= A Bm (all b x b, row-major)
  auto mm_sub = [&](double* Dst, const double* A, const double* Bm) {
    for (int idx = lane; idx < bb; idx += 64) {
      const int r = idx / b, c = idx % b;
      double s = 0;
      for (int k = 0; k < b; ++k) s += A[r * b + k] * Bm[k * b + c];
      tmp[idx] = s;
    }
    __syncthreads();
    for (int idx = lane; idx < bb; idx += 64) Dst[idx] -= tmp[idx];
    __syncthreads();
  };
  // Dst = A Dst
  auto mm_left = [&](const double* A, double* Dst) {
    for (int idx = lane; idx < bb; idx += 64) {
      const int r = idx / b, c = idx % b;
      double s = 0;
      for (int k = 0; k < b; ++k) s += A[r * b + k] * Dst[k * b + c];
      tmp[idx] = s;
    }
    __syncthreads();
    for (int idx = lane; idx < bb; idx += 64) Dst[idx] = tmp[idx];
    __syncthreads();
  };
  for (int e = 0; e < E; ++e) {
    double* D = Di + (int64_t)e * bb;
    double* L1 = Lo + (int64_t)e * bb;
    if constexpr (OI) {
      if (e >= 2) mm_sub(L1, Lo2 + (int64_t)e * bb, Up + (int64_t)(e - 2) * bb);
    }
    if (e > 0) mm_sub(D, L1, Up + (int64_t)(e - 1) * bb);
    if constexpr (OI) {
      if (e >= 2) mm_sub(D, Lo2 + (int64_t)e * bb, Up2 + (int64_t)(e - 2) * bb);
    }
    colw_invert<b>(D, M, fac, &piv_s);
    if (e < E - 1) {
      double* W1 = Up + (int64_t)e * bb;
      if constexpr (OI) {
        if (e >= 1) mm_sub(W1, L1, Up2 + (int64_t)(e - 1) * bb);
      }
      mm_left(D, W1);
    }
    if constexpr (OI) {
      if (e < E - 2) mm_left(D, Up2 + (int64_t)e * bb);
    }
  }
}

// solve (I - ca J) X = rhs with the factored blocks; rhs in X on entry. BW2: block bandwidth
// two (the over-integrated residual; Lo2, Up2 used), otherwise one:
//   forward  y_e = S_e^-1 (r_e - L1_e y_{e-1} - L2_e y_{e-2}),
//   backward x_e = y_e - W1_e x_{e+1} - W2_e x_{e+2}.
// The substitution is a chain over the elements, so the chain itself stays in LDS: row r of
// a block belongs to the four lanes 4r..4r+3 (columns q, q + 4, ... of lane q; their partial
// products are summed across the four lanes), the latest two solutions are in LDS for the
// next elements, each also goes to X for the backward sweep. The block rows and right-hand
// sides of the next PF elements are in flight while one is worked on: a ring of PF register
// slots, refilled right after use, the loads issued unconditionally (clamped to the last
// element) so that the wait for one slot never covers the younger ones. Only LDS ordering is
// needed between the steps (one wavefront); global memory is fenced at the end. Not inlined:
// the ring gets registers of its own instead of sharing the kernel's spilled budget (the
// pointers are then marked global again, or their loads would be flat ones, which every wait
// for an LDS result would also wait for).
typedef const double __attribute__((address_space(1))) gcdouble;
typedef double __attribute__((address_space(1))) gdouble;
template <int P, bool BW2>
__device__ __attribute__((noinline)) void colw_solve(int E, const double* Lo_, const double* Di_, const double* Up_,
                                                     const double* Lo2_, const double* Up2_, double* X_) {
  gcdouble* Lo = (gcdouble*)Lo_;
  gcdouble* Di = (gcdouble*)Di_;
  gcdouble* Up = (gcdouble*)Up_;
  gcdouble* Lo2 = (gcdouble*)Lo2_;
  gcdouble* Up2 = (gcdouble*)Up2_;
  gdouble* X = (gdouble*)X_;
  constexpr int b = 3 * (P + 1);
  constexpr int bb = b * b;
  constexpr int NQ = (b + 3) / 4;   // columns per lane
  constexpr int PF = (P == 4 && BW2) ? 3 : 4;   // elements in flight (the largest blocks: 3, to stay in registers)
  const int lane = wlane();
  const int r = lane >> 2, q = lane & 3;
  const bool row = r < b;
  const int rr = row ? r : 0;       // (lanes past the block's rows load row 0 and use none of it)
  __shared__ double s_x[b], s_x2[b], s_v[b];
  auto seg = [&](gcdouble* blk, double (&o)[NQ]) {
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
      const int k = q + 4 * t;
      o[t] = blk[rr * b + (k < b ? k : b - 1)];
    }
  };
  auto dot4 = [&](const double (&a)[NQ], const double* x) {
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
      const int k = q + 4 * t;
      if (row && k < b) acc += a[t] * x[k];
    }
    acc += wshfl_xor(acc, lane, 1);
    acc += wshfl_xor(acc, lane, 2);
    return acc;
  };
  // forward: slot d holds element e0 + d's L1, S^-1, L2 rows and right-hand side
  {
    double Lr[PF][NQ], Dr[PF][NQ], L2r[PF][NQ], rv[PF];
    auto fetch = [&](int e, int d) {
      e = e < E ? e : E - 1;
      seg(Lo + (int64_t)e * bb, Lr[d]);
      seg(Di + (int64_t)e * bb, Dr[d]);
      if constexpr (BW2) seg(Lo2 + (int64_t)e * bb, L2r[d]);
      rv[d] = X[e * b + rr];
    };
#pragma unroll
    for (int d = 0; d < PF; ++d) fetch(d, d);
    for (int e0 = 0; e0 < E; e0 += PF) {
#pragma unroll
      for (int d = 0; d < PF; ++d) {
        const int e = e0 + d;
        if (e < E) {
          double v = rv[d];
          if (e > 0) v -= dot4(Lr[d], s_x);
          if constexpr (BW2) {
            if (e > 1) v -= dot4(L2r[d], s_x2);
          }
          if (row && q == 0) s_v[r] = v;
          lds_barrier();
          const double y = dot4(Dr[d], s_v);
          if (row) X[e * b + r] = y;   // (every lane of the row: each reads back its own store)
          if (row && q == 0) {
            if constexpr (BW2) s_x2[r] = s_x[r];
            s_x[r] = y;
          }
          lds_barrier();
        }
        fetch(e + PF, d);
      }
    }
  }
  // backward; s_x holds x_{E-1} = y_{E-1}; slot d holds element E - 2 - (i0 + d)'s W1, W2
  // rows and forward solution
  {
    double Wr[PF][NQ], W2r[PF][NQ], xv[PF];
    auto fetch = [&](int e, int d) {
      e = e > 0 ? e : 0;
      seg(Up + (int64_t)e * bb, Wr[d]);
      if constexpr (BW2) seg(Up2 + (int64_t)e * bb, W2r[d]);
      xv[d] = X[e * b + rr];
    };
#pragma unroll
    for (int d = 0; d < PF; ++d) fetch(E - 2 - d, d);
    for (int i0 = 0; i0 < E - 1; i0 += PF) {
#pragma unroll
      for (int d = 0; d < PF; ++d) {
        const int e = E - 2 - (i0 + d);
        if (e >= 0) {
          double x = xv[d] - dot4(Wr[d], s_x);
          if constexpr (BW2) {
            if (e + 2 < E) x -= dot4(W2r[d], s_x2);
          }
          lds_barrier();   // every lane has read s_x, s_x2
          if (row) X[e * b + r] = x;
          if (row && q == 0) {
            if constexpr (BW2) s_x2[r] = s_x[r];
            s_x[r] = x;
          }
          lds_barrier();
        }
        fetch(e - PF, d);
      }
    }
  }
  __syncthreads();   // X is read by other lanes next
}

template <int P, int XP, bool OI>
__device__ __forceinline__ void colw_run(const ColBatch& B, int col, const PhysC& ph, const GllC& gc) {
  constexpr int n = P + 1;
  constexpr int b = 3 * n;
  const int lane = wlane();
  const int E = B.col_E[col];
  const int e0 = B.col_e0[col];
  const int nd = E * b;
  PhysC Pc = ph;
  set_column_phys(Pc, B.cpar, B.euv, col);
  const bool sited = Pc.site[0] != 0.0 || Pc.site[1] != 0.0 || Pc.site[2] != 0.0;
  double* w = B.ws + (int64_t)blockIdx.x * B.ws_stride;
  const int64_t md = B.max_dof;
  double* U = w;
  double* Bv = U + 2 * md;        // (the slot at U + md is spare)
  double* un = Bv + md;
  double* X = un + md;
  double* Rc = X + md;
  double* Rs = Rc + md;           // 3 stage residuals
  double* V = Rs + 3 * md;
  double* Jv = V + md;
  double* fn = Jv + md;           // [maxE][2][3]
  double* fnT = fn + md;
  double* Lo = fnT + md;
  const int64_t blk_len = (int64_t)(md / b + 1) * b * b;
  double* Di = Lo + blk_len;
  double* Up = Di + blk_len;
  double* Lo2 = OI ? Up + blk_len : nullptr;   // block bandwidth two (over-integrated)
  double* Up2 = OI ? Lo2 + blk_len : nullptr;
  double* ug = B.u + B.col_off[col];
  colw_map(nd, un, [&](int i) { return ug[i]; });
  __syncthreads();
  const double ca = B.dt * B.A[0][0];
  int newton_total = 0, builds = 0, status = 0;
  // Chord Newton: the factored stage operator I - dt a_ii J is shared by every SDIRK stage
  // (a_ii is the same) and, with jac_every > 1, by several steps. It is rebuilt at the start
  // of every jac_every-th step, after a step in which a stage needed more than jac_stale
  // iterations, and within a stage when an iteration leaves |G| above jac_slow times its
  // previous value or 12 of the stage's iterations (6 with jac_every 1) have passed since the
  // last build. The iteration path changes, not the converged stages.
  bool stale = true;
  for (int step = 0; step < B.n_steps && status == 0; ++step) {
    const double t = B.t0 + step * B.dt;
    // chord Jacobian at the start of the step (a sited column follows the Sun's direction)
    if (stale || step % B.jac_every == 0) {
      if (sited) sun_direction_dev(Pc, t + B.c[0] * B.dt);
      colw_build_and_factor<P, XP, OI>(B, E, e0, Pc, gc, t + B.c[0] * B.dt, ca, un, V, Jv, fnT, Lo, Di, Up, Lo2,
                                       Up2);
      ++builds;
      stale = false;
    }
    int max_stage_its = 0;
    colw_map(nd, U, [&](int i) { return un[i]; });
    __syncthreads();
    for (int s = 0; s < B.n_stages && status == 0; ++s) {
      const double ti = t + B.c[s] * B.dt;
      if (sited) sun_direction_dev(Pc, ti);
      colw_map(nd, Bv, [&](int i) {
        double bv = un[i];
        for (int j = 0; j < s; ++j) bv += B.dt * B.A[s][j] * Rs[j * md + i];
        return bv;
      });
      __syncthreads();
      colw_residual<P, double, double, double, XP, OI>(B, E, e0, Pc, gc, ti, un, (const double*)nullptr, Rc, fn);
      const double ref = sqrt(colw_stage_residual(nd, un, Rc, ca, Bv, X));
      int it = 0;
      double prev = 0.0;
      int last_build = 0;   // iteration of this stage at which the Jacobian was last rebuilt
      for (;;) {
        colw_residual<P, double, double, double, XP, OI>(B, E, e0, Pc, gc, ti, U, (const double*)nullptr, Rc, fn);
        const double nG = sqrt(colw_stage_residual(nd, U, Rc, ca, Bv, X));
        if (!isfinite(nG)) {
          status = 5;
          break;
        }
        if (nG <= B.rtol * ref) break;
        if (it >= B.max_newton) {
          status = 4;
          break;
        }
        const bool slow = it > 0 && B.jac_every > 1 && nG > B.jac_slow * prev;
        if (slow || it - last_build >= (B.jac_every == 1 ? 6 : 12)) {
          colw_build_and_factor<P, XP, OI>(B, E, e0, Pc, gc, ti, ca, U, V, Jv, fnT, Lo, Di, Up, Lo2, Up2);
          ++builds;
          last_build = it;
        }
        colw_solve<P, OI>(E, Lo, Di, Up, Lo2, Up2, X);
        colw_map(nd, U, [&](int i) { return U[i] + X[i]; });
        __syncthreads();
        prev = nG;
        ++it;
      }
      newton_total += it;
      max_stage_its = max(max_stage_its, it);
      colw_map(nd, Rs + s * md, [&](int i) { return Rc[i]; });
      __syncthreads();
    }
    if (max_stage_its > B.jac_stale) stale = true;
    if (status == 0) {
      colw_map(nd, un, [&](int i) { return U[i]; });
      __syncthreads();
      if (B.filter) {
        const double* F = B.filt[P - 2].F;
        for (int k = lane; k < 3 * E; k += 64) {
          double* x = un + k * n;   // element k / 3, field k % 3
          double y[n];
          for (int a = 0; a < n; ++a) {
            y[a] = 0.0;
            for (int i = 0; i < n; ++i) y[a] += F[a * n + i] * x[i];
          }
          for (int a = 0; a < n; ++a) x[a] = y[a];
        }
        __syncthreads();
      }
    }
  }
  if (status == 0)
    colw_map(nd, ug, [&](int i) { return un[i]; });
  if (lane == 0) {
    B.newton_total[col] = newton_total;
    B.status[col] = status;
    B.jac_builds[col] = builds;
  }
  __syncthreads();
}

}  // namespace

// two waves per SIMD: 256 registers and some scratch spills beat 512 registers at one wave
// (5% on the 4096-column batch)
template <int XP, bool OI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_columns_persistent(ColBatch B, PhysC ph, GllC g2, GllC g3, GllC g4) {
  __shared__ int s_k;
  for (;;) {
    if (threadIdx.x == 0) s_k = atomicAdd(B.counter, 1);
    __syncthreads();
    const int k = s_k;
    __syncthreads();
    if (k >= B.n_col) break;
    const int col = B.order[k];
    switch (B.col_p[col]) {
      case 2: colw_run<2, XP, OI>(B, col, ph, g2); break;
      case 3: colw_run<3, XP, OI>(B, col, ph, g3); break;
      default: colw_run<4, XP, OI>(B, col, ph, g4); break;
    }
  }
}

dg_status_t columns_integrate(dg_mesh_s* m, double t0, double dt, int n_steps, double* u, const dg_solver_opts_t& o,
                              int32_t* newton_host, int32_t* status_host, hipStream_t s) {
  ColBatch B{};
  const int nc = m->n_col;
  if (!m->d_bstate) {
    std::vector<int> colE(nc), colp(nc), e0(nc);
    std::vector<int64_t> off(nc);
    int acc = 0;
    for (int c = 0; c < nc; ++c) {
      colE[c] = m->col_nelem[c];
      colp[c] = m->col_p[c];
      e0[c] = acc;
      acc += colE[c];
      off[c] = m->col_off[c];
    }
    std::vector<int> order(nc);
    for (int c = 0; c < nc; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return (double)colE[a] * (colp[a] + 1) * (colp[a] + 1) > (double)colE[b] * (colp[b] + 1) * (colp[b] + 1);
    });
    DG_HIP_CHECK(hipMalloc(&m->d_bstate, (size_t)nc * 8 * sizeof(int) + 64));
    int* base = m->d_bstate;
    DG_HIP_CHECK(hipMemcpy(base, colE.data(), nc * sizeof(int), hipMemcpyHostToDevice));
    DG_HIP_CHECK(hipMemcpy(base + nc, colp.data(), nc * sizeof(int), hipMemcpyHostToDevice));
    DG_HIP_CHECK(hipMemcpy(base + 2 * nc, e0.data(), nc * sizeof(int), hipMemcpyHostToDevice));
    DG_HIP_CHECK(hipMemcpy(base + 3 * nc, order.data(), nc * sizeof(int), hipMemcpyHostToDevice));
    DG_HIP_CHECK(hipMalloc(&m->d_coloff, nc * sizeof(int64_t)));
    DG_HIP_CHECK(hipMemcpy(m->d_coloff, off.data(), nc * sizeof(int64_t), hipMemcpyHostToDevice));
    int maxd = 0;
    for (int c = 0; c < nc; ++c) maxd = std::max(maxd, colE[c] * 3 * (colp[c] + 1));
    m->col_max_dof = maxd;
  }
  int* base = m->d_bstate;
  const int slots = std::max(1, std::min(nc, m->tune_cols_grid));
  const int64_t md = m->col_max_dof;
  const int64_t blk = (md / 9 + 1) * 15 * 15;   // generous: b >= 9 so md/b <= md/9 elements
  const int64_t stride = 14 * md + (m->col_quad ? 5 : 3) * blk + 64;   // 5 blocks per element over-integrated
  if (m->cols_ws_len < stride * slots) {
    if (m->d_cols_ws) (void)hipFree(m->d_cols_ws);
    m->d_cols_ws = nullptr;
    m->cols_ws_len = 0;
    DG_HIP_CHECK(hipMalloc(&m->d_cols_ws, (size_t)stride * slots * sizeof(double)));
    m->cols_ws_len = stride * slots;
  }
  B.n_col = nc;
  B.col_E = base;
  B.col_p = base + nc;
  B.col_e0 = base + 2 * nc;
  B.order = base + 3 * nc;
  B.newton_total = base + 4 * nc;
  B.status = base + 5 * nc;
  B.jac_builds = base + 6 * nc;
  B.counter = base + 7 * nc;
  B.col_off = m->d_coloff;
  B.geo = m->d_geo;
  B.cpar = m->d_cpar;
  B.euv = m->d_euv_cols;
  B.u = u;
  B.t0 = t0;
  B.dt = dt;
  B.n_steps = n_steps;
  B.max_newton = o.max_newton;
  B.rtol = o.newton_rtol;
  B.filter = o.filter_rate > 0 ? 1 : 0;
  for (int pi = 0; pi < 3; ++pi) B.filt[pi] = make_filter(pi + 2, std::exp(-o.filter_rate * dt));
  B.ws = m->d_cols_ws;
  B.ws_stride = stride;
  B.jac_every = m->cols_jac_every;
  B.jac_slow = 0.01 * m->cols_jac_slow_pct;
  B.jac_stale = m->cols_jac_stale;
  B.quad = m->d_quad;
  B.max_dof = (int)md;
  // DIRK tableau
  {
    double A[3][3] = {}, c[3] = {};
    if (o.scheme == 22) {
      const double g = 1.0 - 1.0 / std::sqrt(2.0);
      A[0][0] = g; A[1][0] = 1.0 - g; A[1][1] = g;
      c[0] = g; c[1] = 1.0;
      B.n_stages = 2;
    } else {
      double g = 0.4;
      for (int it = 0; it < 60; ++it) {
        const double f = ((g - 3.0) * g + 1.5) * g - 1.0 / 6.0;
        const double df = (3.0 * g - 6.0) * g + 1.5;
        g -= f / df;
      }
      A[0][0] = g; A[1][0] = 0.5 * (1.0 - g); A[1][1] = g;
      A[2][0] = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0; A[2][1] = (6.0 * g * g - 20.0 * g + 5.0) / 4.0; A[2][2] = g;
      c[0] = g; c[1] = 0.5 * (1.0 + g); c[2] = 1.0;
      B.n_stages = 3;
    }
    for (int i = 0; i < 3; ++i) {
      B.c[i] = c[i];
      for (int j = 0; j < 3; ++j) B.A[i][j] = A[i][j];
    }
  }
  DG_HIP_CHECK(hipMemsetAsync(B.counter, 0, sizeof(int), s));
  PhysC ph = m->phys;
  sun_direction(ph, t0);
  {
    ProfScope ps(m, 13, s);
    const GllC g2 = make_gllc(2), g3 = make_gllc(3), g4 = make_gllc(4);
    if (m->col_quad == 1) {
      if (ph.xp_mode() == (kXpEuv | kXpComp))
        k_columns_persistent<kXpEuv | kXpComp, true><<<slots, 64, 0, s>>>(B, ph, g2, g3, g4);
      else if (ph.xp_mode() == kXpEuv)
        k_columns_persistent<kXpEuv, true><<<slots, 64, 0, s>>>(B, ph, g2, g3, g4);
      else
        k_columns_persistent<0, true><<<slots, 64, 0, s>>>(B, ph, g2, g3, g4);
    } else if (ph.xp_mode() == (kXpEuv | kXpComp))
      k_columns_persistent<kXpEuv | kXpComp, false><<<slots, 64, 0, s>>>(B, ph, g2, g3, g4);
    else if (ph.xp_mode() == kXpEuv)
      k_columns_persistent<kXpEuv, false><<<slots, 64, 0, s>>>(B, ph, g2, g3, g4);
    else
      k_columns_persistent<0, false><<<slots, 64, 0, s>>>(B, ph, g2, g3, g4);
  }
  DG_HIP_CHECK(hipGetLastError());
  DG_HIP_CHECK(hipStreamSynchronize(s));
  if (newton_host) DG_HIP_CHECK(hipMemcpy(newton_host, B.newton_total, nc * sizeof(int), hipMemcpyDeviceToHost));
  std::vector<int> st(nc);
  DG_HIP_CHECK(hipMemcpy(st.data(), B.status, nc * sizeof(int), hipMemcpyDeviceToHost));
  if (status_host)
    for (int c = 0; c < nc; ++c) status_host[c] = st[c];
  for (int c = 0; c < nc; ++c)
    if (st[c] != 0) {
      set_error("dg_columns_integrate: column " + std::to_string(c) + " failed (status " + std::to_string(st[c]) + ")");
      return st[c] == 5 ? DG_ERR_NAN : DG_ERR_NOCONV;
    }
  return DG_OK;
}

}  // namespace dg
