// The element pass (pass 1) of R(u) and J(u)v on the cubed-sphere shell and its launch
// dispatch, shared by the translation units that instantiate it: the FP64 residual's
// instantiations are compiled on their own (shell_r64.hip), the dual-number and other
// passes with the rest of the shell kernels (shell.hip).
#pragma once
#include <type_traits>

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

// a loaded value required at this point (an empty instruction that reads and writes the
// register): the load is not sunk past it into the branch that stores the value, so the loads
// before a group of pins are issued together. Not volatile: a volatile one counts as a
// possible memory write, after which uniform loads of global data (the EUVAC table, physics
// constants) could no longer be scalar loads.
__device__ inline void pin(double& x) { __asm__("" : "+v"(x)); }
__device__ inline void pin(float& x) { __asm__("" : "+v"(x)); }
__device__ inline void pin(int& x) { __asm__("" : "+v"(x)); }
template <class T> __device__ inline void pin(Dual<T>& x) { pin(x.v); pin(x.d); }

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

// the same with the element's angular connectivity staged in LDS: cn[f] = {neighbour
// cell, its face, the along-edge index map (n entries)} of angular face f
template <int P>
__device__ inline int face_neighbour_lds(const ShellDev& M, const int (*cn)[P + 3], int cell, int k, int f, int a,
                                         int b, int cz, int& jn, int& fn, int& mn) {
  constexpr int n = P + 1, N2 = n * n;
  if (f >= 4) return face_neighbour<P>(M, cell, k, f, a, b, cz, jn, fn, mn);
  const int s = (f < 2) ? b : a;
  const int c2 = cn[f][0];
  fn = cn[f][1];
  const int s2 = cn[f][2 + s];
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

struct NodeGeo {
  int a, b, cz, ja;
  double rk, hk, rc, rp, Jac, x[3], A1[3], A2[3], A3[3];
};

// geometry of node j of an element in radial layer k (angular tables staged in LDS)
template <int P>
__device__ inline NodeGeo node_geo(const ShellDev& M, const GllC& gc, const double (*ang)[Shape<P>::N2], int k,
                                   int j) {
  constexpr int n = P + 1, N2 = n * n;
  NodeGeo g;
  g.a = j % n;
  g.b = (j / n) % n;
  g.cz = j / N2;
  g.ja = g.a + n * g.b;
  g.rk = M.edges[k];
  g.hk = M.edges[k + 1] - g.rk;
  g.rp = 0.5 * g.hk;
  g.rc = g.rk + 0.5 * (gc.x[g.cz] + 1.0) * g.hk;
  for (int d = 0; d < 3; ++d) {
    g.A1[d] = ang[d][g.ja];
    g.A2[d] = ang[3 + d][g.ja];
    g.A3[d] = ang[6 + d][g.ja];
    g.x[d] = g.rc * ang[10 + d][g.ja];
  }
  g.Jac = g.rc * g.rc * g.rp * ang[9][g.ja];
  return g;
}

// auxiliary gradient q at one node: the conservative strong form of the weak LDG
// gradient, q = (1/J) sum_a D_a(J a^a u) + sum_faces Sn (u_hat - u)/(w_end J)
template <int P, class S, class SU, class TV>
__device__ inline void node_gradient(const ShellDev& M, const PhysC& ph, const double* D, const double* xg, double w_end,
                                     const double (*ang)[Shape<P>::N2], const S (*su)[Shape<P>::N], const SU* u,
                                     const TV* v, int cell, int k, const NodeGeo& g, const S* uu, S (*q)[3]) {
  typedef typename Base<S>::type T;
  constexpr int n = P + 1, N = n * n * n, N2 = n * n;
  const int a = g.a, b = g.b, cz = g.cz, ja = g.ja;
  const double rrp = g.rc * g.rp;
  double r2[n];
  for (int i = 0; i < n; ++i) {
    const double ri = g.rk + 0.5 * (xg[i] + 1.0) * g.hk;
    r2[i] = ri * ri;
  }
  const double invJ = recip(g.Jac);
  for (int c = 0; c < 5; ++c) {
    S d1[3], d2[3], d3;
    for (int d = 0; d < 3; ++d) { d1[d] = S(T(0)); d2[d] = S(T(0)); }
    d3 = S(T(0));
    for (int i = 0; i < n; ++i) {
      const S u1 = su[c][i + n * b + N2 * cz];
      const S u2 = su[c][a + n * i + N2 * cz];
      const S u3 = su[c][ja + N2 * i];
      const double Da = D[a * n + i], Db = D[b * n + i], Dc = D[cz * n + i] * r2[i];
      for (int d = 0; d < 3; ++d) {
        d1[d] = d1[d] + u1 * T(Da * ang[d][i + n * b]);
        d2[d] = d2[d] + u2 * T(Db * ang[3 + d][a + n * i]);
      }
      d3 = d3 + u3 * T(Dc);
    }
    for (int d = 0; d < 3; ++d) q[c][d] = (T(rrp) * (d1[d] + d2[d]) + T(g.A3[d]) * d3) * T(invJ);
  }
  const double lfac = 1.0 / (w_end * g.Jac);
  for (int f = 0; f < 6; ++f) {
    const bool on = (f == 0 && a == 0) || (f == 1 && a == n - 1) || (f == 2 && b == 0) || (f == 3 && b == n - 1) ||
                    (f == 4 && cz == 0) || (f == 5 && cz == n - 1);
    if (!on) continue;
    const double side = (f & 1) ? 1.0 : -1.0;
    double Sn[3];
    for (int d = 0; d < 3; ++d)
      Sn[d] = side * (f < 2 ? rrp * g.A1[d] : (f < 4 ? rrp * g.A2[d] : g.rc * g.rc * g.A3[d]));
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
}

// node (a, b, cz) of slot m of face f (inverse of face_slot)
template <int P>
__device__ inline void slot_node(int f, int m, int& a, int& b, int& cz) {
  constexpr int n = P + 1;
  if (f < 2) {
    a = (f == 0) ? 0 : n - 1;
    b = m % n;
    cz = m / n;
  } else if (f < 4) {
    b = (f == 2) ? 0 : n - 1;
    a = m % n;
    cz = m / n;
  } else {
    cz = (f == 4) ? 0 : n - 1;
    a = m % n;
    b = m / n;
  }
}

// The interior-face stabilisation is single valued up to its sign: with
// u_hat = (u + u^-)/2 the term on this side is -|Sn| sigma(u_hat)(u - u_hat) and on the
// neighbour's side -|Sn| sigma(u_hat)(u^- - u_hat) = +|Sn| sigma(u_hat)(u - u_hat). Of
// the two elements of a face, the one with the smaller index (the face's owner)
// evaluates sigma once and folds the neighbour's share into the trace it sends, so
// the trace slot of a face node holds F.Sn - 2 Z with Z = |Sn| sigma(u_hat)(u_hat - u)
// (Z = 0 when the receiving element is the owner).

// XCD-aware order of the blocks of an element-per-block launch. The dispatcher hands
// workgroup b to accelerator die (XCD) b mod 8, each with its own L2. Renumbered, die x runs
// one contiguous range of elements in order, so an element's radial neighbours (e +- 1) and
// its angular neighbours within a panel row or two (e +- n_rad, e +- n_ang n_rad) are being
// processed on the same die at about the same time, and their face values are read from
// that die's L2 instead of from memory. A bijection of [0, G) for every grid size G.
constexpr int kXcds = 8;
__device__ inline int xcd_block(int b, int G) {
  const int q = G / kXcds, r = G % kXcds;
  const int x = b % kXcds, i = b / kXcds;
  return x * q + min(x, r) + i;
}
// the same ranges per die, each run from its end: a pass that follows the element pass
// starts on the elements whose output the die wrote last (the part still in its L2)
__device__ inline int xcd_block_reversed(int b, int G) {
  const int q = G / kXcds, r = G % kXcds;
  const int x = b % kXcds, i = b / kXcds;
  const int count = q + (x < r ? 1 : 0);
  return x * q + min(x, r) + (count - 1 - i);
}

// the r-th set bit of mask (r counted from 0)
__device__ inline int nth_bit(int mask, int r) {
  for (int i = 0; i < r; ++i) mask &= mask - 1;
  return __ffs(mask) - 1;
}

// EPB: elements per block; OCC: minimum waves per SIMD the register allocation must allow.
// RAD (dual numbers only): the radial-line linearisation of the line preconditioner. In
// the derivative parts the tangent at other angular nodes is taken as zero: across the
// angular faces (the neighbour's tangent), in the angular line sums of the gradient and
// of the divergence (only the node's own term); every element takes the stabilisation of
// its own side of the angular faces and sends no angular traces. Radial coupling is
// exact. Lines (cell, a, b) are then independent.
// XP: the extended physics the instantiation contains (kXpEuv, kXpComp; PhysC::xp_mode).
template <int P, int EPB, int OCC, class S, class SU, class TV, class OT, bool RAD = false, int XP = 0>
__global__ __launch_bounds__(Shape<P>::TPE * EPB) __attribute__((amdgpu_waves_per_eu(OCC)))
void shell_pass1(ShellDev M, PhysC ph, GllC gc, double t, const SU* __restrict__ u, const TV* __restrict__ v,
                 OT* __restrict__ R, OT* __restrict__ Fn) {
  typedef Shape<P> Sh;
  typedef typename Base<S>::type T;
  constexpr int n = Sh::n, N = Sh::N, N2 = Sh::N2, TPE = Sh::TPE;
  static_assert(3 * N <= 6 * 5 * N2, "flux staging must fit in the trace buffer");
  __shared__ double s_ang[EPB][13][N2];
  // node (a, b, cz) of a field at a + n b + NS cz: the planes padded by PL so that the line
  // reads of the gradient and divergence (16 distinct addresses per wavefront at p = 3) fall
  // in different LDS banks for the a- and b-lines (without it, four planes share each bank)
  constexpr int PL = (P == 3 && sizeof(S) == 8) ? 2 : 0;
  constexpr int NS = N2 + PL, NP = NS * n;
  __shared__ S s_u[EPB][5][NP];
  // per face slot: u_hat - u (faces 0..5), then Z of the owned faces in the order of their face
  // index (rows 6..10); phase E stages several fields' contravariant fluxes over the whole
  __shared__ S s_fz[EPB][11][5][N2];
  constexpr int kFzStride = 11 * 5 * N2;
  __shared__ int s_nb[EPB][6][N2];   // trace slot of the neighbour's matching face node
  __shared__ int s_cn[EPB][4][P + 3];  // angular connectivity: neighbour cell, its face, index map
  __shared__ double D[n * n];
  const int le = threadIdx.x / TPE;
  const int j = threadIdx.x % TPE;
  const int e = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
  const bool live = e < M.E;
  const bool active = live && (j < N);
  const int cell = live ? e / M.n_rad : 0;
  const int k = live ? e % M.n_rad : 0;
  const double w_end = gc.w[0];
  const int64_t base = (int64_t)e * 5 * N;
  // ---- phase A: the element's own data (the operator D, the angular metric terms, the
  // connectivity, the state, the layer's radii) to LDS. Every load is issued before the first
  // is stored, so that a wavefront waits for memory once (a copy loop would wait once per
  // round); lanes without a value to store read in-range addresses (element min(e, E - 1),
  // node min(j, N - 1)).
  constexpr int NA = (13 * N2 + TPE - 1) / TPE;
  constexpr int NC = 4 * (n + 2);
  static_assert(NC <= TPE, "one connectivity word per thread");
  const int ec = live ? e : M.E - 1;
  const int cc = ec / M.n_rad, kc = ec % M.n_rad;
  double ta[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) ta[i] = M.ang[(int64_t)cc * 13 * N2 + min(j + i * TPE, 13 * N2 - 1)];
  const int jw = min(j, NC - 1), cf = jw / (n + 2), cw = jw % (n + 2);
  const int* cp = cw == 0 ? M.cnbr + cc * 4 + cf : (cw == 1 ? M.cface + cc * 4 + cf : M.cmap + (cc * 4 + cf) * n + cw - 2);
  int tcn = *cp;
  S tu[5];
  const int64_t bc = (int64_t)ec * 5 * N + min(j, N - 1);
  for (int c = 0; c < 5; ++c) tu[c] = load_state<S>(u, v, bc + c * N);
  double e0 = M.edges[kc], e1 = M.edges[kc + 1];
  double tD = gc.D[min((int)threadIdx.x, n * n - 1)];
  // (D's pin first: with it last, the load of D, which reads the argument block, was issued
  // only after the waits for the others)
  pin(tD);
#pragma unroll
  for (int i = 0; i < NA; ++i) pin(ta[i]);
  pin(tcn);
  for (int c = 0; c < 5; ++c) pin(tu[c]);
  pin(e0);
  pin(e1);
  if (threadIdx.x < n * n) D[threadIdx.x] = tD;
  if (live) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = j + i * TPE;
      if (idx < 13 * N2) s_ang[le][idx / N2][idx % N2] = ta[i];
    }
    if (j < NC) s_cn[le][cf][cw] = tcn;
  }
  if (active)
    for (int c = 0; c < 5; ++c) s_u[le][c][j + PL * (j / N2)] = tu[c];
  const double rk = live ? e0 : 0.0;
  const double hk = live ? e1 - e0 : 1.0;
  lds_barrier();
  // owned interior faces (bit f): the neighbour has the larger element index
  int own = 0;
  if (live) {
    for (int f = 0; f < 4; ++f)
      if (RAD || s_cn[le][f][0] * M.n_rad + k > e) own |= 1 << f;
    if (k < M.n_rad - 1) own |= 1 << 5;
  }
  const int n_own = __popc(own);

  // ---- phase B (face-node tasks, owned faces first): numerical trace u_hat - u of every
  // face slot, the neighbour's trace slot, and Z on the owned faces. A thread holds at most
  // NTASK tasks (6 (p+1)^2 face slots over the element's threads: 2 at p = 2, 3, 4); the
  // neighbour values of all of them are requested before any is used, so the gathers of the
  // second task overlap those of the first instead of following them.
  constexpr int NTASK = (6 * N2 + TPE - 1) / TPE;
  {
    int t_f[NTASK], t_m[NTASK], t_r[NTASK], t_jo[NTASK], t_en[NTASK], t_nb[NTASK];
    S t_un[NTASK][5];
#pragma unroll
    for (int q = 0; q < NTASK; ++q) {
      const int tsk = j + q * TPE;
      t_en[q] = -2;                                   // -2: no task
      if (live && tsk < 6 * N2) {
        const int r = tsk / N2, m = tsk % N2;
        const int f = (r < n_own) ? nth_bit(own, r) : nth_bit(~own & 63, r - n_own);
        int a, b, cz;
        slot_node<P>(f, m, a, b, cz);
        int jn, fn, mn;
        const int en = face_neighbour_lds<P>(M, s_cn[le], cell, k, f, a, b, cz, jn, fn, mn);
        t_f[q] = f;
        t_m[q] = m;
        t_r[q] = r;
        t_jo[q] = a + n * b + NS * cz;
        t_en[q] = en;
        if (en >= 0) {
          t_nb[q] = (en * 6 + fn) * 5 * N2 + mn;
          for (int c = 0; c < 5; ++c) t_un[q][c] = load_state<S>(u, v, (int64_t)en * 5 * N + c * N + jn);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NTASK; ++q) {
      if (t_en[q] == -2) continue;
      const int f = t_f[q], m = t_m[q], en = t_en[q];
      S uo[5], du[5];
      for (int c = 0; c < 5; ++c) uo[c] = s_u[le][c][t_jo[q]];
      if (en >= 0) {
        for (int c = 0; c < 5; ++c) du[c] = T(0.5) * (t_un[q][c] - uo[c]);
        if constexpr (RAD) {
          if (f < 4)
            for (int c = 0; c < 5; ++c) du[c].d = T(-0.5) * uo[c].d;
        }
        s_nb[le][f][m] = t_nb[q];
      } else if (ph.bc_mode == 1 || f == 4) {
        S ub[5];
        boundary_state<3, S>(ph, uo, ub);
        for (int c = 0; c < 5; ++c) du[c] = ub[c] - uo[c];
      } else {
        for (int c = 0; c < 5; ++c) du[c] = S(T(0));   // upper boundary: u_hat = u
      }
      for (int c = 0; c < 5; ++c) s_fz[le][f][c][m] = du[c];
    }
    // Z on the owned faces, from the values this thread has just put in LDS (its own
    // slots: no barrier needed), so that the gathered values are dead before sigma
#pragma unroll
    for (int q = 0; q < NTASK; ++q) {
      if (t_en[q] < 0 || t_r[q] >= n_own) continue;
      const int f = t_f[q], m = t_m[q], r = t_r[q];
      int a, b, cz;
      slot_node<P>(f, m, a, b, cz);
      const int dd = f >> 1;
      const int ja = a + n * b;
      const double rc = rk + 0.5 * (gc.x[cz] + 1.0) * hk;
      const double fac = (dd < 2) ? rc * 0.5 * hk : rc * rc;
      const double A0 = s_ang[le][3 * dd][ja], A1 = s_ang[le][3 * dd + 1][ja], A2 = s_ang[le][3 * dd + 2][ja];
      const double Smag = fac * sqrt(A0 * A0 + A1 * A1 + A2 * A2);
      S du[5], uh[5];
      for (int c = 0; c < 5; ++c) {
        du[c] = s_fz[le][f][c][m];
        uh[c] = s_u[le][c][t_jo[q]] + du[c];
      }
      S sm, se;
      sigma<3, S, XP>(ph, uh, sm, se, rc);
      for (int c = 0; c < 5; ++c) {
        const S sg = (c == 0) ? S(T(ph.lam)) : (c == 4 ? se : sm);
        s_fz[le][6 + r][c][m] = T(Smag) * sg * du[c];
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  lds_barrier();

  // ---- phase C (node threads): gradient, pointwise flux and source, contravariant fluxes
  NodeGeo g;
  S Sr[5], G[5][3];
  const int a = j % n, b = (j / n) % n, cz = j / N2;
  if (active) {
    g = node_geo<P>(M, gc, s_ang[le], k, j);
    const double rrp = g.rc * g.rp, rc2 = g.rc * g.rc;
    const double invJ = recip(g.Jac);
    const double lfac = invJ * recip(w_end);
    // metric factors of the three directions at this node
    const double Ja[3][3] = {{rrp * g.A1[0], rrp * g.A1[1], rrp * g.A1[2]},
                             {rrp * g.A2[0], rrp * g.A2[1], rrp * g.A2[2]},
                             {rc2 * g.A3[0], rc2 * g.A3[1], rc2 * g.A3[2]}};
    // line coefficients shared by the five fields: D(a,i) J a^1(i,b), D(b,i) J a^2(a,i), D(cz,i) r_i^2
    double c1[n][3], c2[n][3], c3[n];
    for (int i = 0; i < n; ++i) {
      const double ri = rk + 0.5 * (gc.x[i] + 1.0) * hk;
      c3[i] = D[cz * n + i] * ri * ri;
      for (int d = 0; d < 3; ++d) {
        c1[i][d] = D[a * n + i] * rrp * s_ang[le][d][i + n * b];
        c2[i][d] = D[b * n + i] * rrp * s_ang[le][3 + d][a + n * i];
      }
    }
    S q[5][3];
    for (int c = 0; c < 5; ++c) {
      S g1[3], d3 = S(T(0));
      for (int d = 0; d < 3; ++d) g1[d] = S(T(0));
      for (int i = 0; i < n; ++i) {
        const S u1 = s_u[le][c][i + n * b + NS * cz];
        const S u2 = s_u[le][c][a + n * i + NS * cz];
        const S u3 = s_u[le][c][g.ja + NS * i];
        for (int d = 0; d < 3; ++d) g1[d] = g1[d] + u1 * T(c1[i][d]) + u2 * T(c2[i][d]);
        d3 = d3 + u3 * T(c3[i]);
      }
      if constexpr (RAD) {
        const T vd = s_u[le][c][j + PL * cz].d;
        for (int d = 0; d < 3; ++d) g1[d].d = vd * T(c1[a][d] + c2[b][d]);
      }
      for (int d = 0; d < 3; ++d) q[c][d] = (g1[d] + T(g.A3[d]) * d3) * T(invJ);
    }
    // lift of u_hat - u from the faces through this node
    const bool on[6] = {a == 0, a == n - 1, b == 0, b == n - 1, cz == 0, cz == n - 1};
    for (int f = 0; f < 6; ++f) {
      if (!on[f]) continue;
      const int m = face_slot<P>(f, a, b, cz);
      const double sd = ((f & 1) ? 1.0 : -1.0) * lfac;
      const int dd = f >> 1;
      for (int c = 0; c < 5; ++c) {
        const S du = s_fz[le][f][c][m];
        for (int d = 0; d < 3; ++d) q[c][d] = q[c][d] + du * T(sd * Ja[dd][d]);
      }
    }
    // the node's own state, read back from LDS here rather than held in registers through
    // the face tasks and the gradient
    S uu[5];
    for (int c = 0; c < 5; ++c) uu[c] = s_u[le][c][j + PL * cz];
    // boundary faces: the terms (F - F_hat).Sn are completed here. On the lower face (and
    // every boundary face in bc_mode 1), F_hat.Sn = F(u_b, q).Sn + |Sn| sigma(u_b)(u - u_b)
    // is taken before the node's own flux so that q need not outlive it.
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
      flux_source<3, S, XP>(ph, ub, q, g.x, 0.0, Fb, Sb, false);
      S sm, se;
      sigma<3, S, XP>(ph, ub, sm, se, g.rc);
      for (int c = 0; c < 5; ++c) {
        const S sg = (c == 0) ? S(T(ph.lam)) : (c == 4 ? se : sm);
        Bc[c] = -(Fb[c][0] * T(Sn[0]) + Fb[c][1] * T(Sn[1]) + Fb[c][2] * T(Sn[2])) - T(Smag) * sg * (uu[c] - ub[c]);
      }
    }
    const double Q = heating<3>(ph, g.x, t);
    S F[5][3];
    flux_source<3, S, XP>(ph, uu, q, g.x, Q, F, Sr);
    // the metric terms are read again from LDS rather than kept in registers across the flux
    __asm__ __volatile__("" ::: "memory");
    const double (*ang)[N2] = s_ang[le];
    if (dir || top) {
      double Sn[3];
      for (int d = 0; d < 3; ++d) Sn[d] = bside * ang[6 + d][g.ja];
      if (dir) {
        for (int c = 0; c < 5; ++c)
          Sr[c] = Sr[c] + (F[c][0] * T(Sn[0]) + F[c][1] * T(Sn[1]) + F[c][2] * T(Sn[2]) + Bc[c]) * T(lfac);
      } else {
        // adiabatic, zero normal stress, open: F_hat.Sn = F_inviscid.Sn + lambda (U.Sn) Sn/|Sn|
        // (the penalty on the normal momentum), so (F - F_hat).Sn = F_viscous.Sn - penalty
        S Fi[5][3];
        flux_inviscid<3, S, XP>(ph, uu, Fi, g.rc);
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

  // ---- phase E (node threads): interior-face terms of this side and the traces sent to
  // the neighbours, then the volume divergence one field at a time
  const double invJ = active ? recip(g.Jac) : 0.0;
  const double lfac = invJ * recip(w_end);
  if (active) {
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
        const S z = mine ? s_fz[le][6 + r][c][m] : S(T(0));
        Sr[c] = Sr[c] + (T(0.5) * Fs + z) * T(lfac);
        if (RAD && f < 4)
          Fn[(int64_t)nb + c * N2] = outp(S(T(0)));
        else
          Fn[(int64_t)nb + c * N2] = outp(Fs - T(2) * z);
      }
    }
  }
  lds_barrier();   // every u_hat - u has been read: the trace buffer becomes the flux staging
  // the divergence, FPR fields per LDS round (as many as the face-slot and Z rows hold)
  constexpr int FPR = (kFzStride / (3 * NP)) < 5 ? (kFzStride / (3 * NP)) : 5;
  static_assert(FPR >= 1, "flux staging must fit in the face-slot rows");
  S (*s_G)[3][NP] = reinterpret_cast<S (*)[3][NP]>(&s_fz[le][0][0][0]);
  for (int c0 = 0; c0 < 5; c0 += FPR) {
    if (active)
      for (int cc = 0; cc < FPR && c0 + cc < 5; ++cc)
        for (int dd = 0; dd < 3; ++dd) s_G[cc][dd][j + PL * cz] = G[c0 + cc][dd];
    lds_barrier();
    if (active)
      for (int cc = 0; cc < FPR && c0 + cc < 5; ++cc) {
        const int c = c0 + cc;
        S dv = S(T(0));
        for (int i = 0; i < n; ++i) {
          dv = dv + s_G[cc][0][i + n * b + NS * cz] * T(D[a * n + i]);
          dv = dv + s_G[cc][1][a + n * i + NS * cz] * T(D[b * n + i]);
          dv = dv + s_G[cc][2][g.ja + NS * i] * T(D[cz * n + i]);
        }
        if constexpr (RAD) {
          T dr = G[c][0].d * T(D[a * n + a]) + G[c][1].d * T(D[b * n + b]);
          for (int i = 0; i < n; ++i) dr += s_G[cc][2][g.ja + NS * i].d * T(D[cz * n + i]);
          dv.d = dr;
        }
        R[base + c * N + j] = outp(Sr[c] - dv * T(invJ));
      }
    if (c0 + FPR < 5) lds_barrier();
  }
}

// (profiled: pm->prof on, the interval goes to slot pid)
template <int P, int EPB, int OCC, class S, int XP = 0, class SU, class TV, class OT>
static void launch_p1(const ShellDev& M, const PhysC& ph, const GllC& gc, double t, const SU* u, const TV* v, OT* out,
                      OT* fn, hipStream_t s, dg_mesh_s* pm, int pid) {
  const int blocks = (M.E + EPB - 1) / EPB;
  if (pm->prof) {
    launch_timed(pm, pid, &shell_pass1<P, EPB, OCC, S, SU, TV, OT, false, XP>, dim3(blocks),
                 dim3(Shape<P>::TPE * EPB), s, M, ph, gc, t, u, v, out, fn);
    return;
  }
  shell_pass1<P, EPB, OCC, S, SU, TV, OT, false, XP><<<blocks, Shape<P>::TPE * EPB, 0, s>>>(M, ph, gc, t, u, v, out,
                                                                                             fn);
}

// pass-1 launch configurations (elements per block, minimum waves per SIMD): the
// FP64 residual and the FP32 J v take the tuned table entry of the mesh, the FP64
// J v (dual numbers) runs one element per block with a register budget for two waves
// per SIMD (left free, the allocator reaches 256 + 14 accumulation registers and one wave), and so does every pass of
// a mesh with the EUVAC heating or the variable composition (the one instantiation that
// contains them)
template <int P, class S, class SU, class TV, class OT>
static void dispatch_p1(dg_mesh_s* m, const ShellDev& M, const PhysC& ph, const GllC& gc, double t,
                        const SU* u, const TV* v, OT* out, OT* fn, hipStream_t s, int pid) {
  if (ph.xp_mode() == (kXpEuv | kXpComp)) {
    launch_p1<P, 1, 1, S, kXpEuv | kXpComp>(M, ph, gc, t, u, v, out, fn, s, m, pid);
    return;
  }
  if (ph.xp_mode() == kXpEuv) {
    launch_p1<P, 1, 1, S, kXpEuv>(M, ph, gc, t, u, v, out, fn, s, m, pid);
    return;
  }
  if constexpr (std::is_same<S, Dual<double>>::value) {
    launch_p1<P, 1, 2, S>(M, ph, gc, t, u, v, out, fn, s, m, pid);
    return;
  } else {
  constexpr int maxe = 256 / Shape<P>::TPE;
  const int cfg = m->tune_p1;
  switch (cfg) {
    case 1: launch_p1<P, 1, 1, S>(M, ph, gc, t, u, v, out, fn, s, m, pid); break;
    case 2: launch_p1<P, (maxe >= 2 ? 2 : 1), 1, S>(M, ph, gc, t, u, v, out, fn, s, m, pid); break;
    case 3: launch_p1<P, 1, 3, S>(M, ph, gc, t, u, v, out, fn, s, m, pid); break;
    case 4: launch_p1<P, (maxe >= 2 ? 2 : 1), 3, S>(M, ph, gc, t, u, v, out, fn, s, m, pid); break;
    case 5: launch_p1<P, 1, 4, S>(M, ph, gc, t, u, v, out, fn, s, m, pid); break;
    default: launch_p1<P, maxe, 1, S>(M, ph, gc, t, u, v, out, fn, s, m, pid); break;
  }
  }
}

}  // namespace dg
