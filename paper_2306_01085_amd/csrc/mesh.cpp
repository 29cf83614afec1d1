// Host-side mesh construction: GLL tables, the cubed-sphere shell with factored
// curved geometry, face connectivity, and batches of 1D radial columns.
//
// Shell geometry (section 3.3). A node of angular cell (panel, i, j), radial layer
// k sits at X = r(xi_3) * Ihat(xi_1, xi_2): Ihat is the unit vector of the
// equiangular gnomonic panel point, r is linear in xi_3 inside a layer. For this
// separable map the invariant curl form of the metric terms (Kopriva 2006)
//   J a^i_n = -1/2 e_i . curl_xi I(X_l grad X_m - X_m grad X_l),  (n,m,l) cyclic
// factors exactly into radial factors and angular tables:
//   J a^1 = r r' A1,   A1 = 2 B2
//   J a^2 = r r' A2,   A2 = -2 B1
//   J a^3 = r^2 A3,    A3 = -(d1 B2 - d2 B1)
//   J     = r^2 r' Jang, Jang = d1 Ihat . (d2 Ihat x Ihat)
// with B_k,n = 1/2 (Ihat_l d_k Ihat_m - Ihat_m d_k Ihat_l) on the angular nodes and
// r' = h/2 (the derivative of r^2 along xi_3 is 2 r r' for p >= 2). The kernels
// rebuild every metric term from these tables, so per element only 13 n^2
// angular doubles (shared by all layers of a cell) are stored.
#include <cmath>
#include <cstring>
#include <map>
#include <stdexcept>
#include <tuple>
#include <unordered_map>
#include <utility>

#include "internal.h"

namespace dg {

Gll make_gll(int p) {
  Gll g;
  g.p = p;
  g.n = p + 1;
  const int n = g.n;
  g.x.resize(n);
  g.w.resize(n);
  // Newton on (x P_p - P_{p-1}) from Chebyshev-Gauss-Lobatto guesses
  for (int i = 0; i < n; ++i) g.x[i] = -std::cos(M_PI * i / p);
  for (int it = 0; it < 100; ++it) {
    double change = 0;
    for (int i = 0; i < n; ++i) {
      double x = g.x[i], P0 = 1.0, P1 = x;
      for (int k = 1; k < p; ++k) {
        double P2 = ((2 * k + 1) * x * P1 - k * P0) / (k + 1);
        P0 = P1;
        P1 = P2;
      }
      // P1 = P_p, P0 = P_{p-1}
      double dx = (x * P1 - P0) / ((p + 1) * P1);
      g.x[i] = x - dx;
      change = std::max(change, std::fabs(dx));
    }
    if (change < 1e-17) break;
  }
  g.x[0] = -1.0;
  g.x[p] = 1.0;
  for (int i = 0; i < n; ++i) {
    double x = g.x[i], P0 = 1.0, P1 = x;
    for (int k = 1; k < p; ++k) {
      double P2 = ((2 * k + 1) * x * P1 - k * P0) / (k + 1);
      P0 = P1;
      P1 = P2;
    }
    g.w[i] = 2.0 / (p * (p + 1) * P1 * P1);
  }
  // symmetrise
  for (int i = 0; i < n / 2; ++i) {
    double a = 0.5 * (g.x[n - 1 - i] - g.x[i]);
    g.x[i] = -a;
    g.x[n - 1 - i] = a;
    double w = 0.5 * (g.w[i] + g.w[n - 1 - i]);
    g.w[i] = g.w[n - 1 - i] = w;
  }
  if (n % 2) g.x[n / 2] = 0.0;
  // barycentric differentiation matrix
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (g.x[j] - g.x[k]);
  g.D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0;
    for (int j = 0; j < n; ++j)
      if (j != i) {
        g.D[i * n + j] = (lam[j] / lam[i]) / (g.x[i] - g.x[j]);
        s += g.D[i * n + j];
      }
    g.D[i * n + i] = -s;
  }
  return g;
}

GllC make_gllc(int p) {
  Gll g = make_gll(p);
  GllC c{};
  for (int i = 0; i < g.n * g.n; ++i) c.D[i] = g.D[i];
  for (int i = 0; i < g.n; ++i) {
    c.x[i] = g.x[i];
    c.w[i] = g.w[i];
  }
  return c;
}

QuadC make_quadc(int p) {
  Gll g = make_gll(p);
  const int n = g.n, nq = p + 2;
  QuadC c{};
  c.nq = nq;
  // Gauss-Legendre points: roots of P_nq by Newton from Chebyshev guesses; w = 2 / ((1 - x^2) P'^2)
  for (int i = 0; i < nq; ++i) {
    double x = -std::cos(M_PI * (i + 0.75) / (nq + 0.5)), dP = 1.0;
    for (int it = 0; it < 100; ++it) {
      double P0 = 1.0, P1 = x;
      for (int k = 1; k < nq; ++k) {
        const double P2 = ((2 * k + 1) * x * P1 - k * P0) / (k + 1);
        P0 = P1;
        P1 = P2;
      }
      dP = nq * (x * P1 - P0) / (x * x - 1.0);
      const double dx = P1 / dP;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    c.x[i] = x;
    c.w[i] = 2.0 / ((1.0 - x * x) * dP * dP);
  }
  // Lagrange basis of the GLL nodes at the Gauss points, and its derivative
  for (int gq = 0; gq < nq; ++gq)
    for (int j = 0; j < n; ++j) {
      double l = 1.0;
      for (int k = 0; k < n; ++k)
        if (k != j) l *= (c.x[gq] - g.x[k]) / (g.x[j] - g.x[k]);
      c.V[gq * n + j] = l;
    }
  for (int gq = 0; gq < nq; ++gq)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += c.V[gq * n + k] * g.D[k * n + j];
      c.Dg[gq * n + j] = s;   // l_j' is a degree-p polynomial: interpolate its nodal values
    }
  // exact reference mass matrix and its inverse (Gauss-Jordan with partial pivoting)
  double A[5][10] = {};
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int gq = 0; gq < nq; ++gq) s += c.w[gq] * c.V[gq * n + i] * c.V[gq * n + j];
      A[i][j] = s;
      A[i][n + j] = (i == j) ? 1.0 : 0.0;
    }
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(A[r][k]) > std::fabs(A[piv][k])) piv = r;
    for (int col = 0; col < 2 * n; ++col) std::swap(A[k][col], A[piv][col]);
    const double inv = 1.0 / A[k][k];
    for (int col = 0; col < 2 * n; ++col) A[k][col] *= inv;
    for (int r = 0; r < n; ++r)
      if (r != k) {
        const double f = A[r][k];
        for (int col = 0; col < 2 * n; ++col) A[r][col] -= f * A[k][col];
      }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) c.Mi[i * n + j] = A[i][n + j];
  return c;
}

FiltC make_filter(int p, double sigma) {
  Gll g = make_gll(p);
  const int n = g.n;
  std::vector<double> Pp(n);
  for (int i = 0; i < n; ++i) {
    // Bonnet recursion (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}
    double p0 = 1.0, p1 = g.x[i];
    for (int k = 1; k < p; ++k) {
      const double p2 = ((2.0 * k + 1.0) * g.x[i] * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    Pp[i] = (p == 0) ? 1.0 : p1;
  }
  double nrm = 0;
  for (int i = 0; i < n; ++i) nrm += g.w[i] * Pp[i] * Pp[i];
  FiltC f{};
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i)
      f.F[a * n + i] = (a == i ? 1.0 : 0.0) - (1.0 - sigma) * Pp[a] * g.w[i] * Pp[i] / nrm;
  return f;
}

std::vector<double> radial_edges(double r_bot, double r_top, int n, double stretch) {
  std::vector<double> h(n), e(n + 1);
  if (std::fabs(stretch - 1.0) < 1e-15) {
    for (int k = 0; k < n; ++k) h[k] = (r_top - r_bot) / n;
  } else {
    double h1 = (r_top - r_bot) * (stretch - 1.0) / (std::pow(stretch, n) - 1.0);
    for (int k = 0; k < n; ++k) h[k] = h1 * std::pow(stretch, k);
  }
  e[0] = r_bot;
  double acc = 0;
  for (int k = 0; k < n; ++k) {
    acc += h[k];
    e[k + 1] = r_bot + acc;
  }
  e[n] = r_top;
  return e;
}

// point on the cube for tangent coordinates (a, b); each panel's (alpha, beta,
// outward) frame is right-handed
static void panel_point(int panel, double a, double b, double* P) {
  switch (panel) {
    case 0: P[0] = 1; P[1] = a; P[2] = b; break;
    case 1: P[0] = -a; P[1] = 1; P[2] = b; break;
    case 2: P[0] = -1; P[1] = -a; P[2] = b; break;
    case 3: P[0] = a; P[1] = -1; P[2] = b; break;
    case 4: P[0] = -b; P[1] = a; P[2] = 1; break;
    default: P[0] = b; P[1] = a; P[2] = -1; break;
  }
}

// angular tables of one cell: out[13][n2]
static void cell_tables(const Gll& g, int panel, double a0, double a1, double b0, double b1, double* out) {
  const int n = g.n, n2 = n * n;
  std::vector<double> I(3 * n2), d1(3 * n2), d2(3 * n2);
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) {
      double al = a0 + 0.5 * (g.x[a] + 1.0) * (a1 - a0);
      double be = b0 + 0.5 * (g.x[b] + 1.0) * (b1 - b0);
      double P[3];
      panel_point(panel, std::tan(al), std::tan(be), P);
      double nr = std::sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2]);
      for (int c = 0; c < 3; ++c) I[c * n2 + a + n * b] = P[c] / nr;
    }
  auto deriv = [&](const double* f, double* df, int dir) {
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < n; ++a) {
        double s = 0;
        for (int i = 0; i < n; ++i)
          s += (dir == 0) ? g.D[a * n + i] * f[i + n * b] : g.D[b * n + i] * f[a + n * i];
        df[a + n * b] = s;
      }
  };
  for (int c = 0; c < 3; ++c) {
    deriv(&I[c * n2], &d1[c * n2], 0);
    deriv(&I[c * n2], &d2[c * n2], 1);
  }
  // B_k,n = 1/2 (I_l d_k I_m - I_m d_k I_l), (n, m, l) cyclic
  std::vector<double> B1(3 * n2), B2(3 * n2), dB2(3 * n2), dB1(3 * n2);
  for (int nn = 0; nn < 3; ++nn) {
    int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
    for (int j = 0; j < n2; ++j) {
      B1[nn * n2 + j] = 0.5 * (I[ll * n2 + j] * d1[mm * n2 + j] - I[mm * n2 + j] * d1[ll * n2 + j]);
      B2[nn * n2 + j] = 0.5 * (I[ll * n2 + j] * d2[mm * n2 + j] - I[mm * n2 + j] * d2[ll * n2 + j]);
    }
    deriv(&B2[nn * n2], &dB2[nn * n2], 0);
    deriv(&B1[nn * n2], &dB1[nn * n2], 1);
  }
  for (int nn = 0; nn < 3; ++nn)
    for (int j = 0; j < n2; ++j) {
      out[(0 + nn) * n2 + j] = 2.0 * B2[nn * n2 + j];
      out[(3 + nn) * n2 + j] = -2.0 * B1[nn * n2 + j];
      out[(6 + nn) * n2 + j] = -(dB2[nn * n2 + j] - dB1[nn * n2 + j]);
    }
  for (int j = 0; j < n2; ++j) {
    double x1[3], x2[3], Ih[3];
    for (int c = 0; c < 3; ++c) {
      x1[c] = d1[c * n2 + j];
      x2[c] = d2[c * n2 + j];
      Ih[c] = I[c * n2 + j];
    }
    double cr[3] = {x2[1] * Ih[2] - x2[2] * Ih[1], x2[2] * Ih[0] - x2[0] * Ih[2], x2[0] * Ih[1] - x2[1] * Ih[0]};
    out[9 * n2 + j] = x1[0] * cr[0] + x1[1] * cr[1] + x1[2] * cr[2];
    for (int c = 0; c < 3; ++c) out[(10 + c) * n2 + j] = Ih[c];
  }
}

// along-edge node s of angular face f (0: a=0, 1: a=n-1, 2: b=0, 3: b=n-1) -> angular node
static inline int edge_node(int f, int s, int n) {
  switch (f) {
    case 0: return 0 + n * s;
    case 1: return (n - 1) + n * s;
    case 2: return s;
    default: return s + n * (n - 1);
  }
}

struct Key {
  long long x, y, z;
  bool operator==(const Key& o) const { return x == o.x && y == o.y && z == o.z; }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    return std::hash<long long>()(k.x * 73856093LL ^ k.y * 19349663LL ^ k.z * 83492791LL);
  }
};

// Build the shell: tables and connectivity on the host.
dg_status_t build_shell(dg_mesh_s* m, const dg_mesh_desc_t& d) {
  if (d.p < 2 || d.p > 4 || d.n_ang < 1 || d.n_rad < 1 || !(d.r_top > d.r_bot) || !(d.r_bot > 0) ||
      !(d.stretch > 0)) {
    set_error("dg_mesh_create: shell needs 2 <= p <= 4, n_ang >= 1, n_rad >= 1, 0 < r_bot < r_top, stretch > 0");
    return DG_ERR_ARG;
  }
  Gll g = make_gll(d.p);
  const int n = g.n, n2 = n * n;
  m->p = d.p;
  m->n = n;
  m->N = n * n * n;
  m->N2 = n2;
  m->n_ang = d.n_ang;
  m->n_rad = d.n_rad;
  m->A = 6 * d.n_ang * d.n_ang;
  m->n_elem = (int64_t)m->A * d.n_rad;
  m->dim = 3;
  m->nf = 5;
  m->n_dof = m->n_elem * m->N * 5;
  m->h_edges = radial_edges(d.r_bot, d.r_top, d.n_rad, d.stretch);
  m->h_ang.assign((size_t)m->A * 13 * n2, 0.0);
  const double q = M_PI / 4;
  for (int panel = 0; panel < 6; ++panel)
    for (int j = 0; j < d.n_ang; ++j)
      for (int i = 0; i < d.n_ang; ++i) {
        int cell = (panel * d.n_ang + j) * d.n_ang + i;
        const double step = (2 * q) / d.n_ang;
        double a0 = i * step + (-q), a1 = (i + 1) * step + (-q);
        double b0 = j * step + (-q), b1 = (j + 1) * step + (-q);
        if (i + 1 == d.n_ang) a1 = q;
        if (j + 1 == d.n_ang) b1 = q;
        cell_tables(g, panel, a0, a1, b0, b1, &m->h_ang[(size_t)cell * 13 * n2]);
      }
  // connectivity of angular edges: match edge midpoints (on the unit sphere), then nodes
  std::vector<int> cnbr(m->A * 4, -1), cface(m->A * 4, -1), cmap((size_t)m->A * 4 * n, -1);
  const double Q = 1e7;
  std::unordered_map<Key, std::vector<int>, KeyHash> table;
  std::vector<double> mid((size_t)m->A * 4 * 3);
  for (int cell = 0; cell < m->A; ++cell)
    for (int f = 0; f < 4; ++f) {
      double s3[3] = {0, 0, 0};
      for (int s = 0; s < n; ++s)
        for (int c = 0; c < 3; ++c) s3[c] += m->h_ang[(size_t)cell * 13 * n2 + (10 + c) * n2 + edge_node(f, s, n)];
      for (int c = 0; c < 3; ++c) mid[(cell * 4 + f) * 3 + c] = s3[c] / n;
      Key k{std::llround(s3[0] / n * Q), std::llround(s3[1] / n * Q), std::llround(s3[2] / n * Q)};
      table[k].push_back(cell * 4 + f);
    }
  for (int cell = 0; cell < m->A; ++cell)
    for (int f = 0; f < 4; ++f) {
      const double* me = &mid[(cell * 4 + f) * 3];
      Key k0{std::llround(me[0] * Q), std::llround(me[1] * Q), std::llround(me[2] * Q)};
      int found = -1;
      for (int dx = -1; dx <= 1 && found < 0; ++dx)
        for (int dy = -1; dy <= 1 && found < 0; ++dy)
          for (int dz = -1; dz <= 1 && found < 0; ++dz) {
            auto it = table.find(Key{k0.x + dx, k0.y + dy, k0.z + dz});
            if (it == table.end()) continue;
            for (int cand : it->second) {
              if (cand == cell * 4 + f) continue;
              const double* o = &mid[cand * 3];
              double dd = std::fabs(o[0] - me[0]) + std::fabs(o[1] - me[1]) + std::fabs(o[2] - me[2]);
              if (dd < 1e-10) { found = cand; break; }
            }
          }
      if (found < 0) {
        set_error("dg_mesh_create: unmatched angular edge (internal error)");
        return DG_ERR_ARG;
      }
      int c2 = found / 4, f2 = found % 4;
      cnbr[cell * 4 + f] = c2;
      cface[cell * 4 + f] = f2;
      for (int s = 0; s < n; ++s) {
        const double* Ia = &m->h_ang[(size_t)cell * 13 * n2 + 10 * n2];
        int ja = edge_node(f, s, n);
        int best = -1;
        double bd = 1e300;
        for (int s2 = 0; s2 < n; ++s2) {
          const double* Ib = &m->h_ang[(size_t)c2 * 13 * n2 + 10 * n2];
          int jb = edge_node(f2, s2, n);
          double dd = 0;
          for (int c = 0; c < 3; ++c) dd += std::fabs(Ia[c * n2 + ja] - Ib[c * n2 + jb]);
          if (dd < bd) { bd = dd; best = s2; }
        }
        if (bd > 1e-12) {
          set_error("dg_mesh_create: unmatched edge node (internal error)");
          return DG_ERR_ARG;
        }
        cmap[((size_t)cell * 4 + f) * n + s] = best;
      }
    }
  DG_HIP_CHECK(hipMalloc(&m->d_ang, m->h_ang.size() * sizeof(double)));
  DG_HIP_CHECK(hipMalloc(&m->d_edges, m->h_edges.size() * sizeof(double)));
  DG_HIP_CHECK(hipMalloc(&m->d_cnbr, cnbr.size() * sizeof(int)));
  DG_HIP_CHECK(hipMalloc(&m->d_cface, cface.size() * sizeof(int)));
  DG_HIP_CHECK(hipMalloc(&m->d_cmap, cmap.size() * sizeof(int)));
  DG_HIP_CHECK(hipMemcpy(m->d_ang, m->h_ang.data(), m->h_ang.size() * sizeof(double), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(m->d_edges, m->h_edges.data(), m->h_edges.size() * sizeof(double), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(m->d_cnbr, cnbr.data(), cnbr.size() * sizeof(int), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(m->d_cface, cface.data(), cface.size() * sizeof(int), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(m->d_cmap, cmap.data(), cmap.size() * sizeof(int), hipMemcpyHostToDevice));
  m->fn_len = m->n_elem * 6 * 5 * n2;
  return DG_OK;
}

dg_status_t build_columns(dg_mesh_s* m, const dg_mesh_desc_t& d, const dg_physics_t& ph) {
  if (d.n_col < 1 || !d.col_nelem || !d.col_p || !(d.r_top > d.r_bot) || !(d.stretch > 0)) {
    set_error("dg_mesh_create: columns need n_col >= 1, col_nelem, col_p and r_bot < r_top");
    return DG_ERR_ARG;
  }
  m->dim = 1;
  m->nf = 3;
  m->n_col = d.n_col;
  m->col_nelem.assign(d.col_nelem, d.col_nelem + d.n_col);
  m->col_p.assign(d.col_p, d.col_p + d.n_col);
  m->col_off.assign(d.n_col + 1, 0);
  int64_t E = 0;
  for (int c = 0; c < d.n_col; ++c) {
    if (m->col_nelem[c] < 1 || m->col_p[c] < 2 || m->col_p[c] > 4) {
      set_error("dg_mesh_create: every column needs >= 1 element and 2 <= p <= 4");
      return DG_ERR_ARG;
    }
    m->col_off[c + 1] = m->col_off[c] + (int64_t)m->col_nelem[c] * 3 * (m->col_p[c] + 1);
    E += m->col_nelem[c];
  }
  if (E > 0x7fffffff) {
    set_error("dg_mesh_create: too many elements");
    return DG_ERR_ARG;
  }
  m->n_elem = E;
  m->n_dof = m->col_off[d.n_col];
  std::vector<int64_t> off(E);
  std::vector<int> prev(E), next(E), col(E);
  std::vector<int> plist[3];
  m->elem_p.resize(E);
  m->h_geo.resize(2 * E);
  int64_t e = 0;
  for (int c = 0; c < d.n_col; ++c) {
    const double sc = d.col_stretch ? d.col_stretch[c] : d.stretch;
    if (!(sc > 0)) {
      set_error("dg_mesh_create: column stretch must be positive");
      return DG_ERR_ARG;
    }
    std::vector<double> edges = radial_edges(d.r_bot, d.r_top, m->col_nelem[c], sc);
    int64_t o = m->col_off[c];
    const int p = m->col_p[c];
    for (int k = 0; k < m->col_nelem[c]; ++k, ++e) {
      off[e] = o;
      o += 3 * (p + 1);
      prev[e] = (k == 0) ? -1 : (int)(e - 1);
      next[e] = (k + 1 == m->col_nelem[c]) ? -1 : (int)(e + 1);
      col[e] = c;
      m->elem_p[e] = p;
      m->h_geo[2 * e] = edges[k];
      m->h_geo[2 * e + 1] = edges[k + 1] - edges[k];
      plist[p - 2].push_back((int)e);
    }
  }
  std::vector<double> cpar;
  col_params(ph, d.n_col, cpar);
  DG_HIP_CHECK(hipMalloc(&m->d_off, E * sizeof(int64_t)));
  DG_HIP_CHECK(hipMalloc(&m->d_prev, E * sizeof(int)));
  DG_HIP_CHECK(hipMalloc(&m->d_next, E * sizeof(int)));
  DG_HIP_CHECK(hipMalloc(&m->d_col, E * sizeof(int)));
  DG_HIP_CHECK(hipMalloc(&m->d_geo, 2 * E * sizeof(double)));
  DG_HIP_CHECK(hipMalloc(&m->d_cpar, cpar.size() * sizeof(double)));
  DG_HIP_CHECK(hipMemcpy(m->d_off, off.data(), E * sizeof(int64_t), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(m->d_prev, prev.data(), E * sizeof(int), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(m->d_next, next.data(), E * sizeof(int), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(m->d_col, col.data(), E * sizeof(int), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(m->d_geo, m->h_geo.data(), 2 * E * sizeof(double), hipMemcpyHostToDevice));
  DG_HIP_CHECK(hipMemcpy(m->d_cpar, cpar.data(), cpar.size() * sizeof(double), hipMemcpyHostToDevice));
  for (int i = 0; i < 3; ++i) {
    m->plist_n[i] = (int)plist[i].size();
    if (m->plist_n[i]) {
      DG_HIP_CHECK(hipMalloc(&m->d_plist[i], plist[i].size() * sizeof(int)));
      DG_HIP_CHECK(hipMemcpy(m->d_plist[i], plist[i].data(), plist[i].size() * sizeof(int), hipMemcpyHostToDevice));
    }
  }
  m->fn_len = E * 2 * 3;
  // Gauss tables of the over-integrated residual (degrees 2, 3, 4), read by the column batch
  const QuadC qt[3] = {make_quadc(2), make_quadc(3), make_quadc(4)};
  DG_HIP_CHECK(hipMalloc(&m->d_quad, sizeof(qt)));
  DG_HIP_CHECK(hipMemcpy(m->d_quad, qt, sizeof(qt), hipMemcpyHostToDevice));
  return DG_OK;
}

}  // namespace dg
