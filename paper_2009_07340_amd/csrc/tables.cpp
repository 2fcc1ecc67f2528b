// Host tables: Gauss nodes, Legendre recurrence, 2-D edge-trace basis and
// trace interpolation between orders.  Computed once per handle in float64 (or
// __float128 where the result must be the correctly rounded value).
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace sl {

namespace {

typedef __float128 qd;

qd qabs(qd x) { return x < 0 ? -x : x; }

// P_N(x) and P_N'(x) by the three-term recurrence, in __float128.
void legendre_q(int n, qd x, qd& p, qd& dp) {
  qd p0 = 1, p1 = x;
  if (n == 0) {
    p = 1;
    dp = 0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const qd p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1);
}

// T_N(x) and T_N'(x) = N U_{N-1}(x), in __float128.
void chebyshev_q(int n, qd x, qd& t, qd& dt) {
  qd t0 = 1, t1 = x;
  for (int k = 1; k < n; ++k) {
    const qd t2 = 2 * x * t1 - t0;
    t0 = t1;
    t1 = t2;
  }
  qd u0 = 1, u1 = 2 * x;            // U_0, U_1
  qd u = (n == 1) ? u0 : u1;
  for (int k = 1; k < n - 1; ++k) {
    const qd u2 = 2 * x * u1 - u0;
    u0 = u1;
    u1 = u2;
    u = u1;
  }
  t = t1;
  dt = n * u;
}

}  // namespace

std::vector<double> gauss_nodes(int n, int family) {
  if (n < 1 || n > 64) throw std::invalid_argument("node count out of range");
  std::vector<double> xi(n);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    // i-th largest root x of P_N (or T_N) on [-1, 1]; xi = (1 - x)/2 is increasing in i
    qd x = family == 0 ? (qd)std::cos(pi * (i + 0.75) / (n + 0.5)) : (qd)std::cos(pi * (2 * i + 1) / (2.0 * n));
    for (int it = 0; it < 60; ++it) {
      qd p, dp;
      if (family == 0) legendre_q(n, x, p, dp);
      else chebyshev_q(n, x, p, dp);
      const qd dx = p / dp;
      x -= dx;
      if (qabs(dx) < (qd)1e-33) break;
    }
    xi[i] = (double)((1 - x) / 2);
  }
  return xi;
}

LegendreRec legendre_recurrence() {
  LegendreRec r{};
  for (int k = 0; k < kMaxN; ++k) {
    r.a[k] = std::sqrt((2.0 * k + 3.0) * (2.0 * k + 1.0)) / (k + 1.0);
    r.b[k] = k == 0 ? 0.0 : k * std::sqrt(2.0 * k + 3.0) / ((k + 1.0) * std::sqrt(2.0 * k - 1.0));
  }
  return r;
}

double min_node_spacing(const std::vector<double>& xi) {
  double m = 1.0;
  for (size_t i = 1; i < xi.size(); ++i) m = std::min(m, xi[i] - xi[i - 1]);
  return m;
}

// Lagrange basis through the abscissae `from`, evaluated at x: out[j] = l_j(x).
static void lagrange_row(const std::vector<double>& from, double x, double* out) {
  const int n = (int)from.size();
  for (int j = 0; j < n; ++j) {
    double v = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) v *= (x - from[m]) / (from[j] - from[m]);
    out[j] = v;
  }
}

std::vector<double> quadrature_weights(const std::vector<double>& xi) {
  // the interpolatory rule on [0, 1]: sum_i w_i xi_i^k = 1 / (k + 1), k < n, solved in
  // __float128 by Gaussian elimination with partial pivoting (Gauss weights for GL nodes)
  const int n = (int)xi.size();
  std::vector<qd> A((size_t)n * (n + 1));
  for (int k = 0; k < n; ++k) {
    for (int i = 0; i < n; ++i) {
      qd v = 1;
      for (int e = 0; e < k; ++e) v *= (qd)xi[i];
      A[(size_t)k * (n + 1) + i] = v;
    }
    A[(size_t)k * (n + 1) + n] = (qd)1 / (qd)(k + 1);
  }
  for (int c = 0; c < n; ++c) {
    int pr = c;
    for (int r = c + 1; r < n; ++r)
      if (qabs(A[(size_t)r * (n + 1) + c]) > qabs(A[(size_t)pr * (n + 1) + c])) pr = r;
    for (int j = 0; j <= n; ++j) std::swap(A[(size_t)c * (n + 1) + j], A[(size_t)pr * (n + 1) + j]);
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const qd f = A[(size_t)r * (n + 1) + c] / A[(size_t)c * (n + 1) + c];
      for (int j = c; j <= n; ++j) A[(size_t)r * (n + 1) + j] -= f * A[(size_t)c * (n + 1) + j];
    }
  }
  std::vector<double> w(n);
  for (int i = 0; i < n; ++i) w[i] = (double)(A[(size_t)i * (n + 1) + n] / A[(size_t)i * (n + 1) + i]);
  return w;
}

std::vector<double> barycentric_weights(const std::vector<double>& xi) {
  const int n = (int)xi.size();
  std::vector<double> w(n);
  for (int i = 0; i < n; ++i) {
    long double p = 1.0L;
    for (int m = 0; m < n; ++m)
      if (m != i) p *= (long double)xi[i] - (long double)xi[m];
    w[i] = (double)(1.0L / p);
  }
  return w;
}

std::vector<double> lagrange_matrix(const std::vector<double>& from, const std::vector<double>& to) {
  std::vector<double> L(to.size() * from.size());
  for (size_t i = 0; i < to.size(); ++i) lagrange_row(from, to[i], &L[i * from.size()]);
  return L;
}

// Orthonormal basis U_r (4N x (4N-4), column-major as U[q + 4N*c]) of the
// edge-value vectors that polynomials of Q_{N-1} can take on the W,E,S,N edge
// points.  Those are the vectors whose four edge polynomials (degree N-1
// interpolants through the Gauss abscissae) agree at the four corners, i.e.
// the null space of the 4 x 4N corner-compatibility matrix A.  Householder QR
// of A^T in long double; U_r = the last 4N-4 columns of Q.
std::vector<double> edge_range_basis(int N, const std::vector<double>& xi) {
  const int T = 4 * N;
  std::vector<double> l0(N), l1(N);
  lagrange_row(xi, 0.0, l0.data());
  lagrange_row(xi, 1.0, l1.data());
  // A^T as T x 4 (column c = corner functional); edges blocks W=0, E=1, S=2, N=3
  std::vector<long double> At((size_t)T * 4, 0.0L);
  auto set = [&](int corner, int edge, const std::vector<double>& l, double sign) {
    for (int j = 0; j < N; ++j) At[(size_t)(edge * N + j) * 4 + corner] += sign * l[j];
  };
  set(0, 0, l0, 1.0); set(0, 2, l0, -1.0);   // SW: W at eta=0 equals S at xi=0
  set(1, 1, l0, 1.0); set(1, 2, l1, -1.0);   // SE: E at eta=0 equals S at xi=1
  set(2, 0, l1, 1.0); set(2, 3, l0, -1.0);   // NW: W at eta=1 equals N at xi=0
  set(3, 1, l1, 1.0); set(3, 3, l1, -1.0);   // NE: E at eta=1 equals N at xi=1
  // Householder QR of At (T x 4); accumulate Q (T x T)
  std::vector<long double> Q((size_t)T * T, 0.0L);
  for (int i = 0; i < T; ++i) Q[(size_t)i * T + i] = 1.0L;
  for (int c = 0; c < 4; ++c) {
    long double norm = 0;
    for (int i = c; i < T; ++i) norm += At[(size_t)i * 4 + c] * At[(size_t)i * 4 + c];
    norm = std::sqrt(norm);
    if (norm == 0) throw std::runtime_error("degenerate corner matrix");
    std::vector<long double> v(T, 0.0L);
    const long double a0 = At[(size_t)c * 4 + c];
    const long double alpha = a0 > 0 ? -norm : norm;
    for (int i = c; i < T; ++i) v[i] = At[(size_t)i * 4 + c];
    v[c] -= alpha;
    long double vn = 0;
    for (int i = c; i < T; ++i) vn += v[i] * v[i];
    if (vn == 0) continue;
    // At <- H At
    for (int cc = c; cc < 4; ++cc) {
      long double d = 0;
      for (int i = c; i < T; ++i) d += v[i] * At[(size_t)i * 4 + cc];
      d = 2 * d / vn;
      for (int i = c; i < T; ++i) At[(size_t)i * 4 + cc] -= d * v[i];
    }
    // Q <- Q H
    for (int r = 0; r < T; ++r) {
      long double d = 0;
      for (int i = c; i < T; ++i) d += Q[(size_t)r * T + i] * v[i];
      d = 2 * d / vn;
      for (int i = c; i < T; ++i) Q[(size_t)r * T + i] -= d * v[i];
    }
  }
  const int r = T - 4;
  std::vector<double> U((size_t)T * r);
  for (int c = 0; c < r; ++c)
    for (int q = 0; q < T; ++q) U[(size_t)c * T + q] = (double)Q[(size_t)q * T + (c + 4)];
  return U;
}

// Inverse of an n x n matrix (row-major) by Gauss-Jordan elimination with
// partial pivoting, in long double.
static std::vector<long double> gj_inverse(std::vector<long double> G, int N) {
  std::vector<long double> Inv((size_t)N * N, 0.0L);
  for (int i = 0; i < N; ++i) Inv[i * N + i] = 1.0L;
  for (int c = 0; c < N; ++c) {
    int piv = c;
    for (int r = c + 1; r < N; ++r)
      if (std::fabs(G[r * N + c]) > std::fabs(G[piv * N + c])) piv = r;
    if (piv != c)
      for (int k = 0; k < N; ++k) {
        std::swap(G[c * N + k], G[piv * N + k]);
        std::swap(Inv[c * N + k], Inv[piv * N + k]);
      }
    const long double d = G[c * N + c];
    for (int k = 0; k < N; ++k) {
      G[c * N + k] /= d;
      Inv[c * N + k] /= d;
    }
    for (int r = 0; r < N; ++r) {
      if (r == c) continue;
      const long double f = G[r * N + c];
      if (f == 0.0L) continue;
      for (int k = 0; k < N; ++k) {
        G[r * N + k] -= f * G[c * N + k];
        Inv[r * N + k] -= f * Inv[c * N + k];
      }
    }
  }
  return Inv;
}

std::vector<double> reference_inverses(const std::vector<double>& xi) {
  const int N = (int)xi.size();
  // Vx[i][k] = psi_k(xi_i), the same three-term recurrence as the device tables
  std::vector<long double> V(N * N), G(N * N, 0.0L);
  for (int i = 0; i < N; ++i) {
    const long double x = 2.0L * xi[i] - 1.0L;
    long double pm = 1.0L, pc = 0.0L;
    V[i * N + 0] = 1.0L;
    if (N > 1) {
      pc = std::sqrt(3.0L) * x;
      V[i * N + 1] = pc;
    }
    for (int k = 1; k + 1 < N; ++k) {
      const long double a = std::sqrt((2.0L * k + 3.0L) * (2.0L * k + 1.0L)) / (k + 1.0L);
      const long double b = k * std::sqrt(2.0L * k + 3.0L) / ((k + 1.0L) * std::sqrt(2.0L * k - 1.0L));
      const long double pn = a * x * pc - b * pm;
      pm = pc;
      pc = pn;
      V[i * N + k + 1] = pn;
    }
  }
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b)
      for (int i = 0; i < N; ++i) G[a * N + b] += V[i * N + a] * V[i * N + b];
  const auto Gi = gj_inverse(G, N);
  const auto Vi = gj_inverse(V, N);
  std::vector<double> out(2 * N * N);
  for (int i = 0; i < N * N; ++i) {
    out[i] = (double)Gi[i];
    out[N * N + i] = (double)Vi[i];
  }
  return out;
}

std::vector<double> nullspace_tables(int N, const std::vector<double>& xi) {
  std::vector<double> l0(N), l1(N);
  lagrange_row(xi, 0.0, l0.data());
  lagrange_row(xi, 1.0, l1.data());
  std::vector<double> out(nsp_doubles(N), 0.0);
  for (int a = 0; a < N; ++a) {
    out[nsp_ends(N) + a] = l0[a];
    out[nsp_ends(N) + N + a] = l1[a];
  }
  // C^T C for the corner rows (SW, NW, SE, NE): each row has l_s on one edge and
  // -l_s' on the other, and two rows share an edge only through one end weight
  long double L00 = 0.0L, L01 = 0.0L, L11 = 0.0L;
  for (int a = 0; a < N; ++a) {
    L00 += (long double)l0[a] * l0[a];
    L01 += (long double)l0[a] * l1[a];
    L11 += (long double)l1[a] * l1[a];
  }
  const std::vector<long double> CtC = {2 * L00, L01,       L01,       0.0L,   //
                                        L01,     L00 + L11, 0.0L,      L01,    //
                                        L01,     0.0L,      L00 + L11, L01,    //
                                        0.0L,    L01,       L01,       2 * L11};
  const auto Ci = gj_inverse(CtC, 4);
  for (int i = 0; i < 16; ++i) out[nsp_cinv(N) + i] = (double)Ci[i];
  out[nsp_ll(N)] = (double)L00;
  out[nsp_ll(N) + 1] = (double)L01;
  out[nsp_ll(N) + 2] = (double)L11;
  const auto bw = barycentric_weights(xi);
  for (int a = 0; a < N; ++a) out[nsp_bary(N) + a] = bw[a];
  for (int a = 0; a < N; ++a) {
    const long double x = 2.0L * xi[a] - 1.0L;
    long double pm = 1.0L, pc = 0.0L;
    out[nsp_vx(N) + a * N] = 1.0;
    if (N > 1) {
      pc = std::sqrt(3.0L) * x;
      out[nsp_vx(N) + a * N + 1] = (double)pc;
    }
    for (int k = 1; k + 1 < N; ++k) {
      const long double ak = std::sqrt((2.0L * k + 3.0L) * (2.0L * k + 1.0L)) / (k + 1.0L);
      const long double bk = k * std::sqrt(2.0L * k + 3.0L) / ((k + 1.0L) * std::sqrt(2.0L * k - 1.0L));
      const long double pn = ak * x * pc - bk * pm;
      pm = pc;
      pc = pn;
      out[nsp_vx(N) + a * N + k + 1] = (double)pn;
    }
  }
  const int m = N - 2;
  if (m > 0) {
    long double z = 0.0L;
    for (int a = 0; a < N; ++a) {
      const long double sa = (long double)xi[a] * (1.0L - (long double)xi[a]);
      for (int k = 0; k < m; ++k) {
        const long double v = sa * (long double)out[nsp_vx(N) + a * N + k];
        z += v * v;
      }
    }
    z /= m;
    out[nsp_zz(N)] = (double)(z * z);
  }
  return out;
}

}  // namespace sl
