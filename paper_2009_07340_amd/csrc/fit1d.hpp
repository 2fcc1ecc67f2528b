// One-dimensional element fit for one (element, sample) held in one lane.
//
// Per element and sample (Sec. 5):
//   moved nodes xi*_i = xi_i + (A_i + B_i z)                      (eq. def_dx)
//   carried values f_i = phi_i (1 - dt div u)_i                     (eq. advection_phi)
//   advected interpolant p0 with p0(xi*_i) = f_i                    (eqs. phi_stardef, h_star)
//   traces t = (p0(0), p0(1))                                       (eq. remap_bnd)
//   constrained fit p = argmin sum_i (q(xi*_i) - f_i)^2 s.t. q(0) = g_L, q(1) = g_R
//   new values phi_i = p(xi_i)                                      (eq. phi_star)
//
// Algorithm (range-space Lagrange multipliers on the normal equations):
// basis psi_k(xi - dbar), dbar the mean node displacement; V the N x N basis
// matrix at the moved nodes; G = V^T V = L L^T (Cholesky), c0 = G^-1 V^T f;
// C = [psi(0 - dbar); psi(1 - dbar)] (2 x N); W = G^-1 C^T; S = C W (2 x 2);
// lambda = S^-1 (C c0 - g); c = c0 - W lambda.  Everything that does not
// depend on g (the unconstrained values at the Gauss nodes E c0, the columns
// E W and S) is formed before the boundary values of the neighbours are
// known, so after the exchange only a 2 x 2 solve and N multiply-adds remain.
#pragma once
#include <hip/hip_runtime.h>
#include "sl_internal.hpp"
#include "philox.hpp"

namespace sl {

// The fit arithmetic below may fuse multiply-adds (it is held to the oracle by a
// tolerance); moved positions and edge displacements come from the helpers
// above, which keep contraction off.  Switched off again at the end of the file.
#pragma clang fp contract(fast)

template <int N>
__device__ __forceinline__ void legendre_eval(double t, const LegendreRec& rec, double (&psi)[N]) {
  const double x = 2.0 * t - 1.0;
  psi[0] = 1.0;
  if constexpr (N > 1) psi[1] = rec.a[0] * x;
#pragma unroll
  for (int k = 1; k + 1 < N; ++k) psi[k + 1] = rec.a[k] * x * psi[k] - rec.b[k] * psi[k - 1];
}

// legendre_eval with the compile-time coefficients (the same values, the same
// rounding).
template <int N>
__device__ __forceinline__ void legendre_eval_k(double t, double (&psi)[N]) {
  const double x = 2.0 * t - 1.0;
  psi[0] = 1.0;
  if constexpr (N > 1) psi[1] = kLegA[0] * x;
#pragma unroll
  for (int k = 1; k + 1 < N; ++k) psi[k + 1] = kLegA[k] * x * psi[k] - kLegB[k] * psi[k - 1];
}

template <int N>
struct Fit1DPre {
  double phiu[N];   // unconstrained values at the Gauss nodes, E c0
  double wl[N];     // E G^-1 psi(0 - dbar)
  double wr[N];     // E G^-1 psi(1 - dbar)
  double wm[N];     // E G^-1 m (mass constraint: m . c = the element integral)
  double s00, s01, s11, s02, s12, s22;
  double tL, tR;    // traces of p0
};

// lambda = S^-1 (r0, r1, 0) for the symmetric 3 x 3 system of the boundary and
// mass constraints (cofactors; S is positive definite).
__device__ __forceinline__ void solve3_mass(double s00, double s01, double s11, double s02, double s12, double s22,
                                            double r0, double r1, double& l0, double& l1, double& l2) {
  const double a00 = s11 * s22 - s12 * s12, a01 = s02 * s12 - s01 * s22, a11 = s00 * s22 - s02 * s02;
  const double a02 = s01 * s12 - s02 * s11, a12 = s01 * s02 - s00 * s12;
  const double idet = 1.0 / (s00 * a00 + s01 * a01 + s02 * a02);
  l0 = (a00 * r0 + a01 * r1) * idet;
  l1 = (a01 * r0 + a11 * r1) * idet;
  l2 = (a02 * r0 + a12 * r1) * idet;
}

// Packed lower-triangular index.
__device__ __forceinline__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

template <int N>
__device__ __forceinline__ void chol_solve(const double (&L)[N * (N + 1) / 2], const double (&dinv)[N],
                                           double (&x)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double acc = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) acc -= L[tri(i, k)] * x[k];
    x[i] = acc * dinv[i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double acc = x[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) acc -= L[tri(k, i)] * x[k];
    x[i] = acc * dinv[i];
  }
}

// Phase before the exchange.  xs: moved nodes; f: carried values; xi: Gauss nodes;
// wq: quadrature weights of the nodes (read with the mass constraint only).
template <int N, bool MASS = false>
__device__ __forceinline__ void fit1d_pre(const double (&xs)[N], const double (&f)[N], const double* xi,
                                          const LegendreRec& rec, Fit1DPre<N>& out, const double* wq = nullptr) {
  double dsum = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) dsum += xs[i] - xi[i];
  const double dbar = dsum / N;

  double G[N * (N + 1) / 2];
  double b[N];
#pragma unroll
  for (int k = 0; k < N * (N + 1) / 2; ++k) G[k] = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) b[k] = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double psi[N];
    legendre_eval<N>(xs[i] - dbar, rec, psi);
#pragma unroll
    for (int p = 0; p < N; ++p) {
#pragma unroll
      for (int q = 0; q <= p; ++q) G[tri(p, q)] += psi[p] * psi[q];
      b[p] += psi[p] * f[i];
    }
  }
  // Cholesky G = L L^T in place (column-oriented, Crout order)
  double dinv[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double d = G[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= G[tri(j, k)] * G[tri(j, k)];
    const double ljj = sqrt(d);
    dinv[j] = 1.0 / ljj;
    G[tri(j, j)] = ljj;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      double v = G[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= G[tri(i, k)] * G[tri(j, k)];
      G[tri(i, j)] = v * dinv[j];
    }
  }
  double pl[N], pr[N];
  legendre_eval<N>(0.0 - dbar, rec, pl);
  legendre_eval<N>(1.0 - dbar, rec, pr);
  double wl[N], wr[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    wl[k] = pl[k];
    wr[k] = pr[k];
  }
  // mass row m_k = sum_i wq_i psi_k(xi_i - dbar) (the element's quadrature, exact on Q_{N-1})
  double mk[N], wm[N];
  if constexpr (MASS) {
#pragma unroll
    for (int k = 0; k < N; ++k) mk[k] = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double psi[N];
      legendre_eval<N>(xi[i] - dbar, rec, psi);
#pragma unroll
      for (int k = 0; k < N; ++k) mk[k] += wq[i] * psi[k];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) wm[k] = mk[k];
    chol_solve<N>(G, dinv, wm);
  }
  chol_solve<N>(G, dinv, b);   // b <- c0
  chol_solve<N>(G, dinv, wl);
  chol_solve<N>(G, dinv, wr);
  double tL = 0.0, tR = 0.0, s00 = 0.0, s01 = 0.0, s11 = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    tL += pl[k] * b[k];
    tR += pr[k] * b[k];
    s00 += pl[k] * wl[k];
    s01 += pl[k] * wr[k];
    s11 += pr[k] * wr[k];
  }
  out.tL = tL;
  out.tR = tR;
  out.s00 = s00;
  out.s01 = s01;
  out.s11 = s11;
  if constexpr (MASS) {
    double s02 = 0.0, s12 = 0.0, s22 = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      s02 += pl[k] * wm[k];
      s12 += pr[k] * wm[k];
      s22 += mk[k] * wm[k];
    }
    out.s02 = s02;
    out.s12 = s12;
    out.s22 = s22;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double psi[N];
    legendre_eval<N>(xi[i] - dbar, rec, psi);
    double u = 0.0, a = 0.0, c = 0.0, m = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      u += psi[k] * b[k];
      a += psi[k] * wl[k];
      c += psi[k] * wr[k];
      if constexpr (MASS) m += psi[k] * wm[k];
    }
    out.phiu[i] = u;
    out.wl[i] = a;
    out.wr[i] = c;
    if constexpr (MASS) out.wm[i] = m;
  }
}

// The same fit in nodal form: with V square, the constrained values at the
// moved nodes are a = f - C*^T S^-1 (C* f - g), C* = C V^-1 the Lagrange
// basis of the moved nodes evaluated at the edges and S = C* C*^T, and the
// new values are Phi a with Phi = E V^-1 the Lagrange basis evaluated at the
// Gauss nodes.  Lagrange rows come from the barycentric weights
// w_j = 1 / prod_{m != j} (x*_j - x*_m) and prefix/suffix products, so the
// whole fit costs O(N^2) operations and no N x N matrix is ever stored.
template <int N>
__device__ __forceinline__ void lagrange_row(const double (&xs)[N], const double (&w)[N], double x,
                                             double (&l)[N]) {
  double pre[N];
  pre[0] = 1.0;
#pragma unroll
  for (int m = 1; m < N; ++m) pre[m] = pre[m - 1] * (x - xs[m - 1]);
  double suf = 1.0;
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    l[j] = w[j] * pre[j] * suf;
    suf *= (x - xs[j]);
  }
}

// State of a nodal fit carried across the trace exchange (5N + 5 values).
template <int N>
struct Fit1DNodal {
  double xs[N];     // moved nodes
  double w[N];      // barycentric weights of the moved nodes
  double a[N];      // carried values f (becomes the constrained values a)
  double cl[N];     // C*: Lagrange rows of the moved nodes at xi = 0 ...
  double cr[N];     // ... and at xi = 1
  double cm[N];     // mass row (mass constraint): integral of each Lagrange basis polynomial
  double s00, s01, s11, s02, s12, s22;
  double tL, tR;    // traces of p0
};

// 1 / d for a normal, nonzero d: hardware estimate refined by two Newton steps
// (about 1 ulp; the fit is held to the oracle by a tolerance).
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
#pragma unroll
  for (int k = 0; k < 2; ++k) r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// Reciprocals of the node products, four per reciprocal: 1/a = b c d / (a b c d).
template <int N>
__device__ __forceinline__ void reciprocals(const double (&p)[N], double (&w)[N]) {
#pragma unroll
  for (int g = 0; g + 4 <= N; g += 4) {
    const double ab = p[g] * p[g + 1], cd = p[g + 2] * p[g + 3];
    const double r = recip(ab * cd);
    const double rab = r * ab, rcd = r * cd;
    w[g] = rcd * p[g + 1];
    w[g + 1] = rcd * p[g];
    w[g + 2] = rab * p[g + 3];
    w[g + 3] = rab * p[g + 2];
  }
  constexpr int g = N - N % 4;
  if constexpr (N % 4 == 3) {
    const double ab = p[g] * p[g + 1];
    const double r = recip(ab * p[g + 2]);
    const double rc = r * p[g + 2];
    w[g] = rc * p[g + 1];
    w[g + 1] = rc * p[g];
    w[g + 2] = r * ab;
  } else if constexpr (N % 4 == 2) {
    const double r = recip(p[g] * p[g + 1]);
    w[g] = r * p[g + 1];
    w[g + 1] = r * p[g];
  } else if constexpr (N % 4 == 1) {
    w[g] = recip(p[g]);
  }
}

template <int N, bool MASS = false>
__device__ __forceinline__ void fit1d_nodal_pre(Fit1DNodal<N>& st, const double* xi = nullptr,
                                                const double* wq = nullptr) {
  // p_j = prod_{m != j} (x*_j - x*_m), each difference formed once
  double pj[N];
#pragma unroll
  for (int j = 0; j < N; ++j) pj[j] = 1.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int m = j + 1; m < N; ++m) {
      const double d = st.xs[j] - st.xs[m];
      pj[j] *= d;
      pj[m] *= -d;
    }
  }
  reciprocals<N>(pj, st.w);
  lagrange_row<N>(st.xs, st.w, 0.0, st.cl);
  lagrange_row<N>(st.xs, st.w, 1.0, st.cr);
  double tL = 0.0, tR = 0.0, s00 = 0.0, s01 = 0.0, s11 = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    tL += st.cl[j] * st.a[j];
    tR += st.cr[j] * st.a[j];
    s00 += st.cl[j] * st.cl[j];
    s01 += st.cl[j] * st.cr[j];
    s11 += st.cr[j] * st.cr[j];
  }
  st.tL = tL;
  st.tR = tR;
  st.s00 = s00;
  st.s01 = s01;
  st.s11 = s11;
  if constexpr (MASS) {
    // cm_j = integral of the j-th Lagrange polynomial of the moved nodes = sum_i wq_i l_j(xi_i)
#pragma unroll
    for (int j = 0; j < N; ++j) st.cm[j] = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double row[N];
      lagrange_row<N>(st.xs, st.w, xi[i], row);
#pragma unroll
      for (int j = 0; j < N; ++j) st.cm[j] += wq[i] * row[j];
    }
    double s02 = 0.0, s12 = 0.0, s22 = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      s02 += st.cl[j] * st.cm[j];
      s12 += st.cr[j] * st.cm[j];
      s22 += st.cm[j] * st.cm[j];
    }
    st.s02 = s02;
    st.s12 = s12;
    st.s22 = s22;
  }
}

// After the exchange: a = f - C*^T lambda, lambda = S^-1 (t - g); phi = Phi a.
template <int N, bool MASS = false>
__device__ __forceinline__ void fit1d_nodal_post(Fit1DNodal<N>& st, const double* xi, double gL, double gR,
                                                 double (&phi)[N]) {
  const double r0 = st.tL - gL, r1 = st.tR - gR;
  double l0, l1, l2 = 0.0;
  if constexpr (MASS) {
    // boundary and mass rows: the mass row's residual is zero (the fit keeps p0's integral)
    solve3_mass(st.s00, st.s01, st.s11, st.s02, st.s12, st.s22, r0, r1, l0, l1, l2);
  } else {
    const double idet = recip(st.s00 * st.s11 - st.s01 * st.s01);
    l0 = (st.s11 * r0 - st.s01 * r1) * idet;
    l1 = (st.s00 * r1 - st.s01 * r0) * idet;
  }
  // phi_i = sum_j w_j a_j prod_{m != j} (xi_i - x*_m), with the weights folded
  // into the values once.  With d_m = xi_i - x*_m and P_j = prod_{m < j} d_m the
  // sum is sum_j wa_j P_j prod_{m > j} d_m, a Horner scheme over j:
  // v <- v d_j + wa_j P_j, P <- P d_j (three operations a node pair).
  double wa[N];
#pragma unroll
  for (int j = 0; j < N; ++j)
    wa[j] = st.w[j] * (st.a[j] - (st.cl[j] * l0 + st.cr[j] * l1 + (MASS ? st.cm[j] * l2 : 0.0)));
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double v = wa[0], dprev = xi[i] - st.xs[0], P = 1.0;
#pragma unroll
    for (int j = 1; j < N; ++j) {
      P = (j == 1) ? dprev : P * dprev;
      const double d = xi[i] - st.xs[j];
      v = v * d + wa[j] * P;
      dprev = d;
    }
    phi[i] = v;
  }
}

// Phase after the exchange: new values from the boundary data gL, gR.
template <int N, bool MASS = false>
__device__ __forceinline__ void fit1d_post(const Fit1DPre<N>& pre, double gL, double gR, double (&phi)[N]) {
  const double r0 = pre.tL - gL, r1 = pre.tR - gR;
  if constexpr (MASS) {
    double l0, l1, l2;
    solve3_mass(pre.s00, pre.s01, pre.s11, pre.s02, pre.s12, pre.s22, r0, r1, l0, l1, l2);
#pragma unroll
    for (int i = 0; i < N; ++i) phi[i] = pre.phiu[i] - (pre.wl[i] * l0 + pre.wr[i] * l1 + pre.wm[i] * l2);
  } else {
    const double det = pre.s00 * pre.s11 - pre.s01 * pre.s01;
    const double l0 = (pre.s11 * r0 - pre.s01 * r1) / det;
    const double l1 = (pre.s00 * r1 - pre.s01 * r0) / det;
#pragma unroll
    for (int i = 0; i < N; ++i) phi[i] = pre.phiu[i] - (pre.wl[i] * l0 + pre.wr[i] * l1);
  }
}

// Moved nodes with the contracted-free operation order of the position contract.
template <int N>
__device__ __forceinline__ void move_nodes(const double* xi, const double* A, const double* B, double z,
                                           double (&xs)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) xs[i] = moved_coord(xi[i], A[i], B[i], z);
}

#pragma clang fp contract(off)

}  // namespace sl
