// Two-dimensional step, reference-preconditioned solver.
//
// The same constrained least-squares remap as the factorisation kernels
// (Sec. 5.3, eqs. phi_stardef, h_star, remap_bnd, bnd_update, phi_star), solved
// without forming or factoring the Gram matrix G = V^T V of the fit.
//
// The basis is centred on the mean node displacement, so a uniform
// displacement leaves the moved-node basis matrix equal to the reference one,
// V0 = Vx (x) Vx: the orthonormal Legendre basis at the Gauss nodes.  Its Gram
// matrix is a Kronecker product, G0 = Gx (x) Gx with Gx = Vx^T Vx, and
// G0^-1 = Gx^-1 (x) Gx^-1 costs 2 N^3 operations to apply.  Only the
// non-uniform part of the displacement (velocity and diffusion varying across
// the element) makes G differ from G0, so G0 is an excellent preconditioner:
//
//   phase 1 (unconstrained interpolant p0, traces at the own edge points):
//     preconditioned conjugate gradients on G c = V^T f, preconditioner G0^-1,
//     G applied matrix-free as V^T (V p) from the 1-D Legendre tables;
//   phase 2 (constrained remap):
//     projected preconditioned conjugate gradients on the equality-constrained
//     problem  min |V c - f|^2  s.t.  C_r c = g_r  with the constraint
//     preconditioner [[G0, C_r^T], [C_r, 0]]^-1, applied by the range-space
//     formula with S0 = C_r G0^-1 C_r^T.  Every iterate satisfies the
//     constraints; one final correction restores them to working accuracy.
//
// S0 needs no n x n work either: the edge-point rows of C are tensor products
// of 1-D basis vectors, so C G0^-1 C^T is assembled from two (N+2) x (N+2)
// tables of 1-D quadratic forms, and S0 = U_r^T (C G0^-1 C^T) U_r (matrix
// cores).  S0 is inverted explicitly once per fit (Gauss-Jordan, one barrier
// per pivot), so each iteration only applies dense matrix-vector products.
//
// The iteration count adapts to the fit: zero for a uniform displacement
// (the preconditioner is then exact), a few for the smooth fields of the
// workloads.  Fits that do not reach the tolerance within the iteration limit
// are counted in a device statistic.  Everything is float64.  One workgroup
// (four wavefronts) per fit, all of its data in LDS (N <= 16).
#include "sl_internal.hpp"
#include "philox.hpp"
#include "fit1d.hpp"
#include "blocks.hpp"

namespace sl {

// Solver arithmetic may fuse multiply-adds (the fit is held to the oracle by a
// tolerance); moved positions and edge displacements come from helpers defined
// with contraction off.
#pragma clang fp contract(fast)

using namespace blk;

// LDS layout in doubles.  Phase 1 uses the first part only.
template <int N>
struct LayR {
  static constexpr int n = N * N, TT = 4 * N, R = 4 * N - 4, RB = (R + 15) / 16, RP = 16 * RB, NH = N + 2;
  static constexpr int Rs = R + 1;             // row stride of the dense S0 / S0^-1
  // X1, Y1: the 1-D basis at the moved nodes, stored by basis index with an
  // odd row stride (XS = n + 1) so that lanes walking the nodes and lanes
  // walking the basis index both hit distinct LDS banks.
  static constexpr int XS = n + 1;
  static constexpr int oX1 = 0;
  static constexpr int oY1 = oX1 + N * XS;
  static constexpr int oBx = oY1 + N * XS;
  static constexpr int oBy = oBx + N * N;
  static constexpr int oEv = oBy + N * N;
  static constexpr int oGxi = oEv + 4 * N;
  static constexpr int oB = oGxi + N * N;
  static constexpr int oF = oB + n;
  static constexpr int oXv = oF + n;
  static constexpr int oZ0 = oXv + n;
  static constexpr int oR = oZ0 + n;
  static constexpr int oGv = oR + n;
  static constexpr int oP = oGv + n;
  static constexpr int oQ = oP + n;
  static constexpr int oT1 = oQ + n;
  static constexpr int oT2 = oT1 + n;
  static constexpr int oTr = oT2 + n;          // traces / edge vector
  static constexpr int oUc = oTr + TT;         // edge contractions (phase 1)
  static constexpr int oXs = oUc + TT;
  static constexpr int oYs = oXs + n;
  static constexpr int oRed = oYs + n;
  static constexpr int end1 = oRed + 16;
  // Phase 2.  Regions that are dead at the time hold short-lived data:
  //   [f .. end of phase 1] (f, the iteration vectors, the phase-1 edge vectors,
  //   the moved coordinates) holds Gx^-1 applied to the 1-D edge vectors while
  //   the H tables are formed, then T U_r while S0 is assembled, then the
  //   Gauss-Jordan pivot buffers; the phase-1 edge vectors are the projection's
  //   edge vectors; S0's own space holds the H tables until S0 is written.
  static constexpr int TTs = TT + 1;
  static constexpr int tuMax = TTs * R;
  static constexpr int oTU = oF;                      // T U_r, column stride US
  static constexpr int oSd = (end1 > oTU + tuMax ? end1 : oTU + tuMax);   // S0, then S0^-1 (dense, R x Rs)
  static constexpr int oPiv = oTU;                    // Gauss-Jordan pivot rows, two buffers
  static_assert(8 * R <= oSd - oTU, "pivot buffers must fit in the aliased region");
  static constexpr int oE1 = oTr;
  static constexpr int oE2 = oUc;                     // contraction vectors
  // The projection's two R-vectors sit in the gap between the phase-1 layout
  // and S0 when there is one (dead there after S0 is assembled and inverted).
  static constexpr bool kWinGap = oSd - end1 >= 2 * R;
  static constexpr int oW1 = kWinGap ? end1 : oSd + R * Rs;
  static constexpr int oW2 = oW1 + R;
  static constexpr int oRr = kWinGap ? oSd + R * Rs : oW2 + R;   // g_r = U_r^T g
  // The H tables and the upwinded boundary data g live in S0's space when they
  // fit there: both are dead once T U_r and g_r are formed, before S0 is written.
  static constexpr bool kHinS = 2 * NH * NH + TT <= R * Rs;
  static constexpr int oHx = kHinS ? oSd : oRr + R;
  static constexpr int oHy = oHx + NH * NH;
  static constexpr int oGr = oHy + NH * NH;           // upwinded boundary data g
  // T U_r and U_r^T (T U_r) run on the matrix cores, the entries of
  // T = C G0^-1 C^T formed on the fly from the H tables.  U_r is staged in LDS
  // (column stride TT + 1) when it fits and costs no occupancy (phase-2
  // workgroups a CU, at most 5); otherwise it is read from the cache.
  static constexpr int endR = kHinS ? oRr + R : oGr + TT;
  static constexpr size_t kCU = 160 * 1024, bU = sizeof(double) * (endR + TTs * R), bNoU = sizeof(double) * endR;
  static constexpr bool kUrLds = bU <= 156 * 1024 && (kCU / bU > 5 ? 5 : kCU / bU) >= (kCU / bNoU > 5 ? 5 : kCU / bNoU);
  static constexpr int US = kUrLds ? TTs : TT;        // column stride of U_r as used
  static constexpr int oU = endR;
  static constexpr int end2 = kUrLds ? endR + TTs * R : endR;
  // With U_r staged, the edge operators of the projection use the 4 (R x N)
  // tables M (formed once per fit over the staged U_r, which is not needed
  // afterwards): C_r z and C_r^T y then take two short stages each.
  static constexpr bool kM = kUrLds;
  static_assert(!kM || 4 * R * N <= TTs * R, "M tables replace the staged U_r");
  static_assert(US * R <= oSd - oTU, "T U_r must fit in the aliased region");
  static constexpr size_t bytes1 = sizeof(double) * end1;
  static constexpr size_t bytes2 = sizeof(double) * end2;
  // Workgroups per CU that the LDS admits (one wave per SIMD each): the
  // register budget is asked to admit as many, phase 2 at most 5 (more would
  // spill its registers).
  static constexpr int lds_waves(size_t b, int cap) { return (160 * 1024) / b > (size_t)cap ? cap : (int)((160 * 1024) / b); }
  static constexpr int waves1 = lds_waves(bytes1, 8), waves2 = lds_waves(bytes2, 5);
};

// ---------------------------------------------------------------- helpers

// Sum over the workgroup of a per-thread value; every thread gets the same
// result (fixed summation order).  One barrier: the slots in red are read
// after it and written again only by a later sum, which the callers keep
// behind at least one other barrier (dot products use red, the pair of
// residual norms red + 8).
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane() == 0) red[wave()] = v;
  block_sync();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Two sums at once (one barrier, as above).
__device__ __forceinline__ void block_sum2(double& v0, double& v1, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v0 += __shfl_xor(v0, o, 64);
    v1 += __shfl_xor(v1, o, 64);
  }
  if (lane() == 0) {
    red[wave()] = v0;
    red[4 + wave()] = v1;
  }
  block_sync();
  v0 = (red[0] + red[1]) + (red[2] + red[3]);
  v1 = (red[4] + red[5]) + (red[6] + red[7]);
}

// r^T g and g^T g of the current iterate.  The stopping test uses g^T g: g is
// the preconditioned (projected) residual, about the error of the iterate, and
// its rounding noise enters g^T g only to second order (r^T g carries it to
// first order once the constraints hold r away from zero).
template <int N>
__device__ __forceinline__ void block_rg_gg(const double* r, const double* g, double& rg, double& gg, double* red) {
  double a = 0.0, c = 0.0;
  for (int i = tid(); i < N * N; i += kThreads) {
    a += r[i] * g[i];
    c += g[i] * g[i];
  }
  block_sum2(a, c, red);
  rg = a;
  gg = c;
}

template <int N>
__device__ __forceinline__ double block_dot(const double* a, const double* b, double* red) {
  double v = 0.0;
  for (int i = tid(); i < N * N; i += kThreads) v += a[i] * b[i];
  return block_sum(v, red);
}

// out[i] = (V c)_i
template <int N>
__device__ void r_V(const double* X1, const double* Y1, const double* c, double* out) {
  for (int i = tid(); i < N * N; i += kThreads) {
    double xr[N];
#pragma unroll
    for (int k = 0; k < N; ++k) xr[k] = X1[k * LayR<N>::XS + i];
    double v = 0.0;
#pragma unroll 1
    for (int ly = 0; ly < N; ++ly) {
      double inner = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) inner += xr[k] * c[ly * N + k];
      v += Y1[ly * LayR<N>::XS + i] * inner;
    }
    out[i] = v;
  }
}

// out[p] = (V^T r)_p, p = (ly, k): the N x N matrix Y1 diag(r) X1^T as one
// 16 x 16 float64 matrix-core tile (K = n in steps of 4), by wavefront 0.
template <int N>
__device__ void r_VT_mc(const double* X1, const double* Y1, const double* r, double* out,
                        const double* dotw = nullptr, double* dot_out = nullptr) {
  typedef Mma<double> M64;
  if (wave() != 0) return;
  constexpr int n = N * N, XS = LayR<N>::XS;
  const int l = lane(), lr = l & 15, lk = l >> 4;
  const bool col = lr < N;
  M64::acc_t acc = zacc<double>();
#pragma unroll 4
  for (int kk = 0; kk < (n + 3) / 4; ++kk) {
    const int i = 4 * kk + lk;
    const bool ok = col && i < n;
    const double a = ok ? Y1[lr * XS + i] : 0.0;          // A[ly][i]
    const double b = ok ? r[i] * X1[lr * XS + i] : 0.0;   // B[i][k]
    acc = M64::mma(a, b, acc);
  }
  double d = 0.0;
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const int ly = M64::row(l, s4);
    if (ly < N && col) {
      out[ly * N + lr] = acc[s4];
      if (dotw) d += dotw[ly * N + lr] * acc[s4];
    }
  }
  if (dotw) {   // <dotw, out> from the accumulators, summed across the wavefront
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
    if (l == 0) *dot_out = d;
  }
}

// out = (Gx^-1 (x) Gx^-1) v  (c indexed [ly * N + k]), or minuend - that when
// minuend is given; tmp n doubles.  Two barriers.  With rr given, the
// per-wavefront partial sums of rr . out and out . out are left in
// red2[0..3] and red2[4..7] (readable after the second barrier).
template <int N>
__device__ void r_G0inv(const double* gxi, const double* v, double* tmp, double* out,
                        const double* minuend = nullptr, const double* rr = nullptr, double* red2 = nullptr) {
  for (int p = tid(); p < N * N; p += kThreads) {
    const int k = p % N, ly = p / N;
    double acc = 0.0;
#pragma unroll
    for (int kk = 0; kk < N; ++kk) acc += gxi[k * N + kk] * v[ly * N + kk];
    tmp[p] = acc;
  }
  block_sync();
  double a = 0.0, c = 0.0;
  for (int p = tid(); p < N * N; p += kThreads) {
    const int k = p % N, ly = p / N;
    double acc = 0.0;
#pragma unroll
    for (int ll = 0; ll < N; ++ll) acc += gxi[ly * N + ll] * tmp[ll * N + k];
    const double o = minuend ? minuend[p] - acc : acc;
    out[p] = o;
    if (rr) {
      a += rr[p] * o;
      c += o * o;
    }
  }
  if (rr) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o, 64);
      c += __shfl_xor(c, o, 64);
    }
    if (lane() == 0) {
      red2[wave()] = a;
      red2[4 + wave()] = c;
    }
  }
  block_sync();
}

// out[q] = (C c)_q: the polynomial at own edge point q (W, E, S, N blocks of N)
template <int N>
__device__ void r_C(const double* Bx, const double* By, const double* Ev, const double* c, double* out) {
  for (int q = tid(); q < 4 * N; q += kThreads) {
    const int w = q / N, j = q % N;
    double t = 0.0;
#pragma unroll 1
    for (int ly = 0; ly < N; ++ly) {
      double inner = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const double bx = (w == 0) ? Ev[k] : (w == 1) ? Ev[N + k] : Bx[j * N + k];
        inner += bx * c[ly * N + k];
      }
      const double by = (w < 2) ? By[j * N + ly] : (w == 2) ? Ev[2 * N + ly] : Ev[3 * N + ly];
      t += by * inner;
    }
    out[q] = t;
  }
}

// out[p] = (C^T v)_p
template <int N>
__device__ void r_CT(const double* Bx, const double* By, const double* Ev, const double* v, double* out) {
  for (int p = tid(); p < N * N; p += kThreads) {
    const int k = p % N, ly = p / N;
    const double e0 = Ev[k], e1 = Ev[N + k], f0 = Ev[2 * N + ly], f1 = Ev[3 * N + ly];
    double acc = 0.0;
#pragma unroll 2
    for (int j = 0; j < N; ++j)
      acc += By[j * N + ly] * (e0 * v[j] + e1 * v[N + j]) + Bx[j * N + k] * (f0 * v[2 * N + j] + f1 * v[3 * N + j]);
    out[p] = acc;
  }
}

// out[c] = (U_r^T v)_c, c < R; U column-major 4N x R, column stride US (LDS copy) or
// us (the table in global memory, stride 4N)
template <int N>
__device__ void r_UT(const double* U, const double* v, double* out, int us = LayR<N>::US) {
  using L = LayR<N>;
  for (int c = tid(); c < L::R; c += kThreads) {
    double acc = 0.0;
#pragma unroll 4
    for (int q = 0; q < L::TT; ++q) acc += U[c * us + q] * v[q];
    out[c] = acc;
  }
}

// Carried values of component c's row of the state (eq. advection_phi) into f
// and b = V^T f, for the second and later components of a fit (the first one's
// come with the set-up).  Two barriers.
template <int N>
__device__ void r_rhs(const Params2D& p, double* lds, int e, int64_t row) {
  using L = LayR<N>;
  const int64_t noff = p.noff[e];
  double* f = lds + L::oF;
  for (int i = tid(); i < L::n; i += kThreads) f[i] = p.phi[row * p.nodes + noff + i] * p.src[noff + i];
  block_sync();
  r_VT_mc<N>(lds + L::oX1, lds + L::oY1, f, lds + L::oB);
  block_sync();
}

// Upwinded boundary data of one component row (eq. bnd_update) into gv: at each
// own edge point, the element the interface displacement comes from supplies
// the trace (another order's trace interpolated to this element's abscissae), or
// the Dirichlet ghost value.  No barrier.
template <int N>
__device__ void r_upwind(const Params2D& p, int e, int64_t row, double za, double zb, double* gv) {
  using L = LayR<N>;
  const int64_t eoff = p.eoff[e];
  for (int q = tid(); q < L::TT; q += kThreads) {
    const int ew = q / N, j = q % N;
    const double tq = p.tr[row * p.edges + eoff + q];
    const double zd = (ew < 2) ? za : zb;
    const double disp = edge_disp(p.Af[eoff + q], p.Bf[eoff + q], zd);
    const bool pos = disp > 0.0;
    const bool take_nbr = (ew == 0 || ew == 2) ? pos : !pos;   // W, S: neighbour is the negative side
    double g = tq;
    if (take_nbr) {
      const int nb = p.nbr[4 * e + ew];
      if (nb < 0) {
        g = p.ghost[eoff + q];
      } else {
        const int Ns = p.order[nb];
        const double* src = p.tr + row * p.edges + p.eoff[nb] + (ew ^ 1) * Ns;
        if (Ns == N) {
          g = src[j];
        } else {   // trace of another order: Lagrange interpolation to this element's abscissae
          const double* Lm = p.interp + p.interp_off[N * (kMaxN + 1) + Ns] + j * Ns;
          double acc = 0.0;
          for (int m = 0; m < Ns; ++m) acc += Lm[m] * src[m];
          g = acc;
        }
      }
    }
    gv[q] = g;
  }
}

// out[q] = (U_r w)_q
template <int N>
__device__ void r_U(const double* U, const double* w, double* out) {
  using L = LayR<N>;
  for (int q = tid(); q < L::TT; q += kThreads) {
    double acc = 0.0;
#pragma unroll 4
    for (int c = 0; c < L::R; ++c) acc += U[c * L::US + q] * w[c];
    out[q] = acc;
  }
}

// out = S0^-1 w (dense, row stride Rs)
template <int N>
__device__ void r_Sinv(const double* Sd, const double* w, double* out) {
  using L = LayR<N>;
  for (int c = tid(); c < L::R; c += kThreads) {
    double acc = 0.0;
#pragma unroll 4
    for (int j = 0; j < L::R; ++j) acc += Sd[c * L::Rs + j] * w[j];
    out[c] = acc;
  }
}

// One-dimensional contractions of a coefficient array c[ly][k] with the edge
// basis vectors: out[0..N) = sum_k p0x[k] c[.][k], out[N..2N) with p1x,
// out[2N..3N) = sum_ly p0y[ly] c[ly][.], out[3N..4N) with p1y.
template <int N>
__device__ void r_edge_contract(const double* Ev, const double* c, double* out) {
  for (int o = tid(); o < 4 * N; o += kThreads) {
    const int w = o / N, m = o % N;
    const double* e = Ev + w * N;
    double acc = 0.0;
    if (w < 2) {
#pragma unroll
      for (int k = 0; k < N; ++k) acc += e[k] * c[m * N + k];
    } else {
#pragma unroll
      for (int ly = 0; ly < N; ++ly) acc += e[ly] * c[ly * N + m];
    }
    out[o] = acc;
  }
}

// Traces at the own edge points from the contractions u of r_edge_contract:
// W, E point j = sum_ly By[j][ly] u_{W,E}[ly]; S, N point j = sum_k Bx[j][k] u_{S,N}[k].
template <int N>
__device__ void r_traces_from(const double* Bx, const double* By, const double* u, double* out) {
  for (int q = tid(); q < 4 * N; q += kThreads) {
    const int w = q / N, j = q % N;
    const double* B = (w < 2) ? By + j * N : Bx + j * N;
    const double* v = u + w * N;
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) acc += B[m] * v[m];
    out[q] = acc;
  }
}

// C_r z from the contractions u: w[c] = sum_w sum_m M_w[c][m] u_w[m] - rhs2[c],
// with M_W[c][ly] = sum_j U_W[j][c] By[j][ly] (and E), M_S[c][k] = sum_j U_S[j][c] Bx[j][k]
// (and N), stored as Mm[(w R + c) N + m].
template <int N>
__device__ void r_M_apply(const double* Mm, const double* u, const double* rhs2, double* out) {
  using L = LayR<N>;
  for (int c = tid(); c < L::R; c += kThreads) {
    double acc = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const double* Mr = Mm + (w * L::R + c) * N;
#pragma unroll
      for (int m = 0; m < N; ++m) acc += Mr[m] * u[w * N + m];
    }
    if (rhs2) acc -= rhs2[c];
    out[c] = acc;
  }
}

// y-weighted edge vectors yv[w N + m] = sum_c M_w[c][m] y[c]
template <int N>
__device__ void r_MT_apply(const double* Mm, const double* y, double* yv) {
  using L = LayR<N>;
  for (int o = tid(); o < 4 * N; o += kThreads) {
    const int w = o / N, m = o % N;
    double acc = 0.0;
#pragma unroll 4
    for (int c = 0; c < L::R; ++c) acc += Mm[(w * L::R + c) * N + m] * y[c];
    yv[o] = acc;
  }
}

// C_r^T y from yv: out[(ly, k)] = p0x[k] yW[ly] + p1x[k] yE[ly] + p0y[ly] yS[k] + p1y[ly] yN[k]
template <int N>
__device__ void r_outer_edges(const double* Ev, const double* yv, double* out) {
  for (int p = tid(); p < N * N; p += kThreads) {
    const int k = p % N, ly = p / N;
    out[p] = Ev[k] * yv[ly] + Ev[N + k] * yv[N + ly] + Ev[2 * N + ly] * yv[2 * N + k] + Ev[3 * N + ly] * yv[3 * N + k];
  }
}

// ---------------------------------------------------------------- per-fit set-up

// Moves (eq. def_dx), carried values (eq. advection_phi), centred 1-D tables,
// b = V^T f; returns the mean displacement (dbx, dby) in registers.
template <int N>
__device__ int r_setup(const Params2D& p, double* lds, int e, int64_t s, double za, double zb) {
  using L = LayR<N>;
  constexpr int n = L::n;
  const int t = tid();
  const int64_t noff = p.noff[e];
  double* xs = lds + L::oXs;
  double* ys = lds + L::oYs;
  double* f = lds + L::oF;
  double* red = lds + L::oRed;
  double sx = 0.0, sy = 0.0;
  int esc = 0;
  for (int i = t; i < n; i += kThreads) {
    const int64_t k = noff + i;
    const double x0 = p.xi_node[2 * k], y0 = p.xi_node[2 * k + 1];
    const double xm = moved_coord(x0, p.A[2 * k], p.B[2 * k], za);
    const double ym = moved_coord(y0, p.A[2 * k + 1], p.B[2 * k + 1], zb);
    xs[i] = xm;
    ys[i] = ym;
    f[i] = p.phi[s * p.ncomp * p.nodes + k] * p.src[k];   // component 0 of sample s
    sx += xm - x0;
    sy += ym - y0;
    esc += escaped(xm) + escaped(ym);
  }
  const double* gsrc = p.gxinv + p.gx_off[N];
  double* gxi = lds + L::oGxi;
  for (int i = t; i < N * N; i += kThreads) gxi[i] = gsrc[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_xor(sx, o, 64);
    sy += __shfl_xor(sy, o, 64);
    esc += __shfl_xor(esc, o, 64);
  }
  if (lane() == 0) {
    red[wave()] = sx;
    red[4 + wave()] = sy;
    red[8 + wave()] = (double)esc;
  }
  block_sync();
  const double dbx = (red[0] + red[1] + red[2] + red[3]) / n;
  const double dby = (red[4] + red[5] + red[6] + red[7]) / n;
  const int escapes = (int)((red[8] + red[9]) + (red[10] + red[11]));
  double* X1 = lds + L::oX1;
  double* Y1 = lds + L::oY1;
  double* Bx = lds + L::oBx;
  double* By = lds + L::oBy;
  double* Ev = lds + L::oEv;
  // one basis evaluation an item: the n moved nodes in x, then in y, the N
  // Gauss abscissae of the edges in x and in y, the 4 edge coordinates
  for (int it = t; it < 2 * n + 2 * N + 4; it += kThreads) {
    double arg;
    double* dst;
    int stride = 1;
    if (it < 2 * n) {
      const int dir = it >= n, i = it - dir * n;
      arg = dir ? ys[i] - dby : xs[i] - dbx;
      dst = (dir ? Y1 : X1) + i;
      stride = L::XS;
    } else if (it < 2 * n + 2 * N) {
      const int u = it - 2 * n, dir = u >= N, row = u - dir * N;
      arg = p.xi_tab[N * kMaxN + row] - (dir ? dby : dbx);
      dst = (dir ? By : Bx) + row * N;
    } else {
      const int w = it - 2 * n - 2 * N;
      arg = (w == 0) ? -dbx : (w == 1) ? 1.0 - dbx : (w == 2) ? -dby : 1.0 - dby;
      dst = Ev + w * N;
    }
    double q[N];
    legendre_eval<N>(arg, p.rec, q);
#pragma unroll
    for (int k = 0; k < N; ++k) dst[k * stride] = q[k];
  }
  block_sync();
  r_VT_mc<N>(X1, Y1, f, lds + L::oB);
  block_sync();
  return escapes;
}

// The Wiener increments of sample s in this step (eq. def_dx), drawn only by the
// wavefronts that use them (the node moves and the edge displacements: the
// first max(n, 4N) threads); the others get zeros they never read.
template <int N>
__device__ __forceinline__ Normal2 fit_increments(const Params2D& p, int64_t s) {
  constexpr int kUse = (N * N > 4 * N ? N * N : 4 * N);
  double za = 0.0, zb = 0.0;
  if (__builtin_amdgcn_readfirstlane(tid() >> 6) < (kUse + 63) / 64) {
    const Normal2 d = normal_pair(p.seed, p.stream, (uint64_t)(p.step_ptr ? *p.step_ptr : p.step), (uint64_t)s);
    za = d.a;
    zb = d.b;
  }
  return Normal2{za, zb};
}

// G v = V^T (V v) into out (tmp: n doubles).  Two barriers.
// With dot_out given, <v, G v> is left there too (readable after the return).
template <int N>
__device__ __forceinline__ void r_G(double* lds, const double* v, double* tmp, double* out, double* dot_out = nullptr) {
  using L = LayR<N>;
  r_V<N>(lds + L::oX1, lds + L::oY1, v, tmp);
  block_sync();
  r_VT_mc<N>(lds + L::oX1, lds + L::oY1, tmp, out, dot_out ? v : nullptr, dot_out);
  block_sync();
}

// Diagnostics of one fit: iterations and whether the tolerance was reached
// (per phase), moved nodes outside the element (phase 1 counts the moves) and
// the relative residual left, sqrt(g^T g / x0^T x0).  Called after the fit's
// last barrier: a workgroup barrier waits for the memory operations in flight,
// atomics included.
__device__ __forceinline__ void count_fit(const Params2D& p, int phase, int iters, int unconverged, int escapes,
                                          double resid) {
  if (tid() == 0 && p.stats) {
    unsigned long long* c = stat_slot(p.stats) + 2 * (phase - 1);
    atomicAdd(c, (unsigned long long)iters);
    if (unconverged) atomicAdd(c + 1, (unsigned long long)unconverged);
    stat_add(p.stats, kStatEscapes, (unsigned long long)escapes);
    stat_residual(p.stats, resid);
  }
}

__device__ __forceinline__ double rel_resid(double gg, double xx) {
  return xx > 0.0 ? sqrt(gg / xx) : (gg > 0.0 ? __builtin_inf() : 0.0);
}

// ---------------------------------------------------------------- phase 1

template <int N>
__device__ __forceinline__ void r_phase1_body(const Params2D& p, double* lds, int64_t fit) {
  using L = LayR<N>;
  constexpr int n = L::n;
  const int64_t w = fit / p.M;
  const int64_t s = fit - w * p.M;
  const int e = p.work[w];
  const Normal2 z = fit_increments<N>(p, s);
  const int escapes = r_setup<N>(p, lds, e, s, z.a, z.b);
  const int t = tid();
  const double* gxi = lds + L::oGxi;
  double* b = lds + L::oB;
  double* x = lds + L::oXv;
  double* r = lds + L::oR;
  double* g = lds + L::oGv;
  double* pv = lds + L::oP;
  double* q = lds + L::oQ;
  double* t1 = lds + L::oT1;
  double* red = lds + L::oRed;
  const int64_t eoff = p.eoff[e];
  int its = 0, unconv = 0;
  double rmax = 0.0;
  // the components share the moved nodes and their tables (Sec. 5.3, last paragraph)
  for (int c = 0; c < p.ncomp; ++c) {
  const int64_t row = s * p.ncomp + c;
  if (c > 0) r_rhs<N>(p, lds, e, row);
  // preconditioned conjugate gradients on G c = b from c = G0^-1 b
  r_G0inv<N>(gxi, b, t1, x);
  const double xx = block_dot<N>(x, x, red);
  r_G<N>(lds, x, t1, r);
  for (int i = t; i < n; i += kThreads) r[i] -= b[i];
  block_sync();
  r_G0inv<N>(gxi, r, t1, g, nullptr, r, red + 8);   // with r^T g and g^T g
  double rg = (red[8] + red[9]) + (red[10] + red[11]);
  double gg = (red[12] + red[13]) + (red[14] + red[15]);
  const double stop = p.tol2 * xx;
  int it = 0;
  if (gg > stop) {
    for (int i = t; i < n; i += kThreads) pv[i] = -g[i];
    block_sync();
    for (it = 1; it <= p.max_iter; ++it) {
      r_G<N>(lds, pv, t1, q, red);   // q = G pv and pv^T q
      const double pq = red[0];
      const double alpha = rg / pq;
      for (int i = t; i < n; i += kThreads) {
        x[i] += alpha * pv[i];
        r[i] += alpha * q[i];
      }
      block_sync();
      r_G0inv<N>(gxi, r, t1, g, nullptr, r, red + 8);
      const double rg1 = (red[8] + red[9]) + (red[10] + red[11]);
      gg = (red[12] + red[13]) + (red[14] + red[15]);
      if (gg <= stop) break;
      const double beta = rg1 / rg;
      rg = rg1;
      for (int i = t; i < n; i += kThreads) pv[i] = beta * pv[i] - g[i];
      block_sync();
    }
  }
  // traces of p0 at the own edge points (eq. remap_bnd)
  double* tv = lds + L::oTr;
  double* uc = lds + L::oUc;
  r_edge_contract<N>(lds + L::oEv, x, uc);
  block_sync();
  r_traces_from<N>(lds + L::oBx, lds + L::oBy, uc, tv);
  block_sync();
  for (int qq = t; qq < L::TT; qq += kThreads) p.tr[row * p.edges + eoff + qq] = tv[qq];
  its += it > p.max_iter ? p.max_iter : it;
  unconv += gg <= stop ? 0 : 1;
  rmax = fmax(rmax, rel_resid(gg, xx));
  }
  count_fit(p, 1, its, unconv, escapes, rmax);
}

// ---------------------------------------------------------------- phase 2

// Constraint preconditioner, first block:  out = G0^-1 (r - C_r^T y) with
// y = S0^-1 (C_r G0^-1 r - rhs2); rhs2 may be null (zero).  Leaves
// z0 = G0^-1 r, y (in w2) and C_r^T y (in t2) behind.  Scratch: t1, e1, w1.
template <int N>
__device__ void r_Pproj(double* lds, const double* U, const double* rin, const double* rhs2, double* out) {
  using L = LayR<N>;
  const double* gxi = lds + L::oGxi;
  double* z0 = lds + L::oZ0;
  double* t1 = lds + L::oT1;
  double* t2 = lds + L::oT2;
  double* e1 = lds + L::oE1;
  double* w1 = lds + L::oW1;
  double* w2 = lds + L::oW2;
  const double* Bx = lds + L::oBx;
  const double* By = lds + L::oBy;
  const double* Ev = lds + L::oEv;
  r_G0inv<N>(gxi, rin, t1, z0);
  if constexpr (L::kM) {
    double* u = lds + L::oE2;
    const double* Mm = lds + L::oU;
    r_edge_contract<N>(Ev, z0, u);
    block_sync();
    r_M_apply<N>(Mm, u, rhs2, w1);
    block_sync();
    r_Sinv<N>(lds + L::oSd, w1, w2);
    block_sync();
    r_MT_apply<N>(Mm, w2, u);
    block_sync();
    r_outer_edges<N>(Ev, u, t2);
    block_sync();
  } else {
    r_C<N>(Bx, By, Ev, z0, e1);
    block_sync();
    r_UT<N>(U, e1, w1);
    block_sync();
    if (rhs2) {
      for (int c = tid(); c < L::R; c += kThreads) w1[c] -= rhs2[c];
      block_sync();
    }
    r_Sinv<N>(lds + L::oSd, w1, w2);
    block_sync();
    r_U<N>(U, w2, e1);
    block_sync();
    r_CT<N>(Bx, By, Ev, e1, t2);
    block_sync();
  }
  r_G0inv<N>(gxi, t2, t1, out, z0);
}

// In-place block Gauss-Jordan inversion of the dense SPD matrix S (R x R, row
// stride Rs; R = 4(N - 1) is a multiple of 4): R / 4 steps, each eliminating a
// 4 x 4 pivot block K (SPD, so no pivoting):
//   S_KK <- P^-1,  S_Kj <- P^-1 S_Kj,  S_iK <- -S_iK P^-1,  S_ij <- S_ij - S_iK P^-1 S_Kj.
// Between steps the working matrix keeps the structure of a partial inverse of
// an SPD matrix: its eliminated and remaining diagonal blocks are symmetric and
// the block from eliminated rows to remaining columns is minus the transpose of
// its mirror, so a row's part of the pivot columns is read from the pivot rows
// (negated for rows already eliminated).  Each thread keeps a strided piece of
// one row in registers (TPR threads per row); the pivot rows pass through LDS
// (two buffers, one barrier a step) and every thread solves with the 4 x 4
// pivot block itself (Cholesky, two triangular solves).
template <int N>
__device__ void r_invert_S(double* Sd, double* piv) {
  using L = LayR<N>;
  // two wavefronts hold the matrix up to R = 32 (the per-step pivot solve is
  // repeated by every wavefront that holds rows), the whole workgroup beyond
  constexpr int R = L::R, NTH = R <= 32 ? 128 : kThreads, TPR = NTH / R, kE = (R + TPR - 1) / TPR;
  static_assert(R % 4 == 0, "R is a multiple of 4");
  const int t = tid();
  const int i = t / TPR, chunk = t - i * TPR;
  const bool live = i < R;
  double a[kE];
#pragma unroll
  for (int m = 0; m < kE; ++m) {
    const int j = chunk + TPR * m;
    a[m] = (live && j < R) ? Sd[i * L::Rs + j] : 0.0;
  }
#pragma unroll 1
  for (int k0 = 0; k0 < R; k0 += 4) {
    double* prow = piv + ((k0 >> 2) & 1) * 4 * R;   // [4][R] pivot rows, two buffers
    const bool inK = i >= k0 && i < k0 + 4;
    if (live && inK) {
#pragma unroll
      for (int m = 0; m < kE; ++m) {
        const int j = chunk + TPR * m;
        if (j < R) prow[(i - k0) * R + j] = a[m];
      }
    }
    block_sync();
    if (live) {
      // this row's coefficients x = P^-1 rhs, rhs = S_iK^T (P symmetric) or, for
      // a row of K, the unit vector (x is then that row of P^-1): Cholesky of
      // the 4 x 4 pivot block (lower triangle) and two triangular solves
      double Pl[4][4];
#pragma unroll
      for (int pp = 0; pp < 4; ++pp)
#pragma unroll
        for (int qq = 0; qq <= pp; ++qq) Pl[pp][qq] = prow[pp * R + k0 + qq];
      double dinv[4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        double d = Pl[jj][jj];
#pragma unroll
        for (int kk = 0; kk < jj; ++kk) d -= Pl[jj][kk] * Pl[jj][kk];
        dinv[jj] = rsqrt_nr(d);
#pragma unroll
        for (int ii = jj + 1; ii < 4; ++ii) {
          double v = Pl[ii][jj];
#pragma unroll
          for (int kk = 0; kk < jj; ++kk) v -= Pl[ii][kk] * Pl[jj][kk];
          Pl[ii][jj] = v * dinv[jj];
        }
      }
      const double sg = (i < k0) ? -1.0 : 1.0;
      double x[4];
#pragma unroll
      for (int pp = 0; pp < 4; ++pp) x[pp] = inK ? (i - k0 == pp ? 1.0 : 0.0) : sg * prow[pp * R + i];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        double v = x[ii];
#pragma unroll
        for (int kk = 0; kk < ii; ++kk) v -= Pl[ii][kk] * x[kk];
        x[ii] = v * dinv[ii];
      }
#pragma unroll
      for (int ii = 3; ii >= 0; --ii) {
        double v = x[ii];
#pragma unroll
        for (int kk = ii + 1; kk < 4; ++kk) v -= Pl[kk][ii] * x[kk];
        x[ii] = v * dinv[ii];
      }
#pragma unroll
      for (int m = 0; m < kE; ++m) {
        const int j = chunk + TPR * m;
        const int jj = j < R ? j : 0;
        const bool jK = jj >= k0 && jj < k0 + 4;
        double v;
        if (jK) {
          const int q = jj - k0;
          const double xq = (q == 0) ? x[0] : (q == 1) ? x[1] : (q == 2) ? x[2] : x[3];
          v = inK ? xq : -xq;
        } else {
          const double r0 = prow[jj], r1 = prow[R + jj], r2 = prow[2 * R + jj], r3 = prow[3 * R + jj];
          const double xr = x[0] * r0 + x[1] * r1 + x[2] * r2 + x[3] * r3;
          v = inK ? xr : a[m] - xr;
        }
        a[m] = v;
      }
    }
  }
  if (live) {
#pragma unroll
    for (int m = 0; m < kE; ++m) {
      const int j = chunk + TPR * m;
      if (j < R) Sd[i * L::Rs + j] = a[m];
    }
  }
  block_sync();
}

template <int N>
__device__ __forceinline__ void r_phase2_body(const Params2D& p, double* lds, int64_t fit) {
  using L = LayR<N>;
  constexpr int n = L::n, TT = L::TT, R = L::R, RB = L::RB, NH = L::NH;
  const int64_t w = fit / p.M;
  const int64_t s = fit - w * p.M;
  const int e = p.work[w];
  const Normal2 z = fit_increments<N>(p, s);
  r_setup<N>(p, lds, e, s, z.a, z.b);
  const int t = tid(), wv = wave();
  const int64_t eoff = p.eoff[e];
  const double* U = p.ur + p.ur_off[N];
  if constexpr (L::kUrLds) {
    double* Ul = lds + L::oU;
    for (int i = t; i < TT * R; i += kThreads) Ul[(i / TT) * L::TTs + i % TT] = U[i];
    U = Ul;   // visible to all threads after the barrier that follows the H tables
  }
  const double* gxi = lds + L::oGxi;
  const double* Bx = lds + L::oBx;
  const double* By = lds + L::oBy;
  const double* Ev = lds + L::oEv;
  // 1-D quadratic forms H[a][b] = v_a^T Gx^-1 v_b over {psi(0 - d), psi(1 - d), psi(xi_j - d)}:
  // first W[b] = Gx^-1 v_b (in the space T U_r takes later), then H[a][b] = v_a . W[b]
  double* Hx = lds + L::oHx;
  double* Hy = lds + L::oHy;
  double* Wt = lds + L::oTU;   // [dir][b][N]
  static_assert(2 * NH * N <= L::TTs * R, "W fits where T U_r goes");
  auto hvec = [&](int dir, int a) -> const double* {
    return (a == 0) ? Ev + 2 * dir * N : (a == 1) ? Ev + (2 * dir + 1) * N : (dir == 0 ? Bx : By) + (a - 2) * N;
  };
  for (int idx = t; idx < 2 * NH * N; idx += kThreads) {
    const int db = idx / N, k = idx - db * N, dir = db / NH, bb = db - dir * NH;
    const double* vb = hvec(dir, bb);
    double acc = 0.0;
#pragma unroll
    for (int kk = 0; kk < N; ++kk) acc += gxi[k * N + kk] * vb[kk];
    Wt[idx] = acc;
  }
  block_sync();
  for (int idx = t; idx < 2 * NH * NH; idx += kThreads) {
    const int dir = idx / (NH * NH), ab = idx % (NH * NH), a = ab / NH, bb = ab % NH;
    const double* va = hvec(dir, a);
    const double* wb = Wt + (dir * NH + bb) * N;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) acc += va[k] * wb[k];
    (dir == 0 ? Hx : Hy)[ab] = acc;
  }
  block_sync();
  double* rr = lds + L::oRr;
  // TU = (C G0^-1 C^T) U_r, entry (q1, q2) of C G0^-1 C^T = Hx[xa1][xa2] Hy[ya1][ya2];
  // then S0 = U_r^T TU, dense
  double* TU = lds + L::oTU;
  double* Sd = lds + L::oSd;
  constexpr int Rs = L::Rs;
  typedef Mma<double> M64;
  {
    constexpr int TTs = L::TTs, US = L::US, QB = (TT + 15) / 16;
    const int l = lane(), lr = l & 15, lk = l >> 4;
#pragma unroll 1
    for (int bidx = wv; bidx < QB * RB; bidx += 4) {
      const int I = bidx / RB, C = bidx % RB;
      const int q1 = 16 * I + lr, c = 16 * C + lr;
      const int w1 = q1 / N, j1 = q1 % N;
      const int xa1 = (w1 == 0) ? 0 : (w1 == 1) ? 1 : 2 + j1;
      const int ya1 = (w1 == 2) ? 0 : (w1 == 3) ? 1 : 2 + j1;
      M64::acc_t acc = zacc<double>();
#pragma unroll 4
      for (int kk = 0; kk < TT / 4; ++kk) {
        const int q = 4 * kk + lk;
        const int w2 = q / N, j2 = q % N;
        const int xa2 = (w2 == 0) ? 0 : (w2 == 1) ? 1 : 2 + j2;
        const int ya2 = (w2 == 2) ? 0 : (w2 == 3) ? 1 : 2 + j2;
        const double a = q1 < TT ? Hx[xa1 * NH + xa2] * Hy[ya1 * NH + ya2] : 0.0;
        const double bv = c < R ? U[c * US + q] : 0.0;
        acc = M64::mma(a, bv, acc);
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int row = 16 * I + M64::row(l, s4);
        if (row < TT && c < R) TU[c * TTs + row] = acc[s4];
      }
    }
    block_sync();
    // S0 blocks (I, J), J <= I, written to both triangles
#pragma unroll 1
    for (int bidx = wv; bidx < RB * (RB + 1) / 2; bidx += 4) {
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= bidx) ++I;
      const int J = bidx - I * (I + 1) / 2;
      const int c1 = 16 * I + lr, c2 = 16 * J + lr;
      M64::acc_t acc = zacc<double>();
#pragma unroll 4
      for (int kk = 0; kk < TT / 4; ++kk) {
        const int q = 4 * kk + lk;
        const double a = c1 < R ? U[c1 * US + q] : 0.0;
        const double bv = c2 < R ? TU[c2 * TTs + q] : 0.0;
        acc = M64::mma(a, bv, acc);
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        // lower triangle only, mirrored: the two triangles of a diagonal block
        // are computed separately and need not agree to the last bit
        const int row = 16 * I + M64::row(l, s4), col = c2;
        if (row < R && col < R && row >= col) {
          Sd[row * Rs + col] = acc[s4];
          Sd[col * Rs + row] = acc[s4];
        }
      }
    }
    block_sync();
  }
  if constexpr (L::kM) {
    // M_w = U_w^T B_w (R x N, K = N) on the matrix cores, RB tiles a wavefront,
    // held in registers until every read of the staged U_r is done, then
    // written over it
    const int l = lane(), lr = l & 15, lk = l >> 4;
    M64::acc_t macc[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int tl = wv + 4 * u, w = tl / RB, rt = tl - w * RB;
      const double* Bw = (w < 2) ? By : Bx;
      const int c = 16 * rt + lr;
      M64::acc_t acc = zacc<double>();
#pragma unroll
      for (int st = 0; st < (N + 3) / 4; ++st) {
        const int j = 4 * st + lk;
        const double av = (c < R && j < N) ? U[c * L::TTs + w * N + j] : 0.0;   // A[c][j]
        const double bv = (lr < N && j < N) ? Bw[j * N + lr] : 0.0;             // B[j][m]
        acc = M64::mma(av, bv, acc);
      }
      macc[u] = acc;
    }
    block_sync();
    double* Mm = lds + L::oU;
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int tl = wv + 4 * u, w = tl / RB, rt = tl - w * RB;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int c = 16 * rt + M64::row(l, s4);
        if (c < R && lr < N) Mm[(w * R + c) * N + lr] = macc[u][s4];
      }
    }
  }
  r_invert_S<N>(Sd, lds + L::oPiv);
  // particular solution x0 = first block of [[G0, C_r^T], [C_r, 0]]^-1 [b; g_r]
  double* b = lds + L::oB;
  double* x = lds + L::oXv;
  double* r = lds + L::oR;
  double* g = lds + L::oGv;
  double* pv = lds + L::oP;
  double* q = lds + L::oQ;
  double* t1 = lds + L::oT1;
  double* red = lds + L::oRed;
  const int64_t noff = p.noff[e];
  int its = 0, unconv = 0;
  double rmax = 0.0;
  // the components share everything above: the tables, S0^-1 and the M tables
  // (Sec. 5.3, last paragraph); each has its own carried values and boundary data
  for (int c = 0; c < p.ncomp; ++c) {
  const int64_t row = s * p.ncomp + c;
  if (c > 0) r_rhs<N>(p, lds, e, row);
  {
    double* gvc = lds + L::oE1;            // free here; the projection's scratch later
    r_upwind<N>(p, e, row, z.a, z.b, gvc);
    block_sync();
    r_UT<N>(p.ur + p.ur_off[N], gvc, rr, L::TT);   // g_r = U_r^T g
    block_sync();
  }
  r_Pproj<N>(lds, U, b, rr, x);
  const double xx = block_dot<N>(x, x, red);
  r_G<N>(lds, x, t1, r);
  for (int i = t; i < n; i += kThreads) r[i] -= b[i];
  block_sync();
  r_Pproj<N>(lds, U, r, nullptr, g);
  // residual update: r -= C_r^T y with the projection's multipliers (left in t2
  // by r_Pproj), which leaves g unchanged but keeps r, and with it the
  // rounding noise of the next projections, at the size of the error
  double* t2 = lds + L::oT2;
  for (int i = t; i < n; i += kThreads) r[i] -= t2[i];
  double rg, gg;
  block_rg_gg<N>(r, g, rg, gg, red + 8);
  const double stop = p.tol2 * xx;
  int it = 0;
  if (gg > stop) {
    for (int i = t; i < n; i += kThreads) pv[i] = -g[i];
    block_sync();
    for (it = 1; it <= p.max_iter; ++it) {
      r_G<N>(lds, pv, t1, q, red);   // q = G pv and pv^T q
      const double pq = red[0];
      const double alpha = rg / pq;
      for (int i = t; i < n; i += kThreads) {
        x[i] += alpha * pv[i];
        r[i] += alpha * q[i];
      }
      block_sync();
      r_Pproj<N>(lds, U, r, nullptr, g);
      for (int i = t; i < n; i += kThreads) r[i] -= t2[i];
      double rg1;
      block_rg_gg<N>(r, g, rg1, gg, red + 8);
      if (gg <= stop) break;
      const double beta = rg1 / rg;
      rg = rg1;
      for (int i = t; i < n; i += kThreads) pv[i] = beta * pv[i] - g[i];
      block_sync();
    }
  }
  // restore C_r x = g_r to working accuracy: x -= G0^-1 C_r^T S0^-1 (C_r x - g_r)
  // (after any iteration; the starting iterate satisfies it already)
  if (it > 0) {
    double* zz = lds + L::oZ0;
    double* e1 = lds + L::oE1;
    double* w1 = lds + L::oW1;
    double* w2 = lds + L::oW2;
    if constexpr (L::kM) {
      double* u = lds + L::oE2;
      const double* Mm = lds + L::oU;
      r_edge_contract<N>(Ev, x, u);
      block_sync();
      r_M_apply<N>(Mm, u, rr, w1);
      block_sync();
      r_Sinv<N>(lds + L::oSd, w1, w2);
      block_sync();
      r_MT_apply<N>(Mm, w2, u);
      block_sync();
      r_outer_edges<N>(Ev, u, t2);
      block_sync();
    } else {
      r_C<N>(Bx, By, Ev, x, e1);
      block_sync();
      r_UT<N>(U, e1, w1);
      block_sync();
      for (int c = t; c < R; c += kThreads) w1[c] -= rr[c];
      block_sync();
      r_Sinv<N>(lds + L::oSd, w1, w2);
      block_sync();
      r_U<N>(U, w2, e1);
      block_sync();
      r_CT<N>(Bx, By, Ev, e1, t2);
      block_sync();
    }
    r_G0inv<N>(gxi, t2, t1, zz);
    for (int i = t; i < n; i += kThreads) x[i] -= zz[i];
    block_sync();
  }
  // new values at the Gauss nodes (eq. phi_star)
  for (int i = t; i < n; i += kThreads) {
    const int ix = i % N, iy = i / N;
    double bxr[N];
#pragma unroll
    for (int k = 0; k < N; ++k) bxr[k] = Bx[ix * N + k];
    double v = 0.0;
#pragma unroll 1
    for (int ly = 0; ly < N; ++ly) {
      double inner = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) inner += bxr[k] * x[ly * N + k];
      v += By[iy * N + ly] * inner;
    }
    p.phi[row * p.nodes + noff + i] = v;
  }
  its += it > p.max_iter ? p.max_iter : it;
  unconv += gg <= stop ? 0 : 1;
  rmax = fmax(rmax, rel_resid(gg, xx));
  }
  count_fit(p, 2, its, unconv, 0, rmax);
}

template <int N>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(LayR<N>::waves1))) void fit2r_phase1(Params2D p) {
  extern __shared__ __attribute__((aligned(16))) double lds_r1[];
  r_phase1_body<N>(p, lds_r1, blockIdx.x + p.block0);
}

template <int N>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(LayR<N>::waves2))) void fit2r_phase2(Params2D p) {
  extern __shared__ __attribute__((aligned(16))) double lds_r2[];
  r_phase2_body<N>(p, lds_r2, blockIdx.x + p.block0);
}

template <int N>
static hipError_t launch_r(int phase, const Params2D& p, int64_t nfits, hipStream_t st) {
  const size_t lds = phase == 1 ? LayR<N>::bytes1 : LayR<N>::bytes2;
  const int64_t chunk = (int64_t)1 << 30;
  for (int64_t b0 = 0; b0 < nfits; b0 += chunk) {
    Params2D q = p;
    q.block0 = p.block0 + b0;
    const int64_t nb = (nfits - b0) < chunk ? (nfits - b0) : chunk;
    if (phase == 1)
      hipLaunchKernelGGL((fit2r_phase1<N>), dim3((unsigned)nb), dim3(kThreads), lds, st, q);
    else
      hipLaunchKernelGGL((fit2r_phase2<N>), dim3((unsigned)nb), dim3(kThreads), lds, st, q);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t launch_fit2r(int phase, int N, const Params2D& p, int64_t nfits, hipStream_t st) {
  switch (N) {
    case 2: return launch_r<2>(phase, p, nfits, st);
    case 3: return launch_r<3>(phase, p, nfits, st);
    case 4: return launch_r<4>(phase, p, nfits, st);
    case 5: return launch_r<5>(phase, p, nfits, st);
    case 6: return launch_r<6>(phase, p, nfits, st);
    case 7: return launch_r<7>(phase, p, nfits, st);
    case 8: return launch_r<8>(phase, p, nfits, st);
    case 9: return launch_r<9>(phase, p, nfits, st);
    case 10: return launch_r<10>(phase, p, nfits, st);
    case 11: return launch_r<11>(phase, p, nfits, st);
    case 12: return launch_r<12>(phase, p, nfits, st);
    case 13: return launch_r<13>(phase, p, nfits, st);
    case 14: return launch_r<14>(phase, p, nfits, st);
    case 15: return launch_r<15>(phase, p, nfits, st);
    case 16: return launch_r<16>(phase, p, nfits, st);
    default: return hipErrorInvalidValue;
  }
}

// One order of several problems in one launch: one workgroup per fit of the
// segments (problem, order group) of the argument table, all of order N.
template <int N, int PHASE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(PHASE == 1 ? LayR<N>::waves1 : LayR<N>::waves2)))
void fit2r_multi(Fused2DArgs a) {
  extern __shared__ __attribute__((aligned(16))) double lds_rm[];
  const int64_t item = blockIdx.x;
  int sg = 0;
  while (sg + 1 < a.nseg && item >= a.seg[sg + 1].start) ++sg;
  const Params2D& p = *a.task[a.seg[sg].task];
  const int64_t fit = a.seg[sg].fit0 + (item - a.seg[sg].start);
  if constexpr (PHASE == 1) r_phase1_body<N>(p, lds_rm, fit);
  else r_phase2_body<N>(p, lds_rm, fit);
}

template <int N>
static hipError_t multi_n(int phase, const Fused2DArgs& a, hipStream_t st) {
  const size_t lds = phase == 1 ? LayR<N>::bytes1 : LayR<N>::bytes2;
  if (a.total <= 0) return hipSuccess;
  if (phase == 1) hipLaunchKernelGGL((fit2r_multi<N, 1>), dim3((unsigned)a.total), dim3(kThreads), lds, st, a);
  else hipLaunchKernelGGL((fit2r_multi<N, 2>), dim3((unsigned)a.total), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_fit2r_multi(int phase, int N, const Fused2DArgs& a, hipStream_t st) {
  switch (N) {
    case 2: return multi_n<2>(phase, a, st);
    case 3: return multi_n<3>(phase, a, st);
    case 4: return multi_n<4>(phase, a, st);
    case 5: return multi_n<5>(phase, a, st);
    case 6: return multi_n<6>(phase, a, st);
    case 7: return multi_n<7>(phase, a, st);
    case 8: return multi_n<8>(phase, a, st);
    case 9: return multi_n<9>(phase, a, st);
    case 10: return multi_n<10>(phase, a, st);
    case 11: return multi_n<11>(phase, a, st);
    case 12: return multi_n<12>(phase, a, st);
    case 13: return multi_n<13>(phase, a, st);
    case 14: return multi_n<14>(phase, a, st);
    case 15: return multi_n<15>(phase, a, st);
    case 16: return multi_n<16>(phase, a, st);
    default: return hipErrorInvalidValue;
  }
}

// Persistent fused kernel over every order (2..16) of several problems, as
// the factorisation kernels' fused form: segments largest order first, a
// device work counter, each order outlined with its own registers.
__device__ __forceinline__ int64_t uniform64r(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int N, int PHASE>
__device__ __attribute__((noinline)) void fused_fit_r(const Params2D* pp, int64_t fit) {
  extern __shared__ __attribute__((aligned(16))) double lds_rf[];
  const Params2D& p = *(const Params2D*)(uintptr_t)(uint64_t)uniform64r((int64_t)(uintptr_t)pp);
  fit = uniform64r(fit);
  if constexpr (PHASE == 1) r_phase1_body<N>(p, lds_rf, fit);
  else r_phase2_body<N>(p, lds_rf, fit);
}

template <int PHASE>
__global__ __launch_bounds__(kThreads) void fit2r_fused(Fused2DArgs a) {
  __shared__ int64_t item_sh;
  for (;;) {
    if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(a.counter, 1ull);
    __syncthreads();
    const int64_t item = uniform64r(item_sh);
    __syncthreads();
    if (item >= a.total) break;
    int sg = 0;
    while (sg + 1 < a.nseg && item >= a.seg[sg + 1].start) ++sg;
    const Params2D* p = a.task[a.seg[sg].task];
    const int64_t fit = a.seg[sg].fit0 + (item - a.seg[sg].start);
    switch (a.seg[sg].N) {
      case 2: fused_fit_r<2, PHASE>(p, fit); break;
      case 3: fused_fit_r<3, PHASE>(p, fit); break;
      case 4: fused_fit_r<4, PHASE>(p, fit); break;
      case 5: fused_fit_r<5, PHASE>(p, fit); break;
      case 6: fused_fit_r<6, PHASE>(p, fit); break;
      case 7: fused_fit_r<7, PHASE>(p, fit); break;
      case 8: fused_fit_r<8, PHASE>(p, fit); break;
      case 9: fused_fit_r<9, PHASE>(p, fit); break;
      case 10: fused_fit_r<10, PHASE>(p, fit); break;
      case 11: fused_fit_r<11, PHASE>(p, fit); break;
      case 12: fused_fit_r<12, PHASE>(p, fit); break;
      case 13: fused_fit_r<13, PHASE>(p, fit); break;
      case 14: fused_fit_r<14, PHASE>(p, fit); break;
      case 15: fused_fit_r<15, PHASE>(p, fit); break;
      case 16: fused_fit_r<16, PHASE>(p, fit); break;
      default: break;
    }
    __syncthreads();
  }
}

hipError_t launch_fit2r_fused(int phase, const Fused2DArgs& a, int grid, size_t lds, hipStream_t st) {
  if (phase == 1) hipLaunchKernelGGL((fit2r_fused<1>), dim3(grid), dim3(kThreads), lds, st, a);
  else hipLaunchKernelGGL((fit2r_fused<2>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

int fit2r_fused_occupancy(int phase, size_t lds) {
  int nb = 0;
  hipError_t e = phase == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit2r_fused<1>, kThreads, lds)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit2r_fused<2>, kThreads, lds);
  return e == hipSuccess ? nb : 0;
}

template <int N>
static size_t lds_r(int phase) { return phase == 1 ? LayR<N>::bytes1 : LayR<N>::bytes2; }

size_t fit2r_lds_bytes(int N, int phase) {
  switch (N) {
    case 2: return lds_r<2>(phase);
    case 3: return lds_r<3>(phase);
    case 4: return lds_r<4>(phase);
    case 5: return lds_r<5>(phase);
    case 6: return lds_r<6>(phase);
    case 7: return lds_r<7>(phase);
    case 8: return lds_r<8>(phase);
    case 9: return lds_r<9>(phase);
    case 10: return lds_r<10>(phase);
    case 11: return lds_r<11>(phase);
    case 12: return lds_r<12>(phase);
    case 13: return lds_r<13>(phase);
    case 14: return lds_r<14>(phase);
    case 15: return lds_r<15>(phase);
    case 16: return lds_r<16>(phase);
    default: return 0;
  }
}

}  // namespace sl
