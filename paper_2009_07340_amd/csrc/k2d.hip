// Two-dimensional step: two kernels per step, one wavefront per (element, sample) fit.
//
// Phase 1 (per fit): move the n = N^2 nodes (eq. def_dx), carry the values
// with the source (eq. advection_phi), build the Legendre basis centred on the
// mean displacement, form the Gram matrix G = V^T V on the matrix cores,
// factor it (blocked Cholesky, MFMA panel and trailing updates), solve for
// the advected interpolant p0 (eqs. phi_stardef, h_star) and write its values
// at the element's own 4N edge points (eq. remap_bnd) to the trace buffer.
//
// Phase 2 (per fit, after every trace exists): rebuild and refactor G,
// upwind the boundary data from the neighbours' traces (eq. bnd_update,
// periodic image or Dirichlet ghost), project the trace mismatch onto the
// edge-value space of Q_{N-1} (basis U_r, 4N-4 columns), and apply the
// range-space (Lagrange multiplier) solution of the constrained least-squares
// remap:  c = c0 - G^-1 C_r^T S^-1 (C_r c0 - g_r),  C_r = U_r^T C,
//         S = C_r G^-1 C_r^T = Y^T Y with Y = L^-1 C_r^T,
// then evaluate p at the Gauss nodes (eq. phi_star) into the sample state.
#include "sl_internal.hpp"
#include "philox.hpp"
#include "fit1d.hpp"
#include "fit2d.hpp"

namespace sl {

using namespace f2;

template <int N>
struct Dims {
  static constexpr int n = N * N;
  static constexpr int NB = (n + 15) / 16;
  static constexpr int T = 4 * N;
  static constexpr int R = 4 * N - 4;
  static constexpr int RB = (R + 15) / 16;
  // LDS regions (doubles)
  static constexpr int oG = 0;
  static constexpr int oLinv = oG + NB * (NB + 1) / 2 * BLK;
  static constexpr int oTab = oLinv + NB * BLK;                 // X1, Y1 (phase 1 view) or Y blocks (phase 2)
  static constexpr int tabA = 2 * n * N;
  static constexpr int tabB = NB * RB * BLK;
  static constexpr int oY = oTab;
  static constexpr int oS = oTab + (tabA > tabB ? tabA : tabB);
  static constexpr int oSinv = oS + RB * (RB + 1) / 2 * BLK;
  static constexpr int oBx = oSinv + RB * BLK;
  static constexpr int oBy = oBx + N * N;
  static constexpr int oE = oBy + N * N;                        // ex0, ex1, ey0, ey1
  static constexpr int oF = oE + 4 * N;                         // f (n)
  static constexpr int oC = oF + 16 * NB;                       // b -> c0 (16 NB)
  static constexpr int oW = oC + 16 * NB;                       // work vector (16 NB)
  static constexpr int oTmp = oW + 16 * NB;                     // 16
  static constexpr int oT = oTmp + 16;                          // traces t (T)
  static constexpr int oRho = oT + T;                           // t - g (T)
  static constexpr int oRr = oRho + T;                          // projected mismatch (16 RB)
  static constexpr int oXs = oRr + 16 * RB;                     // moved x (n)
  static constexpr int oYs = oXs + n;                           // moved y (n)
  static constexpr int total = oYs + n;
};

template <int N>
size_t lds_bytes_2d() { return sizeof(double) * Dims<N>::total; }

// Shared part of both phases: nodes, basis tables, Gram matrix, Cholesky, c0,
// and the edge/Gauss-node basis tables.  Returns dbar in (dbx, dby).
template <int N>
__device__ __forceinline__ void fit2d_common(const Params2D& p, double* lds, int e, int64_t s, double za, double zb) {
  using Dm = Dims<N>;
  constexpr int n = Dm::n, NB = Dm::NB;
  const int l = lane_id();
  const int64_t noff = p.noff[e];
  double* X1 = lds + Dm::oTab;
  double* Y1 = X1 + n * N;
  double* f = lds + Dm::oF;
  double* xs = lds + Dm::oXs;
  double* ys = lds + Dm::oYs;
  // moved nodes and carried values; displacement sums for the centring
  double sx = 0.0, sy = 0.0;
  for (int i = l; i < n; i += 64) {
    const int64_t k = noff + i;
    const double x0 = p.xi_node[2 * k], y0 = p.xi_node[2 * k + 1];
    const double x = moved_coord(x0, p.A[2 * k], p.B[2 * k], za);
    const double y = moved_coord(y0, p.A[2 * k + 1], p.B[2 * k + 1], zb);
    xs[i] = x;
    ys[i] = y;
    f[i] = p.phi[s * p.nodes + k] * p.src[k];
    sx += x - x0;
    sy += y - y0;
  }
  const double dbx = wave_sum(sx) / n, dby = wave_sum(sy) / n;
  wave_sync();
  // 1-D basis at the moved nodes
  for (int i = l; i < n; i += 64) {
    double px[N], py[N];
    legendre_eval<N>(xs[i] - dbx, p.rec, px);
    legendre_eval<N>(ys[i] - dby, p.rec, py);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      X1[i * N + k] = px[k];
      Y1[i * N + k] = py[k];
    }
  }
  // basis at the element's own Gauss abscissae and edges (for traces and evaluation)
  double* Bx = lds + Dm::oBx;
  double* By = lds + Dm::oBy;
  double* Ev = lds + Dm::oE;
  if (l < N) {
    double px[N], py[N];
    legendre_eval<N>(p.xi_tab[N * kMaxN + l] - dbx, p.rec, px);
    legendre_eval<N>(p.xi_tab[N * kMaxN + l] - dby, p.rec, py);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      Bx[l * N + k] = px[k];
      By[l * N + k] = py[k];
    }
  } else if (l < N + 4) {
    const int w = l - N;
    double q[N];
    const double t = (w == 0) ? -dbx : (w == 1) ? 1.0 - dbx : (w == 2) ? -dby : 1.0 - dby;
    legendre_eval<N>(t, p.rec, q);
#pragma unroll
    for (int k = 0; k < N; ++k) Ev[w * N + k] = q[k];
  }
  wave_sync();
  // right-hand side b = V^T f, V[i][(k,l)] = X1[i][k] Y1[i][l]
  double* c = lds + Dm::oC;
  for (int q = l; q < 16 * NB; q += 64) {
    double acc = 0.0;
    if (q < n) {
      const int k = q % N, ly = q / N;
      for (int i = 0; i < n; ++i) acc += X1[i * N + k] * Y1[i * N + ly] * f[i];
    }
    c[q] = acc;
  }
  // Gram matrix G = V^T V on the matrix cores, one block row at a time
  double* G = lds + Dm::oG;
#pragma unroll 1
  for (int P = 0; P < NB; ++P) {
    d4 acc[NB];
#pragma unroll
    for (int Q = 0; Q < NB; ++Q) acc[Q] = zero4();
    const int pc = 16 * P + (l & 15);
    const int kP = pc % N, lP = pc / N;
#pragma unroll 1
    for (int kk = 0; kk < 4 * NB; ++kk) {
      const int node = 4 * kk + (l >> 4);
      const bool live = node < n;
      const double a = (live && pc < n) ? X1[node * N + kP] * Y1[node * N + lP] : 0.0;
#pragma unroll
      for (int Q = 0; Q < NB; ++Q) {
        if (Q >= P) {
          const int qc = 16 * Q + (l & 15);
          const double b = (live && qc < n) ? X1[node * N + (qc % N)] * Y1[node * N + (qc / N)] : 0.0;
          acc[Q] = mfma(a, b, acc[Q]);
        }
      }
    }
    // acc[Q] holds G[16P + i][16Q + j]; store as lower block (Q, P), transposed
#pragma unroll
    for (int Q = 0; Q < NB; ++Q) {
      if (Q >= P) {
        double* Bq = G + tblk(Q, P) * BLK;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int i = (l >> 4) + 4 * s4, j = l & 15;
          Bq[j * BS + i] = acc[Q][s4];
        }
      }
    }
  }
  wave_sync();
  cholesky<NB>(G, lds + Dm::oLinv, n);
  forward_solve<NB>(G, lds + Dm::oLinv, c, lds + Dm::oTmp);
  backward_solve<NB>(G, lds + Dm::oLinv, c, lds + Dm::oTmp);   // c = c0
}

// Value of the polynomial with coefficients c at own edge point q (w = q / N, j = q % N).
template <int N>
__device__ __forceinline__ double edge_value(const double* lds, const double* c, int q) {
  using Dm = Dims<N>;
  const double* Bx = lds + Dm::oBx;
  const double* By = lds + Dm::oBy;
  const double* Ev = lds + Dm::oE;
  const int w = q / N, j = q % N;
  double t = 0.0;
#pragma unroll
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
  return t;
}

// Basis value C[q][p] of coefficient p = (k, ly) at own edge point q.
template <int N>
__device__ __forceinline__ double edge_basis(const double* lds, int q, int pidx) {
  using Dm = Dims<N>;
  const double* Bx = lds + Dm::oBx;
  const double* By = lds + Dm::oBy;
  const double* Ev = lds + Dm::oE;
  const int w = q / N, j = q % N, k = pidx % N, ly = pidx / N;
  const double bx = (w == 0) ? Ev[k] : (w == 1) ? Ev[N + k] : Bx[j * N + k];
  const double by = (w < 2) ? By[j * N + ly] : (w == 2) ? Ev[2 * N + ly] : Ev[3 * N + ly];
  return bx * by;
}

__device__ __forceinline__ void fit_index(const Params2D& p, int64_t b, int& e, int64_t& s) {
  const int64_t w = b / p.M;
  s = b - w * p.M;
  e = p.work[w];
}

template <int N>
__global__ __launch_bounds__(64) void fit2d_phase1(Params2D p) {
  extern __shared__ double lds[];
  using Dm = Dims<N>;
  int e;
  int64_t s;
  fit_index(p, blockIdx.x + (int64_t)p.block0, e, s);
  const Normal2 z = normal_pair(p.seed, p.stream, (uint64_t)p.step, (uint64_t)s);
  fit2d_common<N>(p, lds, e, s, z.a, z.b);
  const double* c = lds + Dm::oC;
  const int l = lane_id();
  const int64_t eoff = p.eoff[e];
  for (int q = l; q < Dm::T; q += 64) p.tr[s * p.edges + eoff + q] = edge_value<N>(lds, c, q);
}

template <int N>
__global__ __launch_bounds__(64) void fit2d_phase2(Params2D p) {
  extern __shared__ double lds[];
  using Dm = Dims<N>;
  constexpr int n = Dm::n, NB = Dm::NB, T = Dm::T, R = Dm::R, RB = Dm::RB;
  int e;
  int64_t s;
  fit_index(p, blockIdx.x + (int64_t)p.block0, e, s);
  const Normal2 z = normal_pair(p.seed, p.stream, (uint64_t)p.step, (uint64_t)s);
  fit2d_common<N>(p, lds, e, s, z.a, z.b);
  const int l = lane_id();
  const int64_t eoff = p.eoff[e];
  double* c = lds + Dm::oC;
  double* rho = lds + Dm::oRho;
  double* tt = lds + Dm::oT;
  // upwinded boundary data (eq. bnd_update) and the trace mismatch t - g
  for (int q = l; q < T; q += 64) {
    const int w = q / N, j = q % N;
    const double t = p.tr[s * p.edges + eoff + q];
    const double zd = (w < 2) ? z.a : z.b;
    const double disp = __dadd_rn(p.Af[eoff + q], __dmul_rn(p.Bf[eoff + q], zd));
    const bool pos = disp > 0.0;
    const bool take_nbr = (w == 0 || w == 2) ? pos : !pos;   // W, S: neighbour is the negative side
    double g = t;
    if (take_nbr) {
      const int nb = p.nbr[4 * e + w];
      if (nb < 0) {
        g = p.ghost[eoff + q];
      } else {
        const int Ns = p.order[nb];
        const int opp = w ^ 1;
        const double* src = p.tr + s * p.edges + p.eoff[nb] + opp * Ns;
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
    tt[q] = t;
    rho[q] = t - g;
  }
  wave_sync();
  // projected mismatch rho_r = U_r^T (t - g)
  const double* U = p.ur + p.ur_off[N];   // column-major T x R
  double* rr = lds + Dm::oRr;
  for (int cidx = l; cidx < 16 * RB; cidx += 64) {
    double acc = 0.0;
    if (cidx < R)
      for (int q = 0; q < T; ++q) acc += U[cidx * T + q] * rho[q];
    rr[cidx] = acc;
  }
  // C_r^T = C^T U_r (n x R) into the Y blocks, padded with zeros
  double* Y = lds + Dm::oY;
  for (int idx = l; idx < 16 * NB * 16 * RB; idx += 64) {
    const int pr = idx / (16 * RB), cc = idx % (16 * RB);
    double acc = 0.0;
    if (pr < n && cc < R)
      for (int q = 0; q < T; ++q) acc += edge_basis<N>(lds, q, pr) * U[cc * T + q];
    Y[((pr >> 4) * RB + (cc >> 4)) * BLK + (pr & 15) * BS + (cc & 15)] = acc;
  }
  wave_sync();
  // Y = L^-1 C_r^T, block row by block row
  const double* G = lds + Dm::oG;
  const double* Linv = lds + Dm::oLinv;
  double* Tb = lds + Dm::oS;   // scratch block (S is formed afterwards)
#pragma unroll 1
  for (int kb = 0; kb < NB; ++kb) {
#pragma unroll 1
    for (int C = 0; C < RB; ++C) {
      double* Ykc = Y + (kb * RB + C) * BLK;
      d4 acc = load_acc(Ykc);
#pragma unroll 1
      for (int J = 0; J < kb; ++J) {
        const double* LB = G + tblk(kb, J) * BLK;
        const double* YJ = Y + (J * RB + C) * BLK;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = mfma(-rowpat(LB, kk), colpat(YJ, kk), acc);
      }
      store_acc(Tb, acc);
      wave_sync();
      d4 out = zero4();
      const double* Li = Linv + kb * BLK;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) out = mfma(rowpat(Li, kk), colpat(Tb, kk), out);
      store_acc(Ykc, out);
      wave_sync();
    }
  }
  // S = Y^T Y (R x R, lower blocks)
  double* S = lds + Dm::oS;
#pragma unroll 1
  for (int C1 = 0; C1 < RB; ++C1) {
#pragma unroll 1
    for (int C2 = 0; C2 <= C1; ++C2) {
      d4 acc = zero4();
#pragma unroll 1
      for (int kb = 0; kb < NB; ++kb) {
        const double* A1 = Y + (kb * RB + C1) * BLK;
        const double* A2 = Y + (kb * RB + C2) * BLK;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = mfma(colpat(A1, kk), colpat(A2, kk), acc);
      }
      store_acc(S + tblk(C1, C2) * BLK, acc);
    }
  }
  wave_sync();
  cholesky<RB>(S, lds + Dm::oSinv, R);
  // lambda = S^-1 rho_r
  forward_solve<RB>(S, lds + Dm::oSinv, rr, lds + Dm::oTmp);
  backward_solve<RB>(S, lds + Dm::oSinv, rr, lds + Dm::oTmp);
  // w = Y lambda; x = L^-T w; c = c0 - x
  double* wv = lds + Dm::oW;
  for (int pr = l; pr < 16 * NB; pr += 64) {
    double acc = 0.0;
    const int I = pr >> 4, r = pr & 15;
    for (int C = 0; C < RB; ++C) {
      const double* YB = Y + (I * RB + C) * BLK;
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) acc += YB[r * BS + cc] * rr[16 * C + cc];
    }
    wv[pr] = acc;
  }
  wave_sync();
  backward_solve<NB>(G, Linv, wv, lds + Dm::oTmp);
  for (int pr = l; pr < 16 * NB; pr += 64) c[pr] -= wv[pr];
  wave_sync();
  // new values at the Gauss nodes (eq. phi_star): p(xi_ix, xi_iy)
  const double* Bx = lds + Dm::oBx;
  const double* By = lds + Dm::oBy;
  const int64_t noff = p.noff[e];
  for (int i = l; i < n; i += 64) {
    const int ix = i % N, iy = i / N;
    double v = 0.0;
#pragma unroll
    for (int ly = 0; ly < N; ++ly) {
      double inner = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) inner += Bx[ix * N + k] * c[ly * N + k];
      v += By[iy * N + ly] * inner;
    }
    p.phi[s * p.nodes + noff + i] = v;
  }
}

template <int N>
static hipError_t launch_phase(int phase, const Params2D& p, int64_t nfits, hipStream_t st) {
  const size_t lds = lds_bytes_2d<N>();
  // grids are split so that blockIdx.x stays below 2^31
  const int64_t chunk = (int64_t)1 << 30;
  for (int64_t b0 = 0; b0 < nfits; b0 += chunk) {
    Params2D q = p;
    q.block0 = p.block0 + b0;
    const int64_t nb = (nfits - b0) < chunk ? (nfits - b0) : chunk;
    if (phase == 1)
      hipLaunchKernelGGL(fit2d_phase1<N>, dim3((unsigned)nb), dim3(64), lds, st, q);
    else
      hipLaunchKernelGGL(fit2d_phase2<N>, dim3((unsigned)nb), dim3(64), lds, st, q);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

size_t fit2d_lds_bytes(int N) {
  switch (N) {
    case 2: return lds_bytes_2d<2>();
    case 3: return lds_bytes_2d<3>();
    case 4: return lds_bytes_2d<4>();
    case 5: return lds_bytes_2d<5>();
    case 6: return lds_bytes_2d<6>();
    case 7: return lds_bytes_2d<7>();
    case 8: return lds_bytes_2d<8>();
    case 9: return lds_bytes_2d<9>();
    case 10: return lds_bytes_2d<10>();
    default: return 0;
  }
}

hipError_t launch_fit2d(int phase, int N, const Params2D& p, int64_t nfits, hipStream_t st) {
  switch (N) {
    case 2: return launch_phase<2>(phase, p, nfits, st);
    case 3: return launch_phase<3>(phase, p, nfits, st);
    case 4: return launch_phase<4>(phase, p, nfits, st);
    case 5: return launch_phase<5>(phase, p, nfits, st);
    case 6: return launch_phase<6>(phase, p, nfits, st);
    case 7: return launch_phase<7>(phase, p, nfits, st);
    case 8: return launch_phase<8>(phase, p, nfits, st);
    case 9: return launch_phase<9>(phase, p, nfits, st);
    case 10: return launch_phase<10>(phase, p, nfits, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sl
