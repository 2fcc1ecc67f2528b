// Two-dimensional step: two kernels per step, one workgroup (four wavefronts)
// per (element, sample) fit.
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
//
// Precision modes (template MODE):
//   0  float64 everywhere (Gram, factors, Y and S on v_mfma_f64_16x16x4f64);
//   1  Gram, Cholesky, Y and S in float32 (v_mfma_f32_16x16x4f32), then
//      float64 iterative refinement of the full constrained (KKT) system with
//      float64 residuals b - V^T V c - C_r^T lambda and g_r - C_r c;
//   2  as 1, but the Gram products use bf16 hi/lo splits of V
//      (V^T V ~ Vh^T Vh + Vh^T Vl + Vl^T Vh, v_mfma_f32_16x16x32_bf16,
//      float32 accumulation), with more refinement sweeps.
#include <type_traits>

#include "sl_internal.hpp"
#include "philox.hpp"
#include "fit1d.hpp"
#include "blocks.hpp"

namespace sl {

using namespace blk;

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int N, int MODE>
struct Lay {
  typedef typename std::conditional<MODE == 0, double, float>::type T;
  static constexpr int n = N * N;
  static constexpr int NB = (n + 15) / 16;
  static constexpr int NP = 16 * NB;
  static constexpr int TT = 4 * N;
  static constexpr int R = 4 * N - 4;
  static constexpr int RB = (R + 15) / 16;
  static constexpr int RP = 16 * RB;
  static constexpr size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }
  // byte offsets: [G][float64 scalars][basis tables | Y][S]; phase 1 needs the
  // first three only, so it launches with less LDS (more fits per CU)
  static constexpr size_t oG = 0;
  static constexpr size_t gBytes = sizeof(T) * NB * (NB + 1) / 2 * BLK;
  static constexpr size_t oD = a16(oG + gBytes);
  // double-element offsets relative to oD
  static constexpr int dBx = 0;
  static constexpr int dBy = dBx + N * N;
  static constexpr int dE = dBy + N * N;
  static constexpr int dF = dE + 4 * N;
  static constexpr int dB = dF + NP;
  static constexpr int dC = dB + NP;
  static constexpr int dW = dC + NP;
  static constexpr int dV = dW + NP;
  static constexpr int dTmp = dV + NP;
  static constexpr int dCol = dTmp + 64;
  static constexpr int dT = dCol + 20;
  static constexpr int dG = dT + TT;
  static constexpr int dE1 = dG + TT;
  static constexpr int dE2 = dE1 + TT;
  static constexpr int dRr = dE2 + TT;
  static constexpr int dLam = dRr + RP;
  static constexpr int dDl = dLam + RP;
  static constexpr int dR2 = dDl + RP;
  static constexpr int dXs = dR2 + RP;
  static constexpr int dYs = dXs + n;
  static constexpr int dRed = dYs + n;
  static constexpr int dEnd = dRed + 16;
  static constexpr size_t oTab = a16(oD + sizeof(double) * dEnd);          // X1, Y1 (float64)
  static constexpr size_t tabBytes = sizeof(double) * 2 * n * N;
  static constexpr size_t yBytes = sizeof(double) * NB * RB * BLK;       // Y, S are float64 in every mode
  // float64 mode: Y overwrites the basis tables once G is formed; mixed modes keep them
  static constexpr size_t oY = MODE == 0 ? oTab : a16(oTab + tabBytes);
  static constexpr size_t oS = a16(MODE == 0 ? oTab + (tabBytes > yBytes ? tabBytes : yBytes) : oY + yBytes);
  static constexpr size_t total = a16(oS + sizeof(double) * RB * (RB + 1) / 2 * BLK);
  static constexpr size_t phase1 = a16(oTab + tabBytes);
};

template <int N, int MODE>
struct Ctx {
  using L = Lay<N, MODE>;
  using T = typename L::T;
  char* base;
  __device__ T* G() const { return (T*)(base + L::oG); }
  __device__ double* X1() const { return (double*)(base + L::oTab); }
  __device__ double* Y1() const { return X1() + L::n * N; }
  __device__ double* Y() const { return (double*)(base + L::oY); }
  __device__ double* S() const { return (double*)(base + L::oS); }
  __device__ double* d(int off) const { return (double*)(base + L::oD) + off; }
};

// ---------------------------------------------------------------- float64 operators

// out[i] = (V c)_i, i < n
template <int N, int MODE>
__device__ void op_V(const Ctx<N, MODE>& x, const double* c, double* out) {
  using L = Lay<N, MODE>;
  const double* X1 = x.X1();
  const double* Y1 = x.Y1();
  for (int i = tid(); i < L::n; i += kThreads) {
    double xr[N];
#pragma unroll
    for (int k = 0; k < N; ++k) xr[k] = X1[i * N + k];
    double v = 0.0;
#pragma unroll 1
    for (int ly = 0; ly < N; ++ly) {
      double inner = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) inner += xr[k] * c[ly * N + k];
      v += Y1[i * N + ly] * inner;
    }
    out[i] = v;
  }
}

// out[p] = (V^T r)_p, p < NP (zero padding)
template <int N, int MODE>
__device__ void op_VT(const Ctx<N, MODE>& x, const double* r, double* out) {
  using L = Lay<N, MODE>;
  const double* X1 = x.X1();
  const double* Y1 = x.Y1();
  for (int p = tid(); p < L::NP; p += kThreads) {
    double acc = 0.0;
    if (p < L::n) {
      const int k = p % N, ly = p / N;
#pragma unroll 4
      for (int i = 0; i < L::n; ++i) acc += X1[i * N + k] * Y1[i * N + ly] * r[i];
    }
    out[p] = acc;
  }
}

// out[q] = (C c)_q, the polynomial at own edge point q (W, E, S, N blocks of N)
template <int N, int MODE>
__device__ void op_C(const Ctx<N, MODE>& x, const double* c, double* out) {
  using L = Lay<N, MODE>;
  const double* Bx = x.d(L::dBx);
  const double* By = x.d(L::dBy);
  const double* Ev = x.d(L::dE);
  for (int q = tid(); q < L::TT; q += kThreads) {
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

// out[p] = (C^T v)_p, p < NP
template <int N, int MODE>
__device__ void op_CT(const Ctx<N, MODE>& x, const double* v, double* out) {
  using L = Lay<N, MODE>;
  const double* Bx = x.d(L::dBx);
  const double* By = x.d(L::dBy);
  const double* Ev = x.d(L::dE);
  for (int p = tid(); p < L::NP; p += kThreads) {
    double acc = 0.0;
    if (p < L::n) {
      const int k = p % N, ly = p / N;
      const double e0 = Ev[k], e1 = Ev[N + k], f0 = Ev[2 * N + ly], f1 = Ev[3 * N + ly];
#pragma unroll 2
      for (int j = 0; j < N; ++j)
        acc += By[j * N + ly] * (e0 * v[j] + e1 * v[N + j]) + Bx[j * N + k] * (f0 * v[2 * N + j] + f1 * v[3 * N + j]);
    }
    out[p] = acc;
  }
}

// out[c] = (U_r^T v)_c, c < RP;  U column-major T x R
template <int N, int MODE>
__device__ void op_UT(const double* U, const double* v, double* out) {
  using L = Lay<N, MODE>;
  for (int c = tid(); c < L::RP; c += kThreads) {
    double acc = 0.0;
    if (c < L::R) {
#pragma unroll 4
      for (int q = 0; q < L::TT; ++q) acc += U[c * L::TT + q] * v[q];
    }
    out[c] = acc;
  }
}

// out[q] = (U_r w)_q
template <int N, int MODE>
__device__ void op_U(const double* U, const double* w, double* out) {
  using L = Lay<N, MODE>;
  for (int q = tid(); q < L::TT; q += kThreads) {
    double acc = 0.0;
#pragma unroll 4
    for (int c = 0; c < L::R; ++c) acc += U[c * L::TT + q] * w[c];
    out[q] = acc;
  }
}

// G^-1 v in place with the (storage-precision) factor; whole workgroup calls it.
template <int N, int MODE>
__device__ void g_solve(const Ctx<N, MODE>& x, double* v) {
  using L = Lay<N, MODE>;
  block_sync();
  if (wave() == 0) {
    forward_solve<typename L::T, L::NB>(x.G(), v);
    backward_solve<typename L::T, L::NB>(x.G(), v);
  }
  block_sync();
}

template <int N, int MODE>
__device__ void s_solve(const Ctx<N, MODE>& x, double* v) {
  using L = Lay<N, MODE>;
  block_sync();
  if (wave() == 0) {
    forward_solve<double, L::RB>(x.S(), v);
    backward_solve<double, L::RB>(x.S(), v);
  }
  block_sync();
}

// ---------------------------------------------------------------- shared set-up

// Moved nodes, carried values, centred basis tables, b = V^T f, Gram on the
// matrix cores, Cholesky, c0 (refined in the mixed modes).
template <int N, int MODE>
__device__ int setup_and_factor(const Params2D& p, const Ctx<N, MODE>& x, int e, int64_t s, double za,
                                double zb) {
  using L = Lay<N, MODE>;
  using T = typename L::T;
  constexpr int n = L::n, NB = L::NB;
  const int t = tid();
  const int64_t noff = p.noff[e];
  double* xs = x.d(L::dXs);
  double* ys = x.d(L::dYs);
  double* f = x.d(L::dF);
  double* red = x.d(L::dRed);
  double sx = 0.0, sy = 0.0;
  int esc = 0;
  for (int i = t; i < L::NP; i += kThreads) {
    if (i < n) {
      const int64_t k = noff + i;
      const double x0 = p.xi_node[2 * k], y0 = p.xi_node[2 * k + 1];
      const double xm = moved_coord(x0, p.A[2 * k], p.B[2 * k], za);
      const double ym = moved_coord(y0, p.A[2 * k + 1], p.B[2 * k + 1], zb);
      xs[i] = xm;
      ys[i] = ym;
      f[i] = p.phi[s * p.nodes + k] * p.src[k];
      sx += xm - x0;
      sy += ym - y0;
      esc += escaped(xm) + escaped(ym);
    } else {
      f[i] = 0.0;
    }
  }
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
  double* X1 = x.X1();
  double* Y1 = x.Y1();
  for (int i = t; i < n; i += kThreads) {
    double px[N], py[N];
    legendre_eval<N>(xs[i] - dbx, p.rec, px);
    legendre_eval<N>(ys[i] - dby, p.rec, py);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      X1[i * N + k] = px[k];
      Y1[i * N + k] = py[k];
    }
  }
  double* Bx = x.d(L::dBx);
  double* By = x.d(L::dBy);
  double* Ev = x.d(L::dE);
  if (t < N) {
    double px[N], py[N];
    legendre_eval<N>(p.xi_tab[N * kMaxN + t] - dbx, p.rec, px);
    legendre_eval<N>(p.xi_tab[N * kMaxN + t] - dby, p.rec, py);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      Bx[t * N + k] = px[k];
      By[t * N + k] = py[k];
    }
  } else if (t >= 64 && t < 68) {
    const int w = t - 64;
    double q[N];
    const double a = (w == 0) ? -dbx : (w == 1) ? 1.0 - dbx : (w == 2) ? -dby : 1.0 - dby;
    legendre_eval<N>(a, p.rec, q);
#pragma unroll
    for (int k = 0; k < N; ++k) Ev[w * N + k] = q[k];
  }
  block_sync();
  double* b = x.d(L::dB);
  op_VT<N, MODE>(x, f, b);
  // Gram matrix, lower blocks; block (P, Q), P <= Q, goes to storage block (Q, P) transposed
  T* G = x.G();
  const int l = lane(), w = wave();
  int bi = 0;
#pragma unroll 1
  for (int P = 0; P < NB; ++P) {
#pragma unroll 1
    for (int Q = P; Q < NB; ++Q, ++bi) {
      if ((bi & 3) != w) continue;
      const int pc = 16 * P + (l & 15), qc = 16 * Q + (l & 15);
      const int kP = pc % N, lP = pc / N, kQ = qc % N, lQ = qc / N;
      typename Mma<T>::acc_t acc = zacc<T>();
      if constexpr (MODE == 2) {
#pragma unroll 1
        for (int k32 = 0; k32 < (n + 31) / 32; ++k32) {
          bf8 ah, al, bh, bl;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int node = 32 * k32 + 8 * (l >> 4) + j;
            const bool live = node < n;
            const float va = (live && pc < n) ? (float)(X1[node * N + kP] * Y1[node * N + lP]) : 0.f;
            const float vb = (live && qc < n) ? (float)(X1[node * N + kQ] * Y1[node * N + lQ]) : 0.f;
            ah[j] = (__bf16)va;
            al[j] = (__bf16)(va - (float)ah[j]);
            bh[j] = (__bf16)vb;
            bl[j] = (__bf16)(vb - (float)bh[j]);
          }
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
        }
      } else {
#pragma unroll 1
        for (int kk = 0; kk < 4 * NB; ++kk) {
          const int node = 4 * kk + (l >> 4);
          const bool live = node < n;
          const T a = (live && pc < n) ? (T)(X1[node * N + kP] * Y1[node * N + lP]) : (T)0;
          const T bv = (live && qc < n) ? (T)(X1[node * N + kQ] * Y1[node * N + lQ]) : (T)0;
          acc = Mma<T>::mma(a, bv, acc);
        }
      }
      store_acc_t(G + tblk(Q, P) * BLK, acc);
    }
  }
  block_sync();
  cholesky<T, NB>(G, n);
  // c0 = G^-1 b (refined against float64 residuals in the mixed modes)
  double* c = x.d(L::dC);
  for (int i = t; i < L::NP; i += kThreads) c[i] = b[i];
  g_solve<N, MODE>(x, c);
  if constexpr (MODE != 0) {
    double* v = x.d(L::dV);
    double* w2 = x.d(L::dW);
#pragma unroll 1
    for (int it = 0; it < p.refine; ++it) {
      op_V<N, MODE>(x, c, v);
      block_sync();
      op_VT<N, MODE>(x, v, w2);
      block_sync();
      for (int i = t; i < L::NP; i += kThreads) w2[i] = b[i] - w2[i];
      g_solve<N, MODE>(x, w2);
      for (int i = t; i < L::NP; i += kThreads) c[i] += w2[i];
      block_sync();
    }
  }
  return escapes;
}

__device__ __forceinline__ void fit_index(const Params2D& p, int64_t b, int& e, int64_t& s) {
  const int64_t w = b / p.M;
  s = b - w * p.M;
  e = p.work[w];
}

__device__ __forceinline__ int64_t step_counter(const Params2D& p) { return p.step_ptr ? *p.step_ptr : p.step; }

template <int N, int MODE>
__device__ __forceinline__ void phase1_body(const Params2D& p, char* lds_raw, int64_t fit) {
  using L = Lay<N, MODE>;
  Ctx<N, MODE> x{lds_raw};
  int e;
  int64_t s;
  fit_index(p, fit, e, s);
  const Normal2 z = normal_pair(p.seed, p.stream, (uint64_t)step_counter(p), (uint64_t)(s / p.ncomp));
  const int escapes = setup_and_factor<N, MODE>(p, x, e, s, z.a, z.b);
  double* tv = x.d(L::dT);
  op_C<N, MODE>(x, x.d(L::dC), tv);
  block_sync();
  const int64_t eoff = p.eoff[e];
  for (int q = tid(); q < L::TT; q += kThreads) p.tr[s * p.edges + eoff + q] = tv[q];
  if (tid() == 0) stat_add(p.stats, kStatEscapes, (unsigned long long)escapes);
}

template <int N, int MODE>
__device__ __forceinline__ void phase2_body(const Params2D& p, char* lds_raw, int64_t fit) {
  using L = Lay<N, MODE>;
  using T = typename L::T;
  constexpr int n = L::n, NB = L::NB, TT = L::TT, R = L::R, RB = L::RB;
  Ctx<N, MODE> x{lds_raw};
  int e;
  int64_t s;
  fit_index(p, fit, e, s);
  const Normal2 z = normal_pair(p.seed, p.stream, (uint64_t)step_counter(p), (uint64_t)(s / p.ncomp));
  setup_and_factor<N, MODE>(p, x, e, s, z.a, z.b);
  const int t = tid(), l = lane(), w = wave();
  const int64_t eoff = p.eoff[e];
  double* tv = x.d(L::dT);
  double* gv = x.d(L::dG);
  double* e1 = x.d(L::dE1);
  // upwinded boundary data (eq. bnd_update)
  for (int q = t; q < TT; q += kThreads) {
    const int ew = q / N, j = q % N;
    const double tq = p.tr[s * p.edges + eoff + q];
    const double zd = (ew < 2) ? z.a : z.b;
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
        const double* src = p.tr + s * p.edges + p.eoff[nb] + (ew ^ 1) * Ns;
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
    tv[q] = tq;
    gv[q] = g;
    e1[q] = tq - g;
  }
  block_sync();
  const double* U = p.ur + p.ur_off[N];
  double* rr = x.d(L::dRr);
  op_UT<N, MODE>(U, e1, rr);
  // C_r^T = C^T U_r into the Y blocks:
  //   sum_j By[j][ly] (ex0[k] U_W[j][c] + ex1[k] U_E[j][c]) + sum_j Bx[j][k] (ey0[ly] U_S[j][c] + ey1[ly] U_N[j][c])
  double* Y = x.Y();
  {
    const double* Bx = x.d(L::dBx);
    const double* By = x.d(L::dBy);
    const double* Ev = x.d(L::dE);
    for (int idx = t; idx < L::NP * RB; idx += kThreads) {
      const int pr = idx % L::NP, C = idx / L::NP;
      const int k = pr % N, ly = pr / N;
      const bool live = pr < n;
      const double q0 = live ? Ev[k] : 0.0, q1 = live ? Ev[N + k] : 0.0;
      const double q2 = live ? Ev[2 * N + ly] : 0.0, q3 = live ? Ev[3 * N + ly] : 0.0;
      double by[N], bx[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        by[j] = live ? By[j * N + ly] : 0.0;
        bx[j] = live ? Bx[j * N + k] : 0.0;
      }
      double* Yrow = Y + ((pr >> 4) * RB + C) * BLK + (pr & 15) * BS;
#pragma unroll 1
      for (int cl = 0; cl < 16; ++cl) {
        const int cc = 16 * C + cl;
        double acc = 0.0;
        if (cc < R) {
          const double* Uc = U + cc * TT;
#pragma unroll 2
          for (int j = 0; j < N; ++j)
            acc += by[j] * (q0 * Uc[j] + q1 * Uc[N + j]) + bx[j] * (q2 * Uc[2 * N + j] + q3 * Uc[3 * N + j]);
        }
        Yrow[cl] = acc;
      }
    }
  }
  block_sync();
  // Y = L^-1 C_r^T, one block row at a time; column blocks spread over the
  // wavefronts.  Float64 products in every mode (the factor L is promoted), so
  // that S below is the constraint Schur complement of the factored G to
  // float64 accuracy: S is far worse conditioned than G.
  T* Gm = x.G();
  double* Sm = x.S();
  typedef Mma<double> M64;
#pragma unroll 1
  for (int kb = 0; kb < NB; ++kb) {
#pragma unroll 1
    for (int C = w; C < RB; C += 4) {
      double* Ykc = Y + (kb * RB + C) * BLK;
      M64::acc_t acc = load_acc(Ykc);
#pragma unroll 1
      for (int J = 0; J < kb; ++J) {
        const T* LB = Gm + tblk(kb, J) * BLK;
        const double* YJ = Y + (J * RB + C) * BLK;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = M64::mma(-(double)rowpat(LB, kk), colpat(YJ, kk), acc);
      }
      double* Tb = Sm + C * BLK;   // scratch: S is formed afterwards
      store_acc(Tb, acc);
      wave_sync();
      M64::acc_t out = zacc<double>();
      const T* Li = Gm + tblk(kb, kb) * BLK;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) out = M64::mma((double)rowpat(Li, kk), colpat(Tb, kk), out);
      store_acc(Ykc, out);
    }
    block_sync();
  }
  // S = Y^T Y (lower blocks)
  {
    int bi = 0;
#pragma unroll 1
    for (int C1 = 0; C1 < RB; ++C1) {
#pragma unroll 1
      for (int C2 = 0; C2 <= C1; ++C2, ++bi) {
        if ((bi & 3) != w) continue;
        M64::acc_t acc = zacc<double>();
#pragma unroll 1
        for (int kb = 0; kb < NB; ++kb) {
          const double* A1 = Y + (kb * RB + C1) * BLK;
          const double* A2 = Y + (kb * RB + C2) * BLK;
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) acc = M64::mma(colpat(A1, kk), colpat(A2, kk), acc);
        }
        store_acc(Sm + tblk(C1, C2) * BLK, acc);
      }
    }
  }
  block_sync();
  cholesky<double, RB>(Sm, R);
  // lambda = S^-1 rho_r; c = c0 - L^-T (Y lambda)
  double* lam = x.d(L::dLam);
  for (int i = t; i < L::RP; i += kThreads) lam[i] = rr[i];
  s_solve<N, MODE>(x, lam);
  double* c = x.d(L::dC);
  double* wv = x.d(L::dW);
  for (int pr = t; pr < L::NP; pr += kThreads) {
    double acc = 0.0;
    const int I = pr >> 4, r = pr & 15;
    for (int C = 0; C < RB; ++C) {
      const double* YB = Y + (I * RB + C) * BLK;
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) acc += YB[r * BS + cc] * lam[16 * C + cc];
    }
    wv[pr] = acc;
  }
  block_sync();
  if (w == 0) backward_solve<T, NB>(Gm, wv);
  block_sync();
  for (int pr = t; pr < L::NP; pr += kThreads) c[pr] -= wv[pr];
  block_sync();
  if constexpr (MODE != 0) {
    // float64 refinement of the constrained system
    //   [G  C_r^T] [c     ]   [b  ]
    //   [C_r  0  ] [lambda] = [g_r]
    // with the storage-precision factors as the approximate inverse.
    double* b = x.d(L::dB);
    double* v = x.d(L::dV);
    double* e2 = x.d(L::dE2);
    double* dl = x.d(L::dDl);
    double* r2 = x.d(L::dR2);
#pragma unroll 1
    for (int it = 0; it < p.refine; ++it) {
      op_V<N, MODE>(x, c, v);                 // v = V c
      op_U<N, MODE>(U, lam, e1);              // e1 = U_r lambda
      op_C<N, MODE>(x, c, e2);                // e2 = C c
      block_sync();
      op_VT<N, MODE>(x, v, wv);               // wv = V^T V c
      for (int q = t; q < TT; q += kThreads) e2[q] = gv[q] - e2[q];
      block_sync();
      op_CT<N, MODE>(x, e1, v);               // v = C_r^T lambda
      op_UT<N, MODE>(U, e2, r2);              // r2 = g_r - C_r c
      block_sync();
      for (int i = t; i < L::NP; i += kThreads) wv[i] = b[i] - wv[i] - v[i];   // r1
      g_solve<N, MODE>(x, wv);                // dc0 = G^-1 r1
      op_C<N, MODE>(x, wv, e2);
      block_sync();
      op_UT<N, MODE>(U, e2, dl);              // C_r dc0
      block_sync();
      for (int i = t; i < L::RP; i += kThreads) dl[i] -= r2[i];
      s_solve<N, MODE>(x, dl);                // dlambda
      op_U<N, MODE>(U, dl, e2);
      block_sync();
      op_CT<N, MODE>(x, e2, v);               // C_r^T dlambda
      block_sync();
      g_solve<N, MODE>(x, v);
      double dmax = 0.0, cmax = 0.0;
      for (int i = t; i < L::NP; i += kThreads) {
        const double d = wv[i] - v[i];
        c[i] += d;
        dmax = fmax(dmax, fabs(d));
        cmax = fmax(cmax, fabs(c[i]));
      }
      for (int i = t; i < L::RP; i += kThreads) lam[i] += dl[i];
      if (it == p.refine - 1) {
        // the relative size of the last correction, max |dc| / max |c|, for the diagnostics
        double* red = x.d(L::dRed);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
          cmax = fmax(cmax, __shfl_xor(cmax, o, 64));
        }
        if (l == 0) {
          red[8 + w] = dmax;
          red[12 + w] = cmax;
        }
        block_sync();
        if (t == 0) {
          const double dm = fmax(fmax(red[8], red[9]), fmax(red[10], red[11]));
          const double cm = fmax(fmax(red[12], red[13]), fmax(red[14], red[15]));
          stat_residual(p.stats, cm > 0.0 ? dm / cm : (dm > 0.0 ? __builtin_inf() : 0.0));
        }
      }
      block_sync();
    }
  }
  // new values at the Gauss nodes (eq. phi_star)
  const double* Bx = x.d(L::dBx);
  const double* By = x.d(L::dBy);
  const int64_t noff = p.noff[e];
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
      for (int k = 0; k < N; ++k) inner += bxr[k] * c[ly * N + k];
      v += By[iy * N + ly] * inner;
    }
    p.phi[s * p.nodes + noff + i] = v;
  }
  (void)l;
}

// One kernel per order and phase: one workgroup per fit of the order group.
template <int N, int MODE>
__global__ __launch_bounds__(kThreads) void fit2d_phase1(Params2D p) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  phase1_body<N, MODE>(p, lds_raw, blockIdx.x + p.block0);
}

template <int N, int MODE>
__global__ __launch_bounds__(kThreads) void fit2d_phase2(Params2D p) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  phase2_body<N, MODE>(p, lds_raw, blockIdx.x + p.block0);
}

// Persistent fused kernel over the fits of several orders (and of several
// problems): a fixed grid of workgroups pulls work items from one list through
// a device counter.  The list is made of segments (problem, order group),
// ordered by order, largest first, so the most expensive fits start first and
// the cheap ones fill the tail.  Every workgroup leaves the loop once the
// counter passes the end of the list, so the grid always drains.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// One fit of the fused kernel, outlined so that each order gets its own
// register allocation (the kernel needs as many registers as its largest
// callee, not the union of every order's live values).  Arguments arrive in
// vector registers and are made uniform again; the dynamic LDS is named here
// so that its accesses stay LDS instructions.
template <int N, int MODE, int PHASE>
__device__ __attribute__((noinline)) void fused_fit(const Params2D* pp, int64_t fit) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const uint64_t pv = (uint64_t)uniform64((int64_t)(uintptr_t)pp);
  const Params2D& p = *(const Params2D*)(uintptr_t)pv;
  fit = uniform64(fit);
  if constexpr (PHASE == 1) phase1_body<N, MODE>(p, lds_raw, fit);
  else phase2_body<N, MODE>(p, lds_raw, fit);
}

template <int MODE, int PHASE>
__global__ __launch_bounds__(kThreads) void fit2d_fused(Fused2DArgs a) {
  __shared__ int64_t item_sh;
  for (;;) {
    if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(a.counter, 1ull);
    __syncthreads();
    const int64_t item = uniform64(item_sh);
    __syncthreads();
    if (item >= a.total) break;
    int sg = 0;
    while (sg + 1 < a.nseg && item >= a.seg[sg + 1].start) ++sg;
    const Params2D* p = a.task[a.seg[sg].task];
    const int64_t fit = a.seg[sg].fit0 + (item - a.seg[sg].start);
    switch (a.seg[sg].N) {
      case 2: fused_fit<2, MODE, PHASE>(p, fit); break;
      case 3: fused_fit<3, MODE, PHASE>(p, fit); break;
      case 4: fused_fit<4, MODE, PHASE>(p, fit); break;
      case 5: fused_fit<5, MODE, PHASE>(p, fit); break;
      case 6: fused_fit<6, MODE, PHASE>(p, fit); break;
      case 7: fused_fit<7, MODE, PHASE>(p, fit); break;
      case 8: fused_fit<8, MODE, PHASE>(p, fit); break;
      case 9: fused_fit<9, MODE, PHASE>(p, fit); break;
      case 10: fused_fit<10, MODE, PHASE>(p, fit); break;
      default: break;
    }
    __syncthreads();
  }
}

// Set (set != 0) or advance the device step counters of a batch of problems
// and clear their work counters; a kernel rather than a memset so that it can
// sit inside a captured graph.
__global__ void step_counters_kernel(StepArgs a) {
  const int i = threadIdx.x;
  if (i < a.n) {
    if (a.set) *a.step[i] = a.value[i];
    else *a.step[i] += 1;
    for (int c = 0; c < kWorkCounters; ++c) a.counter[i][c] = 0ull;
  }
}

hipError_t launch_step_counters(const StepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(step_counters_kernel, dim3(1), dim3(kMaxTasks), 0, st, a);
  return hipGetLastError();
}

// One step's normal pairs of a batch of problems, one sample a thread
// (blockIdx.y: the problem), so that the fits of every element read their
// sample's pair instead of drawing it again; also clears each problem's
// counters of phase-1 fits to redo.
__global__ __launch_bounds__(256) void draw_normals_kernel(DrawArgs a) {
  const int t = blockIdx.y;
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < a.n && blockIdx.x == 0 && threadIdx.x <= kMaxN && a.rescue_count[t]) a.rescue_count[t][threadIdx.x] = 0u;
  if (t >= a.n || s >= a.M[t]) return;
  const int64_t step = a.step_ptr[t] ? *a.step_ptr[t] : a.step[t];
  const Normal2 d = normal_pair(a.seed[t], a.stream[t], (uint64_t)step, (uint64_t)s);
  a.z[t][2 * s] = d.a;
  a.z[t][2 * s + 1] = d.b;
}

hipError_t launch_draw_normals(const DrawArgs& a, int64_t maxM, hipStream_t st) {
  if (a.n <= 0 || maxM <= 0) return hipSuccess;
  hipLaunchKernelGGL(draw_normals_kernel, dim3((unsigned)((maxM + 255) / 256), (unsigned)a.n), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int MODE, int PHASE>
static hipError_t fused_one(const Fused2DArgs& a, int grid, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((fit2d_fused<MODE, PHASE>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_fit2d_fused(int phase, int mode, const Fused2DArgs& a, int grid, size_t lds, hipStream_t st) {
  if (phase == 1) {
    if (mode == 0) return fused_one<0, 1>(a, grid, lds, st);
    if (mode == 1) return fused_one<1, 1>(a, grid, lds, st);
    return fused_one<2, 1>(a, grid, lds, st);
  }
  if (mode == 0) return fused_one<0, 2>(a, grid, lds, st);
  if (mode == 1) return fused_one<1, 2>(a, grid, lds, st);
  return fused_one<2, 2>(a, grid, lds, st);
}

template <int MODE, int PHASE>
static int fused_occ(size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit2d_fused<MODE, PHASE>, kThreads, lds) != hipSuccess) return 0;
  return nb;
}

int fit2d_fused_occupancy(int phase, int mode, size_t lds) {
  if (phase == 1) return mode == 0 ? fused_occ<0, 1>(lds) : mode == 1 ? fused_occ<1, 1>(lds) : fused_occ<2, 1>(lds);
  return mode == 0 ? fused_occ<0, 2>(lds) : mode == 1 ? fused_occ<1, 2>(lds) : fused_occ<2, 2>(lds);
}

template <int N, int MODE>
static hipError_t launch_phase(int phase, const Params2D& p, int64_t nfits, hipStream_t st) {
  const size_t lds = phase == 1 ? Lay<N, MODE>::phase1 : Lay<N, MODE>::total;
  const int64_t chunk = (int64_t)1 << 30;
  for (int64_t b0 = 0; b0 < nfits; b0 += chunk) {
    Params2D q = p;
    q.block0 = p.block0 + b0;
    const int64_t nb = (nfits - b0) < chunk ? (nfits - b0) : chunk;
    if (phase == 1)
      hipLaunchKernelGGL((fit2d_phase1<N, MODE>), dim3((unsigned)nb), dim3(kThreads), lds, st, q);
    else
      hipLaunchKernelGGL((fit2d_phase2<N, MODE>), dim3((unsigned)nb), dim3(kThreads), lds, st, q);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

template <int N>
static hipError_t launch_modes(int phase, int mode, const Params2D& p, int64_t nfits, hipStream_t st) {
  switch (mode) {
    case 0: return launch_phase<N, 0>(phase, p, nfits, st);
    case 1: return launch_phase<N, 1>(phase, p, nfits, st);
    case 2: return launch_phase<N, 2>(phase, p, nfits, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
static size_t lds_modes(int mode, int phase) {
  switch (mode) {
    case 0: return phase == 1 ? Lay<N, 0>::phase1 : Lay<N, 0>::total;
    case 1: return phase == 1 ? Lay<N, 1>::phase1 : Lay<N, 1>::total;
    case 2: return phase == 1 ? Lay<N, 2>::phase1 : Lay<N, 2>::total;
    default: return 0;
  }
}

size_t fit2d_lds_bytes(int N, int mode, int phase) {
  switch (N) {
    case 2: return lds_modes<2>(mode, phase);
    case 3: return lds_modes<3>(mode, phase);
    case 4: return lds_modes<4>(mode, phase);
    case 5: return lds_modes<5>(mode, phase);
    case 6: return lds_modes<6>(mode, phase);
    case 7: return lds_modes<7>(mode, phase);
    case 8: return lds_modes<8>(mode, phase);
    case 9: return lds_modes<9>(mode, phase);
    case 10: return lds_modes<10>(mode, phase);
    default: return 0;
  }
}

hipError_t launch_fit2d(int phase, int N, int mode, const Params2D& p, int64_t nfits, hipStream_t st) {
  switch (N) {
    case 2: return launch_modes<2>(phase, mode, p, nfits, st);
    case 3: return launch_modes<3>(phase, mode, p, nfits, st);
    case 4: return launch_modes<4>(phase, mode, p, nfits, st);
    case 5: return launch_modes<5>(phase, mode, p, nfits, st);
    case 6: return launch_modes<6>(phase, mode, p, nfits, st);
    case 7: return launch_modes<7>(phase, mode, p, nfits, st);
    case 8: return launch_modes<8>(phase, mode, p, nfits, st);
    case 9: return launch_modes<9>(phase, mode, p, nfits, st);
    case 10: return launch_modes<10>(phase, mode, p, nfits, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sl
