// Two-dimensional step on a shared geometry: the fast path for constant drift
// and diffusion (and source factor) on a mesh of one order.
//
// With u and D constant, every node of every element of sample s moves by the
// same displacement delta_s = A + B z_s (Sec. 5.2, eq. def_dx).  In the frame
// centred on the mean displacement the moved nodes are then exactly the Gauss
// nodes, so every element of the sample has the same interpolation problem:
// the advected interpolant p0 of an element (eqs. phi_stardef, h_star) is the
// Lagrange interpolant of its carried values f on the Gauss nodes, its own
// traces are t = C* f (eq. remap_bnd) with C* the Lagrange basis evaluated at
// the element's edge points shifted by -delta_s, and the constrained
// least-squares remap (Sec. 5.3) in nodal form is
//     a = f - C_r^T S^-1 (C_r f - U_r^T g),  C_r = U_r^T C*,  S = C_r C_r^T,
// (U_r the orthonormal range basis of the 2-D edge-value map, rank 4N - 4),
// evaluated at the Gauss nodes by Phi = Px (x) Py, the Lagrange basis at the
// nodes shifted by -delta_s (eq. phi_star):
//     phi_new = Phi f + Mg (g - t),  Mg = Phi C_r^T S^-1 U_r^T.
// Everything but f and g is the same for all K elements of a sample, so a
// step is: one small kernel that builds Phi, C* and Mg per sample (one
// workgroup a sample), and two batched dense products over the elements on
// the float64 matrix cores, t = C* F and phi_new = [Phi | Mg] [F; G - T]
// (F the carried values of a tile of elements as columns, G their upwinded
// boundary data gathered from the traces of the neighbours, Sec. 5.3, eq.
// bnd_update).  The source factor (eq. advection_phi) is constant too and is
// folded into Phi and C*.
//
// The operators are stored per sample in the fragment order of
// v_mfma_f64_16x16x4f64 (lane l holds A[l%16][l/16] of a 16 x 4 slice), so a
// wavefront loads each A slice with one coalesced 512-byte read; tiles of
// elements pass through LDS (rows padded to an odd length) so that the B
// slices are read without bank conflicts and the results are written back
// coalesced.
#include "sl_internal.hpp"
#include "philox.hpp"
#include "blocks.hpp"

namespace sl {

#pragma clang fp contract(fast)

using namespace blk;

template <int N>
struct LayS {
  static constexpr int n = N * N, T = 4 * N, R = 4 * N - 4;
  static constexpr int NPB = (n + 15) / 16;          // 16-row blocks of the nodes
  static constexpr int TPB = (T + 15) / 16;          // 16-row blocks of the edge points
  static constexpr int KK = (n + T + 3) / 4;         // 4-wide slices of [Phi | Mg]
  static constexpr int KKc = (n + 3) / 4;            // 4-wide slices of C*
  static constexpr size_t a_doubles = (size_t)NPB * KK * 64;
  static constexpr size_t c_doubles = (size_t)TPB * KKc * 64;
  static constexpr size_t op_doubles = a_doubles + c_doubles + 2;   // + (za, zb)
  // element tile of the product kernels (LDS: the tile's values, padded rows)
  static constexpr int E = n <= 100 ? 64 : 32;
  static constexpr int FS = n + 1;                   // padded row of a tile's values
  static constexpr int GS = T + 1;                   // padded row of a tile's boundary data
  static constexpr size_t tile_bytes = sizeof(double) * (size_t)E * (FS + GS);
  // build kernel LDS (doubles): tables, C_r, S, Y = S^-1 U_r^T, W = C_r^T Y; Mg's
  // first pass reuses the space of C_r and S.  Room for R + 1 constraint rows (the
  // mass constraint adds one).
  static constexpr int RX = R + 1;
  static constexpr int oPx = 0, oPy = oPx + N * N, oEv = oPy + N * N, oMq = oEv + 4 * N;
  static constexpr int CRS = n + 1, SS = RX + 1;
  static constexpr int oCr = oMq + 2 * N;
  static constexpr int oS = oCr + RX * CRS;
  static constexpr int oY = oS + RX * SS;
  static constexpr int oW = oY + RX * T;
  static constexpr int oTmp = oCr;                   // n x T, over C_r and S (dead by then)
  static_assert(n * T <= RX * CRS + RX * SS + RX * T, "the second pass of Mg must fit where C_r, S and Y were");
  static constexpr int bend = oW + n * T;
  static constexpr size_t build_bytes = sizeof(double) * (size_t)(bend + 4);
};

// Lagrange basis of the Gauss nodes xi at x: bw_i prod_{m != i} (x - xi_m).
template <int N>
__device__ __forceinline__ double lagrange_at(const double* xi, const double* bw, int i, double x) {
  double v = bw[i];
#pragma unroll
  for (int m = 0; m < N; ++m)
    if (m != i) v *= (x - xi[m]);
  return v;
}

// C*[q][p] from the 1-D tables: node p = iy*N + ix, edge point q = w*N + j.
template <int N>
__device__ __forceinline__ double cstar(const double* Px, const double* Py, const double* Ev, int q, int p) {
  const int w = q / N, j = q - w * N, iy = p / N, ix = p - iy * N;
  if (w == 0) return Ev[ix] * Py[j * N + iy];             // W: (0, xi_j)
  if (w == 1) return Ev[N + ix] * Py[j * N + iy];         // E: (1, xi_j)
  if (w == 2) return Px[j * N + ix] * Ev[2 * N + iy];     // S: (xi_j, 0)
  return Px[j * N + ix] * Ev[3 * N + iy];                 // N: (xi_j, 1)
}

// One workgroup per sample: the operators of that sample's step.  MASS: one more
// constraint row, the element integral m* (value space) with a zero residual: the
// remap keeps each element's integral of p0 (left out at N = 2, where the boundary
// values fix the polynomial).
template <int N, bool MASS0>
__global__ __launch_bounds__(kThreads) void shared_build(SharedArgs a) {
  using L = LayS<N>;
  constexpr bool MASS = MASS0 && N >= 3;
  constexpr int n = L::n, T = L::T, RB = L::R, R = RB + (MASS ? 1 : 0);
  extern __shared__ __attribute__((aligned(16))) double lb[];
  const int t = tid();
  const int64_t s = blockIdx.x;
  double* op = a.ops + (size_t)s * L::op_doubles;
  double* Px = lb + L::oPx;
  double* Py = lb + L::oPy;
  double* Ev = lb + L::oEv;
  double* Mq = lb + L::oMq;                          // mass row factors: integral of each 1-D Lagrange basis
  double* Cr = lb + L::oCr;
  double* S = lb + L::oS;
  double* Y = lb + L::oY;
  double* W = lb + L::oW;
  double* Tm = lb + L::oTmp;
  double* zsh = lb + L::bend;
  const int64_t step = a.step_ptr ? *a.step_ptr : a.step;
  if (t == 0) {
    const Normal2 z = normal_pair(a.seed, a.stream, (uint64_t)step, (uint64_t)s);
    zsh[0] = z.a;
    zsh[1] = z.b;
    op[L::a_doubles + L::c_doubles] = z.a;
    op[L::a_doubles + L::c_doubles + 1] = z.b;
  }
  block_sync();
  // the uniform displacement, rounded as every moved node's
  const double dx = edge_disp(a.A[0], a.B[0], zsh[0]);
  const double dy = edge_disp(a.A[1], a.B[1], zsh[1]);
  const double* xi = a.xi;
  const double* bw = a.bw;
  for (int it = t; it < 2 * N * N + 4 * N; it += kThreads) {
    if (it < 2 * N * N) {
      const int dir = it >= N * N, r = it - dir * N * N, j = r / N, i = r - j * N;
      (dir ? Py : Px)[r] = lagrange_at<N>(xi, bw, i, xi[j] - (dir ? dy : dx));
    } else {
      const int u = it - 2 * N * N, w = u / N, i = u - w * N;
      const double x = (w == 0) ? -dx : (w == 1) ? 1.0 - dx : (w == 2) ? -dy : 1.0 - dy;
      Ev[u] = lagrange_at<N>(xi, bw, i, x);
    }
  }
  block_sync();
  if constexpr (MASS) {
    // m*[(iy, ix)] = mx[ix] my[iy], mx[i] = sum_j wq_j Px[j][i]: the element's quadrature of the
    // interpolant (the element is [0, 1] - delta in the centred frame, its Gauss nodes xi_j - delta)
    for (int it = t; it < 2 * N; it += kThreads) {
      const int dir = it >= N, i = it - dir * N;
      const double* P = dir ? Py : Px;
      double acc = 0.0;
      for (int j = 0; j < N; ++j) acc += a.wq[j] * P[j * N + i];
      Mq[it] = acc;
    }
  }
  // C* (traces from the carried values, source factor folded in), fragment order
  double* Cf = op + L::a_doubles;
  for (int idx = t; idx < (int)L::c_doubles; idx += kThreads) {
    const int l = idx & 63, rest = idx >> 6, kk = rest % L::KKc, I = rest / L::KKc;
    const int q = 16 * I + (l & 15), p = 4 * kk + (l >> 4);
    Cf[idx] = (q < T && p < n) ? a.src * cstar<N>(Px, Py, Ev, q, p) : 0.0;
  }
  // C_r = U_r^T C*  (U_r column-major T x R), then the mass row
  for (int idx = t; idx < RB * n; idx += kThreads) {
    const int c = idx / n, p = idx - c * n;
    const double* U = a.ur + (size_t)c * T;
    double acc = 0.0;
    for (int q = 0; q < T; ++q) acc += U[q] * cstar<N>(Px, Py, Ev, q, p);
    Cr[c * L::CRS + p] = acc;
  }
  if constexpr (MASS) {
    block_sync();
    for (int p = t; p < n; p += kThreads) Cr[RB * L::CRS + p] = Mq[p % N] * Mq[N + p / N];
  }
  block_sync();
  // S = C_r C_r^T
  for (int idx = t; idx < R * R; idx += kThreads) {
    const int c1 = idx / R, c2 = idx - c1 * R;
    if (c2 > c1) continue;
    double acc = 0.0;
    for (int p = 0; p < n; ++p) acc += Cr[c1 * L::CRS + p] * Cr[c2 * L::CRS + p];
    S[c1 * L::SS + c2] = acc;
    S[c2 * L::SS + c1] = acc;
  }
  block_sync();
  // S^-1 in place by Gauss-Jordan (S is symmetric positive definite: no pivoting)
  constexpr int kPer = (R * R + kThreads - 1) / kThreads;
  for (int k = 0; k < R; ++k) {
    double nv[kPer];
    const double piv = S[k * L::SS + k];
    const double ip = 1.0 / piv;
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int idx = t + m * kThreads;
      nv[m] = 0.0;
      if (idx < R * R) {
        const int i = idx / R, j = idx - i * R;
        const double fik = S[i * L::SS + k], rkj = S[k * L::SS + j];
        if (i == k && j == k) nv[m] = ip;
        else if (i == k) nv[m] = rkj * ip;
        else if (j == k) nv[m] = -fik * ip;
        else nv[m] = S[i * L::SS + j] - fik * (rkj * ip);
      }
    }
    block_sync();
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int idx = t + m * kThreads;
      if (idx < R * R) S[(idx / R) * L::SS + idx % R] = nv[m];
    }
    block_sync();
  }
  // Y = S^-1 [U_r^T; 0]  (R x T; the mass row's right side is zero)
  for (int idx = t; idx < R * T; idx += kThreads) {
    const int c = idx / T, q = idx - c * T;
    double acc = 0.0;
    for (int c2 = 0; c2 < RB; ++c2) acc += S[c * L::SS + c2] * a.ur[(size_t)c2 * T + q];
    Y[idx] = acc;
  }
  block_sync();
  // W = C_r^T Y  (n x T)
  for (int idx = t; idx < n * T; idx += kThreads) {
    const int p = idx / T, q = idx - p * T;
    double acc = 0.0;
    for (int c = 0; c < R; ++c) acc += Cr[c * L::CRS + p] * Y[c * T + q];
    W[idx] = acc;
  }
  block_sync();
  // Mg = (Px (x) Py) W: along x into Tm (over C_r and S), then along y back into W
  for (int idx = t; idx < n * T; idx += kThreads) {
    const int p = idx / T, q = idx - p * T, iy = p / N, jx = p - iy * N;
    double acc = 0.0;
#pragma unroll
    for (int ix = 0; ix < N; ++ix) acc += Px[jx * N + ix] * W[(iy * N + ix) * T + q];
    Tm[idx] = acc;
  }
  block_sync();
  for (int idx = t; idx < n * T; idx += kThreads) {
    const int p = idx / T, q = idx - p * T, jy = p / N, jx = p - jy * N;
    double acc = 0.0;
#pragma unroll
    for (int iy = 0; iy < N; ++iy) acc += Py[jy * N + iy] * Tm[(iy * N + jx) * T + q];
    W[idx] = acc;
  }
  block_sync();
  // [Phi | Mg] in fragment order; Phi[(jy, jx)][(iy, ix)] = src Py[jy][iy] Px[jx][ix]
  for (int idx = t; idx < (int)L::a_doubles; idx += kThreads) {
    const int l = idx & 63, rest = idx >> 6, kk = rest % L::KK, I = rest / L::KK;
    const int p = 16 * I + (l & 15), k = 4 * kk + (l >> 4);
    double v = 0.0;
    if (p < n && k < n) {
      const int jy = p / N, jx = p - jy * N, iy = k / N, ix = k - iy * N;
      v = a.src * (Py[jy * N + iy] * Px[jx * N + ix]);
    } else if (p < n && k < n + T) {
      v = W[p * T + (k - n)];
    }
    op[idx] = v;
  }
}

// Traces of a tile of elements: tr[s][e][q] = (C* f_e)_q.
template <int N>
__global__ __launch_bounds__(kThreads) void shared_traces(SharedArgs a) {
  using L = LayS<N>;
  constexpr int n = L::n, T = L::T, E = L::E, FS = L::FS;
  typedef Mma<double> M64;
  extern __shared__ __attribute__((aligned(16))) double ls[];
  const int t = tid(), l = lane(), wv = wave();
  const int64_t s = blockIdx.y;                      // row: (sample, component)
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (a.K - e0) < E ? (int)(a.K - e0) : E;
  double* F = ls;                                    // [E][FS]
  const double* phi = a.phi + (size_t)s * a.K * n + (size_t)e0 * n;
  for (int idx = t; idx < E * n; idx += kThreads) {
    const int e = idx / n, p = idx - e * n;
    F[e * FS + p] = e < ne ? phi[idx] : 0.0;
  }
  block_sync();
  const double* Cf = a.ops + (size_t)(s / a.ncomp) * L::op_doubles + L::a_doubles;
  constexpr int EB = E / 16, NT = L::TPB * EB;
  M64::acc_t acc[(NT + 3) / 4];
#pragma unroll
  for (int u = 0; u < (NT + 3) / 4; ++u) acc[u] = zacc<double>();
#pragma unroll
  for (int u = 0; u < (NT + 3) / 4; ++u) {
    const int tile = wv + 4 * u;
    if (tile < NT) {
      const int I = tile / EB, J = tile - I * EB;
      for (int kk = 0; kk < L::KKc; ++kk) {
        const double av = Cf[(I * L::KKc + kk) * 64 + l];
        const int p = 4 * kk + (l >> 4);
        const double bv = p < n ? F[(16 * J + (l & 15)) * FS + p] : 0.0;
        acc[u] = M64::mma(av, bv, acc[u]);
      }
    }
  }
  block_sync();
  double* O = ls;                                    // [E][T] over the tile
#pragma unroll
  for (int u = 0; u < (NT + 3) / 4; ++u) {
    const int tile = wv + 4 * u;
    if (tile < NT) {
      const int I = tile / EB, J = tile - I * EB;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int q = 16 * I + M64::row(l, s4), e = 16 * J + (l & 15);
        if (q < T) O[e * T + q] = acc[u][s4];
      }
    }
  }
  block_sync();
  double* tr = a.tr + (size_t)s * a.K * T + (size_t)e0 * T;
  for (int idx = t; idx < ne * T; idx += kThreads) tr[idx] = O[idx];
}

// New values of a tile of elements: phi_e <- Phi f_e + Mg (g_e - t_e).
template <int N>
__global__ __launch_bounds__(kThreads) void shared_update(SharedArgs a) {
  using L = LayS<N>;
  constexpr int n = L::n, T = L::T, E = L::E, FS = L::FS, GS = L::GS;
  typedef Mma<double> M64;
  extern __shared__ __attribute__((aligned(16))) double ls[];
  const int t = tid(), l = lane(), wv = wave();
  const int64_t s = blockIdx.y;                      // row: (sample, component)
  const int64_t e0 = (int64_t)blockIdx.x * E;
  const int ne = (a.K - e0) < E ? (int)(a.K - e0) : E;
  double* F = ls;                                    // [E][FS]
  double* G = ls + E * FS;                           // [E][GS]: g - t
  double* phi = a.phi + (size_t)s * a.K * n + (size_t)e0 * n;
  const double* op = a.ops + (size_t)(s / a.ncomp) * L::op_doubles;
  const double za = op[L::a_doubles + L::c_doubles], zb = op[L::a_doubles + L::c_doubles + 1];
  for (int idx = t; idx < E * n; idx += kThreads) {
    const int e = idx / n, p = idx - e * n;
    F[e * FS + p] = e < ne ? phi[idx] : 0.0;
  }
  // upwinded boundary data minus the own traces (eq. bnd_update)
  const double* tr = a.tr + (size_t)s * a.K * T;
  for (int idx = t; idx < E * T; idx += kThreads) {
    const int el = idx / T, q = idx - el * T;
    double v = 0.0;
    if (el < ne) {
      const int64_t e = e0 + el;
      const int w = q / N, j = q - w * N;
      const double own = tr[e * T + q];
      const double disp = edge_disp(a.Af[e * T + q], a.Bf[e * T + q], w < 2 ? za : zb);
      const bool pos = disp > 0.0;
      const bool take_nbr = (w == 0 || w == 2) ? pos : !pos;   // W, S: the neighbour is the negative side
      if (take_nbr) {
        const int nb = a.nbr[4 * e + w];
        const double g = nb < 0 ? a.ghost[e * T + q] : tr[(int64_t)nb * T + (w ^ 1) * N + j];
        v = g - own;
      }
    }
    G[el * GS + q] = v;
  }
  block_sync();
  constexpr int EB = E / 16, NT = L::NPB * EB;
  M64::acc_t acc[(NT + 3) / 4];
#pragma unroll
  for (int u = 0; u < (NT + 3) / 4; ++u) acc[u] = zacc<double>();
  const double* Af = op;
#pragma unroll
  for (int u = 0; u < (NT + 3) / 4; ++u) {
    const int tile = wv + 4 * u;
    if (tile < NT) {
      const int I = tile / EB, J = tile - I * EB;
      const double* Fe = F + (16 * J + (l & 15)) * FS;
      const double* Ge = G + (16 * J + (l & 15)) * GS;
      for (int kk = 0; kk < L::KK; ++kk) {
        const double av = Af[(I * L::KK + kk) * 64 + l];
        const int k = 4 * kk + (l >> 4);
        const double bv = k < n ? Fe[k] : (k < n + T ? Ge[k - n] : 0.0);
        acc[u] = M64::mma(av, bv, acc[u]);
      }
    }
  }
  block_sync();
  double* O = ls;                                    // [E][n] over the tile
#pragma unroll
  for (int u = 0; u < (NT + 3) / 4; ++u) {
    const int tile = wv + 4 * u;
    if (tile < NT) {
      const int I = tile / EB, J = tile - I * EB;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int p = 16 * I + M64::row(l, s4), e = 16 * J + (l & 15);
        if (p < n) O[e * n + p] = acc[u][s4];
      }
    }
  }
  block_sync();
  for (int idx = t; idx < ne * n; idx += kThreads) phi[idx] = O[idx];
}

template <int N>
static hipError_t launch_shared_n(int stage, const SharedArgs& a, int64_t M, hipStream_t st) {
  using L = LayS<N>;
  const int64_t rows = M * a.ncomp;
  if (rows > 65535 || M < 1 || a.ncomp < 1) return hipErrorInvalidValue;
  const int64_t tiles = (a.K + L::E - 1) / L::E;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  const size_t tb = L::tile_bytes > sizeof(double) * L::E * L::n ? L::tile_bytes : sizeof(double) * L::E * L::n;
  if (stage == 0 && a.mass)
    hipLaunchKernelGGL((shared_build<N, true>), dim3((unsigned)M), dim3(kThreads), L::build_bytes, st, a);
  else if (stage == 0)
    hipLaunchKernelGGL((shared_build<N, false>), dim3((unsigned)M), dim3(kThreads), L::build_bytes, st, a);
  else if (stage == 1)
    hipLaunchKernelGGL((shared_traces<N>), dim3((unsigned)tiles, (unsigned)rows), dim3(kThreads), tb, st, a);
  else
    hipLaunchKernelGGL((shared_update<N>), dim3((unsigned)tiles, (unsigned)rows), dim3(kThreads), tb, st, a);
  return hipGetLastError();
}

size_t shared_op_doubles(int N) {
  switch (N) {
    case 2: return LayS<2>::op_doubles;
    case 3: return LayS<3>::op_doubles;
    case 4: return LayS<4>::op_doubles;
    case 5: return LayS<5>::op_doubles;
    case 6: return LayS<6>::op_doubles;
    case 7: return LayS<7>::op_doubles;
    case 8: return LayS<8>::op_doubles;
    case 9: return LayS<9>::op_doubles;
    case 10: return LayS<10>::op_doubles;
    case 11: return LayS<11>::op_doubles;
    case 12: return LayS<12>::op_doubles;
    default: return 0;
  }
}

hipError_t launch_shared_step(int N, int stage, const SharedArgs& a, int64_t M, hipStream_t st) {
  switch (N) {
    case 2: return launch_shared_n<2>(stage, a, M, st);
    case 3: return launch_shared_n<3>(stage, a, M, st);
    case 4: return launch_shared_n<4>(stage, a, M, st);
    case 5: return launch_shared_n<5>(stage, a, M, st);
    case 6: return launch_shared_n<6>(stage, a, M, st);
    case 7: return launch_shared_n<7>(stage, a, M, st);
    case 8: return launch_shared_n<8>(stage, a, M, st);
    case 9: return launch_shared_n<9>(stage, a, M, st);
    case 10: return launch_shared_n<10>(stage, a, M, st);
    case 11: return launch_shared_n<11>(stage, a, M, st);
    case 12: return launch_shared_n<12>(stage, a, M, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sl
