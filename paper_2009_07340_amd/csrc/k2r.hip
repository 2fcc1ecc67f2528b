// Two-dimensional step, reference-preconditioned solver.
//
// The same constrained least-squares remap as the factorisation kernels
// (Sec. 5.3, eqs. phi_stardef, h_star, remap_bnd, bnd_update, phi_star), solved
// without forming or factoring the Gram matrix G = V^T V of the fit.
//
// Phase 1 (unconstrained interpolant p0, its values at the Gauss nodes and its
// traces at the own edge points): the basis is centred on the mean node
// displacement, so a uniform displacement leaves the moved-node basis matrix
// equal to the reference one, V0 = Vx (x) Vx: the orthonormal Legendre basis at
// the Gauss nodes, whose inverse Vx^-1 (x) Vx^-1 costs 2 N^3 operations to
// apply.  Only the non-uniform part of the displacement (velocity and diffusion
// varying across the element) makes V differ from V0, so Richardson iteration
// on the square system V c = f preconditioned by V0^-1 contracts fast (V c
// applied matrix-free from the 1-D Legendre tables).  A fit whose correction
// shrinks by less than half a step continues with conjugate gradients on the
// normal equations, preconditioned by G0^-1 = Gx^-1 (x) Gx^-1, Gx = Vx^T Vx.
// One-component fits take a lean form without the basis tables at the moved
// nodes and leave the fits that need conjugate gradients to the full form.
//
// Phase 2 (constrained remap) works in null-space form on the (N-2)^2
// coefficients of the part of the correction that vanishes on the edges, with
// a Kronecker preconditioner of the same kind (see the phase-2 section).
//
// The iteration counts adapt to the fit: zero for a uniform displacement (the
// preconditioners are then exact), a few for the smooth fields of the
// workloads.  Fits that do not reach the tolerance within the iteration limit
// are counted in a device statistic.  Everything is float64.  One workgroup
// per fit (one to four wavefronts by order), all of its data in LDS
// (N <= 16).
#include <atomic>

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

// LDS layout of phase 1 in doubles.
template <int N>
struct LayR {
  static constexpr int n = N * N, TT = 4 * N;
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
  static constexpr int oVxi = oGxi + N * N;
  static constexpr int oB = oVxi + N * N;
  static constexpr int oF = oB + n;
  static constexpr int oXv = oF + n;
  static constexpr int oR = oXv + n;
  static constexpr int oGv = oR + n;
  static constexpr int oP = oGv + n;
  static constexpr int oQ = oP + n;
  static constexpr int oT1 = oQ + n;
  static constexpr int oTr = oT1 + n;          // traces
  static constexpr int oUc = oTr + TT;         // edge contractions
  static constexpr int oRed = oUc + TT;
  static constexpr int end1 = oRed + 16;
  static constexpr size_t bytes1 = sizeof(double) * end1;
  // Waves a SIMD that the LDS admits for fits of b bytes on T threads, at most
  // cap: the register budget is asked to admit as many.
  static constexpr int lds_waves(size_t b, int cap, int T = 256) {
    const int w = (int)(((160 * 1024) / b * (size_t)(T / 64) + 3) / 4);
    return w > cap ? cap : w;
  }
  // at most as many as the registers admit without spilling (by order)
  static constexpr int reg_cap1 = N <= 3 ? 8 : N == 4 ? 6 : (N <= 6 || N == 8) ? 5 : 4;
  template <int T> static constexpr int waves1 = lds_waves(bytes1, reg_cap1, T);
};

// ---------------------------------------------------------------- helpers

// A fit runs on T = 64, 128 or 256 threads (one, two or four wavefronts).
// Per-wavefront partial sums in r[0 .. T/64) summed in a fixed order.
template <int T>
__device__ __forceinline__ double wsum(const double* r) {
  if constexpr (T == 256) return (r[0] + r[1]) + (r[2] + r[3]);
  else if constexpr (T == 128) return r[0] + r[1];
  else return r[0];
}

// One DPP lane move of a double (both halves), lanes outside the move or in
// the rows left out of ROWS taking 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_take(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum of v over the wavefront, in every lane (fixed order): quad sums by two
// quad permutations, row sums by row shifts of 4 and 8 (the row's total lands
// in its lanes 12..15), then lane 15 of rows 0 and 2 into rows 1 and 3 and
// lane 31 into rows 2 and 3, so lane 63 holds the total; its value is read
// from there.  The lane moves go through the DPP network, not the LDS.
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_take<0xB1, 0xF>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_take<0x4E, 0xF>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_take<0x114, 0xF>(v);   // row_shr:4
  v += dpp_take<0x118, 0xF>(v);   // row_shr:8
  v += dpp_take<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_take<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return bcast(v, 63);
}

// Sum over the fit's threads of a per-thread value; every thread gets the same
// result (fixed summation order).  One barrier: the slots in red are read
// after it and written again only by a later sum, which the callers keep
// behind at least one other barrier (dot products use red, the pair of
// residual norms red + 8).
template <int T>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_total(v);
  if (lane() == 0) red[wave()] = v;
  block_sync();
  return wsum<T>(red);
}

// Two sums at once (one barrier, as above).
template <int T>
__device__ __forceinline__ void block_sum2(double& v0, double& v1, double* red) {
  v0 = wave_total(v0);
  v1 = wave_total(v1);
  if (lane() == 0) {
    red[wave()] = v0;
    red[4 + wave()] = v1;
  }
  block_sync();
  v0 = wsum<T>(red);
  v1 = wsum<T>(red + 4);
}

// out[i] = (V c)_i
template <int N, int T>
__device__ void r_V(const double* X1, const double* Y1, const double* c, double* out) {
  for (int i = tid(); i < N * N; i += T) {
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
  // four independent accumulator chains (slices kk = u mod 4), summed at the end,
  // so that consecutive matrix-core operations do not wait on each other
  constexpr int KK = (n + 3) / 4;
  M64::acc_t ac[4] = {zacc<double>(), zacc<double>(), zacc<double>(), zacc<double>()};
#pragma unroll
  for (int kk = 0; kk < KK; ++kk) {
    const int i = 4 * kk + lk;
    const bool ok = col && i < n;
    const double a = ok ? Y1[lr * XS + i] : 0.0;          // A[ly][i]
    const double b = ok ? r[i] * X1[lr * XS + i] : 0.0;   // B[i][k]
    ac[kk & 3] = M64::mma(a, b, ac[kk & 3]);
  }
  M64::acc_t acc;
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) acc[s4] = (ac[0][s4] + ac[1][s4]) + (ac[2][s4] + ac[3][s4]);
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
    d = wave_total(d);
    if (l == 0) *dot_out = d;
  }
}

// out[i] = f[i] - (V c)_i
template <int N, int T>
__device__ void r_resid(const double* X1, const double* Y1, const double* c, const double* f, double* out) {
  for (int i = tid(); i < N * N; i += T) {
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
    out[i] = f[i] - v;
  }
}

// d = V0^-1 r = (Vx^-1 (x) Vx^-1) r for values r at the nodes (r[iy N + ix]):
// tmp[iy][k] = sum_ix vxi[k][ix] r[iy][ix], then d[ly][k] = sum_iy vxi[ly][iy] tmp[iy][k];
// x = d, or x += d when add.  Two barriers; the per-wavefront partial sums of
// d . d are left in red2[0..3] (readable after the second barrier).
template <int N, int T>
__device__ void r_V0inv(const double* vxi, const double* r, double* tmp, double* x, bool add, double* red2) {
  for (int p = tid(); p < N * N; p += T) {
    const int k = p % N, iy = p / N;
    double acc = 0.0;
#pragma unroll
    for (int ix = 0; ix < N; ++ix) acc += vxi[k * N + ix] * r[iy * N + ix];
    tmp[p] = acc;
  }
  block_sync();
  double a = 0.0;
  for (int p = tid(); p < N * N; p += T) {
    const int k = p % N, ly = p / N;
    double d = 0.0;
#pragma unroll
    for (int iy = 0; iy < N; ++iy) d += vxi[ly * N + iy] * tmp[iy * N + k];
    x[p] = add ? x[p] + d : d;
    a += d * d;
  }
  a = wave_total(a);
  if (lane() == 0) red2[wave()] = a;
  block_sync();
}

// out = (Gx^-1 (x) Gx^-1) v  (c indexed [ly * N + k]), or minuend - that when
// minuend is given; tmp n doubles.  Two barriers.  With rr given, the
// per-wavefront partial sums of rr . out and out . out are left in
// red2[0..3] and red2[4..7] (readable after the second barrier).
template <int N, int T>
__device__ void r_G0inv(const double* gxi, const double* v, double* tmp, double* out,
                        const double* minuend = nullptr, const double* rr = nullptr, double* red2 = nullptr) {
  for (int p = tid(); p < N * N; p += T) {
    const int k = p % N, ly = p / N;
    double acc = 0.0;
#pragma unroll
    for (int kk = 0; kk < N; ++kk) acc += gxi[k * N + kk] * v[ly * N + kk];
    tmp[p] = acc;
  }
  block_sync();
  double a = 0.0, c = 0.0;
  for (int p = tid(); p < N * N; p += T) {
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
    a = wave_total(a);
    c = wave_total(c);
    if (lane() == 0) {
      red2[wave()] = a;
      red2[4 + wave()] = c;
    }
  }
  block_sync();
}

// Carried values of component c's row of the state (eq. advection_phi) into f,
// for the second and later components of a fit (the first one's come with the
// set-up).  One barrier.
template <int N, int T>
__device__ void r_carried(const Params2D& p, double* lds, const WorkRec* e, int64_t row) {
  using L = LayR<N>;
  const int64_t noff = e->noff;
  double* f = lds + L::oF;
  for (int i = tid(); i < L::n; i += T) f[i] = p.phi[row * p.nodes + noff + i] * p.src[noff + i];
  block_sync();
}

// t - g at the own edge points of one component row into gv: t the own traces
// of p0, g the upwinded boundary data (eq. bnd_update): at each own edge point
// the element the interface displacement comes from supplies the trace
// (another order's trace interpolated to this element's abscissae), or the
// Dirichlet ghost value.  The outside value is loaded before the side is known,
// so that no load waits for the draw.  No barrier.
template <int N, int T>
__device__ void r_jump_data(const Params2D& p, const WorkRec* e, int64_t row, double za, double zb, double* gv, int t0) {
  using L = LayR<N>;
  const int64_t eoff = e->eoff;
  for (int q = t0; q < L::TT; q += T) {
    const int ew = q / N, j = q % N;
    const int64_t nt = e->nbr_tr[ew];
    const double tq = p.tr[row * p.edges + eoff + q];
    double out;
    if (nt < 0) {
      out = p.ghost[eoff + q];
    } else {
      const int Ns = (int)(nt >> 48);
      const double* src = p.tr + row * p.edges + (nt & 0xffffffffffffll);
      if (Ns == N) {
        out = src[j];
      } else {   // trace of another order: Lagrange interpolation to this element's abscissae
        const double* Lm = p.interp + p.interp_off[N * (kMaxN + 1) + Ns] + j * Ns;
        double acc = 0.0;
        for (int m = 0; m < Ns; ++m) acc += Lm[m] * src[m];
        out = acc;
      }
    }
    const double zd = (ew < 2) ? za : zb;
    const bool pos = edge_disp(p.Af[eoff + q], p.Bf[eoff + q], zd) > 0.0;
    const bool take_nbr = (ew == 0 || ew == 2) ? pos : !pos;   // W, S: neighbour is the negative side
    gv[q] = tq - (take_nbr ? out : tq);
  }
}

// One-dimensional contractions of a coefficient array c[ly][k] with the edge
// basis vectors: out[0..N) = sum_k p0x[k] c[.][k], out[N..2N) with p1x,
// out[2N..3N) = sum_ly p0y[ly] c[ly][.], out[3N..4N) with p1y.
template <int N, int T>
__device__ void r_edge_contract(const double* Ev, const double* c, double* out) {
  for (int o = tid(); o < 4 * N; o += T) {
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
template <int N, int T>
__device__ void r_traces_from(const double* Bx, const double* By, const double* u, double* out) {
  for (int q = tid(); q < 4 * N; q += T) {
    const int w = q / N, j = q % N;
    const double* B = (w < 2) ? By + j * N : Bx + j * N;
    const double* v = u + w * N;
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) acc += B[m] * v[m];
    out[q] = acc;
  }
}

// ---------------------------------------------------------------- per-fit set-up

// The mean displacement of a fit's moved nodes, (dbx, dby), from the element
// means of the move coefficients: the same as averaging the moves, up to
// rounding (it only centres the basis).
struct Shift2 {
  double x, y;
};
__device__ __forceinline__ Shift2 mean_shift(const WorkRec* e, Normal2 z) {
  const double* em = e->emean;
  return Shift2{em[0] + em[2] * z.a, em[1] + em[3] * z.b};
}

// This step's Wiener normals of sample s (eq. def_dx), drawn for every sample
// before phase 1 and shared by the elements and both phases.
__device__ __forceinline__ Normal2 fit_increments(const Params2D& p, int64_t s) {
  return Normal2{p.zdraw[2 * s], p.zdraw[2 * s + 1]};
}

// Moves (eq. def_dx), carried values (eq. advection_phi) and the centred 1-D
// tables: item i < n moves node i and evaluates the basis there in x and in y;
// the next 2N items the N Gauss abscissae of the edges in x and in y, the last
// 4 the edge coordinates.  Moved nodes outside the element are counted in the
// statistics (unless the fit is being redone).  One barrier.
template <int N, int T>
__device__ void r_setup(const Params2D& p, double* lds, const WorkRec* e, int64_t s, Normal2 z, bool count = true) {
  using L = LayR<N>;
  constexpr int n = L::n;
  const int t = tid();
  const int64_t noff = e->noff;
  const Shift2 d = mean_shift(e, z);
  double* f = lds + L::oF;
  const double* gsrc = p.gxinv + p.gx_off[N];
  double* gxi = lds + L::oGxi;   // Gx^-1 and Vx^-1, adjacent in both places
  for (int i = t; i < 2 * N * N; i += T) gxi[i] = gsrc[i];
  double* X1 = lds + L::oX1;
  double* Y1 = lds + L::oY1;
  double* Bx = lds + L::oBx;
  double* By = lds + L::oBy;
  double* Ev = lds + L::oEv;
  int esc = 0;
  for (int it = t; it < n + 2 * N + 4; it += T) {
    double q[N];
    if (it < n) {
      const int64_t k = noff + it;
      const double x0 = p.xi_node[2 * k], y0 = p.xi_node[2 * k + 1];
      const double xm = moved_coord(x0, p.A[2 * k], p.B[2 * k], z.a);
      const double ym = moved_coord(y0, p.A[2 * k + 1], p.B[2 * k + 1], z.b);
      f[it] = p.phi[s * p.ncomp * p.nodes + k] * p.src[k];   // component 0 of sample s
      esc += escaped(xm) + escaped(ym);
      legendre_eval_k<N>(xm - d.x, q);
#pragma unroll
      for (int j = 0; j < N; ++j) X1[j * L::XS + it] = q[j];
      legendre_eval_k<N>(ym - d.y, q);
#pragma unroll
      for (int j = 0; j < N; ++j) Y1[j * L::XS + it] = q[j];
    } else {
      double arg;
      double* dst;
      if (it < n + 2 * N) {
        const int u = it - n, dir = u >= N, row = u - dir * N;
        arg = p.xi_tab[N * kMaxN + row] - (dir ? d.y : d.x);
        dst = (dir ? By : Bx) + row * N;
      } else {
        const int w = it - n - 2 * N;
        arg = (w == 0) ? -d.x : (w == 1) ? 1.0 - d.x : (w == 2) ? -d.y : 1.0 - d.y;
        dst = Ev + w * N;
      }
      legendre_eval_k<N>(arg, q);
#pragma unroll
      for (int j = 0; j < N; ++j) dst[j] = q[j];
    }
  }
  if (p.stats && count) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) esc += __shfl_xor(esc, o, 64);
    if (lane() == 0 && esc) stat_add(p.stats, kStatEscapes, (unsigned long long)esc);
  }
  block_sync();
}

// G v = V^T (V v) into out (tmp: n doubles).  Two barriers.
// With dot_out given, <v, G v> is left there too (readable after the return).
template <int N, int T>
__device__ __forceinline__ void r_G(double* lds, const double* v, double* tmp, double* out, double* dot_out = nullptr) {
  using L = LayR<N>;
  r_V<N, T>(lds + L::oX1, lds + L::oY1, v, tmp);
  block_sync();
  r_VT_mc<N>(lds + L::oX1, lds + L::oY1, tmp, out, dot_out ? v : nullptr, dot_out);
  block_sync();
}

// Diagnostics of one fit: iterations and whether the tolerance was reached
// (per phase) and the relative residual left, sqrt(g^T g / x0^T x0) (phase 1's
// set-up counts the moved nodes outside the element).  Called after the fit's
// last barrier: a workgroup barrier waits for the memory operations in flight,
// atomics included.
__device__ __forceinline__ void count_fit(const Params2D& p, int phase, int iters, int unconverged, double resid) {
  if (tid() == 0 && p.stats) {
    unsigned long long* c = stat_slot(p.stats) + 2 * (phase - 1);
    atomicAdd(c, (unsigned long long)iters);
    if (unconverged) atomicAdd(c + 1, (unsigned long long)unconverged);
    stat_residual(p.stats, resid);
  }
}

__device__ __forceinline__ double rel_resid(double gg, double xx) {
  return xx > 0.0 ? sqrt(gg / xx) : (gg > 0.0 ? __builtin_inf() : 0.0);
}

// ---------------------------------------------------------------- phase 1

// p0 = By C Bx^T at the Gauss nodes (C = c[ly][k]) into dst[i], i < n.
template <int N, int T>
__device__ __forceinline__ void r_p0_out(const double* Bx, const double* By, const double* c, double* dst) {
  for (int i = tid(); i < N * N; i += T) {
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
    dst[i] = v;
  }
}

// redo: the fit is one the lean kernel listed (its moved nodes were counted there).
template <int N, int T>
__device__ __forceinline__ void r_phase1_body(const Params2D& p, double* lds, int64_t fit, bool redo = false) {
  using L = LayR<N>;
  constexpr int n = L::n;
  const int64_t w = fit / p.M;
  const int64_t s = fit - w * p.M;
  const WorkRec* e = p.wrec + w;
  const Normal2 z = fit_increments(p, s);
  r_setup<N, T>(p, lds, e, s, z, !redo);
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
  const int64_t eoff = e->eoff;
  const int64_t noff = e->noff;
  int its = 0, unconv = 0;
  double rmax = 0.0;
  // the components share the moved nodes and their tables (Sec. 5.3, last paragraph)
  for (int c = 0; c < p.ncomp; ++c) {
  const int64_t row = s * p.ncomp + c;
  if (c > 0) r_carried<N, T>(p, lds, e, row);
  // Richardson iteration on the square system V c = f, preconditioned by the
  // reference basis matrix: c = V0^-1 f, then c += V0^-1 (f - V c).  Its error
  // contracts by about the non-uniform part of the displacement each step, so
  // the error left after a correction dc is about rho |dc| / (1 - rho), rho the
  // ratio of the last two corrections (of the first correction to c0 at the
  // start): the iteration stops when that estimate, or the correction itself,
  // is below tol |c0|.
  const double* vxi = lds + L::oVxi;
  const double* f = lds + L::oF;
  r_V0inv<N, T>(vxi, f, t1, x, false, red + 8);
  const double xx = wsum<T>(red + 8);
  const double stop = p.tol2 * xx;
  double gg = xx;
  bool slow = false;
  int it;
  for (it = 1; it <= p.max_iter; ++it) {
    r_resid<N, T>(lds + L::oX1, lds + L::oY1, x, f, r);
    block_sync();
    r_V0inv<N, T>(vxi, r, t1, x, true, red + 8);
    const double d1 = wsum<T>(red + 8);
    if (d1 <= stop) {
      gg = d1;
      break;
    }
    slow = d1 > 0.25 * gg;
    if (!slow) {
      const double q = d1 / gg, rq = sqrt(q);
      const double e2 = (d1 * q) / ((1.0 - rq) * (1.0 - rq));   // the estimated error, squared
      if (e2 <= stop) {
        gg = e2;
        break;
      }
    }
    gg = d1;
    if (slow) break;
  }
  // a correction that shrinks by less than half a step: preconditioned
  // conjugate gradients on G c = V^T f (preconditioner G0^-1) from the iterate
  if (slow) {
    its += it;
    if (tid() == 0) stat_add(p.stats, kStatFallbacks, 1ull);
    r_VT_mc<N>(lds + L::oX1, lds + L::oY1, f, b);
    block_sync();
    r_G<N, T>(lds, x, t1, r);
    for (int i = t; i < n; i += T) r[i] -= b[i];
    block_sync();
    r_G0inv<N, T>(gxi, r, t1, g, nullptr, r, red + 8);   // with r^T g and g^T g
    double rg = wsum<T>(red + 8);
    gg = wsum<T>(red + 12);
    it = 0;
    if (gg > stop) {
      for (int i = t; i < n; i += T) pv[i] = -g[i];
      block_sync();
      for (it = 1; it <= p.max_iter; ++it) {
        r_G<N, T>(lds, pv, t1, q, red);   // q = G pv and pv^T q
        const double pq = red[0];
        const double alpha = rg / pq;
        for (int i = t; i < n; i += T) {
          x[i] += alpha * pv[i];
          r[i] += alpha * q[i];
        }
        block_sync();
        r_G0inv<N, T>(gxi, r, t1, g, nullptr, r, red + 8);
        const double rg1 = wsum<T>(red + 8);
        gg = wsum<T>(red + 12);
        if (gg <= stop) break;
        const double beta = rg1 / rg;
        rg = rg1;
        for (int i = t; i < n; i += T) pv[i] = beta * pv[i] - g[i];
        block_sync();
      }
    }
  }
  // p0 at the Gauss nodes into the state row, where phase 2 starts from it
  r_p0_out<N, T>(lds + L::oBx, lds + L::oBy, x, p.phi + row * p.nodes + noff);
  // traces of p0 at the own edge points (eq. remap_bnd)
  double* tv = lds + L::oTr;
  double* uc = lds + L::oUc;
  r_edge_contract<N, T>(lds + L::oEv, x, uc);
  block_sync();
  r_traces_from<N, T>(lds + L::oBx, lds + L::oBy, uc, tv);
  block_sync();
  for (int qq = t; qq < L::TT; qq += T) p.tr[row * p.edges + eoff + qq] = tv[qq];
  its += it > p.max_iter ? p.max_iter : it;
  unconv += gg <= stop ? 0 : 1;
  rmax = fmax(rmax, rel_resid(gg, xx));
  }
  count_fit(p, 1, its, unconv, rmax);
}

// ---------------------------------------------------------------- phase 1, lean form
//
// The same fit for one component without the basis tables at the moved nodes:
// the residual evaluates the basis at each node as it goes, so a fit needs
// about a third of the LDS of the full form and more fits share a compute
// unit.  A fit whose iteration contracts too slowly (where the full form
// turns to conjugate gradients) is listed, and the full form redoes it.

template <int N>
struct LayL {
  static constexpr int n = N * N, TT = 4 * N;
  static constexpr int oXY = 0;              // moved nodes, x then y
  static constexpr int oBx = oXY + 2 * n;
  static constexpr int oBy = oBx + N * N;
  static constexpr int oEv = oBy + N * N;
  static constexpr int oVxi = oEv + 4 * N;
  static constexpr int oF = oVxi + N * N;
  static constexpr int oXv = oF + n;
  static constexpr int oR = oXv + n;
  static constexpr int oT1 = oR + n;
  static constexpr int oTr = oT1 + n;
  static constexpr int oUc = oTr + TT;
  static constexpr int oRed = oUc + TT;
  static constexpr int end = oRed + 16;
  static constexpr size_t bytes = sizeof(double) * end;
  static constexpr int reg_cap = N <= 6 ? 8 : N <= 10 ? 6 : 4;
  template <int T> static constexpr int waves = LayR<N>::lds_waves(bytes, reg_cap, T);
};

// Set-up of the lean form: moves, carried values, Vx^-1 and the tables at the
// Gauss abscissae and edge coordinates.  One barrier.
template <int N, int T>
__device__ void r_setup_lean(const Params2D& p, double* lds, const WorkRec* e, int64_t s, Normal2 z, Shift2 d) {
  using L = LayL<N>;
  constexpr int n = L::n;
  const int t = tid();
  const int64_t noff = e->noff;
  double* f = lds + L::oF;
  double* XY = lds + L::oXY;
  const double* vsrc = p.gxinv + p.gx_off[N] + N * N;
  double* vxi = lds + L::oVxi;
  for (int i = t; i < N * N; i += T) vxi[i] = vsrc[i];
  int esc = 0;
  for (int it = t; it < n + 2 * N + 4; it += T) {
    if (it < n) {
      const int64_t k = noff + it;
      const double xm = moved_coord(p.xi_node[2 * k], p.A[2 * k], p.B[2 * k], z.a);
      const double ym = moved_coord(p.xi_node[2 * k + 1], p.A[2 * k + 1], p.B[2 * k + 1], z.b);
      XY[it] = xm;
      XY[n + it] = ym;
      f[it] = p.phi[s * p.nodes + k] * p.src[k];
      esc += escaped(xm) + escaped(ym);
    } else {
      double arg;
      double* dst;
      if (it < n + 2 * N) {
        const int u = it - n, dir = u >= N, row = u - dir * N;
        arg = p.xi_tab[N * kMaxN + row] - (dir ? d.y : d.x);
        dst = (dir ? lds + L::oBy : lds + L::oBx) + row * N;
      } else {
        const int w = it - n - 2 * N;
        arg = (w == 0) ? -d.x : (w == 1) ? 1.0 - d.x : (w == 2) ? -d.y : 1.0 - d.y;
        dst = lds + L::oEv + w * N;
      }
      double q[N];
      legendre_eval_k<N>(arg, q);
#pragma unroll
      for (int j = 0; j < N; ++j) dst[j] = q[j];
    }
  }
  if (p.stats) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) esc += __shfl_xor(esc, o, 64);
    if (lane() == 0 && esc) stat_add(p.stats, kStatEscapes, (unsigned long long)esc);
  }
  block_sync();
}

// out[i] = f[i] - (V c)_i with the basis evaluated at the moved node i
// (centred on d) as it goes.
template <int N, int T>
__device__ void r_resid_fly(const double* XY, Shift2 d, const double* c, const double* f, double* out) {
  constexpr int n = N * N;
  for (int i = tid(); i < n; i += T) {
    double px[N];
    legendre_eval_k<N>(XY[i] - d.x, px);
    double v = 0.0;
    if constexpr (N <= 10) {   // unrolled: the whole of C is read once
      double py[N];
      legendre_eval_k<N>(XY[n + i] - d.y, py);
#pragma unroll
      for (int ly = 0; ly < N; ++ly) {
        double inner = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) inner += px[k] * c[ly * N + k];
        v += py[ly] * inner;
      }
    } else {   // a row of C at a time, the y basis advanced by its recurrence
      const double yv = 2.0 * (XY[n + i] - d.y) - 1.0;
      double pm = 0.0, pc = 1.0;
#pragma unroll 1
      for (int ly = 0; ly < N; ++ly) {
        double inner = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) inner += px[k] * c[ly * N + k];
        v += pc * inner;
        const double pn = kLegA[ly] * yv * pc - kLegB[ly] * pm;
        pm = pc;
        pc = pn;
      }
    }
    out[i] = f[i] - v;
  }
}

// One fit of one component: the Richardson iteration of the full form; a fit
// that it does not settle is listed (list[atomicAdd(count)]) for the full form
// and writes nothing.
template <int N, int T>
__device__ __forceinline__ void r_phase1_lean(const Params2D& p, double* lds, int64_t fit, uint32_t* list,
                                              unsigned int* count) {
  using L = LayL<N>;
  const int64_t w = fit / p.M;
  const int64_t s = fit - w * p.M;
  const WorkRec* e = p.wrec + w;
  const Normal2 z = fit_increments(p, s);
  const Shift2 d = mean_shift(e, z);
  r_setup_lean<N, T>(p, lds, e, s, z, d);
  const double* vxi = lds + L::oVxi;
  const double* f = lds + L::oF;
  double* x = lds + L::oXv;
  double* r = lds + L::oR;
  double* t1 = lds + L::oT1;
  double* red = lds + L::oRed;
  r_V0inv<N, T>(vxi, f, t1, x, false, red + 8);
  const double xx = wsum<T>(red + 8);
  const double stop = p.tol2 * xx;
  double gg = xx;
  bool slow = false;
  int it;
  for (it = 1; it <= p.max_iter; ++it) {
    r_resid_fly<N, T>(lds + L::oXY, d, x, f, r);
    block_sync();
    r_V0inv<N, T>(vxi, r, t1, x, true, red + 8);
    const double d1 = wsum<T>(red + 8);
    if (d1 <= stop) {
      gg = d1;
      break;
    }
    slow = d1 > 0.25 * gg;
    if (!slow) {
      const double q = d1 / gg, rq = sqrt(q);
      const double e2 = (d1 * q) / ((1.0 - rq) * (1.0 - rq));
      if (e2 <= stop) {
        gg = e2;
        break;
      }
    }
    gg = d1;
    if (slow) break;
  }
  if (slow) {
    if (tid() == 0) list[atomicAdd(count, 1u)] = (uint32_t)fit;
    return;
  }
  const int64_t noff = e->noff;
  const int64_t eoff = e->eoff;
  r_p0_out<N, T>(lds + L::oBx, lds + L::oBy, x, p.phi + s * p.nodes + noff);
  double* tv = lds + L::oTr;
  double* uc = lds + L::oUc;
  r_edge_contract<N, T>(lds + L::oEv, x, uc);
  block_sync();
  r_traces_from<N, T>(lds + L::oBx, lds + L::oBy, uc, tv);
  block_sync();
  for (int qq = tid(); qq < L::TT; qq += T) p.tr[s * p.edges + eoff + qq] = tv[qq];
  count_fit(p, 1, it > p.max_iter ? p.max_iter : it, gg <= stop ? 0 : 1, rel_resid(gg, xx));
}

// ---------------------------------------------------------------- phase 2
//
// Null-space form of the constrained remap.  Phase 1 left p0 at the Gauss nodes
// in the state; p0 fits the carried values at the moved nodes exactly (up to
// the solver tolerance), so for q = p0 - delta the misfit at the moved nodes is
// delta there, and the remap is the delta in Q_{N-1} of least squares at the
// moved nodes whose edge values are the jump j = P (t - g): t the own traces
// of p0, g the upwinded data, P the orthogonal projector onto the edge-value
// vectors of Q_{N-1} (the boundary constraints hold in that range).  Write
//   delta = lift(j) + sum_{k,l} w_{lk} beta_k(x) beta_l(y),
// lift(j) the transfinite interpolant of the four edge traces of j (each the
// degree N-1 interpolant of its N values; it takes the edge values j and lies in
// Q_{N-1}), beta_k(x) = x (1 - x) psi_k(x - dbar_x), k < N - 2 (psi: orthonormal
// Legendre, centred on the mean displacement), which vanish on the edges and
// span, with their y counterparts, the polynomials of Q_{N-1} that vanish
// there.  w solves the (N-2)^2 normal equations
//   (Vz^T Vz) w = -Vz^T lift(j)(moved nodes),  Vz[i][(l,k)] = beta_k(x_i) beta_l(y_i),
// by preconditioned conjugate gradients.  Were the displacement uniform, Vz
// would be the Kronecker product of the 1-D tables Bx[a][k] = beta_k(xi_a + dbar_x)
// and By, so (Bx^T Bx)^-1 (x) (By^T By)^-1 (two (N-2)^2 inverses a fit) is the
// exact inverse there and the preconditioner here.  The new values at the
// Gauss nodes are p0 - lift(j) - sum w beta beta.  The iteration stops when the
// nodal size of its estimated error is below tol times that of p0 and lift(j).

// W: wavefronts a fit (the partial products take one m x m block each).
template <int N, int W = 4>
struct LayZ {
  static constexpr int n = N * N, m = N - 2, mm = m * m, TT = 4 * N;
  static constexpr int mA = m > 0 ? m : 1, mmA = mA * mA;
  static constexpr int ZS = n + 1;            // odd row stride of the bubble tables at the moved nodes
  static constexpr int oXz = 0;               // Xz[k][i] = beta_k(x_i)
  static constexpr int oYz = oXz + mA * ZS;   // Yz[l][i] = beta_l(y_i)
  static constexpr int oGx = oYz + mA * ZS;   // (Bx^T Bx)^-1, m x m row-major
  static constexpr int oGy = oGx + mmA;
  static constexpr int oB = oGy + mmA;        // right side
  static constexpr int oW = oB + mmA;         // iterate
  static constexpr int oR = oW + mmA;         // residual
  static constexpr int oG = oR + mmA;         // preconditioned residual
  static constexpr int oP = oG + mmA;         // search direction
  static constexpr int oT = oP + mmA;         // Kronecker temporary
  static constexpr int oPart = oT + mmA;      // the wavefronts' partial Vz^T products
  static constexpr int oL = oPart + W * mmA;  // n values at the moved nodes
  // the moved nodes' coordinates (x, then y) wait for the lift in the space of
  // R, G, P and T where that holds them: the iteration starts after the lift
  static constexpr bool kXmShared = 4 * mmA >= 2 * n;
  static constexpr int oXm = kXmShared ? oR : oL + n;
  static constexpr int oD = kXmShared ? oL + n : oXm + 2 * n;   // t - g at the own edge points
  static constexpr int oJ = oD + TT;          // the jump and its four corner values
  static constexpr int oMa = oJ + TT + 4;     // mass constraint: ax, ay, hx, hy (m each), a . h
  static constexpr int oRed = oMa + 4 * mA + 1;
  // the projection's edge tables (l0, l1, (C^T C)^-1, l0.l0, l0.l1, l1.l1): in
  // the space of the partial products (free until the first Vz^T product,
  // which follows the projection) where that holds them, else after the rest
  static constexpr int kEdge = 2 * N + 19;
  static constexpr bool kEdgeShared = W * mmA >= kEdge;
  static constexpr int oEdge = kEdgeShared ? oPart : oRed + 16;
  static constexpr int end = oRed + 16 + (kEdgeShared ? 0 : kEdge);
  static constexpr size_t bytes = sizeof(double) * end;
  // at most as many as the registers admit without spilling (by order and fit
  // shape; the general form, with the mass constraint and several components,
  // holds more)
  static constexpr int waves = LayR<N>::lds_waves(bytes, N <= 6 ? (W == 1 ? 6 : 5) : N <= 10 ? 4 : 3, 64 * W);
  static constexpr int waves_general = LayR<N>::lds_waves(bytes, N <= 8 ? 4 : 3, 64 * W);
  static constexpr int waves_multi = LayR<N>::lds_waves(bytes, N <= 6 ? 4 : 3, 64 * W);   // batched launches
  static constexpr int NQ = (n + 3) / 4;   // steps of 4 nodes
};

// out[i] = (Vz c)_i, i < n
template <int N, int T>
__device__ void z_V(const double* Xz, const double* Yz, const double* c, double* out) {
  using L = LayZ<N>;
  constexpr int m = L::m;
  for (int i = tid(); i < L::n; i += T) {
    double xr[m];
#pragma unroll
    for (int k = 0; k < m; ++k) xr[k] = Xz[k * L::ZS + i];
    double v = 0.0;
#pragma unroll 1
    for (int l = 0; l < m; ++l) {
      double inner = 0.0;
#pragma unroll
      for (int k = 0; k < m; ++k) inner += xr[k] * c[l * m + k];
      v += Yz[l * L::ZS + i] * inner;
    }
    out[i] = v;
  }
}

// Partial products Vz^T r over each wavefront's share of the nodes: part[w][(l, k)] =
// sum_{i of w} Yz[l][i] r[i] Xz[k][i], the m x m matrix Yz diag(r) Xz^T as one
// 16 x 16 float64 matrix-core tile per wavefront (K in steps of 4).  With dotw
// given, <dotw, part[w]> goes to dots[w].  No barrier.
template <int N, int T>
__device__ void z_VT_part(const double* Xz, const double* Yz, const double* r, double* part,
                          const double* dotw = nullptr, double* dots = nullptr) {
  typedef Mma<double> M64;
  using L = LayZ<N>;
  constexpr int n = L::n, m = L::m, ZS = L::ZS, KW = (L::NQ + T / 64 - 1) / (T / 64);   // steps a wavefront
  const int w = wave(), l = lane(), lr = l & 15, lk = l >> 4;
  const bool col = lr < m;
  const int lrc = col ? lr : 0;
  M64::acc_t ac[2] = {zacc<double>(), zacc<double>()};
  // every lane loads, so that the loads need no branches and can be issued
  // ahead of the products.  Lanes past the m rows (columns) read row 0: they
  // only feed the tile's rows (columns) beyond m, which are not kept.  Past
  // the last node (at most 4 W + 3 places, only in the last SAFE.. steps) the
  // loads read the next row, or the arrays that follow Yz and r in the
  // workgroup's LDS, and the products take zeros there.
  constexpr int SAFE0 = (n - 3) / 4 - (T / 64 - 1) * KW;   // steps in range for every wavefront
  constexpr int SAFE = SAFE0 < 0 ? 0 : SAFE0 > KW ? KW : SAFE0;
#pragma unroll
  for (int kq = 0; kq < KW; ++kq) {
    const int i = 4 * (w * KW + kq) + lk;
    const double ya = Yz[lrc * ZS + i], xb = Xz[lrc * ZS + i], rb = r[i];
    double a = ya, b = rb * xb;   // A[l][i], B[i][k]
    if (kq >= SAFE) {
      const bool ok = i < n;
      a = ok ? a : 0.0;
      b = ok ? b : 0.0;
    }
    ac[kq & 1] = M64::mma(a, b, ac[kq & 1]);
  }
  double d = 0.0;
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const int ly = M64::row(l, s4);
    if (ly < m && col) {
      const double v = ac[0][s4] + ac[1][s4];
      part[w * L::mmA + ly * m + lr] = v;
      if (dotw) d += dotw[ly * m + lr] * v;
    }
  }
  if (dotw) {
    d = wave_total(d);
    if (l == 0) dots[w] = d;
  }
}

// Inverse of the 1-D preconditioner block Bz^T Bz, Bz[a][k] = s(xi_a + d) psi_k(xi_a)
// with s(x) = x (1 - x) (the bubble table at the Gauss nodes shifted by d, in the
// basis centred on d); Vx: psi_k(xi_a) at [a N + k] (in LDS).  Called by a whole
// wavefront (uniform control flow): lane c < m forms column c of the Gram
// matrix, then Gauss-Jordan elimination without pivoting (the matrix is
// symmetric positive definite: at most two shifted nodes make s vanish, and
// N - 2 >= m rows remain) runs in registers, the pivot column broadcast from its
// lane.  The inverse goes to out0, row-major m x m.  TWO: the upper half of the
// wavefront (lanes 32 + c) forms the block at d1 into out1 at the same time.
template <int N, bool TWO = false>
__device__ __forceinline__ void z_gram_inverse(const double* Vx, const double* xi, double d0, double* out0,
                                               double d1 = 0.0, double* out1 = nullptr) {
  constexpr int m = LayZ<N>::m;
  static_assert(!TWO || m <= 32, "two blocks a wavefront");
  const int h = TWO ? lane() >> 5 : 0;
  const int c = TWO ? lane() & 31 : lane();
  const double d = h ? d1 : d0;
  double col[m];
#pragma unroll
  for (int k = 0; k < m; ++k) col[k] = 0.0;
  if (c < m) {
    // two nodes at a time, so that only two rows of Vx are held
#pragma unroll 2
    for (int a = 0; a < N; ++a) {
      const double xa = xi[a] + d;
      const double sa = xa * (1.0 - xa);
      const double va = (sa * sa) * Vx[a * N + c];
#pragma unroll
      for (int k = 0; k < m; ++k) col[k] += Vx[a * N + k] * va;
    }
  }
#pragma unroll
  for (int k = 0; k < m; ++k) {
    double ak[m];
#pragma unroll
    for (int i = 0; i < m; ++i) ak[i] = TWO ? (h ? bcast(col[i], 32 + k) : bcast(col[i], k)) : bcast(col[i], k);
    // the hardware reciprocal and two Newton steps: the inverse only
    // preconditions, so the last bit of the pivot's reciprocal does not matter
    double pinv = __builtin_amdgcn_rcp(ak[k]);
    pinv = fma(pinv, fma(-ak[k], pinv, 1.0), pinv);
    pinv = fma(pinv, fma(-ak[k], pinv, 1.0), pinv);
    if (c == k) {
#pragma unroll
      for (int i = 0; i < m; ++i) col[i] = (i == k) ? pinv : -ak[i] * pinv;
    } else {
      const double rk = col[k] * pinv;
#pragma unroll
      for (int i = 0; i < m; ++i) col[i] = (i == k) ? rk : col[i] - ak[i] * rk;
    }
  }
  if (c < m) {
    double* out = h ? out1 : out0;
#pragma unroll
    for (int i = 0; i < m; ++i) out[i * m + c] = col[i];
  }
}

// The same inverse with one matrix element a lane, for m^2 <= 64: lane
// (r, c) = (l / m, l % m) forms G[r][c] (the same sums in the same order as
// the column form), then each Gauss-Jordan step takes the pivot by a lane
// read and the pivot row's and column's entries by two lane permutations, so
// a step is one exchange instead of 2m lane reads.  The arithmetic is that of
// the column form, term for term.  TWO: lanes 32 + (r, c) form the block at
// d1 into out1 at the same time (m^2 <= 32).
template <int N, bool TWO = false>
__device__ __forceinline__ void z_gram_inverse_ep(const double* Vx, const double* xi, double d0, double* out0,
                                                  double d1 = 0.0, double* out1 = nullptr) {
  constexpr int m = LayZ<N>::m, mm = m * m;
  static_assert(mm <= 64 && (!TWO || mm <= 32), "one element a lane");
  const int l = lane();
  const int h = TWO ? l >> 5 : 0;
  const int le = TWO ? l & 31 : l;
  const bool live = le < mm;
  const int r = live ? le / m : 0, c = live ? le % m : 0;
  const double d = h ? d1 : d0;
  double a = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double xa = xi[j] + d;
    const double sa = xa * (1.0 - xa);
    a += Vx[j * N + r] * ((sa * sa) * Vx[j * N + c]);
  }
  const int base = h << 5;
#pragma unroll
  for (int k = 0; k < m; ++k) {
    // the pivot of each half, the entry (k, c) of the lane's column and (r, k) of its row
    const double pk0 = bcast(a, k * m + k);
    const double pk = TWO ? (h ? bcast(a, 32 + k * m + k) : pk0) : pk0;
    const int srow = (base + k * m + c) << 2, scol = (base + r * m + k) << 2;
    const double arow = __hiloint2double(__builtin_amdgcn_ds_bpermute(srow, __double2hiint(a)),
                                         __builtin_amdgcn_ds_bpermute(srow, __double2loint(a)));
    const double acol = __hiloint2double(__builtin_amdgcn_ds_bpermute(scol, __double2hiint(a)),
                                         __builtin_amdgcn_ds_bpermute(scol, __double2loint(a)));
    double pinv = __builtin_amdgcn_rcp(pk);
    pinv = fma(pinv, fma(-pk, pinv, 1.0), pinv);
    pinv = fma(pinv, fma(-pk, pinv, 1.0), pinv);
    if (c == k) a = (r == k) ? pinv : -acol * pinv;
    else a = (r == k) ? arow * pinv : a - acol * (arow * pinv);
  }
  if (live) (h ? out1 : out0)[r * m + c] = a;
}

// j = P d (d: the 4N edge data t - g, edges W, E, S, N) and the corner values
// of j (SW, NW, SE, NE) into J[0..4N+4), by one wavefront; tab: the edge
// tables l0 (N), l1 (N), (C^T C)^-1 (16), l0.l0, l0.l1, l1.l1.  P projects onto the
// edge values of Q_{N-1}: the vectors whose edges' polynomials agree at the
// four corners, the null space of C^T with C's columns the corner
// differences; P = I - C (C^T C)^-1 C^T.  C^T d takes the eight end values
// l_s . d_e (lanes 0..7), then lambda = (C^T C)^-1 C^T d, j = d - C lambda, and
// a corner value is the mean of its two edges' end values (equal after the
// projection).  No barrier.
template <int N>
__device__ void z_project(const double* tab, const double* D, double* J) {
  const double* l0 = tab;
  const double* l1 = tab + N;
  const double* Ci = tab + 2 * N;
  const double* Ls = tab + 2 * N + 16;
  const int l = lane();
  double a = 0.0;
  if (l < 8) {   // end value s = l & 1 of edge e = l >> 1
    const double* ls = (l & 1) ? l1 : l0;
    const double* de = D + (l >> 1) * N;
#pragma unroll
    for (int k = 0; k < N; ++k) a += ls[k] * de[k];
  }
  const double aW0 = bcast(a, 0), aW1 = bcast(a, 1), aE0 = bcast(a, 2), aE1 = bcast(a, 3);
  const double aS0 = bcast(a, 4), aS1 = bcast(a, 5), aN0 = bcast(a, 6), aN1 = bcast(a, 7);
  const double y[4] = {aW0 - aS0, aW1 - aN0, aE0 - aS1, aE1 - aN1};   // C^T d
  double lam[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) lam[i] = ((Ci[4 * i] * y[0] + Ci[4 * i + 1] * y[1]) + Ci[4 * i + 2] * y[2]) + Ci[4 * i + 3] * y[3];
  const double sw = lam[0], nw = lam[1], se = lam[2], ne = lam[3];
  for (int q = l; q < 4 * N; q += 64) {
    const int e = q / N, k = q % N;
    double c;   // (C lambda)_q
    if (e == 0) c = l0[k] * sw + l1[k] * nw;
    else if (e == 1) c = l0[k] * se + l1[k] * ne;
    else if (e == 2) c = -(l0[k] * sw + l1[k] * se);
    else c = -(l0[k] * nw + l1[k] * ne);
    J[q] = D[q] - c;
  }
  if (l < 4) {   // the corner values from the end values of j
    const double L00 = Ls[0], L01 = Ls[1], L11 = Ls[2];
    double v;
    if (l == 0) v = (aW0 - (L00 * sw + L01 * nw)) + (aS0 + (L00 * sw + L01 * se));
    else if (l == 1) v = (aW1 - (L01 * sw + L11 * nw)) + (aN0 + (L00 * nw + L01 * ne));
    else if (l == 2) v = (aE0 - (L00 * se + L01 * ne)) + (aS1 + (L01 * sw + L11 * se));
    else v = (aE1 - (L01 * se + L11 * ne)) + (aN1 + (L01 * nw + L11 * ne));
    J[4 * N + l] = 0.5 * v;
  }
}

// s0 = sum_a l_a(x) j0[a] and s1 = sum_a l_a(x) j1[a] for the Lagrange basis of
// the Gauss abscissae in the first form, l_a(x) = w_a prod_{b != a} (x - xi_b),
// from prefix products and a running suffix product.
template <int N>
__device__ __forceinline__ void lagrange_dots(double x, const double* xi, const double* bw, const double* j0,
                                              const double* j1, double& s0, double& s1) {
  double pre[N];
  double pr = 1.0;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    pre[a] = pr;
    pr *= x - xi[a];
  }
  double suf = 1.0, a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int a = N - 1; a >= 0; --a) {
    const double la = (pre[a] * suf) * bw[a];
    a0 += la * j0[a];
    a1 += la * j1[a];
    suf *= x - xi[a];
  }
  s0 = a0;
  s1 = a1;
}

// Transfinite interpolant of the edge traces j (W, E, S, N blocks of N values at
// the Gauss abscissae, then the corners SW, NW, SE, NE) at (x, y).
template <int N>
__device__ __forceinline__ double coons(const double* j, const double* xi, const double* bw, double x, double y) {
  double tw, te, ts, tn;
  lagrange_dots<N>(y, xi, bw, j, j + N, tw, te);
  lagrange_dots<N>(x, xi, bw, j + 2 * N, j + 3 * N, ts, tn);
  const double* cr = j + 4 * N;
  const double x1 = 1.0 - x, y1 = 1.0 - y;
  return (x1 * tw + x * te) + (y1 * ts + y * tn) - (x1 * (y1 * cr[0] + y * cr[1]) + x * (y1 * cr[2] + y * cr[3]));
}

// The same at the Gauss node (xi_a, xi_b), where the Lagrange values are unit vectors.
template <int N>
__device__ __forceinline__ double coons_node(const double* j, int a, int b, double x, double y) {
  const double* cr = j + 4 * N;
  const double x1 = 1.0 - x, y1 = 1.0 - y;
  return (x1 * j[b] + x * j[N + b]) + (y1 * j[2 * N + a] + y * j[3 * N + a]) -
         (x1 * (y1 * cr[0] + y * cr[1]) + x * (y1 * cr[2] + y * cr[3]));
}

// The (N-2)^2-vector work of the bubble iteration runs in wavefront 0 alone,
// each lane taking the entries p = lane, lane + 64, ...; its LDS traffic is
// ordered by wave_sync, and its sums are wavefront shuffles.

// Sum over wavefront 0 (every lane gets it).
__device__ __forceinline__ double wave_sum(double v) { return wave_total(v); }

// out = (Gx (x) Gy) v over v[l m + k] (tmp m^2 doubles), by wavefront 0.  With rr
// given, returns rr . out in rg and out . out in gg.
template <int N>
__device__ __forceinline__ void z_pinv_w0(const double* Gx, const double* Gy, const double* v, double* tmp, double* out,
                                          const double* rr = nullptr, double* rg = nullptr, double* gg = nullptr) {
  constexpr int m = LayZ<N>::m;
  const int l0 = lane();
  for (int p = l0; p < m * m; p += 64) {
    const int k = p % m, l = p / m;
    double acc = 0.0;
#pragma unroll
    for (int kk = 0; kk < m; ++kk) acc += Gx[k * m + kk] * v[l * m + kk];
    tmp[p] = acc;
  }
  wave_sync();
  double a = 0.0, c = 0.0;
  for (int p = l0; p < m * m; p += 64) {
    const int k = p % m, l = p / m;
    double acc = 0.0;
#pragma unroll
    for (int ll = 0; ll < m; ++ll) acc += Gy[l * m + ll] * tmp[ll * m + k];
    out[p] = acc;
    if (rr) {
      a += rr[p] * acc;
      c += acc * acc;
    }
  }
  wave_sync();
  if (rr) {
    *rg = wave_sum(a);
    *gg = wave_sum(c);
  }
}

// MC: the general form, with the mass-constraint code (it runs where p.mass
// is set) and any number of components; without it, one component and no
// constraint, and fewer values held across the fit.
template <int N, int T, bool MC = true>
__device__ __forceinline__ void r_phase2_body(const Params2D& p, double* lds, int64_t fit) {
  constexpr int W = T / 64;
  using L = LayZ<N, W>;
  constexpr int n = L::n, m = L::m, mm = L::mm, mmA = L::mmA;
  static_assert(n <= T, "one node a thread");
  const int64_t w = fit / p.M;
  const int64_t s = fit - w * p.M;
  const WorkRec* e = p.wrec + w;
  const Normal2 z = fit_increments(p, s);
  const int t = tid();
  const bool node = t < n;
  const int64_t noff = e->noff;
  const double* xi = p.xi_tab + N * kMaxN;
  const double* nsp = p.nsp + p.nsp_off[N];
  double* red = lds + L::oRed;
  double* D = lds + L::oD;
  const Shift2 dsh = mean_shift(e, z);
  const double dbx = dsh.x, dby = dsh.y;
  // component 0's jump data first: its loads overlap the moves
  r_jump_data<N, T>(p, e, s * p.ncomp, z.a, z.b, D, t);
  // psi_k(xi_a) for the Gram inverses, in the space of the lift values (free
  // until the lift), and the projection's edge tables
  if constexpr (m > 0)
    for (int i = t; i < N * N; i += T) lds[L::oL + i] = nsp[nsp_vx(N) + i];
  for (int i = t; i < L::kEdge; i += T) lds[L::oEdge + i] = nsp[nsp_ends(N) + i];
  // the moved nodes (eq. def_dx), one a thread
  double xm = 0.0, ym = 0.0;
  if (node) {
    const int64_t k = noff + t;
    xm = moved_coord(p.xi_node[2 * k], p.A[2 * k], p.B[2 * k], z.a);
    ym = moved_coord(p.xi_node[2 * k + 1], p.A[2 * k + 1], p.B[2 * k + 1], z.b);
  }
  double* Xz = lds + L::oXz;
  double* Yz = lds + L::oYz;
  double* XYm = lds + L::oXm;   // the coordinates wait in LDS for the first component's lift
  if (node) {
    XYm[t] = xm;
    XYm[n + t] = ym;
  }
  if constexpr (m > 0) {
    // bubble tables at the moved nodes, one a thread; the two Gram inverses by
    // the last two wavefronts
    if (node) {
      double q[m];
      legendre_eval_k<m>(xm - dbx, q);
      const double sxm = xm * (1.0 - xm);
#pragma unroll
      for (int k = 0; k < m; ++k) Xz[k * L::ZS + t] = sxm * q[k];
      legendre_eval_k<m>(ym - dby, q);
      const double sym = ym * (1.0 - ym);
#pragma unroll
      for (int k = 0; k < m; ++k) Yz[k * L::ZS + t] = sym * q[k];
    }
    block_sync();
    if constexpr (m * m <= 32 && W == 1) {   // both blocks at once, one a half-wavefront
      z_gram_inverse_ep<N, true>(lds + L::oL, xi, dbx, lds + L::oGx, dby, lds + L::oGy);
    } else if constexpr (m * m <= 64 && W == 1) {
      z_gram_inverse_ep<N>(lds + L::oL, xi, dbx, lds + L::oGx);
      z_gram_inverse_ep<N>(lds + L::oL, xi, dby, lds + L::oGy);
    } else if constexpr (m * m <= 64) {
      const int wg = wave() - (W - 2);   // the last two wavefronts
      if (wg >= 0) z_gram_inverse_ep<N>(lds + L::oL, xi, wg ? dby : dbx, lds + (wg ? L::oGy : L::oGx));
    } else if constexpr (W == 1) {
      z_gram_inverse<N, true>(lds + L::oL, xi, dbx, lds + L::oGx, dby, lds + L::oGy);
    } else {
      const int wg = wave() - (W - 2);   // the last two wavefronts
      if (wg >= 0) z_gram_inverse<N>(lds + L::oL, xi, wg ? dby : dbx, lds + (wg ? L::oGy : L::oGx));
    }
  }
  const double zz = nsp[nsp_zz(N)];
  const double* Gx = lds + L::oGx;
  const double* Gy = lds + L::oGy;
  double* Bv = lds + L::oB;
  double* Wv = lds + L::oW;
  double* Rv = lds + L::oR;
  double* Gv = lds + L::oG;
  double* Pv = lds + L::oP;
  double* Tv = lds + L::oT;
  double* part = lds + L::oPart;
  double* Lv = lds + L::oL;
  double* J = lds + L::oJ;
  const double* bw = nsp + nsp_bary(N);
  const double* wq = p.wq_tab + N * kMaxN;   // the element's quadrature weights (mass constraint)
  auto qsum = [&](int j) {
    if constexpr (W == 4) return ((part[j] + part[mmA + j]) + part[2 * mmA + j]) + part[3 * mmA + j];
    else if constexpr (W == 2) return part[j] + part[mmA + j];
    else return part[j];
  };
  int its = 0, unconv = 0;
  double rmax = 0.0;
  // the components share the moved nodes and every table above (Sec. 5.3,
  // last paragraph); each has its own p0, traces and boundary data
  const int ncomp = MC ? p.ncomp : 1;
  for (int c = 0; c < ncomp; ++c) {
    const int64_t row = s * ncomp + c;
    // the thread index, opaque to the compiler here, so that the addresses
    // derived from it are formed again in each pass instead of held (spilled)
    // in registers across the loop
    int tl = t;
    asm volatile("" : "+v"(tl));
    const bool nodel = tl < n;
    if (c > 0) {
      r_jump_data<N, T>(p, e, row, z.a, z.b, D, tl);
      if constexpr (L::kEdgeShared)   // the iteration has overwritten them
        for (int i = tl; i < L::kEdge; i += T) lds[L::oEdge + i] = nsp[nsp_ends(N) + i];
      if constexpr (L::kXmShared) {   // the iteration has overwritten them
        if (nodel) {
          const int64_t k = noff + tl;
          XYm[tl] = moved_coord(p.xi_node[2 * k], p.A[2 * k], p.B[2 * k], z.a);
          XYm[n + tl] = moved_coord(p.xi_node[2 * k + 1], p.A[2 * k + 1], p.B[2 * k + 1], z.b);
        }
      }
    }
    block_sync();
    // j = P (t - g) and its corner values
    if (wave() == 0) z_project<N>(lds + L::oEdge, D, J);
    block_sync();
    double p0v = 0.0, lnode = 0.0, sc = 0.0, mc = 0.0;
    if (nodel) {
      const int ja = tl % N, jb = tl / N;
      p0v = p.phi[row * p.nodes + noff + tl];
      Lv[tl] = coons<N>(J, xi, bw, XYm[tl], XYm[n + tl]);
      lnode = coons_node<N>(J, ja, jb, xi[ja], xi[jb]);
      sc = p0v * p0v + lnode * lnode;
      if (MC && p.mass) mc = (wq[ja] * wq[jb]) * lnode;   // the lift's integral over the element
    }
    if constexpr (MC) block_sum2<T>(sc, mc, red);   // also the barrier after Lv
    else sc = block_sum<T>(sc, red);
    const double scale = sc;
    const double cmass = -mc;     // the bubble part must cancel the lift's integral
    double bub = 0.0;
    if constexpr (m > 0) {
      // b = -Vz^T lift(j); w = (Gx (x) Gy) b; r = Vz^T Vz w - b; g = (Gx (x) Gy) r;
      // then conjugate gradients, three workgroup barriers an iteration
      const double xx = zz > 0.0 ? scale / zz : 0.0;
      const double stop = p.tol2 * xx;
      const bool w0 = wave() == 0;
      double rg = 0.0, gg = 0.0;      // wavefront 0's
      // the mass constraint (G14) is one linear condition a . w = cmass on the
      // bubble coefficients, a[(l, k)] = ay[l] ax[k] the integrals of the bubble
      // functions; its projection in the preconditioner's metric uses
      // h = (Gx (x) Gy) a = hy (x) hx: v -= h (a . v) / (a . h)
      double* Ma = lds + L::oMa;
      if (MC && p.mass && c == 0 && w0) {
        // ax[k] = sum_a wq[a] beta_k(xi_a) (shifted by dbx; ay likewise by dby)
        if (lane() < 2) {
          const int dir = lane();
          double acc[m];
#pragma unroll
          for (int k = 0; k < m; ++k) acc[k] = 0.0;
          for (int a = 0; a < N; ++a) {
            double q[m];
            legendre_eval_k<m>(xi[a] - (dir ? dby : dbx), q);
            const double wa = wq[a] * (xi[a] * (1.0 - xi[a]));
#pragma unroll
            for (int k = 0; k < m; ++k) acc[k] += wa * q[k];
          }
#pragma unroll
          for (int k = 0; k < m; ++k) Ma[dir * m + k] = acc[k];
        }
        wave_sync();
        for (int q = lane(); q < 2 * m; q += 64) {
          const int dir = q >= m, k = q - dir * m;
          const double* G = dir ? Gy : Gx;
          double acc = 0.0;
          for (int kk = 0; kk < m; ++kk) acc += G[k * m + kk] * Ma[dir * m + kk];
          Ma[2 * m + q] = acc;
        }
        wave_sync();
        if (lane() == 0) {
          double sx = 0.0, sy = 0.0;
          for (int k = 0; k < m; ++k) {
            sx += Ma[k] * Ma[2 * m + k];
            sy += Ma[m + k] * Ma[3 * m + k];
          }
          Ma[4 * m] = sx * sy;
        }
        wave_sync();
      }
      // wavefront 0: v -= h (a . v - target) / (a . h), which puts v on a . v = target
      auto mass_project = [&](double* v, double target) {
        double d = 0.0;
        for (int j = lane(); j < mm; j += 64) d += (Ma[m + j / m] * Ma[j % m]) * v[j];
        const double f = (wave_sum(d) - target) / Ma[4 * m];
        for (int j = lane(); j < mm; j += 64) v[j] -= (Ma[3 * m + j / m] * Ma[2 * m + j % m]) * f;
        wave_sync();
      };
      // wavefront 0: with g = (Gx (x) Gy) r given, g -= mu h and r -= mu a, mu = (a . g) / (a . h):
      // g becomes the projected preconditioned residual, and r keeps the size of the
      // error (otherwise its component along a, the constraint's multiplier, grows and
      // its rounding stalls the iteration)
      auto mass_resid = [&](double* r, double* g) {
        double d = 0.0;
        for (int j = lane(); j < mm; j += 64) d += (Ma[m + j / m] * Ma[j % m]) * g[j];
        const double mu = wave_sum(d) / Ma[4 * m];
        for (int j = lane(); j < mm; j += 64) {
          g[j] -= (Ma[3 * m + j / m] * Ma[2 * m + j % m]) * mu;
          r[j] -= (Ma[m + j / m] * Ma[j % m]) * mu;
        }
        wave_sync();
      };
      // wavefront 0: the residual's dot products with the (projected) g
      auto dots = [&](double& rgo, double& ggo) {
        double a = 0.0, b = 0.0;
        for (int j = lane(); j < mm; j += 64) {
          a += Rv[j] * Gv[j];
          b += Gv[j] * Gv[j];
        }
        rgo = wave_sum(a);
        ggo = wave_sum(b);
      };
      z_VT_part<N, T>(Xz, Yz, Lv, part);
      block_sync();
      if (w0) {
        for (int j = lane(); j < mm; j += 64) Bv[j] = -qsum(j);
        wave_sync();
        z_pinv_w0<N>(Gx, Gy, Bv, Tv, Wv);
        if (MC && p.mass) mass_project(Wv, cmass);
      }
      block_sync();
      z_V<N, T>(Xz, Yz, Wv, Lv);
      block_sync();
      z_VT_part<N, T>(Xz, Yz, Lv, part);
      block_sync();
      double* flag = red + 12;
      if (w0) {
        for (int j = lane(); j < mm; j += 64) Rv[j] = qsum(j) - Bv[j];
        wave_sync();
        if (MC && p.mass) {
          z_pinv_w0<N>(Gx, Gy, Rv, Tv, Gv);
          mass_resid(Rv, Gv);
          dots(rg, gg);
        } else {
          z_pinv_w0<N>(Gx, Gy, Rv, Tv, Gv, Rv, &rg, &gg);
        }
        for (int j = lane(); j < mm; j += 64) Pv[j] = -Gv[j];
        if (lane() == 0) flag[0] = (gg > stop && p.max_iter > 0) ? 1.0 : 0.0;
      }
      block_sync();
      int it = 0;
      while (flag[0] != 0.0) {
        ++it;
        z_V<N, T>(Xz, Yz, Pv, Lv);
        block_sync();
        z_VT_part<N, T>(Xz, Yz, Lv, part, Pv, red);   // Vz^T Vz p in parts, <p, .> per part
        block_sync();
        if (w0) {
          const double alpha = rg / wsum<T>(red);
          for (int j = lane(); j < mm; j += 64) {
            Rv[j] += alpha * qsum(j);
            Wv[j] += alpha * Pv[j];
          }
          wave_sync();
          double rg1;
          if (MC && p.mass) {
            z_pinv_w0<N>(Gx, Gy, Rv, Tv, Gv);
            mass_resid(Rv, Gv);
            dots(rg1, gg);
          } else {
            z_pinv_w0<N>(Gx, Gy, Rv, Tv, Gv, Rv, &rg1, &gg);
          }
          const double beta = rg1 / rg;
          rg = rg1;
          for (int j = lane(); j < mm; j += 64) Pv[j] = beta * Pv[j] - Gv[j];
          if (lane() == 0) flag[0] = (gg > stop && it < p.max_iter) ? 1.0 : 0.0;
        }
        block_sync();
      }
      if (w0) {
        its += it;
        unconv += gg <= stop ? 0 : 1;
        rmax = fmax(rmax, rel_resid(gg, xx));
      }
      if (MC && p.mass) {   // the constraint to working accuracy
        if (w0) mass_project(Wv, cmass);
        block_sync();
      }
      if (nodel) {   // the bubbles at the Gauss node (xi_ja, xi_jb)
        const int ja = tl % N, jb = tl / N;
        double zr[m], zc[m];
        legendre_eval_k<m>(xi[ja] - dbx, zr);
        legendre_eval_k<m>(xi[jb] - dby, zc);
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < m; ++l) {
          double inner = 0.0;
#pragma unroll
          for (int k = 0; k < m; ++k) inner += zr[k] * Wv[l * m + k];
          acc += zc[l] * inner;
        }
        bub = ((xi[ja] * (1.0 - xi[ja])) * (xi[jb] * (1.0 - xi[jb]))) * acc;
      }
    }
    // new values at the Gauss nodes (eq. phi_star)
    if (nodel) p.phi[row * p.nodes + noff + tl] = p0v - (lnode + bub);
  }
  count_fit(p, 2, its, unconv, rmax);
}

// Threads a fit of the per-order and batched kernels, by phase and order.
// The persistent fused kernel runs every order on four wavefronts.
template <int N, int PHASE>
constexpr int kFitThreads = PHASE == 1 ? (N <= 8 ? 64 : N <= 12 ? 128 : 256) : (N <= 8 ? 64 : N <= 11 ? 128 : 256);
// The wide fit shape of the per-order kernels: twice the wavefronts a fit, at
// most four (it shortens a fit where there are too few fits to fill the device).
template <int N, int PHASE>
constexpr int kWideThreads = kFitThreads<N, PHASE> < 256 ? 2 * kFitThreads<N, PHASE> : 256;

template <int N, int T>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(LayR<N>::template waves1<T>)))
void fit2r_phase1(Params2D p) {
  extern __shared__ __attribute__((aligned(16))) double lds_r1[];
  r_phase1_body<N, T>(p, lds_r1, blockIdx.x + p.block0);
}

template <int N, int T>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(LayL<N>::template waves<T>)))
void fit2r_phase1_lean(Params2D p) {
  extern __shared__ __attribute__((aligned(16))) double lds_l1[];
  r_phase1_lean<N, T>(p, lds_l1, blockIdx.x + p.block0, p.rescue_list, p.rescue_count);
}

// The listed fits of the lean kernel, redone by the full form: a persistent
// grid that walks the list (usually empty).
template <int N>
__global__ __launch_bounds__((kFitThreads<N, 1>)) __attribute__((amdgpu_waves_per_eu(N >= 15 ? 1 : 2)))
void fit2r_phase1_redo(Params2D p) {
  extern __shared__ __attribute__((aligned(16))) double lds_d1[];
  const unsigned int cnt = *p.rescue_count;
  for (unsigned int j = blockIdx.x; j < cnt; j += gridDim.x) {
    r_phase1_body<N, kFitThreads<N, 1>>(p, lds_d1, (int64_t)p.rescue_list[j], true);
    __syncthreads();
  }
}

template <int N, bool MC, int T>
__global__ __launch_bounds__(T)
__attribute__((amdgpu_waves_per_eu(MC ? LayZ<N, T / 64>::waves_general : LayZ<N, T / 64>::waves)))
void fit2r_phase2(Params2D p) {
  extern __shared__ __attribute__((aligned(16))) double lds_r2[];
  r_phase2_body<N, T, MC>(p, lds_r2, blockIdx.x + p.block0);
}

// T1, T2: threads a fit in phase 1 and 2.  The redo kernel keeps the default
// shape whatever T1 is.
template <int N, int T1, int T2>
static hipError_t launch_r_shape(int phase, const Params2D& p, int64_t nfits, hipStream_t st) {
  const size_t lds = phase == 1 ? LayR<N>::bytes1 : LayZ<N, T2 / 64>::bytes;
  if (phase == 1 && p.rescue_list && p.ncomp == 1 && p.block0 + nfits <= (int64_t)0xffffffff) {
    // lean form, then the full form over the fits it listed
    if (nfits <= 0) return hipSuccess;
    const int64_t chunk = (int64_t)1 << 30;
    for (int64_t b0 = 0; b0 < nfits; b0 += chunk) {
      Params2D q = p;
      q.block0 = p.block0 + b0;
      const int64_t nb = (nfits - b0) < chunk ? (nfits - b0) : chunk;
      hipLaunchKernelGGL((fit2r_phase1_lean<N, T1>), dim3((unsigned)nb), dim3(T1), LayL<N>::bytes, st, q);
      hipError_t err = hipGetLastError();
      if (err != hipSuccess) return err;
    }
    const unsigned grid = (unsigned)(nfits < 2048 ? (nfits > 0 ? nfits : 1) : 2048);
    hipLaunchKernelGGL((fit2r_phase1_redo<N>), dim3(grid), dim3(kFitThreads<N, 1>), LayR<N>::bytes1, st, p);
    return hipGetLastError();
  }
  const int64_t chunk = (int64_t)1 << 30;
  for (int64_t b0 = 0; b0 < nfits; b0 += chunk) {
    Params2D q = p;
    q.block0 = p.block0 + b0;
    const int64_t nb = (nfits - b0) < chunk ? (nfits - b0) : chunk;
    if (phase == 1)
      hipLaunchKernelGGL((fit2r_phase1<N, T1>), dim3((unsigned)nb), dim3(T1), lds, st, q);
    else if (q.mass || q.ncomp > 1)
      hipLaunchKernelGGL((fit2r_phase2<N, true, T2>), dim3((unsigned)nb), dim3(T2), lds, st, q);
    else
      hipLaunchKernelGGL((fit2r_phase2<N, false, T2>), dim3((unsigned)nb), dim3(T2), lds, st, q);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

template <int N>
static hipError_t launch_r(int phase, const Params2D& p, int64_t nfits, hipStream_t st, bool wide) {
  if (wide) return launch_r_shape<N, kWideThreads<N, 1>, kWideThreads<N, 2>>(phase, p, nfits, st);
  return launch_r_shape<N, kFitThreads<N, 1>, kFitThreads<N, 2>>(phase, p, nfits, st);
}

hipError_t launch_fit2r(int phase, int N, const Params2D& p, int64_t nfits, hipStream_t st, bool wide) {
  switch (N) {
    case 2: return launch_r<2>(phase, p, nfits, st, wide);
    case 3: return launch_r<3>(phase, p, nfits, st, wide);
    case 4: return launch_r<4>(phase, p, nfits, st, wide);
    case 5: return launch_r<5>(phase, p, nfits, st, wide);
    case 6: return launch_r<6>(phase, p, nfits, st, wide);
    case 7: return launch_r<7>(phase, p, nfits, st, wide);
    case 8: return launch_r<8>(phase, p, nfits, st, wide);
    case 9: return launch_r<9>(phase, p, nfits, st, wide);
    case 10: return launch_r<10>(phase, p, nfits, st, wide);
    case 11: return launch_r<11>(phase, p, nfits, st, wide);
    case 12: return launch_r<12>(phase, p, nfits, st, wide);
    case 13: return launch_r<13>(phase, p, nfits, st, wide);
    case 14: return launch_r<14>(phase, p, nfits, st, wide);
    case 15: return launch_r<15>(phase, p, nfits, st, wide);
    case 16: return launch_r<16>(phase, p, nfits, st, wide);
    default: return hipErrorInvalidValue;
  }
}

// One order of several problems in one launch: one workgroup per fit of the
// segments (problem, order group) of the argument table, all of order N.
// FAST: every problem has one component and no mass constraint (phase 1 the
// lean form, listing slow fits in each problem's own list; phase 2 without
// the general form).
template <int N, int PHASE, bool FAST>
__global__ __launch_bounds__((kFitThreads<N, PHASE>))
__attribute__((amdgpu_waves_per_eu(PHASE == 1 ? (FAST ? LayL<N>::template waves<kFitThreads<N, 1>> : LayR<N>::template waves1<kFitThreads<N, 1>>)
                                              : (FAST ? LayZ<N, kFitThreads<N, 2> / 64>::waves : LayZ<N, kFitThreads<N, 2> / 64>::waves_multi))))
void fit2r_multi(Fused2DArgs a) {
  extern __shared__ __attribute__((aligned(16))) double lds_rm[];
  const int64_t item = blockIdx.x;
  int sg = 0;
  while (sg + 1 < a.nseg && item >= a.seg[sg + 1].start) ++sg;
  const Params2D& p = *a.task[a.seg[sg].task];
  const int64_t fit = a.seg[sg].fit0 + (item - a.seg[sg].start);
  if constexpr (PHASE == 1 && FAST) r_phase1_lean<N, kFitThreads<N, 1>>(p, lds_rm, fit, p.rescue_list + p.rescue_off[N], p.rescue_count + N);
  else if constexpr (PHASE == 1) r_phase1_body<N, kFitThreads<N, 1>>(p, lds_rm, fit);
  else r_phase2_body<N, kFitThreads<N, 2>, !FAST>(p, lds_rm, fit);
}

// The fits that the lean batched kernel listed, problem by problem, redone by
// the full form (a persistent grid; the lists are usually empty).
template <int N>
__global__ __launch_bounds__((kFitThreads<N, 1>)) __attribute__((amdgpu_waves_per_eu(N >= 15 ? 1 : 2)))
void fit2r_multi_redo(Fused2DArgs a) {
  extern __shared__ __attribute__((aligned(16))) double lds_rr[];
  for (int sg = 0; sg < a.nseg; ++sg) {
    const Params2D& p = *a.task[a.seg[sg].task];
    const unsigned int cnt = p.rescue_count[N];
    const uint32_t* list = p.rescue_list + p.rescue_off[N];
    for (unsigned int j = blockIdx.x; j < cnt; j += gridDim.x) {
      r_phase1_body<N, kFitThreads<N, 1>>(p, lds_rr, (int64_t)list[j], true);
      __syncthreads();
    }
  }
}

template <int N>
static hipError_t multi_n(int phase, const Fused2DArgs& a, bool fast, hipStream_t st) {
  if (a.total <= 0) return hipSuccess;
  if (phase == 1 && fast) {
    hipLaunchKernelGGL((fit2r_multi<N, 1, true>), dim3((unsigned)a.total), dim3(kFitThreads<N, 1>), LayL<N>::bytes, st, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const unsigned grid = (unsigned)(a.total < 2048 ? a.total : 2048);
    hipLaunchKernelGGL((fit2r_multi_redo<N>), dim3(grid), dim3(kFitThreads<N, 1>), LayR<N>::bytes1, st, a);
  } else if (phase == 1) {
    hipLaunchKernelGGL((fit2r_multi<N, 1, false>), dim3((unsigned)a.total), dim3(kFitThreads<N, 1>), LayR<N>::bytes1, st, a);
  } else {
    constexpr size_t lds2 = LayZ<N, kFitThreads<N, 2> / 64>::bytes;
    if (fast) hipLaunchKernelGGL((fit2r_multi<N, 2, true>), dim3((unsigned)a.total), dim3(kFitThreads<N, 2>), lds2, st, a);
    else hipLaunchKernelGGL((fit2r_multi<N, 2, false>), dim3((unsigned)a.total), dim3(kFitThreads<N, 2>), lds2, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_fit2r_multi(int phase, int N, const Fused2DArgs& a, bool fast, hipStream_t st) {
  switch (N) {
    case 2: return multi_n<2>(phase, a, fast, st);
    case 3: return multi_n<3>(phase, a, fast, st);
    case 4: return multi_n<4>(phase, a, fast, st);
    case 5: return multi_n<5>(phase, a, fast, st);
    case 6: return multi_n<6>(phase, a, fast, st);
    case 7: return multi_n<7>(phase, a, fast, st);
    case 8: return multi_n<8>(phase, a, fast, st);
    case 9: return multi_n<9>(phase, a, fast, st);
    case 10: return multi_n<10>(phase, a, fast, st);
    case 11: return multi_n<11>(phase, a, fast, st);
    case 12: return multi_n<12>(phase, a, fast, st);
    case 13: return multi_n<13>(phase, a, fast, st);
    case 14: return multi_n<14>(phase, a, fast, st);
    case 15: return multi_n<15>(phase, a, fast, st);
    case 16: return multi_n<16>(phase, a, fast, st);
    default: return hipErrorInvalidValue;
  }
}

// Persistent form of the reference solver: one kernel per order present, each
// with the grid that fits on the device at once, pulling the fits of that
// order of several problems (segments) from its own device counter and
// running each with the body, fit shape, LDS layout and register budget of the
// batched kernel of that order, so its results are those of the per-order and
// batched kernels bit for bit.  (One kernel over every order would have to
// hold registers for all the orders' bodies at once.)  FAST as for the batched
// kernels; after a FAST phase 1 the batched redo kernel of each order walks the
// fits that the lean form listed.
__device__ __forceinline__ int64_t uniform64r(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

constexpr int kPersistChunk = 16;   // most items a workgroup claims at once

template <int N, int PHASE, bool FAST>
__global__ __launch_bounds__((kFitThreads<N, PHASE>))
__attribute__((amdgpu_waves_per_eu(PHASE == 1 ? (FAST ? LayL<N>::template waves<kFitThreads<N, 1>> : LayR<N>::template waves1<kFitThreads<N, 1>>)
                                              : (FAST ? LayZ<N, kFitThreads<N, 2> / 64>::waves : LayZ<N, kFitThreads<N, 2> / 64>::waves_multi))))
void fit2r_persist(Fused2DArgs a) {
  constexpr int T = kFitThreads<N, PHASE>;
  extern __shared__ __attribute__((aligned(16))) double lds_rp[];
  __shared__ int64_t item_sh;
  for (;;) {
    // a workgroup claims a.chunk consecutive items at a time (one atomic per
    // chunk, not per fit: millions of fits a launch would otherwise queue on
    // one address); every wavefront takes the same chunk and leaves on the
    // same one, so the grid drains once the counter has passed the last item
    int64_t item0;
    if constexpr (T == 64) {
      unsigned long long v = 0ull;
      if (threadIdx.x == 0) v = atomicAdd(a.counter, (unsigned long long)a.chunk);
      item0 = uniform64r((int64_t)v);
    } else {
      if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(a.counter, (unsigned long long)a.chunk);
      __syncthreads();
      item0 = uniform64r(item_sh);
      __syncthreads();
    }
    if (item0 >= a.total) break;
    const int64_t item1 = item0 + a.chunk < a.total ? item0 + a.chunk : a.total;
    int sg = 0;
#pragma unroll 1
    for (int64_t item = item0; item < item1; ++item) {
      while (sg + 1 < a.nseg && item >= a.seg[sg + 1].start) ++sg;
      const Params2D& p = *a.task[a.seg[sg].task];
      const int64_t fit = a.seg[sg].fit0 + (item - a.seg[sg].start);
      if constexpr (PHASE == 1 && FAST) r_phase1_lean<N, T>(p, lds_rp, fit, p.rescue_list + p.rescue_off[N], p.rescue_count + N);
      else if constexpr (PHASE == 1) r_phase1_body<N, T>(p, lds_rp, fit);
      else r_phase2_body<N, T, !FAST>(p, lds_rp, fit);
      __syncthreads();   // the next item reuses the LDS
    }
  }
}

template <int N>
static size_t lds_persist(int phase, bool fast) {
  return phase == 1 ? (fast ? LayL<N>::bytes : LayR<N>::bytes1) : LayZ<N, kFitThreads<N, 2> / 64>::bytes;
}

template <int N>
static int persist_occ(int phase, bool fast) {
  // a property of the kernel and the device model: asked once a process
  static std::atomic<int> known[2][2];
  std::atomic<int>& slot = known[phase - 1][fast ? 1 : 0];
  if (const int v = slot.load(std::memory_order_relaxed)) return v;
  const size_t lds = lds_persist<N>(phase, fast);
  const int T = phase == 1 ? kFitThreads<N, 1> : kFitThreads<N, 2>;
  int nb = 0;
  hipError_t e;
  if (phase == 1) e = fast ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit2r_persist<N, 1, true>, T, lds)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit2r_persist<N, 1, false>, T, lds);
  else e = fast ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit2r_persist<N, 2, true>, T, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit2r_persist<N, 2, false>, T, lds);
  if (e != hipSuccess) return 0;
  slot.store(nb, std::memory_order_relaxed);
  return nb;
}

// grid_req > 0: that many workgroups, else as many as are resident at once
// (occupancy x compute units); never more than the items.
template <int N>
static hipError_t persist_n(int phase, const Fused2DArgs& a, bool fast, int grid_req, int cus, hipStream_t st) {
  if (a.total <= 0) return hipSuccess;
  const size_t lds = lds_persist<N>(phase, fast);
  int64_t grid = grid_req;
  if (grid <= 0) {
    const int occ = persist_occ<N>(phase, fast);
    if (occ <= 0) return hipErrorInvalidConfiguration;
    grid = (int64_t)occ * cus;
  }
  grid = grid < a.total ? grid : a.total;
  // chunks small enough that every workgroup gets about four of them (one
  // item each where there are few), at most kPersistChunk
  Fused2DArgs c = a;
  const int64_t ck = a.total / (4 * grid);
  c.chunk = (int)(ck < 1 ? 1 : ck > kPersistChunk ? kPersistChunk : ck);
  const dim3 g((unsigned)grid), b((unsigned)(phase == 1 ? kFitThreads<N, 1> : kFitThreads<N, 2>));
  if (phase == 1 && fast) hipLaunchKernelGGL((fit2r_persist<N, 1, true>), g, b, lds, st, c);
  else if (phase == 1) hipLaunchKernelGGL((fit2r_persist<N, 1, false>), g, b, lds, st, c);
  else if (fast) hipLaunchKernelGGL((fit2r_persist<N, 2, true>), g, b, lds, st, c);
  else hipLaunchKernelGGL((fit2r_persist<N, 2, false>), g, b, lds, st, c);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || phase != 1 || !fast) return err;
  // the fits that the lean form listed, by the full form
  const unsigned rg = (unsigned)(a.total < 2048 ? a.total : 2048);
  hipLaunchKernelGGL((fit2r_multi_redo<N>), dim3(rg), dim3(kFitThreads<N, 1>), LayR<N>::bytes1, st, a);
  return hipGetLastError();
}

hipError_t launch_fit2r_persist(int phase, int N, const Fused2DArgs& a, bool fast, int grid, int cus, hipStream_t st) {
  switch (N) {
    case 2: return persist_n<2>(phase, a, fast, grid, cus, st);
    case 3: return persist_n<3>(phase, a, fast, grid, cus, st);
    case 4: return persist_n<4>(phase, a, fast, grid, cus, st);
    case 5: return persist_n<5>(phase, a, fast, grid, cus, st);
    case 6: return persist_n<6>(phase, a, fast, grid, cus, st);
    case 7: return persist_n<7>(phase, a, fast, grid, cus, st);
    case 8: return persist_n<8>(phase, a, fast, grid, cus, st);
    case 9: return persist_n<9>(phase, a, fast, grid, cus, st);
    case 10: return persist_n<10>(phase, a, fast, grid, cus, st);
    case 11: return persist_n<11>(phase, a, fast, grid, cus, st);
    case 12: return persist_n<12>(phase, a, fast, grid, cus, st);
    case 13: return persist_n<13>(phase, a, fast, grid, cus, st);
    case 14: return persist_n<14>(phase, a, fast, grid, cus, st);
    case 15: return persist_n<15>(phase, a, fast, grid, cus, st);
    case 16: return persist_n<16>(phase, a, fast, grid, cus, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sl
