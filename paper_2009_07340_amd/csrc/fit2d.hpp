// Building blocks of the two-dimensional element fit: one wavefront (64 lanes)
// owns one (element, sample) fit and keeps its matrices in LDS as 16x16 blocks.
//
// Dense products run on the matrix cores with v_mfma_f64_16x16x4f64:
//   D(16x16) += A(16x4) B(4x16), lane l holds A[l%16][l/16] and B[l/16][l%16]
//   of each 4-wide slice and D[l/16 + 4s][l%16] in accumulator slot s.
// A 16x16 block is stored row-major with a row stride of 17 doubles, so the
// 16 rows of one column fall into distinct LDS banks.
#pragma once
#include <hip/hip_runtime.h>
#include "sl_internal.hpp"

namespace sl {
namespace f2 {

constexpr int BS = 17;            // row stride of a stored block
constexpr int BLK = 16 * BS;      // doubles per stored block

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ void wave_sync() { __syncthreads(); }   // workgroups are one wavefront

// Broadcast lane src's value of x to the whole wavefront (src is wave-uniform).
__device__ __forceinline__ double bcast(double x, int src) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_readlane(lo, src);
  hi = __builtin_amdgcn_readlane(hi, src);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// A-operand / B^T-operand read of X[l%16][4kk + l/16]
__device__ __forceinline__ double rowpat(const double* X, int kk) {
  const int l = lane_id();
  return X[(l & 15) * BS + 4 * kk + (l >> 4)];
}
// B-operand / A^T-operand read of X[4kk + l/16][l%16]
__device__ __forceinline__ double colpat(const double* X, int kk) {
  const int l = lane_id();
  return X[(4 * kk + (l >> 4)) * BS + (l & 15)];
}
__device__ __forceinline__ d4 load_acc(const double* X) {
  const int l = lane_id();
  d4 r;
#pragma unroll
  for (int s = 0; s < 4; ++s) r[s] = X[((l >> 4) + 4 * s) * BS + (l & 15)];
  return r;
}
__device__ __forceinline__ void store_acc(double* X, d4 r) {
  const int l = lane_id();
#pragma unroll
  for (int s = 0; s < 4; ++s) X[((l >> 4) + 4 * s) * BS + (l & 15)] = r[s];
}
__device__ __forceinline__ d4 zero4() {
  d4 r = {0.0, 0.0, 0.0, 0.0};
  return r;
}

// Lower-triangular block (I, J), J <= I, in packed block storage.
__device__ __forceinline__ constexpr int tblk(int I, int J) { return I * (I + 1) / 2 + J; }

// In-place Cholesky of a 16x16 diagonal block whose first m rows/columns are
// live (the rest is padding and becomes identity), and its inverse into Linv.
// Lanes 0..15 hold one row each in registers; each finished column goes
// through a 16-entry LDS vector (col) and is read back with wave-uniform
// addresses, so every lane sees it at the cost of one broadcast LDS read.
__device__ __forceinline__ void factor_diag(double* D, double* Linv, int m, double* col) {
  const int l = lane_id();
  const int r = l & 15;
  double row[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) row[c] = (c <= r) ? D[r * BS + c] : 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (l == j) col[16] = row[j];
    wave_sync();
    const double djj = col[16];
    const double ljj = (j < m) ? sqrt(djj) : 1.0;
    const double inv = 1.0 / ljj;
    double lrj;
    if (r == j) lrj = ljj;
    else if (r > j) lrj = (j < m && r < m) ? row[j] * inv : 0.0;
    else lrj = 0.0;
    row[j] = lrj;
    if (l < 16) col[r] = lrj;
    wave_sync();
#pragma unroll
    for (int c = j + 1; c < 16; ++c) {
      const double lcj = col[c];
      if (r >= c) row[c] -= lrj * lcj;
    }
    wave_sync();
  }
  if (l < 16) {
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) D[r * BS + cc] = row[cc];
  }
  wave_sync();
  // inverse: lane c solves L x = e_c (column c of L^-1); rows of L read with uniform addresses
  double x[16];
  const int c = r;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    double acc = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) acc -= D[i * BS + k] * x[k];
    x[i] = acc / D[i * BS + i];
  }
  if (l < 16) {
#pragma unroll
    for (int i = 0; i < 16; ++i) Linv[i * BS + c] = x[i];
  }
  wave_sync();
}

// Blocked right-looking Cholesky of a packed lower block matrix G (nb x nb
// blocks, live size n, padding -> identity).  Linv receives the inverses of
// the diagonal blocks of L.
template <int NB>
__device__ __forceinline__ void cholesky(double* G, double* Linv, int n, double* col) {
#pragma unroll 1
  for (int kb = 0; kb < NB; ++kb) {
    const int m = n - 16 * kb < 16 ? n - 16 * kb : 16;
    factor_diag(G + tblk(kb, kb) * BLK, Linv + kb * BLK, m, col);
    const double* Li = Linv + kb * BLK;
    // panel: L(I,kb) = G(I,kb) Linv(kb)^T
#pragma unroll 1
    for (int I = kb + 1; I < NB; ++I) {
      double* P = G + tblk(I, kb) * BLK;
      d4 acc = zero4();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = mfma(rowpat(P, kk), rowpat(Li, kk), acc);
      wave_sync();
      store_acc(P, acc);
    }
    wave_sync();
    // trailing update: G(I,J) -= L(I,kb) L(J,kb)^T, kb < J <= I
#pragma unroll 1
    for (int J = kb + 1; J < NB; ++J) {
      const double* LJ = G + tblk(J, kb) * BLK;
#pragma unroll 1
      for (int I = J; I < NB; ++I) {
        const double* LI = G + tblk(I, kb) * BLK;
        double* T = G + tblk(I, J) * BLK;
        d4 acc = load_acc(T);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = mfma(-rowpat(LI, kk), rowpat(LJ, kk), acc);
        store_acc(T, acc);
      }
    }
    wave_sync();
  }
}

// Solve L y = b in place (vector v of length 16*NB in LDS), L from cholesky().
template <int NB>
__device__ __forceinline__ void forward_solve(const double* G, const double* Linv, double* v, double* tmp) {
  const int l = lane_id();
  const int r = l & 15;
#pragma unroll 1
  for (int kb = 0; kb < NB; ++kb) {
    if (l < 16) {
      double t = v[16 * kb + r];
      for (int J = 0; J < kb; ++J) {
        const double* LB = G + tblk(kb, J) * BLK;
#pragma unroll
        for (int c = 0; c < 16; ++c) t -= LB[r * BS + c] * v[16 * J + c];
      }
      tmp[r] = t;
    }
    wave_sync();
    if (l < 16) {
      const double* Li = Linv + kb * BLK;
      double y = 0.0;
#pragma unroll
      for (int c = 0; c <= 15; ++c) y += Li[r * BS + c] * tmp[c];
      v[16 * kb + r] = y;
    }
    wave_sync();
  }
}

// Solve L^T x = y in place.
template <int NB>
__device__ __forceinline__ void backward_solve(const double* G, const double* Linv, double* v, double* tmp) {
  const int l = lane_id();
  const int r = l & 15;
#pragma unroll 1
  for (int kb = NB - 1; kb >= 0; --kb) {
    if (l < 16) {
      double t = v[16 * kb + r];
      for (int J = kb + 1; J < NB; ++J) {
        const double* LB = G + tblk(J, kb) * BLK;   // L(J,kb)^T row r = column r of L(J,kb)
#pragma unroll
        for (int c = 0; c < 16; ++c) t -= LB[c * BS + r] * v[16 * J + c];
      }
      tmp[r] = t;
    }
    wave_sync();
    if (l < 16) {
      const double* Li = Linv + kb * BLK;
      double x = 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c) x += Li[c * BS + r] * tmp[c];
      v[16 * kb + r] = x;
    }
    wave_sync();
  }
}

}  // namespace f2
}  // namespace sl
