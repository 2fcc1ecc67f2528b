// Block linear algebra for the two-dimensional fit, shared by the float64 and
// float32 storage modes.  One workgroup of four wavefronts owns one fit; its
// matrices live in LDS as 16x16 blocks (row stride 17 elements, so the 16 rows
// of a column fall into distinct banks) and every dense block product runs on
// the matrix cores:
//   float64: v_mfma_f64_16x16x4f64, lane l holds A[l%16][l/16], B[l/16][l%16]
//            of a 4-wide slice, D[l/16 + 4s][l%16] in accumulator slot s;
//   float32: v_mfma_f32_16x16x4f32, same A/B lanes, D[4(l/16) + s][l%16].
#pragma once
#include <hip/hip_runtime.h>
#include "sl_internal.hpp"

namespace sl {
namespace blk {

constexpr int BS = 17;            // row stride of a stored block (elements)
constexpr int BLK = 16 * BS;      // elements per stored block
constexpr int kThreads = 256;     // four wavefronts per fit

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int tid() { return threadIdx.x; }
__device__ __forceinline__ int lane() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave() { return threadIdx.x >> 6; }

__device__ __forceinline__ void block_sync() { __syncthreads(); }
// Orders this wavefront's LDS accesses (LDS executes a wavefront's requests in order).
__device__ __forceinline__ void wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <typename T>
struct Mma;

template <>
struct Mma<double> {
  typedef d4 acc_t;
  __device__ static __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int l, int s) { return (l >> 4) + 4 * s; }
};

template <>
struct Mma<float> {
  typedef f4 acc_t;
  __device__ static __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int l, int s) { return 4 * (l >> 4) + s; }
};

template <typename T>
__device__ __forceinline__ typename Mma<T>::acc_t zacc() {
  typename Mma<T>::acc_t r = {0, 0, 0, 0};
  return r;
}

// A-operand (or B^T) read of X[l%16][4kk + l/16]
template <typename T>
__device__ __forceinline__ T rowpat(const T* X, int kk) {
  const int l = lane();
  return X[(l & 15) * BS + 4 * kk + (l >> 4)];
}
// B-operand (or A^T) read of X[4kk + l/16][l%16]
template <typename T>
__device__ __forceinline__ T colpat(const T* X, int kk) {
  const int l = lane();
  return X[(4 * kk + (l >> 4)) * BS + (l & 15)];
}
template <typename T>
__device__ __forceinline__ typename Mma<T>::acc_t load_acc(const T* X) {
  const int l = lane();
  typename Mma<T>::acc_t r;
#pragma unroll
  for (int s = 0; s < 4; ++s) r[s] = X[Mma<T>::row(l, s) * BS + (l & 15)];
  return r;
}
template <typename T>
__device__ __forceinline__ void store_acc(T* X, typename Mma<T>::acc_t r) {
  const int l = lane();
#pragma unroll
  for (int s = 0; s < 4; ++s) X[Mma<T>::row(l, s) * BS + (l & 15)] = r[s];
}
// Store the transpose of an accumulator block.
template <typename T>
__device__ __forceinline__ void store_acc_t(T* X, typename Mma<T>::acc_t r) {
  const int l = lane();
#pragma unroll
  for (int s = 0; s < 4; ++s) X[(l & 15) * BS + Mma<T>::row(l, s)] = r[s];
}

__device__ __forceinline__ constexpr int tblk(int I, int J) { return I * (I + 1) / 2 + J; }

// Broadcast lane src's value to the wavefront (src wave-uniform, a constant after unrolling).
__device__ __forceinline__ double bcast(double x, int src) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_readlane(lo, src);
  hi = __builtin_amdgcn_readlane(hi, src);
  return __hiloint2double(hi, lo);
}

// 1/sqrt(d) to float64 accuracy: the hardware estimate refined by two Newton
// steps (each doubles the correct bits), shorter on the factorisation's critical
// path than a correctly rounded square root followed by a division.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double r = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double e = fma(-d, r * r, 1.0);
    r = fma(0.5 * r, e, r);
  }
  return r;
}

// Cholesky of one 16x16 diagonal block (first m rows live, padding -> identity);
// the block is overwritten with the inverse of its factor, which is all the
// panel update and the triangular solves need.  Executed by one wavefront.
// Lanes 0..15 own a row each in registers; columns travel between lanes with
// readlane broadcasts (no LDS round trips inside the factorisation).
template <typename T>
__device__ __forceinline__ void factor_diag(T* D, int m) {
  const int l = lane();
  const int r = l & 15;
  double row[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) row[c] = (c <= r) ? (double)D[r * BS + c] : 0.0;
  double dinv[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double djj = bcast(row[j], j);
    const double inv = (j < m) ? rsqrt_nr(djj) : 1.0;
    const double ljj = (j < m) ? djj * inv : 1.0;
    dinv[j] = inv;
    double lrj;
    if (r == j) lrj = ljj;
    else if (r > j) lrj = (j < m && r < m) ? row[j] * inv : 0.0;
    else lrj = 0.0;
    row[j] = lrj;
#pragma unroll
    for (int c = j + 1; c < 16; ++c) {
      const double lcj = bcast(lrj, c);
      if (r >= c) row[c] -= lrj * lcj;
    }
  }
  // inverse: lane r solves L x = e_r (column r of L^-1); L[i][k] = readlane(row[k], i)
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    double acc = (i == r) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) acc -= bcast(row[k], i) * x[k];
    x[i] = acc * dinv[i];
  }
  if (l < 16) {
#pragma unroll
    for (int i = 0; i < 16; ++i) D[i * BS + r] = (T)x[i];
  }
  wave_sync();
}

// Blocked right-looking Cholesky of a packed lower block matrix (NB x NB blocks,
// live size n).  Off-diagonal blocks end up holding L, diagonal blocks the
// inverses of L's diagonal blocks.  Whole workgroup; diagonal blocks on
// wavefront 0, panel and trailing blocks spread over the four wavefronts.
template <typename T, int NB>
__device__ __forceinline__ void cholesky(T* G, int n) {
  const int w = wave();
#pragma unroll 1
  for (int kb = 0; kb < NB; ++kb) {
    if (w == 0) {
      const int m = n - 16 * kb < 16 ? n - 16 * kb : 16;
      factor_diag<T>(G + tblk(kb, kb) * BLK, m);
    }
    block_sync();
    const T* Li = G + tblk(kb, kb) * BLK;
#pragma unroll 1
    for (int I = kb + 1 + w; I < NB; I += 4) {
      T* P = G + tblk(I, kb) * BLK;
      typename Mma<T>::acc_t acc = zacc<T>();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = Mma<T>::mma(rowpat(P, kk), rowpat(Li, kk), acc);
      wave_sync();
      store_acc(P, acc);
    }
    block_sync();
    int t = 0;
#pragma unroll 1
    for (int J = kb + 1; J < NB; ++J) {
#pragma unroll 1
      for (int I = J; I < NB; ++I, ++t) {
        if ((t & 3) != w) continue;
        const T* LI = G + tblk(I, kb) * BLK;
        const T* LJ = G + tblk(J, kb) * BLK;
        T* D = G + tblk(I, J) * BLK;
        typename Mma<T>::acc_t acc = load_acc(D);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = Mma<T>::mma(-rowpat(LI, kk), rowpat(LJ, kk), acc);
        store_acc(D, acc);
      }
    }
    block_sync();
  }
}

// Triangular solves with the blocked factor, executed by wavefront 0 (the
// caller brackets them with block_sync).  v: float64 vector of 16*NB entries in
// LDS.  Lanes 0..15 own one row of the current block each.
template <typename T, int NB>
__device__ __forceinline__ void forward_solve(const T* G, double* v) {
  const int l = lane(), r = l & 15;
#pragma unroll 1
  for (int kb = 0; kb < NB; ++kb) {
    double t = v[16 * kb + r];
    for (int J = 0; J < kb; ++J) {
      const T* LB = G + tblk(kb, J) * BLK;
#pragma unroll
      for (int c = 0; c < 16; ++c) t -= (double)LB[r * BS + c] * v[16 * J + c];
    }
    const T* Li = G + tblk(kb, kb) * BLK;
    double y = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) y += (double)Li[r * BS + c] * bcast(t, c);
    if (l < 16) v[16 * kb + r] = y;
    wave_sync();
  }
}

template <typename T, int NB>
__device__ __forceinline__ void backward_solve(const T* G, double* v) {
  const int l = lane(), r = l & 15;
#pragma unroll 1
  for (int kb = NB - 1; kb >= 0; --kb) {
    double t = v[16 * kb + r];
    for (int J = kb + 1; J < NB; ++J) {
      const T* LB = G + tblk(J, kb) * BLK;
#pragma unroll
      for (int c = 0; c < 16; ++c) t -= (double)LB[c * BS + r] * v[16 * J + c];
    }
    const T* Li = G + tblk(kb, kb) * BLK;
    double x = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) x += (double)Li[c * BS + r] * bcast(t, c);
    if (l < 16) v[16 * kb + r] = x;
    wave_sync();
  }
}

}  // namespace blk
}  // namespace sl
