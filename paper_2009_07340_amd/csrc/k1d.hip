// One-dimensional resident step kernel.
//
// Samples never interact (Sec. 5: every Monte-Carlo sample is an independent
// polynomial field), and a 1-D sample of K <= 256 elements is small (K*N
// doubles), so one workgroup owns whole samples for all nsteps steps: each
// lane holds one element's N node values in registers, the element traces are
// exchanged through LDS (one barrier per step, double-buffered), and HBM is
// touched only to load the samples at the start and store them at the end.
//
// Lane l of a 256-lane workgroup works on element e = l % K of sample slot
// l / K; a workgroup carries floor(256 / K) samples.
#include "sl_internal.hpp"
#include "philox.hpp"
#include "fit1d.hpp"

namespace sl {

constexpr int kResidentThreads = 256;

int resident_1d_samples_per_block(int K) { return K <= kResidentThreads ? kResidentThreads / K : 0; }

size_t resident_1d_lds_bytes(int K, int spb) { return sizeof(double) * 2 * 2 * (size_t)spb * K; }

// The Wiener increment of a (sample, step) is the same for every element of
// the sample, so it is drawn once, not once per lane: every P = 256 / spb
// steps the 256 lanes draw the increments of the next P steps of the spb
// samples (lane l: sample slot l / P, step l % P ahead) into zbuf.
// From order 9 to 13 the registers hold two wavefronts a SIMD and the LDS has
// room to stage A and B of the workgroup's elements once, [i][e]
// (lanes read consecutive words): the moves at the top of every step then wait
// on LDS, not on the cache.
template <int N, bool kNodal>
constexpr bool resident_stages_ab() { return kNodal && N >= 9 && N <= 13; }

// MASS: the fit also keeps the element integral of p0 (a third constraint row;
// N = 2 has no room for it: the boundary values fix the linear polynomial).
template <int N, bool kNodal, bool MASS0>
__device__ __forceinline__ void resident_1d_body(const Params1D& p, double* lds_tr, double* zbuf, double* abl,
                                                 int64_t block, int64_t step0, int nsteps) {
  constexpr bool MASS = MASS0 && N >= 3;
  const int K = p.K;
  const int spb = p.samples_per_block;
  const int lane = threadIdx.x;
  const int slot = lane / K;
  const int e = lane - slot * K;
  const int64_t s = block * spb + slot;
  const bool active = slot < spb && s < p.M;
  const int64_t base = s * (int64_t)(K * N) + (int64_t)e * N;

  // A, B and src are shared by all samples and re-read every step (cache hits)
  const double* A = p.A + e * N;
  const double* B = p.B + e * N;
  const double* src = p.src + e * N;
  if constexpr (resident_stages_ab<N, kNodal>()) {
    for (int x = lane; x < K * N; x += kResidentThreads) {
      const int ex = x / N, ix = x - ex * N;
      abl[ix * K + ex] = p.A[x];
      abl[(N + ix) * K + ex] = p.B[x];
    }
    __syncthreads();
  }
  double phi[N];
  // orders 9-12: the source factors stay in registers across the steps (the
  // registers still admit two wavefronts a SIMD); otherwise re-read each step
  constexpr bool kSrcReg = kNodal && N >= 9 && N <= 12;
  double srcv[N];
  double Af0 = 0, Af1 = 0, Bf0 = 0, Bf1 = 0, ghL = 0, ghR = 0;
  if constexpr (kSrcReg) {
#pragma unroll
    for (int i = 0; i < N; ++i) srcv[i] = active ? src[i] : 0.0;
  }
  if (active) {
#pragma unroll
    for (int i = 0; i < N; ++i) phi[i] = p.phi[base + i];
    Af0 = p.Af[2 * e];
    Af1 = p.Af[2 * e + 1];
    Bf0 = p.Bf[2 * e];
    Bf1 = p.Bf[2 * e + 1];
    if (p.dirichlet) {
      ghL = p.ghost[2 * e];
      ghR = p.ghost[2 * e + 1];
    }
  }
  const int stride = spb * K * 2;
  const int P = kResidentThreads / spb;
  int esc = 0;   // moved nodes outside [0, 1] over the launch (diagnostics)
  for (int it = 0; it < nsteps; ++it) {
    double* tr = lds_tr + (it & 1) * stride;
    Fit1DPre<N> pre;          // normal-equation form
    Fit1DNodal<N> nod;        // nodal form
    double z = 0.0, tL = 0.0, tR = 0.0;
    if (it % P == 0) {
      const int zs = lane / P, zk = lane - zs * P;
      const int64_t sz = block * spb + zs;
      if (zs < spb && sz < p.M && it + zk < nsteps)
        zbuf[lane] = normal_pair(p.seed, p.stream, (uint64_t)(step0 + it + zk), (uint64_t)(sz / p.ncomp)).a;
      __syncthreads();
    }
    if (active) {
      z = zbuf[slot * P + it % P];
      if constexpr (kNodal) {
        if constexpr (resident_stages_ab<N, kNodal>()) {
#pragma unroll
          for (int i = 0; i < N; ++i) nod.xs[i] = moved_coord(p.xi[i], abl[i * K + e], abl[(N + i) * K + e], z);
        } else {
          move_nodes<N>(p.xi, A, B, z, nod.xs);
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
          nod.a[i] = phi[i] * (kSrcReg ? srcv[i] : src[i]);
          esc += escaped(nod.xs[i]);
        }
        fit1d_nodal_pre<N, MASS>(nod, p.xi, p.wq);
        tL = nod.tL;
        tR = nod.tR;
      } else {
        double xs[N], f[N];
        move_nodes<N>(p.xi, A, B, z, xs);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          f[i] = phi[i] * src[i];
          esc += escaped(xs[i]);
        }
        fit1d_pre<N, MASS>(xs, f, p.xi, p.rec, pre, p.wq);
        tL = pre.tL;
        tR = pre.tR;
      }
      tr[(slot * K + e) * 2 + 0] = tL;
      tr[(slot * K + e) * 2 + 1] = tR;
    }
    __syncthreads();
    if (active) {
      // upwind (eq. bnd_update): disp > 0 takes the negative-side element
      const double dL = edge_disp(Af0, Bf0, z);
      const double dR = edge_disp(Af1, Bf1, z);
      double nbL, nbR;
      if (e > 0) nbL = tr[(slot * K + e - 1) * 2 + 1];
      else nbL = p.dirichlet ? ghL : tr[(slot * K + K - 1) * 2 + 1];
      if (e < K - 1) nbR = tr[(slot * K + e + 1) * 2 + 0];
      else nbR = p.dirichlet ? ghR : tr[(slot * K) * 2 + 0];
      const double gL = (dL > 0.0) ? nbL : tL;
      const double gR = (dR > 0.0) ? tR : nbR;
      if constexpr (kNodal) fit1d_nodal_post<N, MASS>(nod, p.xi, gL, gR, phi);
      else fit1d_post<N, MASS>(pre, gL, gR, phi);
    }
  }
  if (active) {
#pragma unroll
    for (int i = 0; i < N; ++i) p.phi[base + i] = phi[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) esc += __shfl_xor(esc, o, 64);
  if ((lane & 63) == 0) stat_add(p.stats, kStatEscapes, (unsigned long long)esc);
}

template <int N, bool kNodal, bool MASS>
__global__ __launch_bounds__(kResidentThreads) void resident_1d_kernel(Params1D p) {
  extern __shared__ double lds_tr[];   // [2 buffers][spb][K][2]
  __shared__ double zbuf[kResidentThreads];
  __shared__ double abl[resident_stages_ab<N, kNodal>() ? 2 * N * kResidentThreads : 1];
  resident_1d_body<N, kNodal, MASS>(p, lds_tr, zbuf, abl, blockIdx.x, p.step0, p.nsteps);
}

// Several problems of one order in one launch; workgroup ranges per problem.
template <int N, bool kNodal, bool MASS>
__global__ __launch_bounds__(kResidentThreads) void resident_1d_batch_kernel(Batch1DArgs a) {
  extern __shared__ double lds_tr[];
  __shared__ double zbuf[kResidentThreads];
  __shared__ double abl[resident_stages_ab<N, kNodal>() ? 2 * N * kResidentThreads : 1];
  const int64_t b = blockIdx.x;
  int t = 0;
  while (t + 1 < a.ntasks && b >= a.bstart[t + 1]) ++t;
  resident_1d_body<N, kNodal, MASS>(*a.task[t], lds_tr, zbuf, abl, b - a.bstart[t], a.step0[t], a.nsteps);
}

// Tiled one-dimensional step for meshes of more than 256 elements: one launch
// per step, one 256-lane workgroup per (sample, tile of 254 elements).  Lane
// 1 + i owns element e0 + i of the tile; lanes 0 and 255 recompute the fits
// of the two neighbouring elements (the halo) so that every owned element has
// both neighbour traces without a second pass.  The samples are read from
// phi_in and written to phi_out (the halo elements are read by two tiles, so
// the step cannot update in place).
constexpr int kTile1D = kResidentThreads - 2;

int tiled_1d_tiles(int K) { return (K + kTile1D - 1) / kTile1D; }

template <int N, bool kNodal, bool MASS0>
__global__ __launch_bounds__(kResidentThreads) void tiled_1d_kernel(Params1D p, const double* phi_in,
                                                                    double* phi_out, int64_t step) {
  constexpr bool MASS = MASS0 && N >= 3;
  __shared__ double trL[kResidentThreads], trR[kResidentThreads];
  const int K = p.K;
  const int tiles = (K + kTile1D - 1) / kTile1D;
  const int64_t s = blockIdx.x / tiles;
  const int tile = blockIdx.x - (int)(s * tiles);
  const int e0 = tile * kTile1D;
  const int lane = threadIdx.x;
  int e = e0 + lane - 1;                       // element of this lane (lanes 0 / 255: halo)
  const int owned_end = e0 + kTile1D < K ? e0 + kTile1D : K;
  const bool owned = lane >= 1 && e < owned_end;
  bool live = owned || lane == 0 || e == owned_end;   // own fits, left halo, right halo
  if (e < 0 || e >= K) {
    if (p.dirichlet) live = false;            // beyond the boundary: the ghost value is used
    else e = (e + K) % K;                     // periodic image
  }
  const double z = normal_pair(p.seed, p.stream, (uint64_t)step, (uint64_t)(s / p.ncomp)).a;
  Fit1DNodal<N> nod;
  Fit1DPre<N> pre;
  double tL = 0.0, tR = 0.0;
  int esc = 0;
  if (live) {
    const double* A = p.A + e * N;
    const double* B = p.B + e * N;
    const double* src = p.src + e * N;
    const double* ph = phi_in + s * (int64_t)(K * N) + (int64_t)e * N;
    if constexpr (kNodal) {
      move_nodes<N>(p.xi, A, B, z, nod.xs);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        nod.a[i] = ph[i] * src[i];
        esc += owned ? escaped(nod.xs[i]) : 0;
      }
      fit1d_nodal_pre<N, MASS>(nod, p.xi, p.wq);
      tL = nod.tL;
      tR = nod.tR;
    } else {
      double xs[N], f[N];
      move_nodes<N>(p.xi, A, B, z, xs);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        f[i] = ph[i] * src[i];
        esc += owned ? escaped(xs[i]) : 0;
      }
      fit1d_pre<N, MASS>(xs, f, p.xi, p.rec, pre, p.wq);
      tL = pre.tL;
      tR = pre.tR;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) esc += __shfl_xor(esc, o, 64);
  if ((lane & 63) == 0) stat_add(p.stats, kStatEscapes, (unsigned long long)esc);
  trL[lane] = tL;
  trR[lane] = tR;
  __syncthreads();
  if (owned) {
    const double dL = edge_disp(p.Af[2 * e], p.Bf[2 * e], z);
    const double dR = edge_disp(p.Af[2 * e + 1], p.Bf[2 * e + 1], z);
    const double nbL = (p.dirichlet && e == 0) ? p.ghost[2 * e] : trR[lane - 1];
    const double nbR = (p.dirichlet && e == K - 1) ? p.ghost[2 * e + 1] : trL[lane + 1];
    const double gL = (dL > 0.0) ? nbL : tL;
    const double gR = (dR > 0.0) ? tR : nbR;
    double phi[N];
    if constexpr (kNodal) fit1d_nodal_post<N, MASS>(nod, p.xi, gL, gR, phi);
    else fit1d_post<N, MASS>(pre, gL, gR, phi);
    double* out = phi_out + s * (int64_t)(K * N) + (int64_t)e * N;
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = phi[i];
  }
}

template <int N>
static hipError_t launch_tiled_n(const Params1D& p, const double* in, double* out, int64_t step, hipStream_t st) {
  const int64_t blocks = p.M * (int64_t)tiled_1d_tiles(p.K);
  const dim3 g((unsigned)blocks), b(kResidentThreads);
  if (p.algo == 1 && p.mass) hipLaunchKernelGGL((tiled_1d_kernel<N, false, true>), g, b, 0, st, p, in, out, step);
  else if (p.algo == 1) hipLaunchKernelGGL((tiled_1d_kernel<N, false, false>), g, b, 0, st, p, in, out, step);
  else if (p.mass) hipLaunchKernelGGL((tiled_1d_kernel<N, true, true>), g, b, 0, st, p, in, out, step);
  else hipLaunchKernelGGL((tiled_1d_kernel<N, true, false>), g, b, 0, st, p, in, out, step);
  return hipGetLastError();
}

hipError_t launch_tiled_1d(int N, const Params1D& p, const double* in, double* out, int64_t step, hipStream_t st) {
  switch (N) {
    case 2: return launch_tiled_n<2>(p, in, out, step, st);
    case 3: return launch_tiled_n<3>(p, in, out, step, st);
    case 4: return launch_tiled_n<4>(p, in, out, step, st);
    case 5: return launch_tiled_n<5>(p, in, out, step, st);
    case 6: return launch_tiled_n<6>(p, in, out, step, st);
    case 7: return launch_tiled_n<7>(p, in, out, step, st);
    case 8: return launch_tiled_n<8>(p, in, out, step, st);
    case 9: return launch_tiled_n<9>(p, in, out, step, st);
    case 10: return launch_tiled_n<10>(p, in, out, step, st);
    case 11: return launch_tiled_n<11>(p, in, out, step, st);
    case 12: return launch_tiled_n<12>(p, in, out, step, st);
    case 13: return launch_tiled_n<13>(p, in, out, step, st);
    case 14: return launch_tiled_n<14>(p, in, out, step, st);
    case 15: return launch_tiled_n<15>(p, in, out, step, st);
    case 16: return launch_tiled_n<16>(p, in, out, step, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t launch_batch_n(const Batch1DArgs& a, int algo, size_t lds, hipStream_t st) {
  const int64_t blocks = a.bstart[a.ntasks];
  const dim3 g((unsigned)blocks), b(kResidentThreads);
  const bool mass = algo >= 2;        // algo + 2: with the mass constraint
  if ((algo & 1) == 1 && mass) hipLaunchKernelGGL((resident_1d_batch_kernel<N, false, true>), g, b, lds, st, a);
  else if ((algo & 1) == 1) hipLaunchKernelGGL((resident_1d_batch_kernel<N, false, false>), g, b, lds, st, a);
  else if (mass) hipLaunchKernelGGL((resident_1d_batch_kernel<N, true, true>), g, b, lds, st, a);
  else hipLaunchKernelGGL((resident_1d_batch_kernel<N, true, false>), g, b, lds, st, a);
  return hipGetLastError();
}

hipError_t launch_resident_1d_batch(int N, int algo, const Batch1DArgs& a, size_t lds, hipStream_t st) {
  switch (N) {
    case 2: return launch_batch_n<2>(a, algo, lds, st);
    case 3: return launch_batch_n<3>(a, algo, lds, st);
    case 4: return launch_batch_n<4>(a, algo, lds, st);
    case 5: return launch_batch_n<5>(a, algo, lds, st);
    case 6: return launch_batch_n<6>(a, algo, lds, st);
    case 7: return launch_batch_n<7>(a, algo, lds, st);
    case 8: return launch_batch_n<8>(a, algo, lds, st);
    case 9: return launch_batch_n<9>(a, algo, lds, st);
    case 10: return launch_batch_n<10>(a, algo, lds, st);
    case 11: return launch_batch_n<11>(a, algo, lds, st);
    case 12: return launch_batch_n<12>(a, algo, lds, st);
    case 13: return launch_batch_n<13>(a, algo, lds, st);
    case 14: return launch_batch_n<14>(a, algo, lds, st);
    case 15: return launch_batch_n<15>(a, algo, lds, st);
    case 16: return launch_batch_n<16>(a, algo, lds, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t launch_n(const Params1D& p, hipStream_t st) {
  const int64_t blocks = (p.M + p.samples_per_block - 1) / p.samples_per_block;
  const size_t lds = resident_1d_lds_bytes(p.K, p.samples_per_block);
  const dim3 g((unsigned)blocks), b(kResidentThreads);
  if (p.algo == 1 && p.mass) hipLaunchKernelGGL((resident_1d_kernel<N, false, true>), g, b, lds, st, p);
  else if (p.algo == 1) hipLaunchKernelGGL((resident_1d_kernel<N, false, false>), g, b, lds, st, p);
  else if (p.mass) hipLaunchKernelGGL((resident_1d_kernel<N, true, true>), g, b, lds, st, p);
  else hipLaunchKernelGGL((resident_1d_kernel<N, true, false>), g, b, lds, st, p);
  return hipGetLastError();
}

hipError_t launch_resident_1d(int N, const Params1D& p, hipStream_t st) {
  switch (N) {
    case 2: return launch_n<2>(p, st);
    case 3: return launch_n<3>(p, st);
    case 4: return launch_n<4>(p, st);
    case 5: return launch_n<5>(p, st);
    case 6: return launch_n<6>(p, st);
    case 7: return launch_n<7>(p, st);
    case 8: return launch_n<8>(p, st);
    case 9: return launch_n<9>(p, st);
    case 10: return launch_n<10>(p, st);
    case 11: return launch_n<11>(p, st);
    case 12: return launch_n<12>(p, st);
    case 13: return launch_n<13>(p, st);
    case 14: return launch_n<14>(p, st);
    case 15: return launch_n<15>(p, st);
    case 16: return launch_n<16>(p, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sl
