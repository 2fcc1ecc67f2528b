// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace sl {

constexpr int kMaxN = 16;        // largest nodes per direction supported
constexpr int kMaxAttempts = 64; // polar-method retries before z = 0

// Orthonormal shifted Legendre recurrence on [0, 1]:
//   psi_0 = 1, psi_{k+1}(t) = a_k (2t - 1) psi_k(t) - b_k psi_{k-1}(t),
//   a_k = sqrt((2k+3)(2k+1))/(k+1), b_k = k sqrt(2k+3)/((k+1) sqrt(2k-1)).
struct LegendreRec {
  double a[kMaxN];
  double b[kMaxN];
};

// Step inputs of one handle for the 1-D resident kernel.
struct Params1D {
  const double* A;       // [K][N] (u dt)/h at the nodes
  const double* B;       // [K][N] sqrt((2 D) dt)/h
  const double* src;     // [K][N] 1 - dt div u
  const double* Af;      // [K][2] edge displacement drift part (L, R)
  const double* Bf;      // [K][2] edge displacement diffusion part
  const double* ghost;   // [K][2] Dirichlet ghost values (may be null for periodic)
  double* phi;           // [M][K*N] samples, updated in place
  int K;
  int samples_per_block;
  int dirichlet;
  int nsteps;
  int64_t M;
  int64_t step0;         // Philox step counter of the first step
  uint64_t seed;
  uint32_t stream;
  LegendreRec rec;
  double xi[kMaxN];      // reference nodes
};

// Host launchers (defined in the .hip files).
hipError_t launch_resident_1d(int N, const Params1D& p, hipStream_t st);
size_t resident_1d_lds_bytes(int K, int samples_per_block);
int resident_1d_samples_per_block(int K);

hipError_t launch_mean(const double* phi, double* out, int64_t M, int64_t nodes, hipStream_t st);
hipError_t launch_broadcast(double* phi, const double* phi0, int64_t M, int64_t nodes, hipStream_t st);
hipError_t launch_debug_normals(double* out, uint64_t seed, uint32_t stream, int64_t step,
                                int64_t s0, int64_t ns, hipStream_t st);
hipError_t launch_debug_positions(double* out, const double* xi_node, const double* A, const double* B,
                                  int dim, int64_t nodes, int64_t M, uint64_t seed, uint32_t stream,
                                  int64_t step, hipStream_t st);

}  // namespace sl
