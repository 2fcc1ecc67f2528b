// Sample mean, broadcast of the initial field and the test-aid kernels.
#include "sl_internal.hpp"
#include "philox.hpp"

namespace sl {

// Mean over samples at every node (eq. averaged).  A 256-lane workgroup owns
// 64 consecutive nodes; its 4 wavefronts sum the samples s = w, w+4, ... in
// order (coalesced 512-byte rows per wavefront), then wavefront 0 adds the
// four partial sums in fixed order and divides by M.  The result does not
// depend on the launch, so repeated calls are bitwise identical.
constexpr int kMeanNodes = 64;
constexpr int kMeanWaves = 4;

__global__ __launch_bounds__(kMeanNodes * kMeanWaves) void mean_kernel(const double* __restrict__ phi,
                                                                       double* __restrict__ out, int64_t M,
                                                                       int64_t nodes) {
  __shared__ double part[kMeanWaves][kMeanNodes];
  const int l = threadIdx.x % kMeanNodes;
  const int w = threadIdx.x / kMeanNodes;
  const int64_t node = (int64_t)blockIdx.x * kMeanNodes + l;
  double acc = 0.0;
  if (node < nodes) {
    for (int64_t s = w; s < M; s += kMeanWaves) acc += phi[s * nodes + node];
  }
  part[w][l] = acc;
  __syncthreads();
  if (w == 0 && node < nodes) {
    double t = part[0][l];
#pragma unroll
    for (int k = 1; k < kMeanWaves; ++k) t += part[k][l];
    out[node] = t / (double)M;
  }
}

hipError_t launch_mean(const double* phi, double* out, int64_t M, int64_t nodes, hipStream_t st) {
  const int64_t blocks = (nodes + kMeanNodes - 1) / kMeanNodes;
  hipLaunchKernelGGL(mean_kernel, dim3((unsigned)blocks), dim3(kMeanNodes * kMeanWaves), 0, st, phi, out, M,
                     nodes);
  return hipGetLastError();
}

__global__ void broadcast_kernel(double* __restrict__ phi, const double* __restrict__ phi0, int64_t total,
                                 int64_t nodes) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    phi[i] = phi0[i % nodes];
}

hipError_t launch_broadcast(double* phi, const double* phi0, int64_t M, int64_t nodes, hipStream_t st) {
  const int64_t total = M * nodes;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(broadcast_kernel, dim3((unsigned)blocks), dim3(256), 0, st, phi, phi0, total, nodes);
  return hipGetLastError();
}

__global__ void debug_normals_kernel(double* out, uint64_t seed, uint32_t stream, int64_t step, int64_t s0,
                                     int64_t ns) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) {
    const Normal2 z = normal_pair(seed, stream, (uint64_t)step, (uint64_t)(s0 + i));
    out[2 * i] = z.a;
    out[2 * i + 1] = z.b;
  }
}

hipError_t launch_debug_normals(double* out, uint64_t seed, uint32_t stream, int64_t step, int64_t s0,
                                int64_t ns, hipStream_t st) {
  const int64_t blocks = (ns + 255) / 256;
  hipLaunchKernelGGL(debug_normals_kernel, dim3((unsigned)blocks), dim3(256), 0, st, out, seed, stream, step,
                     s0, ns);
  return hipGetLastError();
}

// Moved reference coordinates with exactly the operations of the step kernels.
__global__ void debug_positions_kernel(double* out, const double* xi_node, const double* A, const double* B,
                                       int dim, int64_t nodes, int64_t M, uint64_t seed, uint32_t stream,
                                       int64_t step) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * nodes) return;
  const int64_t s = i / nodes, node = i - s * nodes;
  const Normal2 z = normal_pair(seed, stream, (uint64_t)step, (uint64_t)s);
  for (int j = 0; j < dim; ++j) {
    const double zj = j == 0 ? z.a : z.b;
    const int64_t k = node * dim + j;
    out[i * dim + j] = moved_coord(xi_node[k], A[k], B[k], zj);
  }
}

hipError_t launch_debug_positions(double* out, const double* xi_node, const double* A, const double* B, int dim,
                                  int64_t nodes, int64_t M, uint64_t seed, uint32_t stream, int64_t step,
                                  hipStream_t st) {
  const int64_t blocks = (M * nodes + 255) / 256;
  hipLaunchKernelGGL(debug_positions_kernel, dim3((unsigned)blocks), dim3(256), 0, st, out, xi_node, A, B, dim,
                     nodes, M, seed, stream, step);
  return hipGetLastError();
}

}  // namespace sl
