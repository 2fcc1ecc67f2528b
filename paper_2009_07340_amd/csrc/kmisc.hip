// Sample mean, broadcast of the initial field and the test-aid kernels.
#include "sl_internal.hpp"
#include "philox.hpp"

#include <mutex>

namespace sl {

// Mean over samples at every node (eq. averaged), in two passes with a fixed
// summation order.  Pass 1: workgroup (x, c) takes 256 consecutive nodes and
// the samples of chunk c, [c*chunk, min(M, (c+1)*chunk)), and sums them in
// sample order, one node a lane (coalesced rows).  With one chunk it writes the
// mean directly; otherwise it writes the partial sum to part[c][node] and pass
// 2 adds the chunks in order and divides by M.  The chunk count depends only
// on (M, nodes) (mean_chunks), so every call with the same sizes, whichever
// entry point makes it and wherever its partial sums live, gives bitwise the
// same result.  Pass 1 also counts the non-finite values it reads.
constexpr int kMeanThreads = 256;

int64_t mean_chunks(int64_t M, int64_t nodes) {
  if (M < 1 || nodes < 1) return 1;
  const int64_t tiles = (nodes + kMeanThreads - 1) / kMeanThreads;
  int64_t C = (2048 + tiles - 1) / tiles;          // about 8 workgroups a compute unit
  C = C < M / 32 ? C : M / 32;                     // at least 32 samples a chunk (partials <= 1/32 of the state)
  const int64_t cap = kMeanScratchDoubles / nodes; // partial sums must fit the scratch bound
  C = C < cap ? C : cap;
  if (C < 1) C = 1;
  const int64_t chunk = (M + C - 1) / C;
  return (M + chunk - 1) / chunk;
}

__global__ __launch_bounds__(kMeanThreads) void mean_pass1(const double* __restrict__ phi, double* __restrict__ dst,
                                                           int64_t M, int64_t nodes, int64_t chunk, int direct,
                                                           unsigned long long* nonfinite) {
  const int64_t node = (int64_t)blockIdx.x * kMeanThreads + threadIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t s0 = c * chunk;
  const int64_t s1 = (s0 + chunk) < M ? (s0 + chunk) : M;
  double acc = 0.0;
  int bad = 0;
  if (node < nodes) {
#pragma unroll 8
    for (int64_t s = s0; s < s1; ++s) {
      const double v = phi[s * nodes + node];
      acc += v;
      bad += __builtin_isfinite(v) ? 0 : 1;
    }
    if (direct) dst[node] = acc / (double)M;
    else dst[c * nodes + node] = acc;
  }
  if (nonfinite) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
    if ((threadIdx.x & 63) == 0 && bad > 0) atomicAdd(nonfinite, (unsigned long long)bad);
  }
}

__global__ __launch_bounds__(kMeanThreads) void mean_pass2(const double* __restrict__ part, double* __restrict__ out,
                                                           int64_t M, int64_t nodes, int64_t C) {
  const int64_t node = (int64_t)blockIdx.x * kMeanThreads + threadIdx.x;
  if (node >= nodes) return;
  double acc = part[node];
  for (int64_t c = 1; c < C; ++c) acc += part[c * nodes + node];
  out[node] = acc / (double)M;
}

__global__ void clear_u64_kernel(unsigned long long* p) { *p = 0ull; }

hipError_t launch_mean(const double* phi, double* out, double* part, int64_t M, int64_t nodes,
                       unsigned long long* nonfinite, hipStream_t st) {
  if (M < 1 || nodes < 1) return hipErrorInvalidValue;
  const int64_t C = mean_chunks(M, nodes);
  if (C > 1 && !part) return hipErrorInvalidValue;
  const int64_t chunk = (M + C - 1) / C;
  const int64_t tiles = (nodes + kMeanThreads - 1) / kMeanThreads;
  if (tiles > 0x7fffffff || C > 65535) return hipErrorInvalidValue;
  if (nonfinite) {
    hipLaunchKernelGGL(clear_u64_kernel, dim3(1), dim3(1), 0, st, nonfinite);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(mean_pass1, dim3((unsigned)tiles, (unsigned)C), dim3(kMeanThreads), 0, st, phi,
                     C > 1 ? part : out, M, nodes, chunk, C > 1 ? 0 : 1, nonfinite);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || C == 1) return e;
  hipLaunchKernelGGL(mean_pass2, dim3((unsigned)tiles), dim3(kMeanThreads), 0, st, part, out, M, nodes, C);
  return hipGetLastError();
}

// Partial sums of the allocation-free mean: one array per device, reserved when
// the library is loaded and held until the process ends.  Host code never
// passes `mean_scratch` itself to a kernel (in host code the name stands for a
// host-side shadow, not a device address): it uses the device address that
// hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) double mean_scratch[kMeanScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
double* g_mean_scratch_ptr[kMaxDevices] = {nullptr};
std::mutex g_mean_scratch_mu;
}  // namespace

hipError_t mean_scratch_device_ptr(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mean_scratch_mu);
  if (!g_mean_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(mean_scratch));
    if (e != hipSuccess) return e;
    g_mean_scratch_ptr[dev] = (double*)p;
  }
  *out = g_mean_scratch_ptr[dev];
  return hipSuccess;
}

// Per-node histogram of the samples (Sec. 5.4: the PDF at each grid point by
// binning).  counts[node][nbins + 2]: column 0 values below lo, 1..nbins the
// bins of width w = (hi - lo) / nbins, nbins + 1 values at or above hi; a value
// v in [lo, hi) goes to bin floor((v - lo) / w) capped at nbins - 1 (a
// correctly rounded subtraction and division, as the oracle); non-finite values
// are skipped.  Workgroup (x, c): 64 consecutive nodes (one a lane) and the
// samples of chunk c, each of the 4 wavefronts taking every fourth sample;
// counts gather in LDS (atomic adds) and are added to the cleared output with
// integer atomics, so the result does not depend on the order.
constexpr int kPdfNodes = 64;

__global__ void clear_u32_kernel(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ __launch_bounds__(256) void pdf_kernel(const double* __restrict__ phi, uint32_t* __restrict__ counts,
                                                  int64_t M, int64_t nodes, int64_t chunk, double lo, double hi,
                                                  double w, int nbins) {
  extern __shared__ uint32_t hist[];     // [kPdfNodes][nbins + 2]
  const int cols = nbins + 2;
  for (int i = threadIdx.x; i < kPdfNodes * cols; i += 256) hist[i] = 0u;
  __syncthreads();
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t node = (int64_t)blockIdx.x * kPdfNodes + l;
  const int64_t s0 = (int64_t)blockIdx.y * chunk;
  const int64_t s1 = (s0 + chunk) < M ? (s0 + chunk) : M;
  if (node < nodes) {
    for (int64_t s = s0 + wv; s < s1; s += 4) {
      const double v = phi[s * nodes + node];
      if (!__builtin_isfinite(v)) continue;
      int col;
      if (v < lo) {
        col = 0;
      } else if (v >= hi) {
        col = nbins + 1;
      } else {
        const double q = floor((v - lo) / w);
        col = 1 + (q < (double)(nbins - 1) ? (int)q : nbins - 1);
      }
      atomicAdd(&hist[l * cols + col], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kPdfNodes * cols; i += 256) {
    const int nl = i / cols;
    const int64_t nd = (int64_t)blockIdx.x * kPdfNodes + nl;
    const uint32_t c = hist[i];
    if (nd < nodes && c) atomicAdd(&counts[nd * cols + (i - nl * cols)], c);
  }
}

size_t pdf_lds_bytes(int nbins) { return sizeof(uint32_t) * kPdfNodes * (size_t)(nbins + 2); }

hipError_t launch_pdf(const double* phi, uint32_t* counts, int64_t M, int64_t nodes, double lo, double hi,
                      int nbins, hipStream_t st) {
  const int64_t total = nodes * (int64_t)(nbins + 2);
  int64_t cb = (total + 255) / 256;
  if (cb > 65536) cb = 65536;
  hipLaunchKernelGGL(clear_u32_kernel, dim3((unsigned)cb), dim3(256), 0, st, counts, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tiles = (nodes + kPdfNodes - 1) / kPdfNodes;
  int64_t C = (2048 + tiles - 1) / tiles;          // about 8 workgroups a compute unit
  C = C < M / 64 ? C : M / 64;                     // at least 64 samples a chunk
  if (C < 1) C = 1;
  if (C > 65535) C = 65535;
  const int64_t chunk = (M + C - 1) / C;
  C = (M + chunk - 1) / chunk;
  const double w = (hi - lo) / nbins;
  hipLaunchKernelGGL(pdf_kernel, dim3((unsigned)tiles, (unsigned)C), dim3(256), pdf_lds_bytes(nbins), st, phi, counts,
                     M, nodes, chunk, lo, hi, w, nbins);
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
