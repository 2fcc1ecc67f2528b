// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace sl {

// Per-handle diagnostics are spread over this many counter slots (by
// workgroup) so that the per-fit atomics of a launch do not all meet at one
// address.  Slot layout (kStatStride words):
//   [0], [1] phase 1: solver iterations summed over fits, fits that hit max_iter
//   [2], [3] phase 2: the same
//   [4] moved nodes that left their element's reference interval [0, 1]
//   [5] largest relative solver residual left by a fit (bits of a non-negative
//       double, so unsigned comparison orders them; NaN sorts above every value)
//   [6] phase-1 fits (per component) whose fixed-point iteration turned to
//       conjugate gradients
constexpr int kStatSlots = 64;
constexpr int kStatStride = 8;
constexpr int kStatEscapes = 4;
constexpr int kStatResidual = 5;
constexpr int kStatFallbacks = 6;

#if defined(__HIPCC__)
__device__ __forceinline__ unsigned long long* stat_slot(unsigned long long* stats) {
  return stats + kStatStride * (blockIdx.x & (kStatSlots - 1));
}
// Add v to counter idx of this workgroup's slot (nothing when v is 0).
__device__ __forceinline__ void stat_add(unsigned long long* stats, int idx, unsigned long long v) {
  if (stats && v) atomicAdd(stat_slot(stats) + idx, v);
}
// Raise the recorded largest residual to r (r >= 0 or NaN).
__device__ __forceinline__ void stat_residual(unsigned long long* stats, double r) {
  if (stats && !(r <= 0.0)) atomicMax(stat_slot(stats) + kStatResidual, (unsigned long long)__double_as_longlong(r));
}
// 1 when a moved reference coordinate lies outside [0, 1].
__device__ __forceinline__ int escaped(double x) { return (x < 0.0 || x > 1.0) ? 1 : 0; }
#endif

constexpr int kMaxN = 16;        // largest nodes per direction supported
constexpr int kMaxAttempts = 64; // polar-method retries before z = 0

// Orthonormal shifted Legendre recurrence on [0, 1]:
//   psi_0 = 1, psi_{k+1}(t) = a_k (2t - 1) psi_k(t) - b_k psi_{k-1}(t),
//   a_k = sqrt((2k+3)(2k+1))/(k+1), b_k = k sqrt(2k+3)/((k+1) sqrt(2k-1)).
struct LegendreRec {
  double a[kMaxN];
  double b[kMaxN];
};

// The same coefficients as compile-time constants, rounded as the host forms
// them (each square root, product and quotient rounded to nearest in turn);
// handle creation checks that the two agree bit for bit.  Kernels that use
// these hold no coefficient in registers: a constant is rematerialised where
// it is needed.
constexpr double kLegA[kMaxN] = {
    0x1.bb67ae8584caap+0, 0x1.efbdeb14f4edap+0, 0x1.f8d6bc21a583cp+0, 0x1.fbfbf7ebc755fp+0,
    0x1.fd6efe4c9b8a5p+0, 0x1.fe3818941c35bp+0, 0x1.feb1347fa3e26p+0, 0x1.feffbfdfebf1fp+0,
    0x1.ff359273d543bp+0, 0x1.ff5c0eb678cbep+0, 0x1.ff78866842d89p+0, 0x1.ff8e2c3c65c25p+0,
    0x1.ff9f0472ace9ep+0, 0x1.ffac61a95fbd2p+0, 0x1.ffb72977c57adp+0, 0x1.ffbffbff7fec0p+0};
constexpr double kLegB[kMaxN] = {
    0x0.0p+0,             0x1.1e3779b97f4a8p+0, 0x1.04b298812c5ccp+0, 0x1.019853f3bf5cap+0,
    0x1.00bafa9e8fc3dp+0, 0x1.00650ed19a3c0p+0, 0x1.003cc41178a0fp+0, 0x1.00275f6f0badep+0,
    0x1.001af6c8b98f3p+0, 0x1.001345bff6204p+0, 0x1.000e40691ddabp+0, 0x1.000ad5c8026d6p+0,
    0x1.00086dfae5feep+0, 0x1.0006afdf9c67ap+0, 0x1.000564c8b46bap+0, 0x1.000469e49acd9p+0};

// Tables of one order for the null-space form of the 2-D constrained remap
// (reference-preconditioned solver), in doubles from the order's offset:
//   [0, N)          barycentric weights 1 / prod_{b != a} (xi_a - xi_b);
//   then N x N      psi_k(xi_a) at [a N + k] (orthonormal shifted Legendre);
//   then 1          the squared mean nodal value of the bubble functions,
//                   ((1/m) sum_{a, k < m} (xi_a (1 - xi_a) psi_k(xi_a))^2)^2, m = N - 2
//                   (the scale of the remap's stopping test);
//   then N, N       l0, l1: the Lagrange weights of the Gauss abscissae at 0 and at 1
//                   (the value at an edge's ends of the polynomial through its data);
//   then 4 x 4      (C^T C)^-1, C the four corner-consistency rows over the edge
//                   points (SW: l0 on W minus l0 on S; NW: l1 on W minus l0 on N;
//                   SE: l0 on E minus l1 on S; NE: l1 on E minus l1 on N), whose null
//                   space is the edge values of Q_{N-1}: the orthogonal projector onto
//                   them is I - C (C^T C)^-1 C^T;
//   then 3          l0.l0, l0.l1, l1.l1.
constexpr int nsp_bary(int N) { return 0; }
constexpr int nsp_vx(int N) { return N; }
constexpr int nsp_zz(int N) { return nsp_vx(N) + N * N; }
constexpr int nsp_ends(int N) { return nsp_zz(N) + 1; }
constexpr int nsp_cinv(int N) { return nsp_ends(N) + 2 * N; }
constexpr int nsp_ll(int N) { return nsp_cinv(N) + 16; }
constexpr int nsp_doubles(int N) { return nsp_ll(N) + 3; }

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
  int algo;              // 0: nodal (Lagrange) form, 1: Legendre normal equations
  int ncomp;             // components: row r of the state draws the increments of sample r / ncomp
  int64_t M;             // rows of K*N values (samples x components)
  int64_t step0;         // Philox step counter of the first step
  uint64_t seed;
  uint32_t stream;
  unsigned long long* stats;   // diagnostics slots (kStatSlots x kStatStride), or null
  int mass;              // 1: the fit also keeps the element integral of p0
  LegendreRec rec;
  double xi[kMaxN];      // reference nodes
  double wq[kMaxN];      // quadrature weights of the reference nodes (element integrals)
};

// Step inputs of one order group for the 2-D phase kernels.
// What a reference-solver fit needs of its element, in work-list order, so
// that a fit reaches it with one load: the element's first node and first edge
// point, per side (W, E, S, N) where the neighbour's facing trace starts in a
// state row, (order << 48) | edge offset, or -1 on a Dirichlet side, and the
// element means of the move coefficients (mean A in x, in y, mean B in x, in y).
struct WorkRec {
  int64_t noff;
  int64_t eoff;
  int64_t nbr_tr[4];
  double emean[4];
};

struct Params2D {
  const double* xi_node;   // [nodes][2] reference coordinates
  const double* A;         // [nodes][2]
  const double* B;         // [nodes][2]
  const double* src;       // [nodes]
  const double* Af;        // [edges]
  const double* Bf;        // [edges]
  const double* ghost;     // [edges]
  const int32_t* order;    // [K]
  const int64_t* noff;     // [K] first node of element e
  const int64_t* eoff;     // [K] first edge point of element e
  const int32_t* nbr;      // [K][4] neighbour across W, E, S, N (-1: Dirichlet boundary)
  const int32_t* work;     // elements of this launch (all of one order)
  const double* xi_tab;    // [(kMaxN+1)][kMaxN] reference nodes of each order
  const double* ur;        // U_r of each order, column-major (4N x (4N-4))
  const int64_t* ur_off;   // [kMaxN+1]
  const double* interp;    // Lagrange matrices between orders (Nd x Ns)
  const int64_t* interp_off;  // [(kMaxN+1)^2], index Nd*(kMaxN+1) + Ns
  double* phi;             // [samples][ncomp][nodes]
  double* tr;              // [samples][ncomp][edges]
  int64_t M, nodes, edges; // M: fits per element of one launch: samples (reference solver, which
                           // loops over the components inside a fit) or samples x ncomp (factorisation)
  int ncomp;
  int64_t block0;          // first fit of this launch within the group
  int64_t step;            // Philox step counter (used when step_ptr is null)
  const int64_t* step_ptr; // device step counter (graph replay), or null
  uint64_t seed;
  uint32_t stream;
  int refine;              // float64 refinement sweeps (mixed-precision modes)
  // reference-preconditioned solver
  const double* gxinv;     // Gx^-1, then Vx^-1, of each order (N x N each, row-major)
  int64_t gx_off[kMaxN + 1];
  const double* nsp;       // null-space tables of each order (layout: nsp_* below)
  int64_t nsp_off[kMaxN + 1];
  double tol2;             // stop when g^T g <= tol2 * x0^T x0 (g: preconditioned residual)
  int max_iter;
  unsigned long long* stats;   // diagnostics slots (kStatSlots x kStatStride, layout above)
  int mass;                // 1: the fit also keeps the element integral of p0 (not on this path)
  const double* wq_tab;    // [(kMaxN+1)][kMaxN] quadrature weights of each order's nodes
  // reference solver: this step's Wiener normals of each sample ([M][2], written
  // by the draw kernel before phase 1) and the element data of each work item
  // (indexed like work)
  const double* zdraw;
  const struct WorkRec* wrec;
  // reference solver, phase 1 of one-component fits: fits whose fixed-point
  // iteration contracts too slowly are listed and redone by a second kernel
  // that holds the full basis tables.  A per-order launch passes its group's
  // slots (fit index within the group) and its order's counter; the device
  // copy holds the handle's whole list and counters (kMaxN + 1), the slots of
  // order N starting at rescue_off[N] (fit index within the handle).  Null:
  // every fit takes the full kernel.
  uint32_t* rescue_list;
  unsigned int* rescue_count;
  int64_t rescue_off[kMaxN + 1];
  LegendreRec rec;
};

// Fused persistent 2-D launch over several problems (each a device copy of its
// Params2D with work pointing at the full order-sorted work list).  Segment k
// covers work items [seg[k].start, seg[k+1].start) (the last one up to total):
// order seg[k].N of problem seg[k].task, fit indices from seg[k].fit0 on.
constexpr int kMaxTasks = 32;
constexpr int kMaxSegs = 64;
struct FusedSeg {
  int64_t start;
  int64_t fit0;
  int32_t task;
  int32_t N;
};
struct Fused2DArgs {
  const Params2D* task[kMaxTasks];
  FusedSeg seg[kMaxSegs];
  int nseg;
  int64_t total;
  unsigned long long* counter;
  int chunk;   // items a workgroup of a persistent reference-solver kernel claims at once
};

// Device step and work counters of up to kMaxTasks problems.
// One step's Wiener normals of up to kMaxTasks 2-D problems (eq. def_dx: one
// pair a sample and step): pair s of problem t goes to z[t][2s], z[t][2s+1].
// The step is *step_ptr[t] when that is set (graph replay), else step[t].
struct DrawArgs {
  double* z[kMaxTasks];
  unsigned int* rescue_count[kMaxTasks];   // kMaxN + 1 counters each, cleared (or null)
  const int64_t* step_ptr[kMaxTasks];
  int64_t step[kMaxTasks];
  int64_t M[kMaxTasks];
  uint64_t seed[kMaxTasks];
  uint32_t stream[kMaxTasks];
  int n;
};

// Work counters of a problem's persistent launches: index 2 N + (phase - 1)
// (the reference solver, one launch per order N; the factorisation kernels'
// single launch uses N = 0).
constexpr int kWorkCounters = 2 * (kMaxN + 1);

struct StepArgs {
  int64_t* step[kMaxTasks];
  unsigned long long* counter[kMaxTasks];   // kWorkCounters per problem
  int64_t value[kMaxTasks];
  int n;
  int set;
};

// Batched 1-D resident launch: problems of one order and form; workgroups
// [bstart[t], bstart[t+1]) belong to problem t.
struct Batch1DArgs {
  const Params1D* task[kMaxTasks];
  int64_t bstart[kMaxTasks + 1];
  int64_t step0[kMaxTasks];
  int ntasks;
  int nsteps;
};

// Shared-geometry 2-D step (constant drift, diffusion and source factor, one
// order): per-sample operators, then batched products over the elements.
struct SharedArgs {
  const double* A;       // [nodes][2]: the first node's values are every node's
  const double* B;       // [nodes][2]
  double src;            // 1 - dt div u, the same at every node
  const double* Af;      // [edges]
  const double* Bf;      // [edges]
  const double* ghost;   // [edges]
  const int32_t* nbr;    // [K][4]
  const double* xi;      // [N] reference nodes
  const double* bw;      // [N] barycentric weights of the reference nodes
  const double* ur;      // U_r, column-major 4N x (4N - 4)
  double* ops;           // [M][shared_op_doubles(N)] per-sample operators
  double* phi;           // [M][ncomp][K n]
  double* tr;            // [M][ncomp][K 4N]
  int64_t K;
  int ncomp;             // row r of phi / tr uses the operators of sample r / ncomp
  int mass;              // 1: the remap also keeps each element's integral of p0
  const double* wq;      // [N] quadrature weights of the reference nodes
  int64_t step;
  const int64_t* step_ptr;
  uint64_t seed;
  uint32_t stream;
};
constexpr int kMaxNShared = 12;   // largest order of the shared-geometry path
size_t shared_op_doubles(int N);
// stage 0: per-sample operators; 1: traces; 2: update of the samples
hipError_t launch_shared_step(int N, int stage, const SharedArgs& a, int64_t M, hipStream_t st);

// Host launchers (defined in the .hip files).
hipError_t launch_fit2d(int phase, int N, int mode, const Params2D& p, int64_t nfits, hipStream_t st);
size_t fit2d_lds_bytes(int N, int mode, int phase);
hipError_t launch_fit2d_fused(int phase, int mode, const Fused2DArgs& a, int grid, size_t lds, hipStream_t st);
int fit2d_fused_occupancy(int phase, int mode, size_t lds);
hipError_t launch_step_counters(const StepArgs& a, hipStream_t st);
hipError_t launch_draw_normals(const DrawArgs& a, int64_t maxM, hipStream_t st);
hipError_t launch_fit2r(int phase, int N, const Params2D& p, int64_t nfits, hipStream_t st, bool wide);
// reference solver, persistent form: the fits of order N of the segments in a,
// grid workgroups (0: as many as are resident at once on `cus` compute units)
// pulling them from a.counter; after a FAST phase 1 also the redo kernel
hipError_t launch_fit2r_persist(int phase, int N, const Fused2DArgs& a, bool fast, int grid, int cus, hipStream_t st);
// fast: every problem of the table has one component and no mass constraint
// (the lean phase-1 kernel with its redo pass; the phase-2 kernel without the
// general form).
hipError_t launch_fit2r_multi(int phase, int N, const Fused2DArgs& a, bool fast, hipStream_t st);
constexpr int kMaxNRef = 16;  // largest order of the reference-preconditioned 2-D solver
constexpr int kMaxN2D = 10;   // largest order of the 2-D LDS-resident fit
hipError_t launch_resident_1d(int N, const Params1D& p, hipStream_t st);
hipError_t launch_tiled_1d(int N, const Params1D& p, const double* in, double* out, int64_t step, hipStream_t st);
int tiled_1d_tiles(int K);
hipError_t launch_resident_1d_batch(int N, int algo, const Batch1DArgs& a, size_t lds, hipStream_t st);
size_t resident_1d_lds_bytes(int K, int samples_per_block);
int resident_1d_samples_per_block(int K);

// Sample mean (two passes, fixed order).  part: partial sums, at least
// mean_chunks(M, nodes) * nodes doubles when that is above 1 (else unused);
// nonfinite (may be null): cleared, then receives the count of non-finite values read.
constexpr int64_t kMeanScratchDoubles = (int64_t)1 << 19;   // bound on the partial sums (4 MiB)
int64_t mean_chunks(int64_t M, int64_t nodes);
hipError_t launch_mean(const double* phi, double* out, double* part, int64_t M, int64_t nodes,
                       unsigned long long* nonfinite, hipStream_t st);
// Device address of this device's allocation-free mean scratch (kMeanScratchDoubles doubles).
hipError_t mean_scratch_device_ptr(double** out);
hipError_t launch_broadcast(double* phi, const double* phi0, int64_t M, int64_t nodes, hipStream_t st);
// Per-node histogram of the samples into counts[nodes][nbins + 2] (cleared first).
constexpr int kPdfMaxBins = 254;
size_t pdf_lds_bytes(int nbins);
hipError_t launch_pdf(const double* phi, uint32_t* counts, int64_t M, int64_t nodes, double lo, double hi,
                      int nbins, hipStream_t st);
hipError_t launch_debug_normals(double* out, uint64_t seed, uint32_t stream, int64_t step,
                                int64_t s0, int64_t ns, hipStream_t st);
hipError_t launch_debug_positions(double* out, const double* xi_node, const double* A, const double* B,
                                  int dim, int64_t nodes, int64_t M, uint64_t seed, uint32_t stream,
                                  int64_t step, hipStream_t st);

}  // namespace sl
