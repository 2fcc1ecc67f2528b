/*
 * sl.h -- C ABI of the MI355X semi-Lagrangian Monte-Carlo library.
 *
 * The library advances Monte-Carlo samples of the drift-diffusion problem of
 * Natarajan, Popov & Jacobs, "A high-order semi-Lagrangian method for the
 * consistent Monte-Carlo solution of stochastic Lagrangian drift-diffusion
 * models coupled with Eulerian discontinuous spectral element method"
 * (arXiv:2009.07340):
 *
 *   dX = u(X) dt + sqrt(2 D(X)) dW                     (Sec. 2, eq. canonical_sde,
 *                                                        D = sigma^2/2, eq. fokkerplanck)
 *
 * by the semi-Lagrangian step of Sec. 5 on a box of equal affine elements with
 * N Gauss nodes per direction (Sec. 3), one polynomial field per sample:
 *   seed at the Gauss nodes (Sec. 5.1), move the nodes by one Euler-Maruyama
 *   step with one Wiener increment per sample (Sec. 5.2, eq. def_dx), carry the
 *   source along (eq. advection_phi), remap by a least-squares fit constrained
 *   by upwinded boundary values (Sec. 5.3, eqs. phi_star, remap_bnd,
 *   bnd_update) and average samples at the nodes (Sec. 5.4, eq. averaged).
 *
 * Conventions shared by every call
 * --------------------------------
 * Status: every function returns an int, 0 (SL_OK) on success or a negative
 * SL_E* code; sl_last_error() gives a message for the calling thread.  No C++
 * exception crosses this interface.  A failed call leaves the handle usable
 * unless it returns SL_EDEVICE.
 *
 * Elements: e = ey*kx + ex (x fastest).  Element e has N_e nodes per
 * direction, n_e = N_e^dim nodes; node i = iy*N_e + ix.  Reference node
 * coordinates xi are the Gauss nodes of the chosen family on [0, 1],
 * correctly rounded to float64.  Physical node coordinates:
 *   x = x0 + hx*(ex + xi_ix),  y = y0 + hy*(ey + xi_iy),  hx = (x1-x0)/kx.
 * Per-sample node arrays are ragged: element e occupies entries
 * [off_e, off_e + n_e) with off_e = sum_{e'<e} n_e'; "nodes" below is the
 * total sum_e n_e per sample.  A vector-valued field (desc.ncomp = C > 1)
 * stores C such arrays per sample, component-major: [sample][component][node];
 * the mean is [component][node] and a sample-range copy [ns][component][node].
 *
 * Edges: 1-D element e has edges L (xi = 0) and R (xi = 1), one point each;
 * 2-D element e has edges W (xi = 0), E (xi = 1), S (eta = 0), N (eta = 1),
 * each with the element's own N_e Gauss abscissae along it, so 4*N_e points,
 * stored edge-major (W points 0..N-1, then E, S, N).  "edge points" below is
 * the total per sample.  The normal component of a velocity at an edge point
 * is its x component on L/R/W/E edges and its y component on S/N edges.
 *
 * Particle positions (bit-exact contract with independent implementations):
 * with z the standard normal of the sample for the step and direction,
 *   A = (u*dt)/h,  B = sqrt((2*D)*dt)/h  (float64, in this order, host side),
 *   xi* = xi + (A + B*z)                  (three roundings, no fused ops).
 * z comes from Philox4x32-10 (Salmon et al., SC'11) with
 * counter (step n, sample s, attempt a, stream id) and key (seed lo, seed hi):
 * words r0..r3 -> k = (r0>>6)*2^26 + (r1>>6), va = (2k+1)*2^-52 - 1, vb from
 * (r2, r3) the same way; polar method: s = va*va + vb*vb (rounded products
 * and sum), accept s < 1 else a+1 (at most 64 attempts, else z = 0);
 * z_a = va*sqrt((-2*log(s))/s), z_b = vb*(same), with log computed by the
 * fixed Cody-Waite + atanh-series recipe documented in the library source.
 * One dimension uses z_a; two dimensions use (z_a, z_b) for (x, y).
 *
 * Memory: pointers named host_* or documented as host are host memory and are
 * read or written before the call returns.  Device pointers are borrowed,
 * never freed by the library.  Handles are not thread-safe: calls on one
 * handle must be serialised by the caller; distinct handles are independent.
 */
#ifndef SL_H
#define SL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SL_ABI_VERSION 3

enum sl_status {
  SL_OK = 0,
  SL_EINVAL = -1,        /* invalid argument or descriptor */
  SL_ENOMEM = -2,        /* device or host allocation failed, or workspace too small (tests can
                            force it: environment SL_FAULT=alloc fails every device allocation
                            of the library, SL_FAULT=host the handle's host allocation; a call
                            that fails this way leaves nothing allocated behind) */
  SL_EDEVICE = -3,       /* a HIP runtime call failed; the handle should be destroyed */
  SL_ENONFINITE = -4,    /* non-finite input values, or non-finite samples met by sl_mean */
  SL_ESTATE = -5,        /* call out of order (e.g. step before fields were set) */
  SL_EUNSUPPORTED = -6   /* valid request this build does not implement */
};

enum { SL_BC_PERIODIC = 0, SL_BC_DIRICHLET = 1 };
enum { SL_CONSTRAIN_BOUNDARY = 0, SL_CONSTRAIN_BOUNDARY_MASS = 1 };
enum { SL_NODES_GL = 0, SL_NODES_CG = 1 };
enum {
  SL_PREC_FP64 = 0,          /* every operation of the fit in float64 */
  SL_PREC_FP32_REFINE = 1,   /* float32 Gram / factorisation, float64 refinement */
  SL_PREC_BF16SPLIT_REFINE = 2 /* bf16 hi/lo split Gram products, float64 refinement */
};

/* Solvers of the 2-D constrained least-squares fit (Sec. 5.3); both give the
 * same remap up to rounding:
 *   SL_SOLVER_FACTOR: Gram matrix V^T V on the matrix cores, blocked Cholesky,
 *     range-space constraint elimination (N <= 10; every precision mode);
 *   SL_SOLVER_REFERENCE: preconditioners built from the undisplaced nodes
 *     (Kronecker products): the unconstrained interpolant by Richardson
 *     iteration on the square interpolation system (conjugate gradients on
 *     the normal equations when that contracts slowly), the constrained remap
 *     in null-space form (the projected boundary jump lifted by transfinite
 *     interpolation, plus conjugate gradients over the (N-2)^2 functions that
 *     vanish on the edges); float64 only; N <= 16;
 *   SL_SOLVER_AUTO: REFERENCE for SL_PREC_FP64, FACTOR for the mixed modes. */
enum { SL_SOLVER_AUTO = 0, SL_SOLVER_FACTOR = 1, SL_SOLVER_REFERENCE = 2 };

typedef struct sl_ctx* sl_handle;

/* Problem description (Sec. 3: box of K = kx*ky affine elements, N nodes
 * per direction; Sec. 5: M Monte-Carlo samples). */
typedef struct sl_mesh_desc {
  int32_t dim;            /* 1 or 2 */
  int32_t kx, ky;         /* elements per direction, >= 1 (ky ignored in 1-D) */
  double x0, x1, y0, y1;  /* box, x1 > x0 (and y1 > y0 in 2-D) */
  int32_t n_uniform;      /* N for every element when order == NULL; 2 <= N <= 16 */
  const int32_t* order;   /* optional host array of K per-element N (copied); 2-D only
                             may mix orders */
  int32_t nodes;          /* SL_NODES_GL (default) or SL_NODES_CG */
  int32_t bc;             /* SL_BC_PERIODIC or SL_BC_DIRICHLET */
  int64_t samples;        /* M >= 1 */
  uint64_t seed;          /* Philox key */
  uint32_t stream_id;     /* fourth Philox counter word (e.g. a request id) */
  int32_t precision;      /* SL_PREC_* */
  int32_t refine_iters;   /* FP64 refinement sweeps for the mixed modes; -1 = default */
  int32_t solver;         /* 2-D least-squares solver, SL_SOLVER_* (0 = automatic) */
  int32_t max_iter;       /* reference solver: iteration limit per fit, 0 = default (32) */
  double tol;             /* reference solver: stop an unconstrained fit when the error its last
                             correction leaves (estimated as that correction times r / (1 - r),
                             r the ratio of the last two corrections), or the correction itself,
                             relative to the starting iterate, is below tol, and the remap when
                             its estimated nodal error, relative to the nodal values, is below
                             tol; 0 = default (1e-13) */
  int32_t constraints;    /* SL_CONSTRAIN_BOUNDARY (0): the remap is constrained by the upwinded
                             boundary values; SL_CONSTRAIN_BOUNDARY_MASS: also by the element's
                             mass, the integral of the advected interpolant p0 over the element
                             (Introduction: a least-squares fit with boundary and mass
                             conservation constraints), so the boundary correction moves no mass
                             into or out of an element; for N = 2 the boundary values fix the
                             polynomial and the mass row is left out.  1-D, the 2-D
                             reference solver and the 2-D shared-geometry path; a 2-D step
                             with the factorisation solver returns SL_EUNSUPPORTED */
  int32_t ncomp;          /* components of a vector-valued field phi* (Sec. 5.3, last paragraph:
                             every component is defined on the same advected points), 1..64;
                             0 means 1.  Every component of a sample takes the same node moves
                             (the sample's Wiener increments) and is remapped on its own, with its
                             own boundary data; the 2-D reference solver shares each fit's
                             geometry, tables and preconditioner inverses across the components */
} sl_mesh_desc;

typedef struct sl_diag_t {
  int64_t steps;              /* Philox step counter n: steps taken since set_fields */
  int64_t samples;            /* M */
  int64_t nodes;              /* nodes per sample */
  int64_t edge_points;        /* edge points per sample */
  double max_disp_ratio;      /* for the last dt: max over nodes and directions of
                                 (|A| + |B|) / (minimum reference node spacing), the
                                 one-sigma displacement measured in node spacings
                                 (Sec. 5.2, eq. 1d_timestep); values well above 1
                                 put the scheme outside its stable range */
  int32_t precision;
  int32_t refine_iters;
  size_t device_bytes;        /* bytes of device memory the handle uses */
  int32_t solver;             /* SL_SOLVER_FACTOR or SL_SOLVER_REFERENCE (2-D) */
  int64_t solver_iterations[2];   /* reference solver, per phase: iterations summed over all fits and
                                     components so far (phase 1 counts each residual evaluation,
                                     the one that confirms a start included) */
  int64_t solver_unconverged[2];  /* reference solver, per phase: fits that stopped at max_iter */
  int64_t escapes;            /* moved nodes (per sample, step, node and direction) whose reference
                                 coordinate left [0, 1] since the handle was created: the step
                                 restriction of Sec. 5.2 (eq. 1d_timestep) keeps particles inside
                                 their element; the library allows the move (the interpolant is
                                 extrapolated, never clamped) and counts it here */
  double max_residual;        /* largest relative residual a fit's solver left since the handle was
                                 created: reference solver, the relative size its tolerance bounds
                                 at its stop (unconstrained fit: the estimated error left, or the
                                 last correction, over the starting iterate; remap: the estimated
                                 nodal error over the nodal values);
                                 factorisation solver in the mixed modes the relative size of the
                                 last float64 refinement correction, max|dc| / max|c|; 0 where
                                 neither applies (1-D, float64 factorisation); NaN if a fit met one */
  int64_t nonfinite;          /* non-finite sample values met by the last sl_mean (0: all finite) */
  int32_t ncomp;              /* components of the field */
  int64_t solver_fallbacks;   /* reference solver: unconstrained fits (per component) whose
                                 fixed-point iteration contracted by less than half a step and
                                 turned to preconditioned conjugate gradients, since the handle
                                 was created */
} sl_diag_t;

/* Device bytes sl_init_mesh needs for this description (state, traces, fields,
 * tables, scratch), for admission control.  Pure host computation. */
int sl_required_bytes(const sl_mesh_desc* desc, size_t* bytes);

/* Create a handle.  desc is validated and copied.  dev_ws: optional device
 * workspace of ws_bytes >= sl_required_bytes() bytes, caller-owned and
 * borrowed for the handle's lifetime (e.g. a torch tensor's data pointer);
 * NULL makes the library allocate.  hip_stream: the hipStream_t every
 * operation of the handle is enqueued on (NULL = the default stream).
 * Uploads the node tables; the handle then needs sl_set_fields. */
int sl_init_mesh(const sl_mesh_desc* desc, void* dev_ws, size_t ws_bytes, void* hip_stream,
                 sl_handle* out);

/* Per-sample sizes: nodes and edge points (of one component), elements, and the
 * number of components (any output pointer may be NULL). */
int sl_sizes(sl_handle h, int64_t* nodes, int64_t* edge_points, int64_t* elements, int32_t* ncomp);

/* Physical coordinates of the nodes ([nodes][dim]) and of the edge points
 * ([edge points][dim]) where the caller samples the fields.  Host buffers.
 * edge_axis (optional, [edge points]) receives 0 for points on x-normal edges
 * and 1 for y-normal edges. */
int sl_node_coords(sl_handle h, double* host_xy);
int sl_edge_coords(sl_handle h, double* host_xy, int32_t* host_edge_axis);

/* Reference nodes of order N for this handle's family (N doubles, host). */
int sl_ref_nodes(sl_handle h, int32_t N, double* host_xi);

/* Fields at the nodes and edge points (Sec. 5.1: available at the quadrature
 * points; Sec. 5.2: div u from the field solver).  Host arrays, copied:
 *   u [nodes][dim] drift; D [nodes] diffusion coefficient (>= 0);
 *   divu [nodes] physical divergence of u, NULL = 0;
 *   un [edge points] normal drift; Dn [edge points] diffusion at edge points;
 *   ghost [edge points] Dirichlet ghost values (required iff bc = DIRICHLET;
 *     only entries on the domain boundary are read);
 *   phi0 [ncomp][nodes] initial field, NULL keeps the current samples; when
 *     given, every sample is set to phi0 and the step counter to 0.
 * Values must be finite (SL_ENONFINITE otherwise). */
int sl_set_fields(sl_handle h, const double* u, const double* D, const double* divu,
                  const double* un, const double* Dn, const double* ghost, const double* phi0);

/* Replace the Dirichlet ghost values ([edge points], host, copied; only entries
 * on the domain boundary are read) for the steps enqueued after this call, for
 * boundary data that change in time (Sec. 5.3: the boundary is treated as an
 * interface with a specified ghost solution).  Waits for the handle's stream.
 * SL_EINVAL for a periodic handle, SL_ENONFINITE for non-finite values. */
int sl_set_ghost(sl_handle h, const double* ghost);

/* Advance every sample nsteps >= 0 steps of size dt > 0 (Sec. 5).  Enqueued on
 * the handle's stream; returns without waiting.  The step counter advances by
 * nsteps. */
int sl_step(sl_handle h, double dt, int32_t nsteps);

/* One batched pass (continuous batching of independent problems): advance nh
 * distinct handles by nsteps steps each, handle i with step dts[i].  Under the
 * first 2-D handle's schedule: fused = 0, the fits of one order from every
 * reference-solver handle share one launch per phase (factorisation handles
 * keep their per-order launches); fused = 1, the handles of one precision
 * mode share one persistent launch per phase (every order in one work list,
 * largest orders first).  The 1-D handles of one order and at most 256
 * elements share one resident launch; larger 1-D meshes step on their own.  Every
 * handle's result is bitwise equal to sl_step on that handle alone under the
 * same schedule (see sl_schedule_t for fused reference-solver handles).  All
 * handles must have been created on the same stream; the batch is enqueued on
 * it and replayed from a cached hipGraph when the first 2-D handle's schedule
 * asks for graphs.  nh = 0 is a no-op; a repeated handle is SL_EINVAL. */
int sl_step_batch(const sl_handle* hs, const double* dts, int32_t nh, int32_t nsteps);

/* Launch schedule of the 2-D step (Sec. 5 fixes only the result, which is the
 * same bit for bit under every schedule, with one exception: the wide fit
 * shape below orders its sums differently and agrees with the others to
 * rounding):
 *   fused = 0: one kernel per order group and phase, one workgroup per fit;
 *   fused = 1: persistent kernels, `grid` workgroups each (0 = as many as fit
 *              on the device at once) pulling fits from device work counters:
 *              factorisation solver one kernel per phase over all orders;
 *              reference solver one kernel per phase and order present, with
 *              that order's per-order fit shape and body;
 *   graph = 1: the step is captured once as a hipGraph (device step counter,
 *              counters cleared by a kernel) and replayed nsteps times;
 *   wide = 1:  fit shape of the reference solver's per-order kernels (fused = 0,
 *              a handle stepped alone): every fit of order <= 12 runs on
 *              twice the default wavefronts (orders <= 8: two instead of one;
 *              9..12: four instead of two), which shortens a fit where there are
 *              too few fits to fill the device.  The sums are ordered
 *              differently, so the result agrees with the default shape to
 *              rounding.  Other solvers, schedules and batches ignore it.
 * ms_per_step is what sl_autotune measured (0 if set by hand).  The 1-D step
 * is one resident launch for all steps whatever the schedule. */
typedef struct sl_schedule_t {
  int32_t fused;
  int32_t graph;
  int32_t grid;
  float ms_per_step;
  int32_t shared;   /* 1: the shared-geometry path (below); fused, graph, grid and wide are then unused */
  int32_t wide;     /* 1: the wide fit shape (above) */
} sl_schedule_t;

/* Shared-geometry path (schedule.shared = 1; 2-D meshes of one order N <= 12,
 * at most 65535 samples): when drift, diffusion and div u are the same at every
 * node, every element of a sample moves by the same displacement (Sec. 5.2,
 * eq. def_dx), so in the frame centred on it all elements share one
 * interpolation problem.  Per step and sample one small kernel builds the
 * remap as two operators, the interpolation Phi to the Gauss nodes and the
 * boundary correction Mg (range-space multipliers of the constrained least
 * squares, Sec. 5.3), plus the trace operator C*; the elements of the sample
 * are then advanced as dense products on the float64 matrix cores:
 * t = C* f, phi_new = Phi f + Mg (g - t) with g the upwinded traces (eq.
 * bnd_update).  The result agrees with the general path to rounding.  A step
 * on this path returns SL_EUNSUPPORTED when the mesh or the fields do not
 * qualify.  It never replaces the general path on its own. */
int sl_set_schedule(sl_handle h, const sl_schedule_t* s);
int sl_get_schedule(sl_handle h, sl_schedule_t* s);

/* Autotuner: time every candidate schedule (per-order in both fit shapes for
 * the reference solver / fused with several grid sizes, each direct and as a
 * graph) over trial_steps steps of size dt
 * and keep the fastest.  The samples and the step counter are restored
 * afterwards (a temporary device copy of the samples is allocated for that).
 * cache_path (may be NULL) names a text file of earlier choices keyed by
 * dimension, elements per order, samples and precision: a hit applies the
 * stored schedule without timing, a miss appends the new choice.  The chosen
 * schedule is returned in *out (may be NULL). */
int sl_autotune(sl_handle h, double dt, int32_t trial_steps, const char* cache_path, sl_schedule_t* out);

/* Sample mean at every node (eq. averaged): out[nodes].  out_is_device != 0:
 * out is a device pointer and the call is asynchronous on the handle's
 * stream (the count of non-finite samples it met is in sl_diag().nonfinite
 * afterwards); otherwise out is host memory, the call waits and returns
 * SL_ENONFINITE (with out written) when any sample value was not finite.
 * The sum runs in a fixed order (samples in chunks whose count depends only
 * on the sizes, the chunks added in order), so repeated calls agree bit for
 * bit.  Uses partial sums in the handle's workspace. */
int sl_mean(sl_handle h, double* out, int32_t out_is_device);

/* Per-node PDF of the samples by binning (Sec. 5.4: the PDF of the solution at
 * each grid point from the samples).  counts[nodes][nbins + 2] (uint32):
 * column 0 counts values below lo, columns 1..nbins the bins of width
 * w = (hi - lo) / nbins, column nbins + 1 values at or above hi.  A value v in
 * [lo, hi) goes to bin floor((v - lo) / w), capped at nbins - 1 (float64,
 * correctly rounded subtraction and division, so the bin of every value is
 * defined exactly); non-finite values are not counted.  Counts are exact
 * integers whatever the launch.  1 <= nbins <= 254, finite lo < hi,
 * samples < 2^32.  out_is_device != 0: counts is a device pointer and the call
 * is asynchronous; otherwise host memory, a temporary device buffer is
 * allocated and the call waits. */
int sl_pdf(sl_handle h, double lo, double hi, int32_t nbins, uint32_t* counts, int32_t out_is_device);

/* Re-seeding (Sec. 5.4, eq. re-seed): every sample is set to the sample mean at
 * the nodes (the same mean as sl_mean).  Enqueued on the handle's stream; the
 * step counter is unchanged, so the next step draws the Wiener increments it
 * would have drawn anyway.  The paper re-seeds every 100 steps of its
 * Dirichlet cases; the caller chooses when (e.g. sl_step(h, dt, 100) then
 * sl_reseed(h)).  Non-finite samples met by the mean are counted in
 * sl_diag().nonfinite. */
int sl_reseed(sl_handle h);

/* Copy ns samples starting at s0 ([ns][nodes]) out of / into the handle (for
 * checkpoints and subset checks).  Host buffers unless *_is_device != 0. */
int sl_get_samples(sl_handle h, int64_t s0, int64_t ns, double* out, int32_t out_is_device);
int sl_set_samples(sl_handle h, int64_t s0, int64_t ns, const double* in, int32_t in_is_device);

/* Step counter n (the first Philox counter word of the next step). */
int sl_get_step(sl_handle h, int64_t* n);
int sl_set_step(sl_handle h, int64_t n);

/* Test aids.  sl_debug_normals: z (z_a, z_b) of samples [s0, s0+ns) at step
 * n, computed by the device generator: out[ns][2], host.
 * sl_debug_positions: moved reference coordinates xi* the next step would
 * produce with step size dt, by the same device code as the step:
 * out[samples][nodes][dim], host. */
int sl_debug_normals(sl_handle h, int64_t n, int64_t s0, int64_t ns, double* out);
int sl_debug_positions(sl_handle h, double dt, double* out);

/* Per-kernel device time, for measurement.  sl_profile(h, 1) starts
 * recording HIP events around every launch on the handle's stream and clears
 * the totals; sl_profile(h, 0) stops.  sl_kernel_time(h, name, &launches,
 * &ms) reads the totals for a kernel name (see the library source for the
 * names), waiting for the stream first. */
int sl_profile(sl_handle h, int32_t enable);
int sl_kernel_time(sl_handle h, const char* name, int64_t* launches, double* ms);

int sl_diag(sl_handle h, sl_diag_t* out);
int sl_sync(sl_handle h);                 /* wait for the handle's stream */
/* Move the handle to another HIP stream (NULL = the null stream); waits for
 * the work pending on the old one first.  Lets a caller initialise a handle
 * on a private stream and then join it to a batch stream. */
int sl_set_stream(sl_handle h, void* hip_stream);
/* Free and total bytes of the current device (hipMemGetInfo), for admission. */
int sl_mem_info(size_t* free_bytes, size_t* total_bytes);
const char* sl_last_error(void);          /* thread-local message of the last failure */

/* Allocation-free sample mean, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc) and hold their own sample arrays: the variant of sl_mean that
 * needs no handle and allocates nothing.
 *   phi: device array [samples][nodes] (float64, borrowed, read only);
 *   out: device array [nodes], receives the mean (same summation order as
 *     sl_mean, so the two agree bit for bit for the same sizes and values);
 *   nonfinite: optional device uint64, cleared and then set to the count of
 *     non-finite values read (NULL: not counted);
 *   hip_stream: the stream to enqueue on (NULL = the null stream); the call
 *     returns without waiting.
 * The partial sums live in one static device array per GPU of the library
 * (4 MiB, kept until the process ends); the chunk count is chosen so that
 * they always fit it (for more than 2^19 nodes the mean takes one pass and
 * uses no scratch), so no size is rejected for lack of scratch.  Calls on one
 * GPU share that array: calls that overlap in time on one GPU (two streams,
 * two threads) race and must be serialised by the caller.  Errors: SL_EINVAL
 * for null pointers or sizes < 1 or above 2^40 (or samples * nodes > 9e15),
 * SL_EDEVICE when a launch fails. */
int sl_mean_noalloc(const double* phi, int64_t samples, int64_t nodes, double* out, uint64_t* nonfinite,
                    void* hip_stream);
int sl_destroy(sl_handle h);              /* waits, frees what the library allocated */

#ifdef __cplusplus
}
#endif
#endif /* SL_H */
