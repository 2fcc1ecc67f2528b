// C ABI of the library (declared in include/sl.h): handle lifetime, argument
// checks, host-side step coefficients, workspace layout and kernel dispatch.
#include "../../include/sl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "sl_internal.hpp"
#include "tables.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define SL_HIP(call)                                                                                  \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) return fail(SL_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct KStat {
  int64_t launches = 0;
  double ms = 0.0;
};

struct PendingEvent {
  std::string name;
  hipEvent_t a, b;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t stats_bytes() { return sizeof(unsigned long long) * sl::kStatSlots * sl::kStatStride; }

// Allocation-failure injection for tests: SL_FAULT=alloc makes every device
// allocation of the library fail (SL_ENOMEM), SL_FAULT=host the host allocation
// of a handle's context.  Read at each allocation.
bool fault_is(const char* what) {
  const char* f = std::getenv("SL_FAULT");
  return f && std::strcmp(f, what) == 0;
}

hipError_t dev_malloc(void** p, size_t bytes) {
  *p = nullptr;
  if (fault_is("alloc")) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

// Sizes derived from a descriptor (shared by sl_required_bytes and sl_init_mesh).
struct Layout {
  int dim = 1, kx = 1, ky = 1, K = 1;
  std::vector<int> order;
  std::vector<int64_t> noff, eoff;
  int64_t nodes = 0, edges = 0, M = 0;
  int nc = 1;                       // components of the field (vector-valued phi*)
  bool mass = false;                // mass constraint beside the boundary constraints
  int64_t MV = 0;                   // rows of `nodes` values in the state: M * nc
  int maxN = 0;
  bool uniform = true;
  std::vector<int> orders;          // distinct orders present, increasing
  size_t ur_doubles = 0, interp_doubles = 0;
  // byte offsets in the workspace
  size_t o_phi, o_phi2, o_tr, o_xi, o_A, o_B, o_src, o_Af, o_Bf, o_ghost, o_mean, o_phi0;
  size_t o_order, o_noff, o_eoff, o_nbr, o_work, o_xitab, o_ur, o_uroff, o_interp, o_interpoff;
  size_t o_params, o_dstep, o_ctr, o_nonf, o_stats, o_mpart, o_gxinv, o_nsp, o_sops, o_bw, o_wqtab, o_z, o_wrec, o_rlist, o_rcount, total;
  bool shared_capable = false;      // one order <= kMaxNShared in 2-D: the shared-geometry path can run
  int solver = SL_SOLVER_FACTOR;    // effective 2-D solver
  size_t gx_doubles = 0, nsp_doubles = 0;
  int max_iter = 32;
  double tol = 1e-13;
};

int make_layout(const sl_mesh_desc* d, Layout& L) {
  if (!d) return fail(SL_EINVAL, "null descriptor");
  if (d->dim != 1 && d->dim != 2) return fail(SL_EINVAL, "dim must be 1 or 2");
  if (d->kx < 1 || (d->dim == 2 && d->ky < 1)) return fail(SL_EINVAL, "kx, ky must be >= 1");
  if (!(d->x1 > d->x0) || (d->dim == 2 && !(d->y1 > d->y0))) return fail(SL_EINVAL, "empty box");
  if (!std::isfinite(d->x0) || !std::isfinite(d->x1) || !std::isfinite(d->y0) || !std::isfinite(d->y1))
    return fail(SL_EINVAL, "non-finite box");
  if (d->samples < 1) return fail(SL_EINVAL, "samples must be >= 1");
  if (d->nodes != SL_NODES_GL && d->nodes != SL_NODES_CG) return fail(SL_EINVAL, "unknown node family");
  if (d->bc != SL_BC_PERIODIC && d->bc != SL_BC_DIRICHLET) return fail(SL_EINVAL, "unknown boundary condition");
  if (d->precision < SL_PREC_FP64 || d->precision > SL_PREC_BF16SPLIT_REFINE)
    return fail(SL_EINVAL, "unknown precision mode");
  if (d->solver < SL_SOLVER_AUTO || d->solver > SL_SOLVER_REFERENCE) return fail(SL_EINVAL, "unknown solver");
  if (d->max_iter < 0 || d->max_iter > 100000) return fail(SL_EINVAL, "max_iter must be in [0, 100000]");
  if (!(d->tol >= 0.0) || !std::isfinite(d->tol) || d->tol >= 1.0) return fail(SL_EINVAL, "tol must be in [0, 1)");
  if (d->solver == SL_SOLVER_REFERENCE && d->precision != SL_PREC_FP64)
    return fail(SL_EINVAL, "the reference-preconditioned solver runs in float64 only");
  L.solver = d->solver == SL_SOLVER_FACTOR ? SL_SOLVER_FACTOR
             : d->solver == SL_SOLVER_REFERENCE ? SL_SOLVER_REFERENCE
             : (d->precision == SL_PREC_FP64 ? SL_SOLVER_REFERENCE : SL_SOLVER_FACTOR);
  if (d->max_iter > 0) L.max_iter = d->max_iter;
  if (d->tol > 0.0) L.tol = d->tol;
  L.dim = d->dim;
  L.kx = d->kx;
  L.ky = d->dim == 2 ? d->ky : 1;
  const int64_t K64 = (int64_t)L.kx * L.ky;
  if (K64 > (1 << 26)) return fail(SL_EINVAL, "too many elements");
  L.K = (int)K64;
  L.order.resize(L.K);
  for (int e = 0; e < L.K; ++e) {
    const int N = d->order ? d->order[e] : d->n_uniform;
    if (N < 2 || N > sl::kMaxN) return fail(SL_EINVAL, "element order N must be in [2, 16]");
    L.order[e] = N;
  }
  L.maxN = *std::max_element(L.order.begin(), L.order.end());
  L.uniform = std::all_of(L.order.begin(), L.order.end(), [&](int n) { return n == L.order[0]; });
  L.noff.resize(L.K + 1);
  L.eoff.resize(L.K + 1);
  L.noff[0] = L.eoff[0] = 0;
  for (int e = 0; e < L.K; ++e) {
    const int N = L.order[e];
    L.noff[e + 1] = L.noff[e] + (L.dim == 1 ? N : N * N);
    L.eoff[e + 1] = L.eoff[e] + (L.dim == 1 ? 2 : 4 * N);
  }
  L.nodes = L.noff[L.K];
  L.edges = L.eoff[L.K];
  L.M = d->samples;
  if (d->ncomp < 0 || d->ncomp > 64) return fail(SL_EINVAL, "ncomp must be in [0, 64] (0 means 1)");
  if (d->constraints != SL_CONSTRAIN_BOUNDARY && d->constraints != SL_CONSTRAIN_BOUNDARY_MASS)
    return fail(SL_EINVAL, "unknown constraint set");
  L.mass = d->constraints == SL_CONSTRAIN_BOUNDARY_MASS;
  L.nc = d->ncomp > 1 ? d->ncomp : 1;
  L.MV = L.M * L.nc;
  for (int N : L.order)
    if (std::find(L.orders.begin(), L.orders.end(), N) == L.orders.end()) L.orders.push_back(N);
  std::sort(L.orders.begin(), L.orders.end());
  if (L.dim == 2) {
    for (int N : L.orders) L.ur_doubles += (size_t)(4 * N) * (4 * N - 4);
    for (int Nd : L.orders)
      for (int Ns : L.orders)
        if (Nd != Ns) L.interp_doubles += (size_t)Nd * Ns;
    for (int N : L.orders) L.gx_doubles += (size_t)2 * N * N;
    for (int N : L.orders) L.nsp_doubles += (size_t)sl::nsp_doubles(N);
  }
  if ((double)L.MV * (double)L.nodes * 8.0 > 250e9) return fail(SL_ENOMEM, "state exceeds device memory");
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.o_phi = take(sizeof(double) * (size_t)L.MV * L.nodes);
  // 1-D meshes of more than 256 elements step out of place (tiled kernel)
  L.o_phi2 = take(L.dim == 1 && L.K > 256 ? sizeof(double) * (size_t)L.MV * L.nodes : 0);
  L.o_tr = take(L.dim == 2 ? sizeof(double) * (size_t)L.MV * L.edges : 0);
  L.o_xi = take(sizeof(double) * L.nodes * L.dim);
  L.o_A = take(sizeof(double) * L.nodes * L.dim);
  L.o_B = take(sizeof(double) * L.nodes * L.dim);
  L.o_src = take(sizeof(double) * L.nodes);
  L.o_Af = take(sizeof(double) * L.edges);
  L.o_Bf = take(sizeof(double) * L.edges);
  L.o_ghost = take(sizeof(double) * L.edges);
  L.o_mean = take(sizeof(double) * L.nc * L.nodes);
  L.o_phi0 = take(sizeof(double) * L.nc * L.nodes);
  L.o_order = take(sizeof(int32_t) * L.K);
  L.o_noff = take(sizeof(int64_t) * L.K);
  L.o_eoff = take(sizeof(int64_t) * L.K);
  L.o_nbr = take(sizeof(int32_t) * 4 * (size_t)L.K);
  L.o_work = take(sizeof(int32_t) * L.K);
  L.o_xitab = take(sizeof(double) * (sl::kMaxN + 1) * sl::kMaxN);
  L.o_ur = take(sizeof(double) * (L.ur_doubles + 1));
  L.o_uroff = take(sizeof(int64_t) * (sl::kMaxN + 1));
  L.o_interp = take(sizeof(double) * (L.interp_doubles + 1));
  L.o_interpoff = take(sizeof(int64_t) * (sl::kMaxN + 1) * (sl::kMaxN + 1));
  L.o_params = take(std::max(sizeof(sl::Params1D), sizeof(sl::Params2D)));
  L.o_dstep = take(sizeof(int64_t));
  L.o_ctr = take(sl::kWorkCounters * sizeof(unsigned long long));
  L.o_nonf = take(sizeof(unsigned long long));
  L.o_stats = take(stats_bytes());
  {
    const int64_t C = sl::mean_chunks(L.M, L.nc * L.nodes);     // partial sums of the sample mean
    L.o_mpart = take(C > 1 ? sizeof(double) * (size_t)C * L.nc * L.nodes : 0);
  }
  L.o_gxinv = take(sizeof(double) * (L.gx_doubles + 1));
  L.o_nsp = take(sizeof(double) * (L.nsp_doubles + 1));
  L.o_wqtab = take(sizeof(double) * (sl::kMaxN + 1) * sl::kMaxN);
  L.shared_capable = L.dim == 2 && L.uniform && L.maxN <= sl::kMaxNShared;
  L.o_sops = take(L.shared_capable ? sizeof(double) * (size_t)L.M * sl::shared_op_doubles(L.maxN) : 0);
  L.o_bw = take(sizeof(double) * sl::kMaxN);
  L.o_z = take(L.dim == 2 ? sizeof(double) * 2 * (size_t)L.M : 0);
  L.o_wrec = take(L.dim == 2 ? sizeof(sl::WorkRec) * (size_t)L.K : 0);
  // phase-1 fits to redo (reference solver, one component): one slot a fit
  const bool lean = L.dim == 2 && L.solver == SL_SOLVER_REFERENCE && L.nc == 1;
  L.o_rlist = take(lean ? sizeof(uint32_t) * (size_t)L.K * (size_t)L.M : 0);
  L.o_rcount = take(lean ? sizeof(unsigned int) * (sl::kMaxN + 1) : 0);
  L.total = o;
  return SL_OK;
}

}  // namespace

struct sl_ctx {
  sl_mesh_desc desc{};
  Layout L;
  double hx = 1, hy = 1;
  int family = 0;
  hipStream_t stream = nullptr;
  bool own_ws = false;
  char* ws = nullptr;
  double *phi = nullptr, *phi2 = nullptr, *tr = nullptr, *xi_node = nullptr, *A = nullptr, *B = nullptr, *src = nullptr;
  double *Af = nullptr, *Bf = nullptr, *ghost = nullptr, *mean = nullptr, *phi0 = nullptr;
  // 2-D tables
  int32_t *d_order = nullptr, *d_nbr = nullptr, *d_work = nullptr;
  int64_t *d_noff = nullptr, *d_eoff = nullptr, *d_uroff = nullptr, *d_interpoff = nullptr;
  double *d_xitab = nullptr, *d_ur = nullptr, *d_interp = nullptr;
  std::vector<std::pair<int, std::pair<int64_t, int64_t>>> groups;   // (N, (first work index, count))
  std::map<int, std::vector<double>> xi_tab;    // reference nodes per order
  int64_t gx_off[sl::kMaxN + 1] = {0};          // offsets of the reference Gram inverses
  int64_t nsp_off[sl::kMaxN + 1] = {0};         // offsets of the null-space tables
  sl::LegendreRec rec{};
  // host copies of the fields
  std::vector<double> u, D, divu, un, Dn, ghost_h;
  std::vector<double> hA, hB, hsrc, hAf, hBf;
  std::vector<int32_t> work_h;           // the work list (elements grouped by order)
  std::vector<sl::WorkRec> hwrec;        // host copy of the work records
  bool fields_set = false;
  bool coeff_valid = false;
  double coeff_dt = 0.0;
  double max_disp_ratio = 0.0;
  int64_t step = 0;
  int algo_1d = 0;      // 0 nodal form, 1 Legendre normal equations (SL_1D_FIT=normal, for tests)
  // launch schedule and its device-side state
  uint64_t id = 0;                       // unique per handle (graph cache keys)
  sl_schedule_t sched{0, 0, 0, 0.f};
  sl::Params1D p1{};                     // step inputs (host copies; device copies at d_p1 / d_p2)
  sl::Params2D p2{};
  sl::Params1D* d_p1 = nullptr;
  sl::Params2D* d_p2 = nullptr;
  int64_t* d_step = nullptr;             // device step counter (fused / graph schedules)
  unsigned long long* d_ctr = nullptr;   // work counters of the persistent launches (phase, order)
  unsigned long long* d_stats = nullptr; // diagnostics slots (solver statistics, escapes, residuals)
  unsigned long long* d_nonf = nullptr;  // non-finite values seen by the last sample mean
  double* d_mpart = nullptr;             // partial sums of the sample mean
  double* d_gxinv = nullptr;
  double* d_nsp = nullptr;
  double* d_sops = nullptr;              // shared-geometry path: per-sample operators
  double* d_bw = nullptr;                // barycentric weights of the (single) order's nodes
  double* d_wqtab = nullptr;             // [(kMaxN+1)][kMaxN] quadrature weights of each order's nodes
  double* d_z = nullptr;                 // [M][2] this step's Wiener normals (reference solver)
  sl::WorkRec* d_wrec = nullptr;         // [K] element data of each work item (reference solver)
  uint32_t* d_rlist = nullptr;           // phase-1 fits to redo, by order group (null: none)
  unsigned int* d_rcount = nullptr;      // [kMaxN + 1] their counts, by order
  bool shared_geometry = false;          // the current step coefficients are the same at every node
  hipStream_t cap_stream = nullptr;      // private stream for graph capture
  // measurement
  bool profile = false;
  std::vector<PendingEvent> pending;
  std::map<std::string, KStat> kstats;
};

namespace {

int check_handle(sl_handle h) {
  if (!h) return fail(SL_EINVAL, "null handle");
  return SL_OK;
}

// Record an event pair around a launch when profiling is on.
struct ProfScope {
  sl_ctx* h;
  PendingEvent ev;
  bool on;
  ProfScope(sl_ctx* h_, const char* name) : h(h_), on(h_->profile) {
    if (on) {
      ev.name = name;
      (void)hipEventCreate(&ev.a);
      (void)hipEventCreate(&ev.b);
      (void)hipEventRecord(ev.a, h->stream);
    }
  }
  ~ProfScope() {
    if (on) {
      (void)hipEventRecord(ev.b, h->stream);
      h->pending.push_back(ev);
    }
  }
};

void drain_events(sl_ctx* h) {
  if (h->pending.empty()) return;
  (void)hipStreamSynchronize(h->stream);
  for (auto& p : h->pending) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    auto& k = h->kstats[p.name];
    k.launches += 1;
    k.ms += ms;
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  h->pending.clear();
}

// Step coefficients for dt (position contract, host side):
//   A = (u*dt)/h, B = sqrt((2*D)*dt)/h, src = 1 - dt*divu,
//   Af = (un*dt)/h_axis, Bf = sqrt((2*Dn)*dt)/h_axis.
int update_coefficients(sl_ctx* h, double dt) {
  if (h->coeff_valid && h->coeff_dt == dt) return SL_OK;
  const Layout& L = h->L;
  const double hdir[2] = {h->hx, h->hy};
  h->hA.resize(L.nodes * L.dim);
  h->hB.resize(L.nodes * L.dim);
  h->hsrc.resize(L.nodes);
  double maxratio = 0.0;
  for (int e = 0; e < L.K; ++e) {
    const int N = L.order[e];
    const double spacing = sl::min_node_spacing(h->xi_tab[N]);
    for (int64_t k = L.noff[e]; k < L.noff[e + 1]; ++k) {
      const double sq = std::sqrt((2.0 * h->D[k]) * dt);
      for (int j = 0; j < L.dim; ++j) {
        const double a = (h->u[k * L.dim + j] * dt) / hdir[j];
        const double b = sq / hdir[j];
        h->hA[k * L.dim + j] = a;
        h->hB[k * L.dim + j] = b;
        maxratio = std::max(maxratio, (std::fabs(a) + std::fabs(b)) / spacing);
      }
      h->hsrc[k] = 1.0 - dt * (h->divu.empty() ? 0.0 : h->divu[k]);
    }
  }
  h->hAf.resize(L.edges);
  h->hBf.resize(L.edges);
  for (int e = 0; e < L.K; ++e) {
    const int N = L.order[e];
    for (int64_t q = L.eoff[e]; q < L.eoff[e + 1]; ++q) {
      const int64_t local = q - L.eoff[e];
      const int axis = (L.dim == 1 || local < 2 * N) ? 0 : 1;
      h->hAf[q] = (h->un[q] * dt) / hdir[axis];
      h->hBf[q] = std::sqrt((2.0 * h->Dn[q]) * dt) / hdir[axis];
    }
  }
  SL_HIP(hipMemcpyAsync(h->A, h->hA.data(), sizeof(double) * h->hA.size(), hipMemcpyHostToDevice, h->stream));
  SL_HIP(hipMemcpyAsync(h->B, h->hB.data(), sizeof(double) * h->hB.size(), hipMemcpyHostToDevice, h->stream));
  SL_HIP(hipMemcpyAsync(h->src, h->hsrc.data(), sizeof(double) * h->hsrc.size(), hipMemcpyHostToDevice, h->stream));
  SL_HIP(hipMemcpyAsync(h->Af, h->hAf.data(), sizeof(double) * h->hAf.size(), hipMemcpyHostToDevice, h->stream));
  SL_HIP(hipMemcpyAsync(h->Bf, h->hBf.data(), sizeof(double) * h->hBf.size(), hipMemcpyHostToDevice, h->stream));
  if (L.dim == 2) {
    // element means of A and B per direction into the work records: the mean
    // displacement of a fit's moved nodes is then mean(A) + mean(B) z, up to
    // rounding
    for (size_t w = 0; w < h->work_h.size(); ++w) {
      const int e = h->work_h[w];
      long double sa[2] = {0, 0}, sb[2] = {0, 0};
      for (int64_t k = L.noff[e]; k < L.noff[e + 1]; ++k)
        for (int j = 0; j < 2; ++j) {
          sa[j] += h->hA[k * 2 + j];
          sb[j] += h->hB[k * 2 + j];
        }
      const long double n = (long double)(L.noff[e + 1] - L.noff[e]);
      for (int j = 0; j < 2; ++j) {
        h->hwrec[w].emean[j] = (double)(sa[j] / n);
        h->hwrec[w].emean[2 + j] = (double)(sb[j] / n);
      }
    }
    SL_HIP(hipMemcpyAsync(h->d_wrec, h->hwrec.data(), sizeof(sl::WorkRec) * h->hwrec.size(), hipMemcpyHostToDevice,
                          h->stream));
  }
  SL_HIP(hipStreamSynchronize(h->stream));   // host vectors may be reused right after
  h->coeff_valid = true;
  h->coeff_dt = dt;
  h->max_disp_ratio = maxratio;
  // shared geometry: every node moves by the same displacement and carries the same source factor
  bool same = L.dim == 2 && L.uniform;
  for (int64_t k = 1; same && k < L.nodes; ++k)
    same = h->hA[2 * k] == h->hA[0] && h->hA[2 * k + 1] == h->hA[1] && h->hB[2 * k] == h->hB[0] &&
           h->hB[2 * k + 1] == h->hB[1] && h->hsrc[k] == h->hsrc[0];
  h->shared_geometry = same;
  return SL_OK;
}


// ---------------------------------------------------------------- launch schedules

const char* kernel_label(const sl_ctx* h, int phase) {
  if (h->L.solver == SL_SOLVER_REFERENCE) return phase == 1 ? "fit2r_phase1" : "fit2r_phase2";
  return phase == 1 ? "fit2d_phase1" : "fit2d_phase2";
}

int default_refine(int precision) {
  return precision == SL_PREC_FP32_REFINE ? 2 : precision == SL_PREC_BF16SPLIT_REFINE ? 3 : 0;
}

// Step inputs of a handle (device pointers into its workspace); the device
// copy is what the fused and batched kernels read.
void build_params(sl_ctx* h) {
  const Layout& L = h->L;
  if (L.dim == 2) {
    sl::Params2D& p = h->p2;
    p = sl::Params2D{};
    p.xi_node = h->xi_node;
    p.A = h->A;
    p.B = h->B;
    p.src = h->src;
    p.Af = h->Af;
    p.Bf = h->Bf;
    p.ghost = h->ghost;
    p.order = h->d_order;
    p.noff = h->d_noff;
    p.eoff = h->d_eoff;
    p.nbr = h->d_nbr;
    p.work = h->d_work;
    p.xi_tab = h->d_xitab;
    p.ur = h->d_ur;
    p.ur_off = h->d_uroff;
    p.interp = h->d_interp;
    p.interp_off = h->d_interpoff;
    p.phi = h->phi;
    p.tr = h->tr;
    // the reference solver loops over the components inside a fit; the
    // factorisation kernels take every (sample, component) row as a fit
    p.M = L.solver == SL_SOLVER_REFERENCE ? L.M : L.MV;
    p.ncomp = L.nc;
    p.nodes = L.nodes;
    p.edges = L.edges;
    p.block0 = 0;
    p.step = 0;
    p.step_ptr = h->d_step;
    p.seed = h->desc.seed;
    p.stream = h->desc.stream_id;
    p.refine = h->desc.refine_iters >= 0 ? h->desc.refine_iters : default_refine(h->desc.precision);
    p.gxinv = h->d_gxinv;
    for (int N = 0; N <= sl::kMaxN; ++N) p.gx_off[N] = h->gx_off[N];
    p.nsp = h->d_nsp;
    for (int N = 0; N <= sl::kMaxN; ++N) p.nsp_off[N] = h->nsp_off[N];
    p.tol2 = L.tol * L.tol;
    p.max_iter = L.max_iter;
    p.stats = h->d_stats;
    p.rec = h->rec;
    p.mass = L.mass ? 1 : 0;
    p.wq_tab = h->d_wqtab;
    p.zdraw = h->d_z;
    p.rescue_list = h->d_rlist;
    p.rescue_count = h->d_rcount;
    for (const auto& g : h->groups) p.rescue_off[g.first] = g.second.first * p.M;
    p.wrec = h->d_wrec;
  } else {
    sl::Params1D& p = h->p1;
    p = sl::Params1D{};
    p.A = h->A;
    p.B = h->B;
    p.src = h->src;
    p.Af = h->Af;
    p.Bf = h->Bf;
    p.ghost = h->ghost;
    p.phi = h->phi;
    p.K = L.K;
    p.samples_per_block = sl::resident_1d_samples_per_block(L.K);
    p.dirichlet = h->desc.bc == SL_BC_DIRICHLET;
    p.nsteps = 0;
    p.algo = h->algo_1d;
    p.M = L.MV;                 // one row per (sample, component), each drawing its sample's increments
    p.ncomp = L.nc;
    p.step0 = 0;
    p.seed = h->desc.seed;
    p.stream = h->desc.stream_id;
    p.stats = h->d_stats;
    p.rec = h->rec;
    p.mass = L.mass ? 1 : 0;
    const auto& xi = h->xi_tab[L.order[0]];
    for (size_t i = 0; i < xi.size(); ++i) p.xi[i] = xi[i];
    const auto wq = sl::quadrature_weights(xi);
    for (size_t i = 0; i < wq.size(); ++i) p.wq[i] = wq[i];
  }
}

int device_cus() {
  int d = 0, c = 0;
  if (hipGetDevice(&d) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || c <= 0) return 256;
  return c;
}

// Set (set = 1, to each handle's host step counter) or advance the device
// step counters of the handles and clear their work counters.
int enqueue_counters(const std::vector<sl_ctx*>& hs, int set, hipStream_t st) {
  for (size_t c0 = 0; c0 < hs.size(); c0 += sl::kMaxTasks) {
    sl::StepArgs a{};
    a.set = set;
    a.n = (int)std::min<size_t>(sl::kMaxTasks, hs.size() - c0);
    for (int i = 0; i < a.n; ++i) {
      a.step[i] = hs[c0 + i]->d_step;
      a.counter[i] = hs[c0 + i]->d_ctr;
      a.value[i] = hs[c0 + i]->step;
    }
    SL_HIP(sl::launch_step_counters(a, st));
  }
  return SL_OK;
}

// This step's normal pairs of the reference-solver handles among hs, read by
// both phases.  devstep: the draw reads each handle's device step counter
// (graph capture), else it takes the host counter plus `ahead`.
int enqueue_draw(const std::vector<sl_ctx*>& hs, bool devstep, int64_t ahead, hipStream_t st) {
  std::vector<sl_ctx*> ref;
  for (sl_ctx* h : hs)
    if (h->L.solver == SL_SOLVER_REFERENCE) ref.push_back(h);
  for (size_t c0 = 0; c0 < ref.size(); c0 += sl::kMaxTasks) {
    sl::DrawArgs a{};
    a.n = (int)std::min<size_t>(sl::kMaxTasks, ref.size() - c0);
    int64_t maxM = 0;
    for (int i = 0; i < a.n; ++i) {
      sl_ctx* h = ref[c0 + i];
      a.z[i] = h->d_z;
      a.rescue_count[i] = h->d_rcount;
      a.step_ptr[i] = devstep ? h->d_step : nullptr;
      a.step[i] = h->step + ahead;
      a.M[i] = h->p2.M;
      a.seed[i] = h->p2.seed;
      a.stream[i] = h->p2.stream;
      maxM = std::max<int64_t>(maxM, h->p2.M);
    }
    SL_HIP(sl::launch_draw_normals(a, maxM, st));
  }
  return SL_OK;
}

// Per-order launches of one phase for one handle.  devstep: the kernels read
// the device step counter (graph capture), else the host counter `step`.
int enqueue_perorder(sl_ctx* h, int phase, bool devstep, int64_t step, hipStream_t st) {
  sl::Params2D p = h->p2;
  p.step_ptr = devstep ? h->d_step : nullptr;
  p.step = step;
  for (const auto& g : h->groups) {
    p.work = h->d_work + g.second.first;
    p.wrec = h->d_wrec ? h->d_wrec + g.second.first : nullptr;
    p.block0 = 0;
    // the group's slots of the phase-1 redo list
    p.rescue_list = h->d_rlist ? h->d_rlist + g.second.first * h->p2.M : nullptr;
    p.rescue_count = h->d_rcount ? h->d_rcount + g.first : nullptr;
    if (h->L.solver == SL_SOLVER_REFERENCE)
      SL_HIP(sl::launch_fit2r(phase, g.first, p, g.second.second * h->p2.M, st, h->sched.wide != 0));
    else
      SL_HIP(sl::launch_fit2d(phase, g.first, h->desc.precision, p, g.second.second * h->p2.M, st));
  }
  return SL_OK;
}

// Persistent launches of one phase of the reference solver over a batch of
// handles, per chunk of kMaxTasks handles / kMaxSegs order segments: one
// launch per order present, largest first, each pulling the chunk's fits of
// that order from its own counter of the chunk's first handle.
int enqueue_fused_ref(const std::vector<sl_ctx*>& m, int phase, int grid_req, hipStream_t st) {
  size_t i = 0;
  while (i < m.size()) {
    size_t j = i, nseg = 0;
    while (j < m.size() && j - i < (size_t)sl::kMaxTasks && nseg + m[j]->groups.size() <= (size_t)sl::kMaxSegs)
      nseg += m[j++]->groups.size();
    bool fast = true;   // every handle takes the lean phase 1 and the one-component phase 2
    for (size_t t = i; t < j; ++t) fast = fast && m[t]->d_rlist && !m[t]->L.mass;
    for (int N = sl::kMaxNRef; N >= 2; --N) {
      sl::Fused2DArgs a{};
      int64_t start = 0;
      for (size_t t = i; t < j; ++t) {
        a.task[t - i] = m[t]->d_p2;
        for (const auto& g : m[t]->groups)
          if (g.first == N && g.second.second > 0) {
            a.seg[a.nseg++] = sl::FusedSeg{start, g.second.first * m[t]->p2.M, (int32_t)(t - i), N};
            start += g.second.second * m[t]->p2.M;
          }
      }
      a.total = start;
      if (start <= 0) continue;
      a.counter = m[i]->d_ctr + 2 * N + (phase - 1);
      SL_HIP(sl::launch_fit2r_persist(phase, N, a, fast, grid_req, device_cus(), st));
    }
    i = j;
  }
  return SL_OK;
}

// Persistent fused launches of one phase over a batch of 2-D handles: the
// reference solver's by enqueue_fused_ref; for the factorisation solver one
// launch per precision mode (and per chunk of kMaxTasks handles / kMaxSegs
// order segments), each chunk pulling work from its first handle's counter.
int enqueue_fused(const std::vector<sl_ctx*>& hs, int phase, int grid_req, hipStream_t st) {
  {
    std::vector<sl_ctx*> ref;
    for (sl_ctx* h : hs)
      if (h->L.solver == SL_SOLVER_REFERENCE) ref.push_back(h);
    if (int rc = enqueue_fused_ref(ref, phase, grid_req, st)) return rc;
  }
  for (int mode = 0; mode <= 2; ++mode) {
    std::vector<sl_ctx*> m;
    for (sl_ctx* h : hs)
      if (h->L.solver != SL_SOLVER_REFERENCE && h->desc.precision == mode) m.push_back(h);
    size_t i = 0;
    while (i < m.size()) {
      // take handles while the chunk's segments fit
      size_t j = i, nseg = 0;
      while (j < m.size() && j - i < (size_t)sl::kMaxTasks && nseg + m[j]->groups.size() <= (size_t)sl::kMaxSegs)
        nseg += m[j++]->groups.size();
      sl::Fused2DArgs a{};
      struct S { int N, task; int64_t fit0, count; };
      std::vector<S> segs;
      for (size_t t = i; t < j; ++t) {
        a.task[t - i] = m[t]->d_p2;
        for (const auto& g : m[t]->groups)
          segs.push_back({g.first, (int)(t - i), g.second.first * m[t]->p2.M, g.second.second * m[t]->p2.M});
      }
      std::stable_sort(segs.begin(), segs.end(), [](const S& x, const S& y) { return x.N > y.N; });
      int64_t start = 0;
      size_t lds = 0;
      a.nseg = 0;
      for (const S& g : segs) {
        if (g.count == 0) continue;
        a.seg[a.nseg] = sl::FusedSeg{start, g.fit0, g.task, g.N};
        ++a.nseg;
        start += g.count;
        lds = std::max(lds, sl::fit2d_lds_bytes(g.N, mode, phase));
      }
      a.total = start;
      a.counter = m[i]->d_ctr + (phase - 1);
      if (a.total > 0) {
        const int occ = sl::fit2d_fused_occupancy(phase, mode, lds);
        if (occ <= 0) return fail(SL_EDEVICE, "fused kernel does not fit on a compute unit");
        int64_t grid = grid_req > 0 ? grid_req : (int64_t)occ * device_cus();
        grid = std::min<int64_t>(grid, a.total);
        SL_HIP(sl::launch_fit2d_fused(phase, mode, a, (int)grid, lds, st));
      }
      i = j;
    }
  }
  return SL_OK;
}

// Batched launches of one phase, one per order: the reference-solver fits of
// every handle that have order N go into one launch (chunks of kMaxTasks
// handles); factorisation handles get their per-order launches.
int enqueue_multi(const std::vector<sl_ctx*>& hs, int phase, hipStream_t st) {
  std::vector<sl_ctx*> ref;
  for (sl_ctx* h : hs) {
    if (h->L.solver == SL_SOLVER_REFERENCE) ref.push_back(h);
    else if (int rc = enqueue_perorder(h, phase, true, 0, st)) return rc;
  }
  for (int N = sl::kMaxNRef; N >= 2; --N) {
    std::vector<std::pair<sl_ctx*, std::pair<int64_t, int64_t>>> segs;   // (handle, (fit0, count))
    for (sl_ctx* h : ref)
      for (const auto& g : h->groups)
        if (g.first == N && g.second.second > 0)
          segs.push_back({h, {g.second.first * h->p2.M, g.second.second * h->p2.M}});
    for (size_t c0 = 0; c0 < segs.size(); c0 += sl::kMaxTasks) {
      sl::Fused2DArgs a{};
      const size_t nc = std::min<size_t>(sl::kMaxTasks, segs.size() - c0);
      int64_t start = 0;
      for (size_t i = 0; i < nc; ++i) {
        a.task[i] = segs[c0 + i].first->d_p2;
        a.seg[i] = sl::FusedSeg{start, segs[c0 + i].second.first, (int32_t)i, N};
        start += segs[c0 + i].second.second;
      }
      a.nseg = (int)nc;
      a.total = start;
      if (start > 0x7fffffff) return fail(SL_EUNSUPPORTED, "too many fits of one order in one batch");
      bool fast = true;
      for (size_t i = 0; i < nc; ++i) fast = fast && segs[c0 + i].first->d_rlist && !segs[c0 + i].first->L.mass;
      SL_HIP(sl::launch_fit2r_multi(phase, N, a, fast, st));
    }
  }
  return SL_OK;
}

// One whole step (both phases and the counter advance) on the device step counters.
int enqueue_device_step(const std::vector<sl_ctx*>& hs, int fused, int grid, hipStream_t st, sl_ctx* prof) {
  {
    std::unique_ptr<ProfScope> ps(prof ? new ProfScope(prof, "draw_normals") : nullptr);
    if (int rc = enqueue_draw(hs, true, 0, st)) return rc;
  }
  for (int phase = 1; phase <= 2; ++phase) {
    const char* name = fused ? (phase == 1 ? "fit2d_fused_phase1" : "fit2d_fused_phase2")
                       : hs.size() > 1 ? (phase == 1 ? "fit2d_batch_phase1" : "fit2d_batch_phase2")
                                       : kernel_label(hs[0], phase);
    std::unique_ptr<ProfScope> ps(prof ? new ProfScope(prof, name) : nullptr);
    if (fused) {
      if (int rc = enqueue_fused(hs, phase, grid, st)) return rc;
    } else if (hs.size() > 1) {
      if (int rc = enqueue_multi(hs, phase, st)) return rc;
    } else {
      if (int rc = enqueue_perorder(hs[0], phase, true, 0, st)) return rc;
    }
  }
  return enqueue_counters(hs, 0, st);
}

// Graph cache: one captured step per (handles, schedule), least recently used first out.
struct GraphEntry {
  std::vector<uint64_t> ids;
  int fused, grid, wide;
  hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::list<GraphEntry> g_graphs;
constexpr size_t kMaxGraphs = 16;
uint64_t g_next_id = 1;

void purge_graphs(uint64_t id) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto it = g_graphs.begin(); it != g_graphs.end();) {
    if (std::find(it->ids.begin(), it->ids.end(), id) != it->ids.end()) {
      (void)hipGraphExecDestroy(it->exec);
      it = g_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

int get_graph(const std::vector<sl_ctx*>& hs, int fused, int grid, hipGraphExec_t* out) {
  std::vector<uint64_t> ids;
  for (sl_ctx* h : hs) ids.push_back(h->id);
  // the fit shape of a handle that runs its per-order kernels alone
  const int wide = !fused && hs.size() == 1 ? hs[0]->sched.wide : 0;
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
      if (it->ids == ids && it->fused == fused && it->grid == grid && it->wide == wide) {
        g_graphs.splice(g_graphs.begin(), g_graphs, it);
        *out = it->exec;
        return SL_OK;
      }
  }
  sl_ctx* h0 = hs[0];
  if (!h0->cap_stream) SL_HIP(hipStreamCreateWithFlags(&h0->cap_stream, hipStreamNonBlocking));
  SL_HIP(hipStreamBeginCapture(h0->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_device_step(hs, fused, grid, h0->cap_stream, nullptr);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(h0->cap_stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return fail(SL_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(ec));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return fail(SL_EDEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(ei));
  std::lock_guard<std::mutex> lk(g_graph_mu);
  g_graphs.push_front(GraphEntry{ids, fused, grid, wide, exec});
  while (g_graphs.size() > kMaxGraphs) {
    (void)hipGraphExecDestroy(g_graphs.back().exec);
    g_graphs.pop_back();
  }
  *out = exec;
  return SL_OK;
}

// nsteps steps of a set of 2-D handles (coefficients already current) under a schedule.
int step_2d(const std::vector<sl_ctx*>& hs, int32_t nsteps, int fused, int graph, int grid, hipStream_t st) {
  sl_ctx* h0 = hs[0];
  if (!fused && !graph && hs.size() == 1) {
    // per-order kernels with the host step counter
    for (int it = 0; it < nsteps; ++it) {
      if (h0->L.solver == SL_SOLVER_REFERENCE) {
        ProfScope ps(h0, "draw_normals");
        if (int rc = enqueue_draw(hs, false, it, st)) return rc;
      }
      for (int phase = 1; phase <= 2; ++phase) {
        ProfScope ps(h0, kernel_label(h0, phase));
        if (int rc = enqueue_perorder(h0, phase, false, h0->step + it, st)) return rc;
      }
    }
  } else {
    if (int rc = enqueue_counters(hs, 1, st)) return rc;
    if (graph && !h0->profile) {
      hipGraphExec_t exec = nullptr;
      if (int rc = get_graph(hs, fused, grid, &exec)) return rc;
      for (int it = 0; it < nsteps; ++it) SL_HIP(hipGraphLaunch(exec, st));
    } else {
      // direct launches (also what profiling uses, so that every kernel is timed)
      for (int it = 0; it < nsteps; ++it)
        if (int rc = enqueue_device_step(hs, fused, grid, st, h0->profile ? h0 : nullptr)) return rc;
    }
  }
  for (sl_ctx* h : hs) h->step += nsteps;
  return SL_OK;
}

// Batched resident 1-D launches: one per (order, fit form), chunks of kMaxTasks.
int step_1d(sl_ctx* h, int32_t nsteps, hipStream_t st);

int step_1d_batch(const std::vector<sl_ctx*>& hs, int32_t nsteps, hipStream_t st) {
  std::map<std::pair<int, int>, std::vector<sl_ctx*>> by;
  std::vector<sl_ctx*> tiled;
  for (sl_ctx* h : hs) {
    if (h->L.K > 256) tiled.push_back(h);
    else by[{h->L.order[0], h->algo_1d + 2 * h->p1.mass}].push_back(h);
  }
  for (sl_ctx* h : tiled)
    if (int rc = step_1d(h, nsteps, st)) return rc;
  for (auto& kv : by) {
    const auto& v = kv.second;
    for (size_t c0 = 0; c0 < v.size(); c0 += sl::kMaxTasks) {
      sl::Batch1DArgs a{};
      a.ntasks = (int)std::min<size_t>(sl::kMaxTasks, v.size() - c0);
      a.nsteps = nsteps;
      size_t lds = 0;
      a.bstart[0] = 0;
      for (int t = 0; t < a.ntasks; ++t) {
        sl_ctx* h = v[c0 + t];
        const int spb = h->p1.samples_per_block;
        a.task[t] = h->d_p1;
        a.step0[t] = h->step;
        a.bstart[t + 1] = a.bstart[t] + (h->L.MV + spb - 1) / spb;
        lds = std::max(lds, sl::resident_1d_lds_bytes(h->L.K, spb));
      }
      ProfScope ps(v[c0], "resident_1d_batch");
      SL_HIP(sl::launch_resident_1d_batch(kv.first.first, kv.first.second, a, lds, st));
    }
  }
  for (auto& kv : by)
    for (sl_ctx* h : kv.second) h->step += nsteps;
  return SL_OK;
}

// nsteps 1-D steps of one handle: one resident launch for all steps (K <= 256),
// else one tiled launch per step, out of place, ending in the primary buffer.
int step_1d(sl_ctx* h, int32_t nsteps, hipStream_t st) {
  const Layout& L = h->L;
  const int N = L.order[0];
  sl::Params1D p = h->p1;
  p.nsteps = nsteps;
  p.step0 = h->step;
  if (L.K <= 256) {
    ProfScope ps(h, "resident_1d");
    SL_HIP(sl::launch_resident_1d(N, p, st));
  } else {
    double* buf[2] = {h->phi, h->phi2};
    for (int it = 0; it < nsteps; ++it) {
      ProfScope ps(h, "tiled_1d");
      SL_HIP(sl::launch_tiled_1d(N, p, buf[it & 1], buf[(it + 1) & 1], h->step + it, st));
    }
    if (nsteps & 1)
      SL_HIP(hipMemcpyAsync(h->phi, h->phi2, sizeof(double) * (size_t)L.MV * L.nodes, hipMemcpyDeviceToDevice, st));
  }
  h->step += nsteps;
  return SL_OK;
}

// nsteps steps on the shared-geometry path (per-sample operators, then the
// batched trace and update products), host step counter.
int step_shared(sl_ctx* h, int32_t nsteps) {
  const Layout& L = h->L;
  if (!L.shared_capable)
    return fail(SL_EUNSUPPORTED, "the shared-geometry path needs a 2-D mesh of one order N <= 12");
  if (!h->shared_geometry)
    return fail(SL_EUNSUPPORTED, "the shared-geometry path needs the same drift, diffusion and source factor at every node");
  if (L.MV > 65535) return fail(SL_EUNSUPPORTED, "the shared-geometry path runs at most 65535 samples x components");
  const int N = L.order[0];
  sl::SharedArgs a{};
  a.A = h->A;
  a.B = h->B;
  a.src = h->hsrc[0];
  a.Af = h->Af;
  a.Bf = h->Bf;
  a.ghost = h->ghost;
  a.nbr = h->d_nbr;
  a.xi = h->d_xitab + N * sl::kMaxN;
  a.bw = h->d_bw;
  a.ur = h->d_ur;   // one order in the mesh: its U_r is the first table
  a.ops = h->d_sops;
  a.phi = h->phi;
  a.tr = h->tr;
  a.K = L.K;
  a.ncomp = L.nc;
  a.mass = L.mass ? 1 : 0;
  a.wq = h->d_wqtab + N * sl::kMaxN;
  a.step_ptr = nullptr;
  a.seed = h->desc.seed;
  a.stream = h->desc.stream_id;
  static const char* const names[3] = {"shared_build", "shared_traces", "shared_update"};
  for (int it = 0; it < nsteps; ++it) {
    a.step = h->step + it;
    for (int stage = 0; stage < 3; ++stage) {
      ProfScope ps(h, names[stage]);
      SL_HIP(sl::launch_shared_step(N, stage, a, L.M, h->stream));
    }
  }
  h->step += nsteps;
  return SL_OK;
}

std::string tune_key(const sl_ctx* h) {
  std::ostringstream k;
  const Layout& L = h->L;
  k << "dim=" << L.dim << ";K=" << L.kx << "x" << L.ky << ";orders=";
  for (const auto& g : h->groups) k << g.first << ":" << g.second.second << ",";
  k << ";M=" << L.M << ";nc=" << L.nc << ";prec=" << h->desc.precision << ";refine=" << h->p2.refine << ";bc=" << h->desc.bc
    << ";solver=" << L.solver;
  return k.str();
}

}  // namespace

extern "C" {

int sl_required_bytes(const sl_mesh_desc* desc, size_t* bytes) {
  if (!bytes) return fail(SL_EINVAL, "null output");
  Layout L;
  const int rc = make_layout(desc, L);
  if (rc) return rc;
  *bytes = L.total;
  return SL_OK;
}

int sl_init_mesh(const sl_mesh_desc* desc, void* dev_ws, size_t ws_bytes, void* hip_stream, sl_handle* out) {
  if (!out) return fail(SL_EINVAL, "null output handle");
  *out = nullptr;
  std::unique_ptr<sl_ctx> h(fault_is("host") ? nullptr : new (std::nothrow) sl_ctx());
  if (!h) return fail(SL_ENOMEM, "host allocation failed");
  int rc = make_layout(desc, h->L);
  if (rc) return rc;
  const Layout& L = h->L;
  if (L.dim == 1 && !L.uniform) return fail(SL_EUNSUPPORTED, "1-D meshes need a uniform order");
  if (L.dim == 2 && L.solver == SL_SOLVER_FACTOR && L.maxN > sl::kMaxN2D)
    return fail(SL_EUNSUPPORTED, "the factorisation solver supports N <= 10; use the float64 reference solver for N <= 16");
  if (L.dim == 1 && desc->precision != SL_PREC_FP64)
    return fail(SL_EUNSUPPORTED, "the 1-D fit runs in float64 only (it has no dense contraction to lower)");
  h->desc = *desc;
  h->desc.order = nullptr;
  h->hx = (desc->x1 - desc->x0) / L.kx;
  h->hy = L.dim == 2 ? (desc->y1 - desc->y0) / L.ky : 1.0;
  h->family = desc->nodes == SL_NODES_CG ? 1 : 0;
  h->stream = (hipStream_t)hip_stream;
  for (int N : L.order)
    if (!h->xi_tab.count(N)) h->xi_tab[N] = sl::gauss_nodes(N, h->family);
  h->rec = sl::legendre_recurrence();
  for (int k = 0; k < sl::kMaxN; ++k)
    if (h->rec.a[k] != sl::kLegA[k] || h->rec.b[k] != sl::kLegB[k])
      return fail(SL_EUNSUPPORTED, "the host's Legendre recurrence differs from the compiled constants");
  if (const char* a = std::getenv("SL_1D_FIT")) h->algo_1d = std::strcmp(a, "normal") == 0 ? 1 : 0;
  if (dev_ws) {
    if (ws_bytes < L.total) return fail(SL_ENOMEM, "workspace smaller than sl_required_bytes");
    h->ws = (char*)dev_ws;
  } else {
    void* p = nullptr;
    if (dev_malloc(&p, L.total) != hipSuccess) return fail(SL_ENOMEM, "hipMalloc of the workspace failed");
    h->ws = (char*)p;
    h->own_ws = true;
  }
  h->phi = (double*)(h->ws + L.o_phi);
  h->phi2 = (double*)(h->ws + L.o_phi2);
  h->tr = (double*)(h->ws + L.o_tr);
  h->xi_node = (double*)(h->ws + L.o_xi);
  h->A = (double*)(h->ws + L.o_A);
  h->B = (double*)(h->ws + L.o_B);
  h->src = (double*)(h->ws + L.o_src);
  h->Af = (double*)(h->ws + L.o_Af);
  h->Bf = (double*)(h->ws + L.o_Bf);
  h->ghost = (double*)(h->ws + L.o_ghost);
  h->mean = (double*)(h->ws + L.o_mean);
  h->phi0 = (double*)(h->ws + L.o_phi0);
  h->d_order = (int32_t*)(h->ws + L.o_order);
  h->d_noff = (int64_t*)(h->ws + L.o_noff);
  h->d_eoff = (int64_t*)(h->ws + L.o_eoff);
  h->d_nbr = (int32_t*)(h->ws + L.o_nbr);
  h->d_work = (int32_t*)(h->ws + L.o_work);
  h->d_xitab = (double*)(h->ws + L.o_xitab);
  h->d_ur = (double*)(h->ws + L.o_ur);
  h->d_uroff = (int64_t*)(h->ws + L.o_uroff);
  h->d_interp = (double*)(h->ws + L.o_interp);
  h->d_interpoff = (int64_t*)(h->ws + L.o_interpoff);
  h->d_p1 = (sl::Params1D*)(h->ws + L.o_params);
  h->d_p2 = (sl::Params2D*)(h->ws + L.o_params);
  h->d_step = (int64_t*)(h->ws + L.o_dstep);
  h->d_ctr = (unsigned long long*)(h->ws + L.o_ctr);
  h->d_stats = (unsigned long long*)(h->ws + L.o_stats);
  h->d_nonf = (unsigned long long*)(h->ws + L.o_nonf);
  h->d_mpart = (double*)(h->ws + L.o_mpart);
  h->d_gxinv = (double*)(h->ws + L.o_gxinv);
  h->d_nsp = (double*)(h->ws + L.o_nsp);
  h->d_sops = (double*)(h->ws + L.o_sops);
  h->d_wqtab = (double*)(h->ws + L.o_wqtab);
  h->d_bw = (double*)(h->ws + L.o_bw);
  h->d_z = (double*)(h->ws + L.o_z);
  h->d_wrec = (sl::WorkRec*)(h->ws + L.o_wrec);
  const bool lean = L.dim == 2 && L.solver == SL_SOLVER_REFERENCE && L.nc == 1;
  h->d_rlist = lean ? (uint32_t*)(h->ws + L.o_rlist) : nullptr;
  h->d_rcount = lean ? (unsigned int*)(h->ws + L.o_rcount) : nullptr;
  // element tables, work list grouped by order, node tables, U_r and trace interpolation
  std::vector<int32_t> nbr(4 * (size_t)L.K, -1), work;
  for (int e = 0; e < L.K; ++e) {
    const int ex = e % L.kx, ey = e / L.kx;
    const int dx[4] = {-1, 1, 0, 0}, dy[4] = {0, 0, -1, 1};
    for (int w = 0; w < 4; ++w) {
      int nx = ex + dx[w], ny = ey + dy[w];
      if (desc->bc == SL_BC_PERIODIC) {
        nx = (nx + L.kx) % L.kx;
        ny = (ny + L.ky) % L.ky;
        nbr[4 * e + w] = ny * L.kx + nx;
      } else if (nx >= 0 && nx < L.kx && ny >= 0 && ny < L.ky) {
        nbr[4 * e + w] = ny * L.kx + nx;
      }
    }
  }
  for (auto it = L.orders.rbegin(); it != L.orders.rend(); ++it) {   // largest fits first
    const int N = *it;
    const int64_t first = (int64_t)work.size();
    for (int e = 0; e < L.K; ++e)
      if (L.order[e] == N) work.push_back(e);
    h->groups.push_back({N, {first, (int64_t)work.size() - first}});
  }
  std::vector<double> xitab((sl::kMaxN + 1) * sl::kMaxN, 0.0), wqtab((sl::kMaxN + 1) * sl::kMaxN, 0.0);
  for (int N = 1; N <= sl::kMaxN; ++N) {
    const auto xi = sl::gauss_nodes(N, h->family);
    for (int i = 0; i < N; ++i) xitab[N * sl::kMaxN + i] = xi[i];
  }
  for (int N : L.orders) {
    const auto w = sl::quadrature_weights(h->xi_tab[N]);
    for (int i = 0; i < N; ++i) wqtab[N * sl::kMaxN + i] = w[i];
  }
  std::vector<double> ur(L.ur_doubles + 1, 0.0), interp(L.interp_doubles + 1, 0.0);
  std::vector<int64_t> uroff(sl::kMaxN + 1, 0), interpoff((sl::kMaxN + 1) * (sl::kMaxN + 1), 0);
  if (L.dim == 2) {
    size_t o = 0;
    for (int N : L.orders) {
      const auto U = sl::edge_range_basis(N, h->xi_tab[N]);
      uroff[N] = (int64_t)o;
      std::copy(U.begin(), U.end(), ur.begin() + o);
      o += U.size();
    }
    o = 0;
    for (int Nd : L.orders)
      for (int Ns : L.orders)
        if (Nd != Ns) {
          const auto Lm = sl::lagrange_matrix(h->xi_tab[Ns], h->xi_tab[Nd]);
          interpoff[Nd * (sl::kMaxN + 1) + Ns] = (int64_t)o;
          std::copy(Lm.begin(), Lm.end(), interp.begin() + o);
          o += Lm.size();
        }
  }
  std::vector<double> gx(L.gx_doubles + 1, 0.0);
  if (L.dim == 2) {
    size_t o = 0;
    for (int N : L.orders) {
      const auto G = sl::reference_inverses(h->xi_tab[N]);
      h->gx_off[N] = (int64_t)o;
      std::copy(G.begin(), G.end(), gx.begin() + o);
      o += G.size();
    }
  }
  std::vector<double> nsp(L.nsp_doubles + 1, 0.0);
  if (L.dim == 2) {
    size_t o = 0;
    for (int N : L.orders) {
      const auto T = sl::nullspace_tables(N, h->xi_tab[N]);
      h->nsp_off[N] = (int64_t)o;
      std::copy(T.begin(), T.end(), nsp.begin() + o);
      o += T.size();
    }
  }
  std::vector<double> bw(sl::kMaxN, 0.0);
  {
    const auto w = sl::barycentric_weights(h->xi_tab[L.order[0]]);
    std::copy(w.begin(), w.end(), bw.begin());
  }
  std::vector<int64_t> noff64(L.noff.begin(), L.noff.end() - 1), eoff64(L.eoff.begin(), L.eoff.end() - 1);
  std::vector<int32_t> order32(L.order.begin(), L.order.end());
  // work records (2-D): the element's offsets and, per side, the neighbour's
  // facing trace (across W (E, S, N) the neighbour's E (W, N, S) block of Ns
  // values, packed with Ns); the move-coefficient means come with the step
  // coefficients
  h->work_h = work;
  h->hwrec.assign(L.dim == 2 ? work.size() : 0, sl::WorkRec{});
  for (size_t w = 0; w < h->hwrec.size(); ++w) {
    const int e = work[w];
    sl::WorkRec& r = h->hwrec[w];
    r.noff = L.noff[e];
    r.eoff = L.eoff[e];
    for (int sd = 0; sd < 4; ++sd) {
      const int nb = nbr[4 * (size_t)e + sd];
      const int64_t Ns = nb < 0 ? 0 : L.order[nb];
      r.nbr_tr[sd] = nb < 0 ? -1 : (Ns << 48) | (L.eoff[nb] + (int64_t)(sd ^ 1) * Ns);
    }
  }
  struct Up { void* dst; const void* src; size_t bytes; };
  const Up ups[] = {
      {h->d_order, order32.data(), sizeof(int32_t) * L.K}, {h->d_noff, noff64.data(), sizeof(int64_t) * L.K},
      {h->d_eoff, eoff64.data(), sizeof(int64_t) * L.K}, {h->d_nbr, nbr.data(), sizeof(int32_t) * nbr.size()},
      {h->d_work, work.data(), sizeof(int32_t) * work.size()}, {h->d_xitab, xitab.data(), sizeof(double) * xitab.size()},
      {h->d_ur, ur.data(), sizeof(double) * ur.size()}, {h->d_uroff, uroff.data(), sizeof(int64_t) * uroff.size()},
      {h->d_interp, interp.data(), sizeof(double) * interp.size()},
      {h->d_interpoff, interpoff.data(), sizeof(int64_t) * interpoff.size()},
      {h->d_gxinv, gx.data(), sizeof(double) * gx.size()}, {h->d_nsp, nsp.data(), sizeof(double) * nsp.size()},
      {h->d_bw, bw.data(), sizeof(double) * bw.size()},
      {h->d_wqtab, wqtab.data(), sizeof(double) * wqtab.size()},
      {h->d_wrec, h->hwrec.data(), sizeof(sl::WorkRec) * h->hwrec.size()}};
  for (const auto& u : ups) {
    if (u.bytes == 0) continue;
    if (hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, h->stream) != hipSuccess) {
      if (h->own_ws) (void)hipFree(h->ws);
      return fail(SL_EDEVICE, "table upload failed");
    }
  }
  if (hipStreamSynchronize(h->stream) != hipSuccess) {
    if (h->own_ws) (void)hipFree(h->ws);
    return fail(SL_EDEVICE, "table upload failed");
  }
  // reference coordinates of every node, [nodes][dim]
  std::vector<double> xin(L.nodes * L.dim);
  for (int e = 0; e < L.K; ++e) {
    const int N = L.order[e];
    const auto& xi = h->xi_tab[N];
    const int n = L.dim == 1 ? N : N * N;
    for (int i = 0; i < n; ++i) {
      const int64_t k = L.noff[e] + i;
      xin[k * L.dim + 0] = xi[i % N];
      if (L.dim == 2) xin[k * L.dim + 1] = xi[i / N];
    }
  }
  build_params(h.get());
  hipError_t e1 = hipMemcpyAsync(h->xi_node, xin.data(), sizeof(double) * xin.size(), hipMemcpyHostToDevice, h->stream);
  hipError_t e2 = hipMemsetAsync(h->phi, 0, sizeof(double) * (size_t)L.MV * L.nodes, h->stream);
  hipError_t e4 = L.dim == 2 ? hipMemcpyAsync(h->d_p2, &h->p2, sizeof(sl::Params2D), hipMemcpyHostToDevice, h->stream)
                             : hipMemcpyAsync(h->d_p1, &h->p1, sizeof(sl::Params1D), hipMemcpyHostToDevice, h->stream);
  hipError_t e5 = hipMemsetAsync(h->ws + L.o_dstep, 0, L.o_stats + stats_bytes() - L.o_dstep, h->stream);
  hipError_t e3 = hipStreamSynchronize(h->stream);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess || e5 != hipSuccess) {
    if (h->own_ws) (void)hipFree(h->ws);
    return fail(SL_EDEVICE, "initial upload failed");
  }
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    h->id = g_next_id++;
  }
  *out = h.release();
  return SL_OK;
}

int sl_sizes(sl_handle h, int64_t* nodes, int64_t* edge_points, int64_t* elements, int32_t* ncomp) {
  if (int rc = check_handle(h)) return rc;
  if (nodes) *nodes = h->L.nodes;
  if (edge_points) *edge_points = h->L.edges;
  if (elements) *elements = h->L.K;
  if (ncomp) *ncomp = h->L.nc;
  return SL_OK;
}

int sl_ref_nodes(sl_handle h, int32_t N, double* host_xi) {
  if (int rc = check_handle(h)) return rc;
  if (N < 1 || N > 64 || !host_xi) return fail(SL_EINVAL, "bad order or null output");
  const auto xi = sl::gauss_nodes(N, h->family);
  std::memcpy(host_xi, xi.data(), sizeof(double) * N);
  return SL_OK;
}

int sl_node_coords(sl_handle h, double* xy) {
  if (int rc = check_handle(h)) return rc;
  if (!xy) return fail(SL_EINVAL, "null output");
  const Layout& L = h->L;
  for (int e = 0; e < L.K; ++e) {
    const int N = L.order[e];
    const int ex = e % L.kx, ey = e / L.kx;
    const auto& xi = h->xi_tab[N];
    const int n = L.dim == 1 ? N : N * N;
    for (int i = 0; i < n; ++i) {
      const int64_t k = L.noff[e] + i;
      xy[k * L.dim] = h->desc.x0 + h->hx * (ex + xi[i % N]);
      if (L.dim == 2) xy[k * L.dim + 1] = h->desc.y0 + h->hy * (ey + xi[i / N]);
    }
  }
  return SL_OK;
}

int sl_edge_coords(sl_handle h, double* xy, int32_t* axis) {
  if (int rc = check_handle(h)) return rc;
  const Layout& L = h->L;
  for (int e = 0; e < L.K; ++e) {
    const int N = L.order[e];
    const int ex = e % L.kx, ey = e / L.kx;
    const auto& xi = h->xi_tab[N];
    if (L.dim == 1) {
      for (int w = 0; w < 2; ++w) {
        const int64_t q = L.eoff[e] + w;
        if (xy) xy[q] = h->desc.x0 + h->hx * (ex + (w == 0 ? 0.0 : 1.0));
        if (axis) axis[q] = 0;
      }
    } else {
      for (int w = 0; w < 4; ++w)
        for (int j = 0; j < N; ++j) {
          const int64_t q = L.eoff[e] + w * N + j;
          double rx, ry;
          if (w == 0) { rx = 0.0; ry = xi[j]; }
          else if (w == 1) { rx = 1.0; ry = xi[j]; }
          else if (w == 2) { rx = xi[j]; ry = 0.0; }
          else { rx = xi[j]; ry = 1.0; }
          if (xy) {
            xy[2 * q] = h->desc.x0 + h->hx * (ex + rx);
            xy[2 * q + 1] = h->desc.y0 + h->hy * (ey + ry);
          }
          if (axis) axis[q] = w < 2 ? 0 : 1;
        }
    }
  }
  return SL_OK;
}

int sl_set_fields(sl_handle h, const double* u, const double* D, const double* divu, const double* un,
                  const double* Dn, const double* ghost, const double* phi0) {
  if (int rc = check_handle(h)) return rc;
  const Layout& L = h->L;
  if (!u || !D || !un || !Dn) return fail(SL_EINVAL, "u, D, un and Dn are required");
  if (h->desc.bc == SL_BC_DIRICHLET && !ghost) return fail(SL_EINVAL, "Dirichlet boundaries need ghost values");
  auto finite = [](const double* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(p[i])) return false;
    return true;
  };
  if (!finite(u, L.nodes * L.dim) || !finite(D, L.nodes) || (divu && !finite(divu, L.nodes)) ||
      !finite(un, L.edges) || !finite(Dn, L.edges) || (ghost && !finite(ghost, L.edges)) ||
      (phi0 && !finite(phi0, L.nc * L.nodes)))
    return fail(SL_ENONFINITE, "non-finite field values");
  for (int64_t i = 0; i < L.nodes; ++i)
    if (D[i] < 0) return fail(SL_EINVAL, "D must be >= 0");
  for (int64_t i = 0; i < L.edges; ++i)
    if (Dn[i] < 0) return fail(SL_EINVAL, "Dn must be >= 0");
  h->u.assign(u, u + L.nodes * L.dim);
  h->D.assign(D, D + L.nodes);
  if (divu) h->divu.assign(divu, divu + L.nodes);
  else h->divu.assign(L.nodes, 0.0);
  h->un.assign(un, un + L.edges);
  h->Dn.assign(Dn, Dn + L.edges);
  h->ghost_h.assign(L.edges, 0.0);
  if (ghost) h->ghost_h.assign(ghost, ghost + L.edges);
  SL_HIP(hipMemcpyAsync(h->ghost, h->ghost_h.data(), sizeof(double) * L.edges, hipMemcpyHostToDevice, h->stream));
  if (phi0) {
    SL_HIP(hipMemcpyAsync(h->phi0, phi0, sizeof(double) * L.nc * L.nodes, hipMemcpyHostToDevice, h->stream));
    SL_HIP(sl::launch_broadcast(h->phi, h->phi0, L.M, L.nc * L.nodes, h->stream));
    h->step = 0;
  }
  SL_HIP(hipStreamSynchronize(h->stream));
  h->coeff_valid = false;
  h->fields_set = true;
  return SL_OK;
}

int sl_set_ghost(sl_handle h, const double* ghost) {
  if (int rc = check_handle(h)) return rc;
  if (!h->fields_set) return fail(SL_ESTATE, "sl_set_fields must come before sl_set_ghost");
  if (h->desc.bc != SL_BC_DIRICHLET) return fail(SL_EINVAL, "ghost values need Dirichlet boundaries");
  if (!ghost) return fail(SL_EINVAL, "null ghost values");
  const Layout& L = h->L;
  for (int64_t i = 0; i < L.edges; ++i)
    if (!std::isfinite(ghost[i])) return fail(SL_ENONFINITE, "non-finite ghost values");
  // the device copy may still be read by enqueued steps: wait before overwriting the staging copy
  SL_HIP(hipStreamSynchronize(h->stream));
  h->ghost_h.assign(ghost, ghost + L.edges);
  SL_HIP(hipMemcpyAsync(h->ghost, h->ghost_h.data(), sizeof(double) * L.edges, hipMemcpyHostToDevice, h->stream));
  SL_HIP(hipStreamSynchronize(h->stream));
  return SL_OK;
}

int sl_step(sl_handle h, double dt, int32_t nsteps) {
  if (int rc = check_handle(h)) return rc;
  if (!h->fields_set) return fail(SL_ESTATE, "sl_set_fields must come before sl_step");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(SL_EINVAL, "dt must be finite and > 0");
  if (nsteps < 0) return fail(SL_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return SL_OK;
  if (int rc = update_coefficients(h, dt)) return rc;
  const Layout& L = h->L;
  if (h->sched.shared) return step_shared(h, nsteps);
  if (L.dim == 2 && L.mass && L.solver != SL_SOLVER_REFERENCE)
    return fail(SL_EUNSUPPORTED, "in 2-D the mass constraint runs with the reference solver or on the shared-geometry path");
  if (L.dim == 2) return step_2d({h}, nsteps, h->sched.fused, h->sched.graph, h->sched.grid, h->stream);
  return step_1d(h, nsteps, h->stream);
}

int sl_step_batch(const sl_handle* hs, const double* dts, int32_t nh, int32_t nsteps) {
  if (nh < 0 || nsteps < 0) return fail(SL_EINVAL, "nh and nsteps must be >= 0");
  if (nh == 0 || nsteps == 0) return SL_OK;
  if (!hs || !dts) return fail(SL_EINVAL, "null batch arrays");
  std::vector<sl_ctx*> one, two;
  for (int i = 0; i < nh; ++i) {
    sl_ctx* h = hs[i];
    if (!h) return fail(SL_EINVAL, "null handle in batch");
    for (int j = 0; j < i; ++j)
      if (hs[j] == h) return fail(SL_EINVAL, "a handle appears twice in the batch");
    if (!h->fields_set) return fail(SL_ESTATE, "sl_set_fields must come before sl_step_batch");
    if (!(dts[i] > 0) || !std::isfinite(dts[i])) return fail(SL_EINVAL, "dt must be finite and > 0");
    if (h->stream != hs[0]->stream) return fail(SL_EINVAL, "all handles of a batch must share one stream");
    if (h->L.dim == 2 && ((h->L.mass && h->L.solver != SL_SOLVER_REFERENCE) || h->sched.shared))
      return fail(SL_EUNSUPPORTED, "batches take the general path; a 2-D handle of the shared-geometry schedule, or with the mass constraint and the factorisation solver, steps alone");
    (h->L.dim == 2 ? two : one).push_back(h);
  }
  for (int i = 0; i < nh; ++i)
    if (int rc = update_coefficients(hs[i], dts[i])) return rc;
  hipStream_t st = hs[0]->stream;
  if (!one.empty())
    if (int rc = step_1d_batch(one, nsteps, st)) return rc;
  if (!two.empty())
    if (int rc = step_2d(two, nsteps, two[0]->sched.fused, two[0]->sched.graph, two[0]->sched.grid, st)) return rc;
  return SL_OK;
}

int sl_set_schedule(sl_handle h, const sl_schedule_t* s) {
  if (int rc = check_handle(h)) return rc;
  if (!s) return fail(SL_EINVAL, "null schedule");
  if ((s->fused != 0 && s->fused != 1) || (s->graph != 0 && s->graph != 1) || s->grid < 0 || s->grid > (1 << 24) ||
      (s->shared != 0 && s->shared != 1) || (s->wide != 0 && s->wide != 1))
    return fail(SL_EINVAL, "schedule: fused, graph, shared and wide are 0 or 1, 0 <= grid <= 2^24");
  h->sched = *s;
  return SL_OK;
}

int sl_get_schedule(sl_handle h, sl_schedule_t* s) {
  if (int rc = check_handle(h)) return rc;
  if (!s) return fail(SL_EINVAL, "null output");
  *s = h->sched;
  return SL_OK;
}

int sl_autotune(sl_handle h, double dt, int32_t trial_steps, const char* cache_path, sl_schedule_t* out) {
  if (int rc = check_handle(h)) return rc;
  if (!h->fields_set) return fail(SL_ESTATE, "sl_set_fields must come before sl_autotune");
  if (!(dt > 0) || !std::isfinite(dt) || trial_steps < 1) return fail(SL_EINVAL, "dt > 0 and trial_steps >= 1 required");
  const Layout& L = h->L;
  if (L.dim == 1) {   // one resident launch for all steps: nothing to choose
    if (out) *out = h->sched;
    return SL_OK;
  }
  const std::string key = tune_key(h);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      sl_schedule_t c{};
      if (ls >> k >> c.fused >> c.graph >> c.grid >> c.ms_per_step && k == key) {
        if (!(ls >> c.wide)) c.wide = 0;   // lines written before the fit shape was a choice
        if (int rc = sl_set_schedule(h, &c)) return rc;
        if (out) *out = h->sched;
        return SL_OK;
      }
    }
  }
  if (int rc = update_coefficients(h, dt)) return rc;
  // keep the samples and the step counter; trial steps advance both
  const size_t bytes = sizeof(double) * (size_t)L.MV * L.nodes;
  void* snap = nullptr;
  if (dev_malloc(&snap, bytes) != hipSuccess) return fail(SL_ENOMEM, "no device memory for the autotuner's copy of the samples");
  const int64_t step0 = h->step;
  const sl_schedule_t keep = h->sched;
  const bool prof = h->profile;
  h->profile = false;
  int rc = SL_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<sl_schedule_t> cand;
  // the wide fit shape changes the per-order reference-solver kernels of
  // orders up to 12 only
  bool shape = L.solver == SL_SOLVER_REFERENCE;
  if (shape) {
    shape = false;
    for (const auto& g : h->groups) shape = shape || (g.first <= 12 && g.second.second > 0);
  }
  for (int fused = 0; fused <= 1; ++fused)
    for (int graph = 0; graph <= 1; ++graph) {
      if (!fused) {
        cand.push_back({0, graph, 0, 0.f, 0, 0});
        if (shape) cand.push_back({0, graph, 0, 0.f, 0, 1});
      } else {
        cand.push_back({1, graph, 0, 0.f});                    // every resident workgroup
        cand.push_back({1, graph, device_cus(), 0.f});         // one per compute unit
        cand.push_back({1, graph, 2 * device_cus(), 0.f});
      }
    }
  sl_schedule_t best{0, 0, 0, 0.f};
  float best_ms = -1.f;
  auto fail_dev = [&](hipError_t e) { return fail(SL_EDEVICE, std::string("autotune: ") + hipGetErrorString(e)); };
  hipError_t e = hipMemcpyAsync(snap, h->phi, bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) rc = fail_dev(e);
  for (size_t c = 0; c < cand.size() && rc == SL_OK; ++c) {
    h->sched = cand[c];
    rc = step_2d({h}, 1, cand[c].fused, cand[c].graph, cand[c].grid, h->stream);   // warm-up (and capture)
    if (rc) break;
    if ((e = hipEventRecord(e0, h->stream)) != hipSuccess) { rc = fail_dev(e); break; }
    rc = step_2d({h}, trial_steps, cand[c].fused, cand[c].graph, cand[c].grid, h->stream);
    if (rc) break;
    if ((e = hipEventRecord(e1, h->stream)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
      rc = fail_dev(e);
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= trial_steps;
    if (best_ms < 0 || ms < best_ms) {
      best_ms = ms;
      best = cand[c];
      best.ms_per_step = ms;
    }
  }
  // restore the samples and the step counter whatever happened
  e = hipMemcpyAsync(h->phi, snap, bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(snap);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  h->step = step0;
  h->profile = prof;
  if (rc == SL_OK && e != hipSuccess) rc = fail_dev(e);
  if (rc) {
    h->sched = keep;
    return rc;
  }
  h->sched = best;
  if (cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    o << key << " " << best.fused << " " << best.graph << " " << best.grid << " " << best.ms_per_step << " " << best.wide << "\n";
  }
  if (out) *out = best;
  return SL_OK;
}

int sl_mean(sl_handle h, double* out, int32_t out_is_device) {
  if (int rc = check_handle(h)) return rc;
  if (!out) return fail(SL_EINVAL, "null output");
  const Layout& L = h->L;
  double* dst = out_is_device ? out : h->mean;
  {
    ProfScope ps(h, "mean");
    SL_HIP(sl::launch_mean(h->phi, dst, h->d_mpart, L.M, L.nc * L.nodes, h->d_nonf, h->stream));
  }
  if (!out_is_device) {
    unsigned long long bad = 0;
    SL_HIP(hipMemcpyAsync(out, h->mean, sizeof(double) * L.nc * L.nodes, hipMemcpyDeviceToHost, h->stream));
    SL_HIP(hipMemcpyAsync(&bad, h->d_nonf, sizeof(bad), hipMemcpyDeviceToHost, h->stream));
    SL_HIP(hipStreamSynchronize(h->stream));
    if (bad) return fail(SL_ENONFINITE, std::to_string(bad) + " non-finite sample values at the nodes");
  }
  return SL_OK;
}

int sl_pdf(sl_handle h, double lo, double hi, int32_t nbins, uint32_t* counts, int32_t out_is_device) {
  if (int rc = check_handle(h)) return rc;
  if (!counts) return fail(SL_EINVAL, "null output");
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo)) return fail(SL_EINVAL, "need finite lo < hi");
  if (!std::isfinite((hi - lo) / (double)std::max(nbins, 1)) || !((hi - lo) / std::max(nbins, 1) > 0.0))
    return fail(SL_EINVAL, "bin width (hi - lo) / nbins must be a positive finite number");
  if (nbins < 1 || nbins > sl::kPdfMaxBins) return fail(SL_EINVAL, "nbins must be in [1, 254]");
  const Layout& L = h->L;
  if (L.M > 0xffffffffll) return fail(SL_EINVAL, "more samples than a 32-bit count holds");
  const size_t bytes = sizeof(uint32_t) * (size_t)L.nc * L.nodes * (nbins + 2);
  uint32_t* dst = counts;
  void* tmp = nullptr;
  if (!out_is_device) {
    if (dev_malloc(&tmp, bytes) != hipSuccess) return fail(SL_ENOMEM, "no device memory for the histogram");
    dst = (uint32_t*)tmp;
  }
  hipError_t e;
  {
    ProfScope ps(h, "pdf");
    e = sl::launch_pdf(h->phi, dst, L.M, L.nc * L.nodes, lo, hi, nbins, h->stream);
  }
  if (e == hipSuccess && !out_is_device) {
    e = hipMemcpyAsync(counts, dst, bytes, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  }
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return fail(SL_EDEVICE, std::string("pdf: ") + hipGetErrorString(e));
  return SL_OK;
}

int sl_reseed(sl_handle h) {
  if (int rc = check_handle(h)) return rc;
  if (!h->fields_set) return fail(SL_ESTATE, "sl_set_fields must come before sl_reseed");
  const Layout& L = h->L;
  {
    ProfScope ps(h, "reseed");
    SL_HIP(sl::launch_mean(h->phi, h->mean, h->d_mpart, L.M, L.nc * L.nodes, h->d_nonf, h->stream));
    SL_HIP(sl::launch_broadcast(h->phi, h->mean, L.M, L.nc * L.nodes, h->stream));
  }
  return SL_OK;
}

int sl_get_samples(sl_handle h, int64_t s0, int64_t ns, double* out, int32_t out_is_device) {
  if (int rc = check_handle(h)) return rc;
  const Layout& L = h->L;
  if (!out || s0 < 0 || ns < 0 || s0 + ns > L.M) return fail(SL_EINVAL, "sample range out of bounds");
  SL_HIP(hipMemcpyAsync(out, h->phi + s0 * L.nc * L.nodes, sizeof(double) * ns * L.nc * L.nodes,
                        out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
  if (!out_is_device) SL_HIP(hipStreamSynchronize(h->stream));
  return SL_OK;
}

int sl_set_samples(sl_handle h, int64_t s0, int64_t ns, const double* in, int32_t in_is_device) {
  if (int rc = check_handle(h)) return rc;
  const Layout& L = h->L;
  if (!in || s0 < 0 || ns < 0 || s0 + ns > L.M) return fail(SL_EINVAL, "sample range out of bounds");
  SL_HIP(hipMemcpyAsync(h->phi + s0 * L.nc * L.nodes, in, sizeof(double) * ns * L.nc * L.nodes,
                        in_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
  SL_HIP(hipStreamSynchronize(h->stream));
  return SL_OK;
}

int sl_get_step(sl_handle h, int64_t* n) {
  if (int rc = check_handle(h)) return rc;
  if (!n) return fail(SL_EINVAL, "null output");
  *n = h->step;
  return SL_OK;
}

int sl_set_step(sl_handle h, int64_t n) {
  if (int rc = check_handle(h)) return rc;
  if (n < 0 || n > 0xFFFFFFFFll) return fail(SL_EINVAL, "step counter out of range");
  h->step = n;
  return SL_OK;
}

int sl_debug_normals(sl_handle h, int64_t n, int64_t s0, int64_t ns, double* out) {
  if (int rc = check_handle(h)) return rc;
  if (!out || ns < 0 || s0 < 0 || n < 0) return fail(SL_EINVAL, "bad arguments");
  if (ns == 0) return SL_OK;
  double* d = nullptr;
  if (dev_malloc((void**)&d, sizeof(double) * 2 * ns) != hipSuccess) return fail(SL_ENOMEM, "no device memory for the normals");
  hipError_t e = sl::launch_debug_normals(d, h->desc.seed, h->desc.stream_id, n, s0, ns, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d, sizeof(double) * 2 * ns, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(SL_EDEVICE, hipGetErrorString(e));
  return SL_OK;
}

int sl_debug_positions(sl_handle h, double dt, double* out) {
  if (int rc = check_handle(h)) return rc;
  if (!h->fields_set) return fail(SL_ESTATE, "fields not set");
  if (!out || !(dt > 0)) return fail(SL_EINVAL, "bad arguments");
  if (int rc = update_coefficients(h, dt)) return rc;
  const Layout& L = h->L;
  const size_t n = (size_t)L.M * L.nodes * L.dim;
  double* d = nullptr;
  if (dev_malloc((void**)&d, sizeof(double) * n) != hipSuccess) return fail(SL_ENOMEM, "no device memory for the positions");
  hipError_t e = sl::launch_debug_positions(d, h->xi_node, h->A, h->B, L.dim, L.nodes, L.M, h->desc.seed,
                                            h->desc.stream_id, h->step, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(SL_EDEVICE, hipGetErrorString(e));
  return SL_OK;
}

int sl_profile(sl_handle h, int32_t enable) {
  if (int rc = check_handle(h)) return rc;
  drain_events(h);
  if (enable) h->kstats.clear();
  h->profile = enable != 0;
  return SL_OK;
}

int sl_kernel_time(sl_handle h, const char* name, int64_t* launches, double* ms) {
  if (int rc = check_handle(h)) return rc;
  if (!name) return fail(SL_EINVAL, "null name");
  drain_events(h);
  auto it = h->kstats.find(name);
  if (launches) *launches = it == h->kstats.end() ? 0 : it->second.launches;
  if (ms) *ms = it == h->kstats.end() ? 0.0 : it->second.ms;
  return SL_OK;
}

int sl_diag(sl_handle h, sl_diag_t* out) {
  if (int rc = check_handle(h)) return rc;
  if (!out) return fail(SL_EINVAL, "null output");
  std::memset(out, 0, sizeof(*out));
  out->steps = h->step;
  out->samples = h->L.M;
  out->ncomp = h->L.nc;
  out->nodes = h->L.nodes;
  out->edge_points = h->L.edges;
  out->max_disp_ratio = h->max_disp_ratio;
  out->precision = h->desc.precision;
  out->refine_iters = h->desc.refine_iters >= 0 ? h->desc.refine_iters
                      : (h->desc.precision == SL_PREC_FP32_REFINE ? 2 : h->desc.precision == SL_PREC_BF16SPLIT_REFINE ? 3 : 0);
  out->device_bytes = h->L.total;
  out->solver = h->L.dim == 2 ? h->L.solver : 0;
  std::vector<unsigned long long> st(sl::kStatSlots * sl::kStatStride);
  unsigned long long nonf = 0;
  SL_HIP(hipStreamSynchronize(h->stream));
  SL_HIP(hipMemcpy(st.data(), h->d_stats, stats_bytes(), hipMemcpyDeviceToHost));
  SL_HIP(hipMemcpy(&nonf, h->d_nonf, sizeof(nonf), hipMemcpyDeviceToHost));
  unsigned long long rmax = 0;
  for (int k = 0; k < sl::kStatSlots; ++k) {
    const unsigned long long* c = st.data() + (size_t)k * sl::kStatStride;
    for (int ph = 0; ph < 2; ++ph) {
      out->solver_iterations[ph] += (int64_t)c[2 * ph];
      out->solver_unconverged[ph] += (int64_t)c[2 * ph + 1];
    }
    out->escapes += (int64_t)c[sl::kStatEscapes];
    out->solver_fallbacks += (int64_t)c[sl::kStatFallbacks];
    rmax = std::max(rmax, c[sl::kStatResidual]);
  }
  std::memcpy(&out->max_residual, &rmax, sizeof(double));
  out->nonfinite = (int64_t)nonf;
  return SL_OK;
}

int sl_sync(sl_handle h) {
  if (int rc = check_handle(h)) return rc;
  SL_HIP(hipStreamSynchronize(h->stream));
  return SL_OK;
}

int sl_set_stream(sl_handle h, void* hip_stream) {
  if (int rc = check_handle(h)) return rc;
  drain_events(h);
  SL_HIP(hipStreamSynchronize(h->stream));
  h->stream = (hipStream_t)hip_stream;
  return SL_OK;
}

int sl_mem_info(size_t* free_bytes, size_t* total_bytes) {
  if (!free_bytes || !total_bytes) return fail(SL_EINVAL, "null output");
  SL_HIP(hipMemGetInfo(free_bytes, total_bytes));
  return SL_OK;
}

const char* sl_last_error(void) { return g_last_error.c_str(); }

int sl_mean_noalloc(const double* phi, int64_t samples, int64_t nodes, double* out, uint64_t* nonfinite,
                    void* hip_stream) {
  if (!phi || !out) return fail(SL_EINVAL, "null sample or output pointer");
  if (samples < 1 || nodes < 1) return fail(SL_EINVAL, "samples and nodes must be >= 1");
  if (nodes > ((int64_t)1 << 40) || samples > ((int64_t)1 << 40) || (double)samples * (double)nodes > 9.0e15)
    return fail(SL_EINVAL, "sizes beyond the supported range (samples, nodes <= 2^40, samples * nodes <= 9e15)");
  const int64_t C = sl::mean_chunks(samples, nodes);
  if (C > 1 && C * nodes > sl::kMeanScratchDoubles)
    return fail(SL_EINVAL, "partial sums exceed the allocation-free scratch bound");
  double* part = nullptr;
  if (C > 1) SL_HIP(sl::mean_scratch_device_ptr(&part));
  SL_HIP(sl::launch_mean(phi, out, part, samples, nodes, (unsigned long long*)nonfinite, (hipStream_t)hip_stream));
  return SL_OK;
}

int sl_destroy(sl_handle h) {
  if (!h) return SL_OK;
  (void)hipStreamSynchronize(h->stream);
  drain_events(h);
  purge_graphs(h->id);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->own_ws && h->ws) (void)hipFree(h->ws);
  delete h;
  return SL_OK;
}

}  // extern "C"
