"""ctypes binding of the C ABI in include/sl.h (argument marshalling only).

Every function of the header is exposed under the same name.  Arrays are
numpy float64/int32 arrays (host) or integer device pointers (torch
``tensor.data_ptr()``).  A negative status raises ``SLError`` with the
library's message.  The library must have been built (``__graft_entry__.build``
or ``python -m paper_2009_07340_amd.build_lib``); without it, importing this
module raises ImportError: there is no fallback implementation.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsl_mi355x.so")

SL_OK, SL_EINVAL, SL_ENOMEM, SL_EDEVICE, SL_ENONFINITE, SL_ESTATE, SL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SL_BC_PERIODIC, SL_BC_DIRICHLET = 0, 1
SL_CONSTRAIN_BOUNDARY, SL_CONSTRAIN_BOUNDARY_MASS = 0, 1
SL_NODES_GL, SL_NODES_CG = 0, 1
SL_PREC_FP64, SL_PREC_FP32_REFINE, SL_PREC_BF16SPLIT_REFINE = 0, 1, 2

SL_SOLVER_AUTO, SL_SOLVER_FACTOR, SL_SOLVER_REFERENCE = 0, 1, 2
SOLVERS = {"auto": SL_SOLVER_AUTO, "factor": SL_SOLVER_FACTOR, "reference": SL_SOLVER_REFERENCE}

PRECISIONS = {"fp64": SL_PREC_FP64, "fp32_refine": SL_PREC_FP32_REFINE, "bf16split_refine": SL_PREC_BF16SPLIT_REFINE}


class sl_mesh_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("kx", C.c_int32), ("ky", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("n_uniform", C.c_int32), ("order", C.POINTER(C.c_int32)), ("nodes", C.c_int32),
                ("bc", C.c_int32), ("samples", C.c_int64), ("seed", C.c_uint64), ("stream_id", C.c_uint32),
                ("precision", C.c_int32), ("refine_iters", C.c_int32), ("solver", C.c_int32),
                ("max_iter", C.c_int32), ("tol", C.c_double), ("constraints", C.c_int32), ("ncomp", C.c_int32)]


class sl_diag_t(C.Structure):
    _fields_ = [("steps", C.c_int64), ("samples", C.c_int64), ("nodes", C.c_int64), ("edge_points", C.c_int64),
                ("max_disp_ratio", C.c_double), ("precision", C.c_int32), ("refine_iters", C.c_int32),
                ("device_bytes", C.c_size_t), ("solver", C.c_int32), ("solver_iterations", C.c_int64 * 2),
                ("solver_unconverged", C.c_int64 * 2), ("escapes", C.c_int64), ("max_residual", C.c_double),
                ("nonfinite", C.c_int64), ("ncomp", C.c_int32), ("solver_fallbacks", C.c_int64)]


class sl_schedule_t(C.Structure):
    _fields_ = [("fused", C.c_int32), ("graph", C.c_int32), ("grid", C.c_int32), ("ms_per_step", C.c_float),
                ("shared", C.c_int32), ("wide", C.c_int32)]


class SLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sl error {code}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library {LIB_PATH} is missing; build it with __graft_entry__.build()")
# A process can hold only one HIP runtime: PyTorch wheels carry their own, and a
# second one loaded beside it cannot open the device.  When torch is installed
# its runtime is loaded first, so the library binds to it and device pointers
# and streams from torch are valid here.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = C.CDLL(LIB_PATH)

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_SIGS = {
    "sl_required_bytes": [C.POINTER(sl_mesh_desc), C.POINTER(C.c_size_t)],
    "sl_init_mesh": [C.POINTER(sl_mesh_desc), _P, C.c_size_t, _P, C.POINTER(_P)],
    "sl_sizes": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)],
    "sl_node_coords": [_P, _P],
    "sl_edge_coords": [_P, _P, _P],
    "sl_ref_nodes": [_P, C.c_int32, _P],
    "sl_set_fields": [_P, _P, _P, _P, _P, _P, _P, _P],
    "sl_step": [_P, C.c_double, C.c_int32],
    "sl_set_ghost": [_P, _P],
    "sl_step_batch": [_P, _P, C.c_int32, C.c_int32],
    "sl_mean": [_P, _P, C.c_int32],
    "sl_reseed": [_P],
    "sl_pdf": [_P, C.c_double, C.c_double, C.c_int32, _P, C.c_int32],
    "sl_get_samples": [_P, C.c_int64, C.c_int64, _P, C.c_int32],
    "sl_set_samples": [_P, C.c_int64, C.c_int64, _P, C.c_int32],
    "sl_get_step": [_P, C.POINTER(C.c_int64)],
    "sl_set_step": [_P, C.c_int64],
    "sl_debug_normals": [_P, C.c_int64, C.c_int64, C.c_int64, _P],
    "sl_debug_positions": [_P, C.c_double, _P],
    "sl_profile": [_P, C.c_int32],
    "sl_kernel_time": [_P, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)],
    "sl_diag": [_P, C.POINTER(sl_diag_t)],
    "sl_sync": [_P],
    "sl_set_stream": [_P, _P],
    "sl_mem_info": [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
    "sl_set_schedule": [_P, C.POINTER(sl_schedule_t)],
    "sl_get_schedule": [_P, C.POINTER(sl_schedule_t)],
    "sl_autotune": [_P, C.c_double, C.c_int32, C.c_char_p, C.POINTER(sl_schedule_t)],
    "sl_destroy": [_P],
    "sl_mean_noalloc": [_P, C.c_int64, C.c_int64, _P, _P, _P],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.sl_last_error.argtypes = []
_lib.sl_last_error.restype = C.c_char_p

EXPORTED = sorted(list(_SIGS) + ["sl_last_error"])


def _check(rc):
    if rc != SL_OK:
        raise SLError(rc, _lib.sl_last_error().decode())
    return rc


def _ptr(a):
    """Host numpy array or device integer pointer -> void*."""
    if a is None:
        return None
    if isinstance(a, int):
        return C.c_void_p(a)
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def make_desc(dim, kx, ky=1, box=(0.0, 1.0, 0.0, 1.0), order=8, nodes="gl", bc="periodic", samples=1,
              seed=0, stream_id=0, precision="fp64", refine_iters=-1, solver="auto", max_iter=0, tol=0.0, ncomp=1,
              mass=False):
    d = sl_mesh_desc()
    d.dim, d.kx, d.ky = dim, kx, ky if dim == 2 else 1
    d.x0, d.x1, d.y0, d.y1 = (float(v) for v in box)
    keep = None
    if np.isscalar(order):
        d.n_uniform, d.order = int(order), None
    else:
        keep = np.ascontiguousarray(order, dtype=np.int32)
        d.n_uniform = int(keep[0])
        d.order = keep.ctypes.data_as(C.POINTER(C.c_int32))
    d.nodes = SL_NODES_GL if nodes == "gl" else SL_NODES_CG
    d.bc = SL_BC_PERIODIC if bc == "periodic" else SL_BC_DIRICHLET
    d.samples, d.seed, d.stream_id = int(samples), int(seed) & (2 ** 64 - 1), int(stream_id)
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.refine_iters = int(refine_iters)
    d.solver = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    d.max_iter, d.tol = int(max_iter), float(tol)
    d.ncomp = int(ncomp)
    d.constraints = 1 if mass else 0
    d._keep = keep
    return d


# --- the C ABI, one wrapper per function ---------------------------------------------

def sl_required_bytes(desc):
    out = C.c_size_t()
    _check(_lib.sl_required_bytes(C.byref(desc), C.byref(out)))
    return out.value


def sl_init_mesh(desc, dev_ws=None, ws_bytes=0, hip_stream=None):
    h = C.c_void_p()
    _check(_lib.sl_init_mesh(C.byref(desc), _ptr(dev_ws), ws_bytes, _ptr(hip_stream), C.byref(h)))
    return h


def sl_sizes(h):
    """(nodes, edge points, elements) of one component."""
    n, e, k, c = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
    _check(_lib.sl_sizes(h, C.byref(n), C.byref(e), C.byref(k), C.byref(c)))
    return n.value, e.value, k.value


def sl_ncomp(h):
    c = C.c_int32()
    _check(_lib.sl_sizes(h, None, None, None, C.byref(c)))
    return c.value


def _row(h):
    """Values per sample: nodes x components."""
    nodes, _, _ = sl_sizes(h)
    return nodes * sl_ncomp(h)


def sl_node_coords(h, dim):
    nodes, _, _ = sl_sizes(h)
    out = np.empty((nodes, dim))
    _check(_lib.sl_node_coords(h, _ptr(out)))
    return out


def sl_edge_coords(h, dim):
    _, edges, _ = sl_sizes(h)
    out = np.empty((edges, dim))
    axis = np.empty(edges, dtype=np.int32)
    _check(_lib.sl_edge_coords(h, _ptr(out), _ptr(axis)))
    return out, axis


def sl_ref_nodes(h, N):
    out = np.empty(N)
    _check(_lib.sl_ref_nodes(h, int(N), _ptr(out)))
    return out


def sl_set_fields(h, u, D, divu, un, Dn, ghost=None, phi0=None):
    nodes, edges, _ = sl_sizes(h)
    arrs = [_f64(u), _f64(D, nodes), None if divu is None else _f64(divu, nodes), _f64(un, edges),
            _f64(Dn, edges), None if ghost is None else _f64(ghost, edges),
            None if phi0 is None else _f64(phi0, nodes * sl_ncomp(h))]
    _check(_lib.sl_set_fields(h, *[_ptr(a) for a in arrs]))


def sl_set_ghost(h, ghost):
    _, edges, _ = sl_sizes(h)
    _check(_lib.sl_set_ghost(h, _ptr(_f64(ghost, edges))))


def sl_step(h, dt, nsteps):
    _check(_lib.sl_step(h, float(dt), int(nsteps)))


def sl_step_batch(hs, dts, nsteps):
    arr = (C.c_void_p * len(hs))(*[x.value if isinstance(x, C.c_void_p) else x for x in hs])
    d = _f64(dts, len(hs))
    _check(_lib.sl_step_batch(C.cast(arr, C.c_void_p), _ptr(d), len(hs), int(nsteps)))


def sl_mean(h, out=None):
    """Host mean (numpy) when out is None; else out is a device pointer (int)."""
    if out is None:
        res = np.empty(_row(h))
        _check(_lib.sl_mean(h, _ptr(res), 0))
        return res
    _check(_lib.sl_mean(h, _ptr(out), 1))
    return None


def sl_pdf(h, lo, hi, nbins, out=None):
    """Per-node histogram counts (nodes, nbins + 2) as uint32 numpy; or into a device pointer."""
    if out is None:
        res = np.empty((_row(h), int(nbins) + 2), dtype=np.uint32)
        _check(_lib.sl_pdf(h, float(lo), float(hi), int(nbins), _ptr(res), 0))
        return res
    _check(_lib.sl_pdf(h, float(lo), float(hi), int(nbins), _ptr(out), 1))
    return None


def sl_reseed(h):
    _check(_lib.sl_reseed(h))


def sl_get_samples(h, s0, ns, out=None):
    nodes = _row(h)
    if out is None:
        res = np.empty((ns, nodes))
        _check(_lib.sl_get_samples(h, int(s0), int(ns), _ptr(res), 0))
        return res
    _check(_lib.sl_get_samples(h, int(s0), int(ns), _ptr(out), 1))
    return None


def sl_set_samples(h, s0, data):
    if isinstance(data, tuple):      # (device pointer, ns)
        ptr, ns = data
        _check(_lib.sl_set_samples(h, int(s0), int(ns), _ptr(ptr), 1))
        return
    nodes = _row(h)
    a = _f64(data)
    ns = a.size // nodes
    _check(_lib.sl_set_samples(h, int(s0), ns, _ptr(a), 0))


def sl_get_step(h):
    n = C.c_int64()
    _check(_lib.sl_get_step(h, C.byref(n)))
    return n.value


def sl_set_step(h, n):
    _check(_lib.sl_set_step(h, int(n)))


def sl_debug_normals(h, n, s0, ns):
    out = np.empty((ns, 2))
    _check(_lib.sl_debug_normals(h, int(n), int(s0), int(ns), _ptr(out)))
    return out


def sl_debug_positions(h, dt, samples, dim):
    nodes, _, _ = sl_sizes(h)
    out = np.empty((samples, nodes, dim))
    _check(_lib.sl_debug_positions(h, float(dt), _ptr(out)))
    return out


def sl_profile(h, enable):
    _check(_lib.sl_profile(h, 1 if enable else 0))


def sl_kernel_time(h, name):
    n, ms = C.c_int64(), C.c_double()
    _check(_lib.sl_kernel_time(h, name.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value


def sl_diag(h):
    d = sl_diag_t()
    _check(_lib.sl_diag(h, C.byref(d)))
    out = {}
    for k, _ in d._fields_:
        v = getattr(d, k)
        out[k] = list(v) if isinstance(v, C.Array) else v
    return out


def _sched_dict(s):
    return {"fused": s.fused, "graph": s.graph, "grid": s.grid, "ms_per_step": s.ms_per_step, "shared": s.shared,
            "wide": s.wide}


def sl_set_schedule(h, fused=0, graph=0, grid=0, shared=0, wide=0):
    s = sl_schedule_t(int(fused), int(graph), int(grid), 0.0, int(shared), int(wide))
    _check(_lib.sl_set_schedule(h, C.byref(s)))


def sl_get_schedule(h):
    s = sl_schedule_t()
    _check(_lib.sl_get_schedule(h, C.byref(s)))
    return _sched_dict(s)


def sl_autotune(h, dt, trial_steps=3, cache_path=None):
    s = sl_schedule_t()
    path = None if cache_path is None else os.fspath(cache_path).encode()
    _check(_lib.sl_autotune(h, float(dt), int(trial_steps), path, C.byref(s)))
    return _sched_dict(s)


def sl_mean_noalloc(phi_dev, samples, nodes, out_dev, nonfinite_dev=None, hip_stream=None):
    """Allocation-free mean of a device array [samples][nodes] into out_dev (device pointers as ints)."""
    _check(_lib.sl_mean_noalloc(_ptr(phi_dev), int(samples), int(nodes), _ptr(out_dev), _ptr(nonfinite_dev),
                                _ptr(hip_stream)))


def sl_sync(h):
    _check(_lib.sl_sync(h))


def sl_set_stream(h, hip_stream):
    _check(_lib.sl_set_stream(h, _ptr(hip_stream)))


def sl_mem_info():
    f, t = C.c_size_t(), C.c_size_t()
    _check(_lib.sl_mem_info(C.byref(f), C.byref(t)))
    return f.value, t.value


def sl_last_error():
    return _lib.sl_last_error().decode()


def sl_destroy(h):
    _check(_lib.sl_destroy(h))
