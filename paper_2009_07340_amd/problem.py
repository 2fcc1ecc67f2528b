"""One library handle for one workload: descriptor, fields from the library's own
coordinates, stepping and readback.  Argument marshalling only; every step of
the method runs in the HIP library."""
import numpy as np

from . import binding as B


class Problem:
    def __init__(self, wl, precision="fp64", samples=None, seed=None, stream_id=0, dev_ws=None,
                 ws_bytes=0, hip_stream=None, nodes="gl", refine_iters=-1, solver="auto", ncomp=1):
        self.wl = wl
        self.M = int(samples if samples is not None else wl.samples)
        self.desc = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, wl.order if np.isscalar(wl.order) else wl.order_array(),
                                nodes=nodes, bc=wl.bc, samples=self.M,
                                seed=wl.seed if seed is None else seed, stream_id=stream_id,
                                precision=precision, refine_iters=refine_iters, solver=solver, ncomp=ncomp)
        self.ncomp = int(ncomp)
        self.h = B.sl_init_mesh(self.desc, dev_ws, ws_bytes, hip_stream)
        self.nodes, self.edges, self.K = B.sl_sizes(self.h)

    @staticmethod
    def required_bytes(wl, precision="fp64", samples=None, solver="auto", ncomp=1):
        d = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, wl.order if np.isscalar(wl.order) else wl.order_array(),
                        bc=wl.bc, samples=int(samples if samples is not None else wl.samples), precision=precision,
                        solver=solver, ncomp=ncomp)
        return B.sl_required_bytes(d)

    def coords(self):
        xy = B.sl_node_coords(self.h, self.wl.dim)
        exy, axis = B.sl_edge_coords(self.h, self.wl.dim)
        return xy, exy, axis

    def set_fields(self, t=0.0, with_phi0=True):
        xy, exy, axis = self.coords()
        a = self.wl.sample_fields(xy, exy, axis, t)
        phi0 = None
        if with_phi0:
            # component c starts from the workload's field scaled by 1 + c/10 (synthetic components)
            phi0 = np.concatenate([a["phi0"] * (1.0 + 0.1 * c) for c in range(self.ncomp)])
        B.sl_set_fields(self.h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], phi0)
        return a

    def step(self, dt, nsteps):
        B.sl_step(self.h, dt, nsteps)

    def mean(self):
        return B.sl_mean(self.h)

    def samples(self, s0=0, ns=None):
        return B.sl_get_samples(self.h, s0, self.M - s0 if ns is None else ns)

    def sync(self):
        B.sl_sync(self.h)

    def close(self):
        if self.h is not None:
            B.sl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
