"""Continuous-batching request loop over the C ABI.

Independent drift-diffusion problems arrive over time.  A request is
admitted when a slot is free and its device footprint (``sl_required_bytes``:
samples, traces, fields, tables) fits in what the admitted requests leave of
the memory budget; its particle and field state then stays resident on the
device until it finishes.  Every iteration advances all admitted requests by
a common chunk of steps in ONE ``sl_step_batch`` call (the 2-D fits of one
order from every request share one launch per phase, or with ``fused`` all
orders share one persistent launch; 1-D problems of one order share one
resident launch), so requests that arrive while others run join the next iteration and
their work overlaps on the device.  While a chunk runs, the host prepares and
uploads newly admitted requests on a separate stream.

Each request's result is the sample mean of its field at the nodes (eq.
averaged); it does not depend on what else was in the batch (the Philox
counters are per request, per sample and per step), which the tests check bit
for bit.  A request that fails (unsupported shape, allocation failure,
non-finite result) is reported with its error and leaves the others untouched.

The module is a driver: all arithmetic of the method runs in the HIP library.
"""
from collections import deque
from dataclasses import dataclass, field
import time

import numpy as np

from . import workloads as W

# status codes of the C ABI (include/sl.h) that argument checks return before
# anything is enqueued
_EINVAL, _ESTATE = -1, -5


@dataclass
class Request:
    id: int
    arrival: float               # seconds after the start of the run
    wl: object                   # workloads.Workload
    dt: float
    steps: int
    precision: str = "fp64"
    # filled in by the server
    footprint: int = 0
    admitted: float = None
    done: float = None
    error: str = None
    mean: np.ndarray = None
    nodes: int = 0
    remaining: int = 0
    h: object = field(default=None, repr=False)

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival

    @property
    def node_updates(self):
        return self.nodes * self.wl.samples * self.steps


def requests_from_stream(stream, precision="fp64", steps_scale=1.0):
    """Request objects from ``workloads.serving_requests`` dicts.  precision is
    the 2-D mode: "fp64" runs the reference-preconditioned solver (every order
    up to 16; the fastest 2-D path), the mixed modes run the factorisation
    solver (orders up to 10).  The 1-D fit has no dense contraction and runs in
    float64 whatever the requested mode."""
    out = []
    for r in stream:
        wl = W.request_workload(r)
        steps = max(1, int(round(r["steps"] * steps_scale)))
        out.append(Request(r["id"], r["arrival"], wl, r["dt"], steps,
                           "fp64" if r["dim"] == 1 else precision))
    return out


class Server:
    """backend: the binding module (or a stand-in with the same functions)."""

    def __init__(self, backend=None, budget_bytes=None, max_active=32, chunk_steps=16, graph=True, fused=False,
                 max_bypass_wait=5.0, batch_stream=None, admit_stream=None, clock=time.perf_counter,
                 sleep=time.sleep):
        if backend is None:
            from . import binding as backend
        self.B = backend
        if budget_bytes is None:
            free, _ = self.B.sl_mem_info()
            budget_bytes = int(0.9 * free)
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.chunk_steps = int(chunk_steps)
        self.graph = 1 if graph else 0
        self.fused = 1 if fused else 0
        self.max_bypass_wait = float(max_bypass_wait)
        self.batch_stream = batch_stream
        self.admit_stream = admit_stream
        self.clock = clock
        self.sleep = sleep
        self.used = 0
        self.peak_used = 0
        self.iterations = 0
        self.peak_active = 0
        self.batch_log = []          # request ids of every batched call

    # ---------------------------------------------------------------- requests
    def _desc(self, r):
        wl = r.wl
        order = wl.order if np.isscalar(wl.order) else wl.order_array()
        return self.B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=wl.samples,
                                seed=wl.seed, precision=r.precision)

    def footprint(self, r):
        if not r.footprint:
            r.footprint = int(self.B.sl_required_bytes(self._desc(r)))
        return r.footprint

    def _start(self, r):
        """Create the handle on the admission stream, upload fields, join the batch stream."""
        B = self.B
        h = B.sl_init_mesh(self._desc(r), None, 0, self.admit_stream)
        try:
            nodes, _, _ = B.sl_sizes(h)
            xy = B.sl_node_coords(h, r.wl.dim)
            exy, axis = B.sl_edge_coords(h, r.wl.dim)
            a = r.wl.sample_fields(xy, exy, axis, 0.0)
            B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
            B.sl_set_schedule(h, self.fused, self.graph, 0)
            B.sl_set_stream(h, self.batch_stream)
        except Exception:
            B.sl_destroy(h)
            raise
        r.h, r.nodes, r.remaining = h, nodes, r.steps

    def _admit(self, queue, n_active, now):
        """First fit in arrival order; later requests may pass a waiting one
        until it has waited max_bypass_wait seconds."""
        admitted = []
        blocked_head = False
        for r in list(queue):
            if n_active + len(admitted) >= self.max_active:
                break
            try:
                fp = self.footprint(r)
            except Exception as e:          # invalid descriptor
                r.error = f"rejected: {e}"
                queue.remove(r)
                continue
            if fp > self.budget:
                r.error = f"rejected: footprint {fp} B exceeds the budget {self.budget} B"
                queue.remove(r)
                continue
            if self.used + fp > self.budget:
                if now - r.arrival >= self.max_bypass_wait:
                    blocked_head = True
                if blocked_head:
                    break
                continue
            queue.remove(r)
            try:
                self._start(r)
            except Exception as e:
                r.error = f"failed at admission: {e}"
                continue
            r.admitted = now
            self.used += fp
            self.peak_used = max(self.peak_used, self.used)
            admitted.append(r)
        return admitted

    def _retire(self, r, now):
        try:
            m = self.B.sl_mean(r.h)
            if np.all(np.isfinite(m)):
                r.mean = m
            else:
                r.error = "non-finite result"
        except Exception as e:
            r.error = f"failed at readback: {e}"
        r.done = now
        self.B.sl_destroy(r.h)
        r.h = None
        self.used -= r.footprint

    # ---------------------------------------------------------------- loop
    def run(self, requests):
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue, active = [], []
        t0 = self._t0 = self.clock()
        while pending or queue or active:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            launched = False
            if active:
                chunk = min(self.chunk_steps, min(r.remaining for r in active))
                self.batch_log.append([r.id for r in active])
                before = [self.B.sl_get_step(r.h) for r in active]
                try:
                    self.B.sl_step_batch([r.h for r in active], [r.dt for r in active], chunk)
                    launched = True
                except Exception as err:
                    launched = self._recover(active, before, chunk, err)
                for r in active:
                    r.remaining -= chunk
                self.iterations += 1
            new = self._admit(queue, len(active), self.clock() - t0)
            if launched:
                live = [r for r in active if r.h is not None]
                if live:
                    self.B.sl_sync(live[0].h)
            now = self.clock() - t0
            still = []
            for r in active:
                if r.h is None:
                    continue
                if r.remaining <= 0:
                    self._retire(r, now)
                else:
                    still.append(r)
            active = still + new
            self.peak_active = max(self.peak_active, len(active))
            if not active and not queue and pending:
                self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
            elif not active and queue and not new:
                # nothing runs and nothing fits: only possible if the budget shrank
                for r in queue:
                    r.error = "rejected: no memory to admit"
                queue.clear()
        return requests

    def _recover(self, active, before, chunk, err):
        """A batch that raised.  A request whose step counter advanced by the chunk
        finished it.  When the batch failed its argument checks (SL_EINVAL or
        SL_ESTATE, raised before anything is enqueued) and no counter moved, no
        step ran: each request is stepped again alone, so one bad request cannot
        poison the rest.  Otherwise a request whose counter did not advance may
        hold a partly advanced state (some of its launches ran) and is failed,
        never stepped again.  Returns whether any request holds enqueued work."""
        code = getattr(err, "code", None)
        steps = [self.B.sl_get_step(r.h) for r in active]
        nothing_ran = code in (_EINVAL, _ESTATE) and steps == before
        launched = False
        for r, b, now_step in zip(active, before, steps):
            if now_step == b + chunk:
                launched = True
                continue
            if nothing_ran:
                try:
                    self.B.sl_step_batch([r.h], [r.dt], chunk)
                    launched = True
                    continue
                except Exception as e:
                    msg = f"failed in step: {e}"
            else:
                msg = f"failed in step: the batch failed ({err}) and this request's state may be partly advanced"
            self._fail(r, msg)
        return launched

    def _fail(self, r, msg):
        r.error = msg
        try:
            self.B.sl_destroy(r.h)
        finally:
            r.h = None
            self.used -= r.footprint
            r.done = self.clock() - self._t0


def summarize(requests, makespan=None):
    done = [r for r in requests if r.mean is not None]
    lat = np.array([r.latency for r in done]) if done else np.zeros(0)
    wait = np.array([r.admitted - r.arrival for r in done]) if done else np.zeros(0)
    if makespan is None and done:
        makespan = max(r.done for r in done) - min(r.arrival for r in requests)
    nu = float(sum(r.node_updates for r in done))
    return {
        "requests": len(requests),
        "completed": len(done),
        "failed": sum(1 for r in requests if r.error),
        "errors": sorted({r.error.split(":")[0] for r in requests if r.error}),
        "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
        "p50_queue_wait_s": float(np.percentile(wait, 50)) if wait.size else None,
        "makespan_s": makespan,
        "node_updates_per_s": nu / makespan if makespan else None,
        "completed_per_s": len(done) / makespan if makespan else None,
    }
