"""Host logic of the serving loop (admission by footprint, slots, isolation of a
failing request, latency accounting) against a stand-in backend on the CPU.
The GPU test of the loop (each result the same alone and in the mix) is in
test_gpu_serve.py."""
import numpy as np
import pytest

from paper_2009_07340_amd import serve, workloads as W


class FakeBackend:
    """Same function names as the binding; a handle is a dict.  Footprint =
    8 bytes per node value; a step advances a per-handle counter."""

    class SLError(RuntimeError):
        def __init__(self, msg, code=-3):
            super().__init__(msg)
            self.code = code

    def __init__(self, free=10 ** 9, fail_dims=(), nan_ids=(), batch_fault=None):
        self.free = free
        self.live = {}
        self.next = 1
        self.batches = []
        self.fail_dims = fail_dims
        self.nan_ids = set(nan_ids)
        # batch_fault(call index, handles) -> None, or (code, handles advanced before the error)
        self.batch_fault = batch_fault
        self.calls = 0

    def make_desc(self, dim, kx, ky, box, order, bc, samples, seed, precision):
        N = int(order) if np.isscalar(order) else int(np.max(order))
        return dict(dim=dim, nodes=kx * ky * N ** dim, samples=samples, seed=seed)

    def sl_required_bytes(self, d):
        return 8 * d["nodes"] * d["samples"]

    def sl_mem_info(self):
        return self.free, self.free

    def sl_init_mesh(self, d, ws, nbytes, stream):
        if d["dim"] in self.fail_dims:
            raise self.SLError("unsupported")
        h = self.next
        self.next += 1
        self.live[h] = dict(desc=d, steps=0)
        return h

    def sl_sizes(self, h):
        return self.live[h]["desc"]["nodes"], 1, 1

    def sl_node_coords(self, h, dim):
        return np.zeros((self.live[h]["desc"]["nodes"], dim))

    def sl_edge_coords(self, h, dim):
        return np.zeros((1, dim)), np.zeros(1, dtype=np.int32)

    def sl_set_fields(self, h, *a):
        pass

    def sl_set_schedule(self, h, *a):
        pass

    def sl_set_stream(self, h, s):
        pass

    def sl_step_batch(self, hs, dts, n):
        assert len(set(hs)) == len(hs)
        self.calls += 1
        fault = self.batch_fault(self.calls, list(hs)) if self.batch_fault else None
        if fault is not None:
            code, advanced = fault
            for h in advanced:              # the part of the batch that ran before the error
                self.live[h]["steps"] += n
            raise self.SLError("injected batch failure", code)
        self.batches.append(list(hs))
        for h in hs:
            self.live[h]["steps"] += n

    def sl_get_step(self, h):
        return self.live[h]["steps"]

    def sl_sync(self, h):
        pass

    def sl_mean(self, h):
        d = self.live[h]["desc"]
        v = float(self.live[h]["steps"])
        return np.full(d["nodes"], np.nan if d["seed"] in self.nan_ids else v)

    def sl_destroy(self, h):
        del self.live[h]


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 0.001
        return self.t

    def sleep(self, s):
        self.t += s


def _reqs(n, dim=1, K=8, N=4, M=16, steps=10, gap=0.01):
    out = []
    for i in range(n):
        wl = W.c1_1d_const() if dim == 1 else W.c3_2d_const()
        wl.kx, wl.ky, wl.order, wl.samples, wl.seed = K, (1 if dim == 1 else K), N, M, 1000 + i
        out.append(serve.Request(i, i * gap, wl, 1e-4, steps))
    return out


def test_every_request_completes_with_its_own_step_count():
    fb, clk = FakeBackend(), Clock()
    reqs = _reqs(10, steps=7) + _reqs(5, steps=23, gap=0.003)
    for i, r in enumerate(reqs):
        r.id = i
    srv = serve.Server(fb, budget_bytes=10 ** 8, max_active=4, chunk_steps=5, clock=clk, sleep=clk.sleep)
    srv.run(reqs)
    assert all(r.error is None for r in reqs)
    for r in reqs:
        assert np.all(r.mean == r.steps), (r.id, r.mean[0], r.steps)
        assert r.done >= r.admitted >= r.arrival
    assert max(len(b) for b in fb.batches) <= 4
    assert srv.peak_active == 4
    assert not fb.live and srv.used == 0


def test_admission_respects_the_memory_budget_and_rejects_oversize():
    fb, clk = FakeBackend(), Clock()
    reqs = _reqs(6, K=8, N=4, M=16)           # 8*32*16 = 4096 B each
    big = _reqs(1, K=64, N=16, M=64)[0]       # far above the budget
    big.id = 99
    srv = serve.Server(fb, budget_bytes=3 * 4096, max_active=10, chunk_steps=3, clock=clk, sleep=clk.sleep)
    srv.run(reqs + [big])
    assert "exceeds the budget" in big.error
    assert srv.peak_used <= 3 * 4096
    assert max(len(b) for b in fb.batches) <= 3
    assert all(r.mean is not None for r in reqs)


def test_a_failing_request_does_not_poison_the_batch():
    fb, clk = FakeBackend(fail_dims=(2,), nan_ids={1003}), Clock()
    reqs = _reqs(6) + _reqs(2, dim=2, K=2, N=3)
    for i, r in enumerate(reqs):
        r.id = i
    srv = serve.Server(fb, budget_bytes=10 ** 8, max_active=8, chunk_steps=4, clock=clk, sleep=clk.sleep)
    srv.run(reqs)
    assert all("admission" in r.error for r in reqs[6:])
    assert reqs[3].error == "non-finite result"
    assert all(r.mean is not None for i, r in enumerate(reqs[:6]) if i != 3)
    s = serve.summarize(reqs)
    assert s["completed"] == 5 and s["failed"] == 3
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_late_arrivals_join_a_running_batch():
    fb, clk = FakeBackend(), Clock()
    reqs = _reqs(2, steps=200, gap=0.0) + _reqs(2, steps=5, gap=0.0)
    reqs[2].arrival = reqs[3].arrival = 0.05
    for i, r in enumerate(reqs):
        r.id = i
    srv = serve.Server(fb, budget_bytes=10 ** 8, max_active=8, chunk_steps=2, clock=clk, sleep=clk.sleep)
    srv.run(reqs)
    joined = [b for b in fb.batches if len(b) == 4]
    assert joined, "late requests never shared a batch with running ones"
    assert reqs[2].done < reqs[0].done


def test_stream_requests_keep_the_specified_shapes():
    stream = W.serving_requests(n=50, kmax=64, mmax=128)
    for prec in ("fp64", "fp32_refine"):
        reqs = serve.requests_from_stream(stream, precision=prec)
        for r, d in zip(reqs, stream):
            assert (r.wl.dim, r.wl.kx, r.wl.ky, r.wl.samples, r.steps) == (d["dim"], d["kx"], d["ky"], d["M"], d["steps"])
            assert r.precision == ("fp64" if d["dim"] == 1 else prec)


def test_a_batch_that_fails_midway_never_steps_a_request_twice():
    """A device error after part of a batch ran: requests whose step counter
    advanced keep going; the others may hold partly advanced state and fail
    instead of being stepped again."""
    def fault(call, hs):
        return (-3, hs[:2]) if call == 3 and len(hs) >= 4 else None
    fb, clk = FakeBackend(batch_fault=fault), Clock()
    reqs = _reqs(5, steps=12, gap=0.0)
    srv = serve.Server(fb, budget_bytes=10 ** 8, max_active=8, chunk_steps=4, clock=clk, sleep=clk.sleep)
    srv.run(reqs)
    ok = [r for r in reqs if r.error is None]
    bad = [r for r in reqs if r.error is not None]
    assert len(ok) == 2 and len(bad) == 3
    for r in ok:                        # exactly the requested steps: none repeated
        assert np.all(r.mean == r.steps), (r.id, r.mean[0])
    assert all("partly advanced" in r.error for r in bad)
    assert not fb.live and srv.used == 0


def test_a_batch_rejected_by_its_argument_checks_is_retried_request_by_request():
    """SL_EINVAL before anything was enqueued: every request is stepped alone once."""
    def fault(call, hs):
        return (-1, []) if call == 2 else None
    fb, clk = FakeBackend(batch_fault=fault), Clock()
    reqs = _reqs(4, steps=8, gap=0.0)
    srv = serve.Server(fb, budget_bytes=10 ** 8, max_active=8, chunk_steps=4, clock=clk, sleep=clk.sleep)
    srv.run(reqs)
    assert all(r.error is None for r in reqs)
    for r in reqs:
        assert np.all(r.mean == r.steps), (r.id, r.mean[0])
