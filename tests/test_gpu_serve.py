"""The serving loop on the GPU: requests of the specified stream's shapes
(scaled to test size) arrive while others run, share batched launches, and
each result is bitwise the one the request gets when it runs alone."""
import numpy as np
import pytest

from oracle import sl
from paper_2009_07340_amd import serve, workloads as W

from helpers import oracle_mesh, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _alone(B, r):
    wl = r.wl
    order = wl.order if np.isscalar(wl.order) else wl.order_array()
    d = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=wl.samples, seed=wl.seed,
                    precision=r.precision)
    h = B.sl_init_mesh(d)
    try:
        xy = B.sl_node_coords(h, wl.dim)
        exy, axis = B.sl_edge_coords(h, wl.dim)
        a = wl.sample_fields(xy, exy, axis, 0.0)
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
        B.sl_step(h, r.dt, r.steps)
        return B.sl_mean(h), a
    finally:
        B.sl_destroy(h)


def test_each_request_is_the_same_alone_and_in_the_mix(B):
    stream = W.serving_requests(n=40, rate=50.0, kmax=36, mmax=48)
    reqs = serve.requests_from_stream(stream, steps_scale=0.04)
    for r in reqs:
        r.arrival *= 0.25          # 200 requests/s
    reqs[0].steps = 3000           # a long request that is on the device while the others arrive
    srv = serve.Server(B, budget_bytes=2 << 30, max_active=12, chunk_steps=4)
    srv.run(reqs)
    s = serve.summarize(reqs)
    print(s, f"peak active {srv.peak_active}, iterations {srv.iterations}", flush=True)
    ok = [r for r in reqs if r.mean is not None]
    assert len(ok) == len(reqs), [r.error for r in reqs if r.error]
    # later arrivals were admitted into the running batch of the long request
    joined = {i for ids in srv.batch_log if 0 in ids for i in ids if i != 0}
    assert len(joined) >= 20, sorted(joined)
    assert srv.peak_active >= 2
    for r in ok:
        want, _ = _alone(B, r)
        assert np.array_equal(r.mean, want), (r.id, r.wl.dim, r.precision)
    # the smallest 1-D request against the oracle
    r = min((r for r in ok if r.wl.dim == 1), key=lambda r: r.node_updates)
    mesh = oracle_mesh(r.wl)
    _, a = _alone(B, r)
    f = sl.Fields(u=a["u"], D=a["D"], divu=a["divu"], un=a["un"], Dn=a["Dn"], ghost=a["ghost"])
    ref = sl.run(mesh, f, a["phi0"], r.dt, r.steps, r.wl.seed, np.arange(r.wl.samples))
    assert rel_l2(r.mean, sl.mean(ref)) < 1e-11


def test_mixed_precision_requests_in_the_mix(B):
    """2-D requests in the float32 + refinement mode (factorisation solver) mixed
    with float64 ones; orders above 10 are rejected cleanly in that mode."""
    stream = W.serving_requests(n=24, rate=100.0, kmax=25, mmax=32, seed=5)
    reqs = serve.requests_from_stream(stream, precision="fp32_refine", steps_scale=0.03)
    srv = serve.Server(B, budget_bytes=1 << 30, max_active=8, chunk_steps=3)
    srv.run(reqs)
    for r in reqs:
        if r.error:
            assert "admission" in r.error and r.wl.dim == 2 and int(r.wl.order) > 10, r.error
        else:
            want, _ = _alone(B, r)
            assert np.array_equal(r.mean, want), r.id
    assert sum(r.mean is not None for r in reqs) >= 12


def test_serving_with_separate_admission_and_batch_streams(B):
    torch = pytest.importorskip("torch")
    s_batch, s_admit = torch.cuda.Stream(), torch.cuda.Stream()
    stream = W.serving_requests(n=12, rate=200.0, kmax=16, mmax=32, seed=77)
    reqs = serve.requests_from_stream(stream, steps_scale=0.03)
    srv = serve.Server(B, budget_bytes=1 << 30, max_active=6, chunk_steps=3,
                       batch_stream=s_batch.cuda_stream, admit_stream=s_admit.cuda_stream)
    srv.run(reqs)
    assert all(r.mean is not None for r in reqs), [r.error for r in reqs]
    for r in reqs:
        want, _ = _alone(B, r)
        assert np.array_equal(r.mean, want), r.id
