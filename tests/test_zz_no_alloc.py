"""The allocation-free sample mean (sl_mean_noalloc) against sl_mean, through the
C ABI: bitwise equal on two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _mean_via_handle(B, K, M, seed):
    """sl_mean of a 1-D handle holding random samples; returns (samples, mean)."""
    wl = W.c1_1d_const()
    wl.kx, wl.samples = K, M
    mesh, f, phi0, a = oracle_inputs(wl)
    desc = B.make_desc(1, K, order=wl.order, samples=M, seed=wl.seed)
    h = B.sl_init_mesh(desc)
    try:
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], None, a["phi0"])
        x = np.random.default_rng(seed).standard_normal((M, mesh.total_nodes)) + 1.0
        B.sl_set_samples(h, 0, x)
        return x, B.sl_mean(h)
    finally:
        B.sl_destroy(h)


@pytest.mark.parametrize("sizes", [((256, 1000), (16, 300)), ((16, 64), (16, 40)), ((256, 512), (3, 5))])
def test_no_alloc_mean_equals_sl_mean_on_two_calls(B, sizes):
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    for call, (K, M) in enumerate(sizes):
        x, want = _mean_via_handle(B, K, M, seed=17 + call)
        phi = torch.from_numpy(x).to(dev)
        out = torch.full((x.shape[1],), np.nan, dtype=torch.float64, device=dev)
        bad = torch.full((1,), 12345, dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        B.sl_mean_noalloc(phi.data_ptr(), M, x.shape[1], out.data_ptr(), bad.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(f"call {call}: K={K} M={M}: max |noalloc - sl_mean| = {np.max(np.abs(got - want)):.3e}")
        assert np.array_equal(got, want)
        assert int(bad.item()) == 0
        # a non-finite value is counted
        phi[M - 1, 0] = float("nan")
        B.sl_mean_noalloc(phi.data_ptr(), M, x.shape[1], out.data_ptr(), bad.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        assert int(bad.item()) == 1
