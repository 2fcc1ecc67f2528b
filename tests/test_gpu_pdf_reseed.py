"""Per-node PDF by binning (sl_pdf) and re-seeding (sl_reseed) on the GPU against
the oracle, through the C ABI.  Bin counts are integers decided by float64
arithmetic done the same way on both sides: they must match exactly."""
import numpy as np
import pytest

from oracle import sl
from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _handle(B, wl, a, M):
    desc = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, wl.order, bc=wl.bc, samples=M, seed=wl.seed)
    h = B.sl_init_mesh(desc)
    B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
    return h


@pytest.mark.parametrize("K,M,nbins", [(16, 64, 10), (16, 5000, 254), (256, 300, 1), (3, 7, 33)])
def test_pdf_counts_equal_the_oracle_exactly(B, K, M, nbins):
    wl = W.c1_1d_const()
    wl.kx = K
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, M)
    try:
        g = np.random.default_rng(K * 31 + M)
        x = g.standard_normal((M, mesh.total_nodes))
        lo, hi = -1.7, 2.1
        w = (hi - lo) / nbins
        # values on the edges, next to them and non-finite ones
        edge = lo + w * np.arange(nbins + 1)
        x.flat[:edge.size] = edge
        x.flat[edge.size:2 * edge.size] = np.nextafter(edge, -np.inf)
        x.flat[2 * edge.size] = np.nan
        x.flat[2 * edge.size + 1] = np.inf
        x.flat[2 * edge.size + 2] = -np.inf
        B.sl_set_samples(h, 0, x)
        got = B.sl_pdf(h, lo, hi, nbins)
    finally:
        B.sl_destroy(h)
    want = sl.pdf_counts(x, lo, hi, nbins)
    assert np.array_equal(got.astype(np.int64), want)
    assert int(got.sum()) == int(np.isfinite(x).sum())


def test_pdf_of_an_evolved_ensemble(B):
    wl = W.c1_1d_const()
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, 64)
    try:
        B.sl_step(h, wl.dt, 40)
        x = B.sl_get_samples(h, 0, 64)
        got = B.sl_pdf(h, 0.0, 1.0, 20)
    finally:
        B.sl_destroy(h)
    assert np.array_equal(got.astype(np.int64), sl.pdf_counts(x, 0.0, 1.0, 20))


@pytest.mark.parametrize("lo,hi,nbins", [(1.0, 1.0, 4), (2.0, 1.0, 4), (0.0, 1.0, 0), (0.0, 1.0, 255),
                                          (0.0, float("inf"), 4), (float("nan"), 1.0, 4)])
def test_pdf_rejects_bad_bins(B, lo, hi, nbins):
    wl = W.c1_1d_const()
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, 4)
    try:
        with pytest.raises(B.SLError) as ei:
            B.sl_pdf(h, lo, hi, nbins)
        assert ei.value.code == B.SL_EINVAL
    finally:
        B.sl_destroy(h)


@pytest.mark.parametrize("dim", [1, 2])
def test_reseeding_matches_the_oracle(B, dim):
    """Eq. re-seed every 3 steps (sl_step then sl_reseed) against the oracle's run(reseed_every=3)."""
    if dim == 1:
        wl = W.c2_1d_sine()
        wl.kx, wl.order, wl.dt, M = 12, 7, 2e-6, 9
    else:
        wl = W.c4_2d_rotation(kx=3, ky=3, samples=5, steps=7)
        wl.order, wl.dt, M = 6, 1e-4, 5
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, M)
    try:
        for chunk in (3, 3, 1):
            B.sl_step(h, wl.dt, chunk)
            if chunk == 3:
                B.sl_reseed(h)
        got = B.sl_get_samples(h, 0, M)
        assert B.sl_get_step(h) == 7
    finally:
        B.sl_destroy(h)
    ref = sl.run(mesh, f, phi0, wl.dt, 7, wl.seed, np.arange(M), reseed_every=3)
    err = rel_l2(got, ref)
    node = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"re-seeding {dim}-D: rel L2 {err:.2e}, max node {node:.2e}")
    assert err < 1e-11 and node < 1e-11
