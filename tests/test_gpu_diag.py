"""Diagnostics of the C ABI on the GPU: escape counts (against the oracle's
positions), solver residuals, the non-finite flag of the sample mean, injected
allocation failures, and the two-pass sample mean against the oracle."""
import numpy as np
import pytest

from oracle import sl
from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _handle(B, wl, a, solver="auto", precision="fp64"):
    order = wl.order if np.isscalar(wl.order) else wl.order_array()
    desc = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=wl.samples, seed=wl.seed,
                       solver=solver, precision=precision)
    h = B.sl_init_mesh(desc)
    B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
    return h


def _exact_mean_bound(B, x):
    """The mean from an exactly rounded sum (math.fsum per node, then / M) and the
    error any summation order may add in float64: gamma_{M-1} sum|x| / M per node
    (u = 2^-53, gamma_k = k u / (1 - k u)), plus the roundings of the divisions and
    of the exact sum."""
    import math
    M = x.shape[0]
    ref = np.array([math.fsum(col) for col in x.T]) / M
    u = 2.0 ** -53
    gamma = (M - 1) * u / (1 - (M - 1) * u)
    bound = gamma * np.sum(np.abs(x), axis=0) / M * (1 + u) + 3 * u * np.abs(ref)
    return ref, bound


def _oracle_escapes(mesh, f, wl, dt, steps, samples):
    """Coordinates of moved nodes outside [0, 1], counted per sample, step, node and direction."""
    n = 0
    for k in range(steps):
        z = sl.wiener_normals(mesh, wl.seed, k, np.arange(samples))
        xs = sl.positions(mesh, f, dt, z)
        n += int(np.count_nonzero((xs < 0.0) | (xs > 1.0)))
    return n


@pytest.mark.parametrize("K,algo", [(16, "nodal"), (16, "normal"), (300, "nodal")])
def test_escape_count_1d_matches_the_oracle(B, K, algo, monkeypatch):
    if algo == "normal":
        monkeypatch.setenv("SL_1D_FIT", "normal")
    wl = W.c1_1d_const()
    wl.kx, wl.samples = K, 40
    dt = 1e-4 * (16.0 / K) ** 2 * 4          # a one-sigma move of ~0.05 h: outer nodes leave
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a)
    try:
        B.sl_step(h, dt, 12)
        d = B.sl_diag(h)
    finally:
        B.sl_destroy(h)
    want = _oracle_escapes(mesh, f, wl, dt, 12, wl.samples)
    print(f"1-D K={K} {algo}: escapes {d['escapes']} (oracle {want})")
    assert want > 0
    assert d["escapes"] == want


@pytest.mark.parametrize("solver,precision", [("reference", "fp64"), ("factor", "fp64"), ("factor", "fp32_refine")])
def test_escape_count_and_residual_2d(B, solver, precision):
    wl = W.c4_2d_rotation(kx=4, ky=4, samples=6, steps=4)
    wl.order = np.array([6, 8, 10, 6, 8, 6, 10, 8, 10, 6, 8, 6, 8, 10, 6, 8], dtype=np.int32)
    dt = 1e-3                                 # moves of ~0.02 h: the outer nodes of N = 10 leave
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, solver=solver, precision=precision)
    try:
        B.sl_step(h, dt, 4)
        d = B.sl_diag(h)
    finally:
        B.sl_destroy(h)
    want = _oracle_escapes(mesh, f, wl, dt, 4, wl.samples)
    print(f"2-D {solver} {precision}: escapes {d['escapes']} (oracle {want}), max residual {d['max_residual']:.3e}")
    assert want > 0
    assert d["escapes"] == want
    if solver == "reference":
        assert d["solver_unconverged"] == [0, 0]
        assert 0.0 < d["max_residual"] <= 1e-13          # the solver's own stopping bound
    elif precision == "fp64":
        assert d["max_residual"] == 0.0
    else:
        assert 0.0 < d["max_residual"] < 1e-9


def test_no_escapes_for_small_moves(B):
    wl = W.c1_1d_const()
    wl.samples = 16
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a)
    try:
        B.sl_step(h, 1e-7, 20)
        assert B.sl_diag(h)["escapes"] == _oracle_escapes(mesh, f, wl, 1e-7, 20, 16) == 0
    finally:
        B.sl_destroy(h)


@pytest.mark.parametrize("K,M", [(16, 64), (256, 1000), (16, 1)])
def test_nonfinite_samples_are_flagged_by_the_mean(B, K, M):
    wl = W.c1_1d_const()
    wl.kx, wl.samples = K, M
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a)
    try:
        nodes = mesh.total_nodes
        s = B.sl_get_samples(h, 0, M)
        bad = s.copy()
        bad[M - 1, 3] = np.nan
        bad[M // 2, nodes - 1] = np.inf
        B.sl_set_samples(h, 0, bad)
        with pytest.raises(B.SLError) as ei:
            B.sl_mean(h)
        assert ei.value.code == B.SL_ENONFINITE
        nexp = 2 if M > 1 else 2
        assert B.sl_diag(h)["nonfinite"] == nexp
        B.sl_set_samples(h, 0, s)
        m = B.sl_mean(h)
        assert B.sl_diag(h)["nonfinite"] == 0
        ref, bound = _exact_mean_bound(B, s)
        assert np.all(np.abs(m - ref) <= bound)
    finally:
        B.sl_destroy(h)


@pytest.mark.parametrize("K,M", [(256, 1000), (256, 33), (16, 4096), (3, 7)])
def test_two_pass_mean_matches_the_oracle(B, K, M):
    """Random sample values through sl_set_samples: the chunked mean is within the
    float64 summation bound of the exactly summed mean (as the oracle's sequential
    mean is), and repeated calls are bitwise equal."""
    wl = W.c1_1d_const()
    wl.kx, wl.samples = K, M
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a)
    try:
        x = np.random.default_rng(K * 7919 + M).standard_normal((M, mesh.total_nodes)) + 3.0
        B.sl_set_samples(h, 0, x)
        m1 = B.sl_mean(h)
        m2 = B.sl_mean(h)
        assert np.array_equal(m1, m2)
        ref, bound = _exact_mean_bound(B, x)
        assert np.all(np.abs(m1 - ref) <= bound)
        assert np.all(np.abs(sl.mean(x) - ref) <= bound)
    finally:
        B.sl_destroy(h)


def test_mean_of_one_sample_is_the_sample(B):
    wl = W.c1_1d_const()
    wl.samples = 1
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a)
    try:
        B.sl_step(h, wl.dt, 5)
        assert np.array_equal(B.sl_mean(h), B.sl_get_samples(h, 0, 1)[0])
    finally:
        B.sl_destroy(h)


def test_injected_allocation_failures_leave_the_handle_working(B, monkeypatch):
    """SL_FAULT=alloc: the autotuner's and the debug calls' device allocations fail
    with SL_ENOMEM, free device memory is unchanged, and the handle then steps
    exactly as an untouched one."""
    wl = W.c4_2d_rotation(kx=4, ky=4, samples=4, steps=2)
    wl.order = 6
    mesh, f, phi0, a = oracle_inputs(wl)
    h1, h2 = _handle(B, wl, a), _handle(B, wl, a)
    try:
        B.sl_sync(h1)
        free0, _ = B.sl_mem_info()
        monkeypatch.setenv("SL_FAULT", "alloc")
        for call in (lambda: B.sl_autotune(h1, wl.dt, 1), lambda: B.sl_debug_positions(h1, wl.dt, 4, 2),
                     lambda: B.sl_debug_normals(h1, 0, 0, 4), lambda: B.sl_init_mesh(B.make_desc(1, 4, order=4))):
            with pytest.raises(B.SLError) as ei:
                call()
            assert ei.value.code == B.SL_ENOMEM
        monkeypatch.delenv("SL_FAULT")
        free1, _ = B.sl_mem_info()
        assert free1 == free0
        B.sl_step(h1, wl.dt, 3)
        B.sl_step(h2, wl.dt, 3)
        assert np.array_equal(B.sl_get_samples(h1, 0, 4), B.sl_get_samples(h2, 0, 4))
        assert B.sl_get_step(h1) == 3
    finally:
        B.sl_destroy(h1)
        B.sl_destroy(h2)
