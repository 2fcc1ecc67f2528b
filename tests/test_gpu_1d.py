"""GPU parity of the 1-D path against the FP64 oracle (runs through the C ABI)."""
import numpy as np
import pytest

from oracle import rng, sl
from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-11      # relative L2, float64 path (measurement plan)


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _handle(B, wl, mesh, arrays, samples=None, seed=None, stream_id=0):
    desc = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, wl.order if np.isscalar(wl.order) else wl.order_array(),
                       bc=wl.bc, samples=samples or wl.samples, seed=wl.seed if seed is None else seed,
                       stream_id=stream_id)
    h = B.sl_init_mesh(desc)
    a = arrays
    B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
    return h


def test_device_normals_bitwise_equal_oracle(B):
    wl = W.c1_1d_const()
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, mesh, a, seed=0x123456789ABCDEF, stream_id=7)
    try:
        for step in (0, 1, 999, 2 ** 32 - 1):
            got = B.sl_debug_normals(h, step, 5, 3000)
            za, zb = rng.normal_pair(0x123456789ABCDEF, step, np.arange(5, 3005), stream=7)
            assert np.array_equal(got[:, 0], za), step
            assert np.array_equal(got[:, 1], zb), step
    finally:
        B.sl_destroy(h)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_node_coordinates_and_positions_bitwise(B, name):
    wl = W.WORKLOADS[name]()
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, mesh, a, samples=16)
    try:
        np.testing.assert_array_equal(B.sl_node_coords(h, 1), mesh.node_coords())
        exy, axis = B.sl_edge_coords(h, 1)
        np.testing.assert_array_equal(exy, mesh.edge_coords())
        for N in (2, 8, 12, 16):
            np.testing.assert_array_equal(B.sl_ref_nodes(h, N), np.asarray(__import__("oracle.tables").tables.nodes(N)))
        B.sl_set_step(h, 37)
        got = B.sl_debug_positions(h, wl.dt, 16, 1)
        z = sl.wiener_normals(mesh, wl.seed, 37, np.arange(16))
        ref = sl.positions(mesh, f, wl.dt, z)
        assert np.array_equal(got, ref)
    finally:
        B.sl_destroy(h)


def _parity(B, wl, nsteps, samples_checked, M=None):
    mesh, f, phi0, a = oracle_inputs(wl)
    M = M or wl.samples
    h = _handle(B, wl, mesh, a, samples=M)
    try:
        B.sl_step(h, wl.dt, nsteps)
        got = B.sl_get_samples(h, 0, M)
        mean = B.sl_mean(h)
        assert B.sl_get_step(h) == nsteps
    finally:
        B.sl_destroy(h)
    ref = sl.run(mesh, f, phi0, wl.dt, nsteps, wl.seed, np.asarray(samples_checked))
    err = rel_l2(got[samples_checked], ref)
    print(f"{wl.name}: {nsteps} steps, samples {list(samples_checked)[:4]}..: rel L2 {err:.3e}", flush=True)
    return got, mean, ref, err


@pytest.fixture(params=["nodal", "normal"])
def algo(request, monkeypatch):
    """The 1-D fit in nodal (Lagrange) form and in Legendre normal-equation form."""
    monkeypatch.setenv("SL_1D_FIT", request.param)
    return request.param


def test_c1_full_parity_and_mean(B, algo):
    wl = W.c1_1d_const()
    got, mean, ref, err = _parity(B, wl, wl.steps, np.arange(wl.samples))
    assert err < TOL
    assert rel_l2(mean, sl.mean(ref)) < TOL
    assert np.all(np.isfinite(got))


def test_c2_parity_sample_subset(B, algo):
    wl = W.c2_1d_sine()
    idx = np.array([0, 1, 511, 1023])
    got, mean, ref, err = _parity(B, wl, 200, idx)
    assert err < TOL


@pytest.mark.slow
def test_c2_parity_full_length(B):
    """All 1000 steps of the 1-D sinusoidal workload on a few samples."""
    wl = W.c2_1d_sine()
    got, mean, ref, err = _parity(B, wl, wl.steps, np.array([3, 700]))
    assert err < TOL


def test_small_ragged_cases(B, algo):
    """K not dividing the 256-lane workgroup, M not filling the last workgroup, several N."""
    for K, N, M in ((3, 2, 5), (7, 5, 37), (24, 9, 11), (200, 4, 3), (256, 16, 2), (1, 6, 4)):
        wl = W.c2_1d_sine()
        wl.kx, wl.order, wl.samples, wl.dt = K, N, M, 2e-6
        mesh, f, phi0, a = oracle_inputs(wl)
        got, mean, ref, err = _parity(B, wl, 7, np.arange(M))
        assert err < TOL, (K, N, M, err)


def test_every_order_parity(B):
    """Every order 2..16 of the resident kernel (nodal form), each with its own
    register and LDS plan (staged step coefficients at orders 9-13, source
    factors held in registers at 9-12): a mesh of 20 elements (12 samples a
    workgroup, Wiener draws refilled every 21 steps), 25 samples (two full
    workgroups and a partial one), 45 steps (two refills); relative L2 and the
    largest node error both within the tolerance."""
    for N in range(2, 17):
        wl = W.c2_1d_sine()
        wl.kx, wl.order, wl.samples, wl.dt = 20, N, 25, 2e-6
        got, mean, ref, err = _parity(B, wl, 45, np.arange(25))
        node = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        assert err < TOL and node < TOL, (N, err, node)


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_tiled_meshes_beyond_256_elements(B, algo, bc):
    """More elements than one workgroup holds: tiles of 254 elements with a
    recomputed halo, out-of-place steps (odd and even counts), ragged last tile."""
    for K, N, M, steps in ((300, 5, 3, 3), (509, 12, 2, 4), (762, 4, 2, 1)):
        wl = W.c2_1d_sine()
        wl.kx, wl.order, wl.samples, wl.dt = K, N, M, 2e-7
        if bc == "dirichlet":
            wl.bc = "dirichlet"
            wl.ghost = lambda x, y, t: 0.3 + 0.0 * x
        got, mean, ref, err = _parity(B, wl, steps, np.arange(M))
        assert err < TOL, (K, N, M, bc, err)
        assert rel_l2(mean, sl.mean(got)) < 1e-14


def test_dirichlet_parity(B, algo):
    wl = W.Workload("dir", 1, 12, 1, 7, 9, 1e-5, 15, 4,
                    u=lambda x, y: (0.7 + 0.3 * np.sin(6 * x), np.zeros(np.shape(x))),
                    D=lambda x, y: 0.004 * (1 + 0.5 * np.cos(3 * x)), divu=lambda x, y: 1.8 * np.cos(6 * x),
                    phi0=lambda x, y: 1.0 + np.sin(3 * x), bc="dirichlet",
                    ghost=lambda x, y, t: 1.0 + np.sin(3 * x) + 0.01)
    got, mean, ref, err = _parity(B, wl, wl.steps, np.arange(wl.samples))
    assert err < TOL


def test_checkpoint_resume_and_determinism(B):
    wl = W.c2_1d_sine()
    wl.kx, wl.samples = 64, 32
    mesh, f, phi0, a = oracle_inputs(wl)
    h1 = _handle(B, wl, mesh, a)
    h2 = _handle(B, wl, mesh, a)
    try:
        B.sl_step(h1, wl.dt, 40)
        B.sl_step(h2, wl.dt, 20)
        ck = B.sl_get_samples(h2, 0, wl.samples)
        n = B.sl_get_step(h2)
        # restore into a fresh handle and continue
        h3 = _handle(B, wl, mesh, a)
        B.sl_set_samples(h3, 0, ck)
        B.sl_set_step(h3, n)
        B.sl_step(h3, wl.dt, 20)
        r1 = B.sl_get_samples(h1, 0, wl.samples)
        r3 = B.sl_get_samples(h3, 0, wl.samples)
        B.sl_destroy(h3)
        assert np.array_equal(r1, r3)
        B.sl_step(h2, wl.dt, 20)
        assert np.array_equal(B.sl_get_samples(h2, 0, wl.samples), r1)
    finally:
        B.sl_destroy(h1)
        B.sl_destroy(h2)


def test_sample_results_do_not_depend_on_sample_count(B):
    wl = W.c1_1d_const()
    mesh, f, phi0, a = oracle_inputs(wl)
    hs = [_handle(B, wl, mesh, a, samples=m) for m in (16, 64)]
    try:
        for h in hs:
            B.sl_step(h, wl.dt, 30)
        r16 = B.sl_get_samples(hs[0], 0, 16)
        r64 = B.sl_get_samples(hs[1], 0, 64)
        assert np.array_equal(r16, r64[:16])
    finally:
        for h in hs:
            B.sl_destroy(h)


def test_step_argument_errors(B):
    wl = W.c1_1d_const()
    mesh, f, phi0, a = oracle_inputs(wl)
    desc = B.make_desc(1, wl.kx, order=wl.order, samples=4)
    h = B.sl_init_mesh(desc)
    try:
        with pytest.raises(B.SLError) as ei:
            B.sl_step(h, wl.dt, 1)          # fields not set
        assert ei.value.code == B.SL_ESTATE
        bad = dict(a)
        bad["D"] = a["D"].copy()
        bad["D"][3] = np.nan
        with pytest.raises(B.SLError) as ei:
            B.sl_set_fields(h, bad["u"], bad["D"], bad["divu"], bad["un"], bad["Dn"], None, bad["phi0"])
        assert ei.value.code == B.SL_ENONFINITE
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], None, a["phi0"])
        for dt in (0.0, -1.0, float("nan")):
            with pytest.raises(B.SLError):
                B.sl_step(h, dt, 1)
        with pytest.raises(B.SLError):
            B.sl_get_samples(h, 3, 2)
        B.sl_step(h, wl.dt, 0)
        assert B.sl_get_step(h) == 0
    finally:
        B.sl_destroy(h)
