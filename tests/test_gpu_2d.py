"""GPU parity of the 2-D path (MFMA Gram, blocked Cholesky, range-space constraints)
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import sl
from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _handle(B, wl, a, samples=None, precision="fp64", refine=-1, solver="auto"):
    order = wl.order if np.isscalar(wl.order) else wl.order_array()
    desc = B.make_desc(2, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=samples or wl.samples, seed=wl.seed,
                       precision=precision, refine_iters=refine, solver=solver)
    h = B.sl_init_mesh(desc)
    B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
    return h


def _parity(B, wl, nsteps, samples_checked, precision="fp64", refine=-1, solver="auto"):
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, precision=precision, refine=refine, solver=solver)
    try:
        B.sl_step(h, wl.dt, nsteps)
        got = B.sl_get_samples(h, 0, wl.samples)
        diag = B.sl_diag(h)
    finally:
        B.sl_destroy(h)
    ref = sl.run(mesh, f, phi0, wl.dt, nsteps, wl.seed, np.asarray(samples_checked))
    err = rel_l2(got[samples_checked], ref)
    print(f"{wl.name} {wl.kx}x{wl.ky} {precision} solver {diag['solver']}: {nsteps} steps: rel L2 {err:.3e}; "
          f"iterations {diag['solver_iterations']}, unconverged {diag['solver_unconverged']}", flush=True)
    if diag["solver"] == 2:
        assert diag["solver_unconverged"] == [0, 0]
    return got, ref, err


def _small(N, kx=3, ky=3, samples=3, bc="periodic", rot=False):
    wl = W.c4_2d_rotation(kx=kx, ky=ky, samples=samples, steps=3) if rot else W.c3_2d_const()
    wl.kx, wl.ky, wl.samples, wl.order = kx, ky, samples, N
    wl.phi0 = lambda x, y: np.exp(np.cos(2 * np.pi * x) + 0.5 * np.sin(2 * np.pi * (y - 0.2)))
    if bc == "dirichlet":
        wl.bc = "dirichlet"
        wl.ghost = lambda x, y, t: np.exp(np.cos(2 * np.pi * x) + 0.5 * np.sin(2 * np.pi * (y - 0.2))) + 0.01
    return wl


def test_positions_bitwise_2d(B):
    wl = W.c4_2d_rotation(kx=8, ky=8, samples=5, steps=1)
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a)
    try:
        np.testing.assert_array_equal(B.sl_node_coords(h, 2), mesh.node_coords())
        exy, axis = B.sl_edge_coords(h, 2)
        np.testing.assert_array_equal(exy, mesh.edge_coords())
        B.sl_set_step(h, 11)
        got = B.sl_debug_positions(h, wl.dt, 5, 2)
        z = sl.wiener_normals(mesh, wl.seed, 11, np.arange(5))
        assert np.array_equal(got, sl.positions(mesh, f, wl.dt, z))
    finally:
        B.sl_destroy(h)


@pytest.mark.parametrize("N,solver", [(N, "factor") for N in range(2, 11)] +
                         [(N, "reference") for N in range(2, 17)])
def test_small_periodic_parity_every_order(B, N, solver):
    wl = _small(N, rot=True)
    got, ref, err = _parity(B, wl, 3, np.arange(wl.samples), solver=solver)
    assert err < TOL, (N, solver, err)


def test_slowly_contracting_fits_are_redone_by_the_full_form(B):
    """A rotation step long enough that many element fits' fixed-point
    iteration contracts by less than half a step: the per-order kernels list
    those fits and the full form (with conjugate gradients) redoes them.  The
    result matches the oracle, every fit converges, the fallbacks are counted,
    and the batched launch (the full form for every fit) agrees to rounding.
    Orders 4 and 6 on one mesh, so that two order groups keep their own lists."""
    wl = W.c4_2d_rotation(kx=3, ky=3, samples=6, steps=1)
    wl.order = np.where(np.arange(wl.K) % 2 == 0, 6, 4).astype(np.int32)
    wl.dt = 0.01
    mesh, f, phi0, a = oracle_inputs(wl)
    hs = [_handle(B, wl, a, solver="reference") for _ in range(3)]
    try:
        B.sl_step(hs[0], wl.dt, 1)
        B.sl_step_batch(hs[1:], [wl.dt, wl.dt], 1)
        got = B.sl_get_samples(hs[0], 0, wl.samples)
        batch = B.sl_get_samples(hs[1], 0, wl.samples)
        d = B.sl_diag(hs[0])
        db = B.sl_diag(hs[1])
    finally:
        for h in hs:
            B.sl_destroy(h)
    ref = sl.run(mesh, f, phi0, wl.dt, 1, wl.seed, np.arange(4))
    err = rel_l2(got[:4], ref)
    print(f"fallbacks {d['solver_fallbacks']} (batched {db['solver_fallbacks']}), iterations {d['solver_iterations']}, "
          f"unconverged {d['solver_unconverged']}, rel L2 {err:.3e}, vs batched {rel_l2(got, batch):.3e}", flush=True)
    assert d["solver_fallbacks"] > 0 and d["solver_fallbacks"] == db["solver_fallbacks"]
    assert d["solver_unconverged"] == [0, 0]
    assert err < TOL
    assert rel_l2(got, batch) < 1e-13


@pytest.mark.parametrize("solver", ["factor", "reference"])
def test_rectangular_mesh_and_rotation(B, solver):
    wl = _small(6, kx=4, ky=2, samples=4, rot=True)
    got, ref, err = _parity(B, wl, 4, np.arange(4), solver=solver)
    assert err < TOL


@pytest.mark.parametrize("N,solver", [(3, "factor"), (8, "factor"), (3, "reference"), (8, "reference"),
                                      (13, "reference")])
def test_dirichlet_parity_2d(B, N, solver):
    wl = _small(N, kx=3, ky=2, samples=2, bc="dirichlet")
    got, ref, err = _parity(B, wl, 3, np.arange(2), solver=solver)
    assert err < TOL


@pytest.mark.parametrize("solver", ["factor", "reference"])
def test_mixed_order_parity(B, solver):
    """Neighbours of different order: traces interpolated between Gauss abscissae."""
    wl = W.c4_2d_rotation(kx=4, ky=4, samples=3, steps=3)
    wl.order = np.array([6, 8, 10, 6, 8, 6, 10, 8, 10, 6, 8, 6, 8, 10, 6, 8], dtype=np.int32)
    wl.dt = 2e-4
    got, ref, err = _parity(B, wl, 3, np.arange(3), solver=solver)
    assert err < TOL


def test_mixed_high_orders_reference_solver(B):
    """Orders up to 16 side by side (reference solver only)."""
    wl = W.c4_2d_rotation(kx=3, ky=3, samples=2, steps=2)
    wl.order = np.array([11, 16, 12, 14, 13, 15, 16, 11, 12], dtype=np.int32)
    wl.dt = 5e-5
    got, ref, err = _parity(B, wl, 2, np.arange(2), solver="reference")
    assert err < TOL


def test_reference_solver_iterations(B):
    """A uniform displacement (constant fields) makes the preconditioners exact:
    phase 1 takes the one residual evaluation that confirms its start (Richardson
    iteration counts each), phase 2 none; the rotation needs a few per fit and
    every fit converges."""
    wl = W.c3_2d_const()
    wl.kx = wl.ky = 8
    wl.samples = 4
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, solver="reference")
    try:
        B.sl_step(h, wl.dt, 2)
        d = B.sl_diag(h)
    finally:
        B.sl_destroy(h)
    fits = wl.K * wl.samples * 2
    print("constant fields:", d["solver_iterations"], "iterations over", fits, "fits per phase", flush=True)
    assert d["solver_unconverged"] == [0, 0]
    assert d["solver_iterations"][0] == fits and d["solver_iterations"][1] <= fits // 10
    wl = W.c4_2d_rotation(kx=8, ky=8, samples=4, steps=2)
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, solver="reference")
    try:
        B.sl_step(h, wl.dt, 2)
        d = B.sl_diag(h)
    finally:
        B.sl_destroy(h)
    fits = wl.K * wl.samples * 2
    print("rotation:", d["solver_iterations"], "iterations over", fits, "fits per phase", flush=True)
    assert d["solver_unconverged"] == [0, 0]
    assert d["solver_iterations"][1] <= 6 * fits


@pytest.mark.parametrize("solver", ["factor", "reference"])
def test_c3_full_size_sample_subset(B, solver):
    wl = W.c3_2d_const()
    got, ref, err = _parity(B, wl, 2, np.array([0, 255]), solver=solver)
    assert err < TOL
    assert np.all(np.isfinite(got))


@pytest.mark.slow
@pytest.mark.parametrize("solver", ["factor", "reference"])
def test_c4_full_size_one_sample(B, solver):
    wl = W.c4_2d_rotation()
    got, ref, err = _parity(B, wl, 1, np.array([511]), solver=solver)
    assert err < TOL


def test_c4_full_size_reference_solver_subset(B):
    """The 128 x 128 mixed-order rotation at full size (all 512 samples on the
    device), two samples checked against the oracle."""
    wl = W.c4_2d_rotation()
    got, ref, err = _parity(B, wl, 1, np.array([0, 301]), solver="reference")
    assert err < TOL


def test_2d_mean_and_determinism(B):
    wl = _small(5, kx=4, ky=3, samples=17)
    mesh, f, phi0, a = oracle_inputs(wl)
    h1, h2 = _handle(B, wl, a), _handle(B, wl, a)
    try:
        B.sl_step(h1, wl.dt, 4)
        B.sl_step(h2, wl.dt, 2)
        B.sl_step(h2, wl.dt, 2)
        r1 = B.sl_get_samples(h1, 0, 17)
        assert np.array_equal(r1, B.sl_get_samples(h2, 0, 17))
        m = B.sl_mean(h1)
        assert rel_l2(m, sl.mean(r1)) < 1e-14
    finally:
        B.sl_destroy(h1)
        B.sl_destroy(h2)


MODES = ["fp32_refine", "bf16split_refine"]


@pytest.mark.parametrize("precision", MODES)
@pytest.mark.parametrize("N", [3, 6, 8, 10])
def test_mixed_precision_small_parity(B, precision, N):
    """float32 / bf16-split factorisations with float64 refinement reach the float64 tolerance."""
    wl = _small(N, samples=2, rot=True)
    got, ref, err = _parity(B, wl, 3, np.arange(2), precision=precision)
    assert err < TOL, (precision, N, err)


@pytest.mark.parametrize("precision", MODES)
def test_mixed_precision_mixed_order_and_dirichlet(B, precision):
    wl = W.c4_2d_rotation(kx=4, ky=4, samples=2, steps=3)
    wl.order = np.array([6, 8, 10, 6, 8, 6, 10, 8, 10, 6, 8, 6, 8, 10, 6, 8], dtype=np.int32)
    wl.dt = 2e-4
    got, ref, err = _parity(B, wl, 2, np.arange(2), precision=precision)
    assert err < TOL
    wl = _small(5, kx=3, ky=2, samples=2, bc="dirichlet")
    got, ref, err = _parity(B, wl, 2, np.arange(2), precision=precision)
    assert err < TOL


@pytest.mark.parametrize("precision", MODES)
def test_mixed_precision_c3_subset(B, precision):
    wl = W.c3_2d_const()
    got, ref, err = _parity(B, wl, 2, np.array([7]), precision=precision)
    assert err < TOL


def test_refinement_is_what_recovers_accuracy(B):
    """Without refinement sweeps the float32 path is only float32-accurate."""
    wl = _small(8, samples=2, rot=True)
    _, _, err0 = _parity(B, wl, 2, np.arange(2), precision="fp32_refine", refine=0)
    _, _, err3 = _parity(B, wl, 2, np.arange(2), precision="fp32_refine", refine=3)
    assert err0 > 1e-9
    assert err3 < TOL


@pytest.mark.parametrize("precision", MODES)
def test_mixed_precision_all_samples_agree_with_fp64(B, precision):
    """Every sample of the 64x64 workload (large displacements included) stays finite and
    matches the float64 GPU path; sample 131 is also checked against the oracle."""
    wl = W.c3_2d_const()
    mesh, f, phi0, a = oracle_inputs(wl)
    out = {}
    for prec in ("fp64", precision):
        h = _handle(B, wl, a, precision=prec)
        try:
            B.sl_step(h, wl.dt, 4)
            out[prec] = B.sl_get_samples(h, 0, wl.samples)
        finally:
            B.sl_destroy(h)
    assert np.all(np.isfinite(out[precision]))
    err = rel_l2(out[precision], out["fp64"])
    print(f"{precision} vs fp64, all {wl.samples} samples, 4 steps: rel L2 {err:.3e}", flush=True)
    assert err < TOL
    ref = sl.run(mesh, f, phi0, wl.dt, 4, wl.seed, np.array([131]))
    assert rel_l2(out[precision][[131]], ref) < TOL


@pytest.mark.parametrize("solver", ["factor", "reference"])
def test_serving_shapes_large_displacements(B, solver):
    """2-D requests of the serving stream (coarse meshes, sinusoidal drift, the
    largest time step the stream allows): the preconditioner is far from exact
    here, the solver must still converge to the oracle's remap."""
    reqs = [r for r in W.serving_requests(n=120, kmax=25, mmax=40) if r["dim"] == 2]
    reqs = [r for r in reqs if r["N"] <= (10 if solver == "factor" else 16)][:6]
    assert len(reqs) >= 4
    for r in reqs:
        wl = W.request_workload(r)
        wl.samples = 2
        got, ref, err = _parity(B, wl, 2, np.arange(2), solver=solver)
        assert err < TOL, (r["id"], r["N"], r["kx"], err)
