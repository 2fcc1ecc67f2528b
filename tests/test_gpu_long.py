"""GPU parity at the 2-D workloads' own lengths and on the paths the short tests
miss, through the C ABI.

* The 64x64 constant-drift workload over 50 and 200 steps and the 128x128
  mixed-order rotation over 20 steps, sample 0 against the oracle's values
  stored by tests/golden/make_long_runs.py (the oracle needs seconds a step on
  these meshes).  The library runs two samples (global indices 0 and 1, the
  same Philox counters as the full runs; samples never interact).
* 1-D orders 13-16 at a one-sigma displacement of one node spacing (the limit
  of eq. 1d_timestep), both fit forms.
* Chebyshev-Gauss nodes (eq. gaussquad's family) in 1-D and 2-D.
Every check bounds the relative L2 error and the largest node error by 1e-11.
"""
import glob
import os

import numpy as np
import pytest

from oracle import sl, tables
from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs, oracle_mesh, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-11
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _check(got, ref, what):
    err = rel_l2(got, ref)
    node = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"{what}: rel L2 {err:.3e}, max node error / max |ref| {node:.3e}", flush=True)
    assert err < TOL and node < TOL, (what, err, node)


def _golden(name):
    files = sorted(glob.glob(os.path.join(GOLDEN, f"long_{name}_s0_n*.npz")))
    return [np.load(f, allow_pickle=False) for f in files]


@pytest.mark.parametrize("key", ["c3", "c4"])
def test_long_runs_against_stored_oracle_values(B, key):
    wl = W.WORKLOADS[key]()
    runs = _golden(wl.name)
    assert runs, f"no stored oracle runs for {wl.name}"
    mesh = oracle_mesh(wl)
    order = wl.order if np.isscalar(wl.order) else wl.order_array()
    desc = B.make_desc(2, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=2, seed=wl.seed)
    h = B.sl_init_mesh(desc)
    try:
        nodes, _, _ = B.sl_sizes(h)
        assert nodes == mesh.total_nodes
        _, _, _, a = oracle_inputs(wl, mesh)
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
        done = 0
        for g in sorted(runs, key=lambda g: int(g["steps"])):
            assert float(g["dt"]) == wl.dt and int(g["sample"]) == 0
            B.sl_step(h, wl.dt, int(g["steps"]) - done)
            done = int(g["steps"])
            got = B.sl_get_samples(h, 0, 1)[0]
            _check(got[g["idx"]], g["values"], f"{wl.name} sample 0 after {done} steps")
        d = B.sl_diag(h)
        assert d["solver_unconverged"] == [0, 0]
        assert np.all(np.isfinite(B.sl_get_samples(h, 0, 2)))
    finally:
        B.sl_destroy(h)


@pytest.mark.parametrize("algo", ["nodal", "normal"])
@pytest.mark.parametrize("N", [13, 14, 15, 16])
def test_1d_high_orders_at_one_node_spacing(B, N, algo, monkeypatch):
    """A one-sigma move of one (smallest) node spacing per step: sqrt(2 D dt) / h = min gap."""
    if algo == "normal":
        monkeypatch.setenv("SL_1D_FIT", "normal")
    xi = np.asarray(tables.nodes(N))
    gap = float(np.min(np.diff(np.concatenate([[0.0], xi, [1.0]]))))
    K, M, dt = 8, 6, 1e-5
    h = 1.0 / K
    D = (gap * h) ** 2 / (2 * dt)
    wl = W.Workload("hi", 1, K, 1, N, M, dt, 3, 21,
                    u=lambda x, y: (np.zeros(np.shape(x)), np.zeros(np.shape(x))), D=W.const(D),
                    divu=W.const(0.0), phi0=lambda x, y: np.exp(np.sin(2 * np.pi * x)))
    mesh, f, phi0, a = oracle_inputs(wl)
    desc = B.make_desc(1, K, order=N, samples=M, seed=wl.seed)
    hd = B.sl_init_mesh(desc)
    try:
        B.sl_set_fields(hd, a["u"], a["D"], a["divu"], a["un"], a["Dn"], None, a["phi0"])
        B.sl_step(hd, dt, 3)
        got = B.sl_get_samples(hd, 0, M)
        assert B.sl_diag(hd)["escapes"] > 0          # the move reaches the edges
    finally:
        B.sl_destroy(hd)
    ref = sl.run(mesh, f, phi0, dt, 3, wl.seed, np.arange(M))
    _check(got, ref, f"1-D N={N} {algo} at one node spacing")


@pytest.mark.parametrize("dim,N,solver", [(1, 8, "auto"), (1, 13, "auto"), (2, 6, "reference"), (2, 9, "reference"),
                                          (2, 7, "factor")])
def test_chebyshev_gauss_nodes(B, dim, N, solver):
    if dim == 1:
        wl = W.c2_1d_sine()
        wl.kx, wl.order, wl.samples, wl.dt = 12, N, 5, 2e-6
    else:
        wl = W.c4_2d_rotation(kx=4, ky=3, samples=3, steps=3)
        wl.order, wl.dt = N, 1e-4
    mesh = oracle_mesh(wl, family="cg")
    mesh, f, phi0, a = oracle_inputs(wl, mesh)
    desc = B.make_desc(dim, wl.kx, wl.ky, wl.box, N, nodes="cg", bc=wl.bc, samples=wl.samples, seed=wl.seed,
                       solver=solver)
    h = B.sl_init_mesh(desc)
    try:
        np.testing.assert_array_equal(B.sl_node_coords(h, dim), mesh.node_coords())
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
        B.sl_step(h, wl.dt, 3)
        got = B.sl_get_samples(h, 0, wl.samples)
    finally:
        B.sl_destroy(h)
    ref = sl.run(mesh, f, phi0, wl.dt, 3, wl.seed, np.arange(wl.samples))
    _check(got, ref, f"Chebyshev-Gauss {dim}-D N={N} {solver}")
