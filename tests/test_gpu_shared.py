"""Shared-geometry 2-D path (constant drift, diffusion and source factor, one
order): per-sample operators and batched float64 matrix-core products, against
the oracle through the C ABI, on every order it supports, with Dirichlet
boundaries, a source factor, and over the 64x64 workload's own 50 and 200 steps
(stored oracle values)."""
import glob
import os

import numpy as np
import pytest

from oracle import sl
from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs, oracle_mesh, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-11
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _handle(B, wl, a, M, shared=1):
    order = wl.order if np.isscalar(wl.order) else wl.order_array()
    desc = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=M, seed=wl.seed)
    h = B.sl_init_mesh(desc)
    B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
    B.sl_set_schedule(h, 0, 0, 0, shared)
    return h


def _check(got, ref, what):
    err = rel_l2(got, ref)
    node = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"{what}: rel L2 {err:.2e}, max node {node:.2e}", flush=True)
    assert err < TOL and node < TOL, (what, err, node)


def _const_wl(N, kx=4, ky=3, M=5, bc="periodic", divu=0.0, dt=1e-4):
    wl = W.c3_2d_const()
    wl.kx, wl.ky, wl.order, wl.samples, wl.dt = kx, ky, N, M, dt
    wl.divu = W.const(divu)
    wl.phi0 = lambda x, y: np.exp(np.cos(2 * np.pi * x) + 0.5 * np.sin(2 * np.pi * (y - 0.2)))
    if bc == "dirichlet":
        wl.bc = "dirichlet"
        wl.ghost = lambda x, y, t: np.exp(np.cos(2 * np.pi * x) + 0.5 * np.sin(2 * np.pi * (y - 0.2))) + 0.01
    return wl


@pytest.mark.parametrize("N", list(range(2, 13)))
def test_shared_path_matches_the_oracle_every_order(B, N):
    wl = _const_wl(N)
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, wl.samples)
    try:
        B.sl_step(h, wl.dt, 3)
        got = B.sl_get_samples(h, 0, wl.samples)
        assert B.sl_diag(h)["steps"] == 3
    finally:
        B.sl_destroy(h)
    ref = sl.run(mesh, f, phi0, wl.dt, 3, wl.seed, np.arange(wl.samples))
    _check(got, ref, f"shared N={N}")


@pytest.mark.parametrize("bc,divu", [("dirichlet", 0.0), ("periodic", 0.7), ("dirichlet", -1.3)])
def test_shared_path_dirichlet_and_source_factor(B, bc, divu):
    wl = _const_wl(7, kx=5, ky=4, M=4, bc=bc, divu=divu)
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, wl.samples)
    try:
        B.sl_step(h, wl.dt, 4)
        got = B.sl_get_samples(h, 0, wl.samples)
    finally:
        B.sl_destroy(h)
    ref = sl.run(mesh, f, phi0, wl.dt, 4, wl.seed, np.arange(wl.samples))
    _check(got, ref, f"shared {bc} div u={divu}")


def test_shared_path_equals_the_general_path_on_a_ragged_tile(B):
    """70 x 3 elements (tiles of 64 elements with a ragged last tile), 9 samples."""
    wl = _const_wl(8, kx=70, ky=3, M=9)
    mesh, f, phi0, a = oracle_inputs(wl)
    h1, h2 = _handle(B, wl, a, 9, shared=1), _handle(B, wl, a, 9, shared=0)
    try:
        B.sl_step(h1, wl.dt, 5)
        B.sl_step(h2, wl.dt, 5)
        g1, g2 = B.sl_get_samples(h1, 0, 9), B.sl_get_samples(h2, 0, 9)
    finally:
        B.sl_destroy(h1)
        B.sl_destroy(h2)
    _check(g1, g2, "shared vs general path")


def test_shared_path_over_the_64x64_workload_length(B):
    wl = W.c3_2d_const()
    runs = sorted((np.load(f, allow_pickle=False) for f in glob.glob(os.path.join(GOLDEN, f"long_{wl.name}_s0_n*.npz"))),
                  key=lambda g: int(g["steps"]))
    assert runs
    mesh = oracle_mesh(wl)
    _, _, _, a = oracle_inputs(wl, mesh)
    h = _handle(B, wl, a, 2)
    try:
        done = 0
        for g in runs:
            B.sl_step(h, wl.dt, int(g["steps"]) - done)
            done = int(g["steps"])
            got = B.sl_get_samples(h, 0, 1)[0]
            _check(got[g["idx"]], g["values"], f"shared {wl.name} after {done} steps")
    finally:
        B.sl_destroy(h)


def test_shared_path_refuses_what_it_cannot_run(B):
    # varying drift (rotation): not a shared geometry
    wl = W.c4_2d_rotation(kx=3, ky=3, samples=2, steps=1)
    wl.order = 6
    mesh, f, phi0, a = oracle_inputs(wl)
    h = _handle(B, wl, a, 2)
    try:
        with pytest.raises(B.SLError) as ei:
            B.sl_step(h, wl.dt, 1)
        assert ei.value.code == B.SL_EUNSUPPORTED
        B.sl_set_schedule(h, 0, 0, 0, 0)
        B.sl_step(h, wl.dt, 1)                       # the general path still runs
    finally:
        B.sl_destroy(h)
    # mixed orders and 1-D meshes
    wl = W.c4_2d_rotation(kx=2, ky=2, samples=2, steps=1)
    wl.order = np.array([6, 8, 6, 8], dtype=np.int32)
    wl.u = lambda x, y: (np.full(np.shape(x), 1.0), np.full(np.shape(x), 0.5))
    wl.D = W.const(0.002)
    mesh, f, phi0, a = oracle_inputs(wl)
    for w in (wl, W.c1_1d_const()):
        m2, f2, p2, a2 = oracle_inputs(w)
        h = _handle(B, w, a2, 2)
        try:
            with pytest.raises(B.SLError) as ei:
                B.sl_step(h, w.dt, 1)
            assert ei.value.code == B.SL_EUNSUPPORTED
        finally:
            B.sl_destroy(h)
