"""The mass-conservation constraint (descriptor constraints = boundary + mass) on the
GPU against the oracle's constrained fit with the mass row, through the C ABI: 1-D
(both fit forms, resident and tiled), the 2-D general path (reference solver: one
more linear condition on the bubble coefficients of its null-space remap) and the
2-D shared-geometry path.  The fit
keeps each element's integral of p0, so the remap moves no mass across an
element's boundary; the oracle's mass row is pinned against an mpmath KKT solve
with exact integrals (test_oracle_pins.py)."""
import numpy as np
import pytest

from oracle import sl
from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs, oracle_mesh, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _run(B, wl, a, steps, shared=0, solver="auto", ncomp=1):
    order = wl.order if np.isscalar(wl.order) else wl.order_array()
    desc = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=wl.samples, seed=wl.seed, mass=True,
                       solver=solver, ncomp=ncomp)
    h = B.sl_init_mesh(desc)
    try:
        phi0 = a["phi0"] if ncomp == 1 else np.concatenate([a["phi0"] * (1.0 + 0.1 * c) for c in range(ncomp)])
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], phi0)
        if shared:
            B.sl_set_schedule(h, 0, 0, 0, 1)
        B.sl_step(h, wl.dt, steps)
        return B.sl_get_samples(h, 0, wl.samples)
    finally:
        B.sl_destroy(h)


def _check(got, ref, what):
    err = rel_l2(got, ref)
    node = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"{what}: rel L2 {err:.2e}, max node {node:.2e}")
    assert err < TOL and node < TOL, (what, err, node)


@pytest.mark.parametrize("algo,K,N", [("nodal", 20, 2), ("nodal", 20, 3), ("nodal", 20, 8), ("nodal", 24, 12),
                                      ("nodal", 16, 16), ("normal", 20, 9), ("nodal", 300, 6), ("normal", 300, 5)])
def test_mass_constrained_1d_matches_the_oracle(B, algo, K, N, monkeypatch):
    if algo == "normal":
        monkeypatch.setenv("SL_1D_FIT", "normal")
    wl = W.c2_1d_sine()
    wl.kx, wl.order, wl.samples, wl.dt = K, N, 5, 2e-6 if K < 256 else 2e-7
    mesh = oracle_mesh(wl)
    mesh.mass = True
    mesh, f, phi0, a = oracle_inputs(wl, mesh)
    got = _run(B, wl, a, 6)
    ref = sl.run(mesh, f, phi0, wl.dt, 6, wl.seed, np.arange(wl.samples))
    _check(got, ref, f"mass 1-D {algo} K={K} N={N}")
    if N >= 3:
        plain = sl.run(oracle_mesh(wl), f, phi0, wl.dt, 6, wl.seed, np.arange(wl.samples))
        assert np.max(np.abs(plain - ref)) > 1e-14       # the constraint changes the result


@pytest.mark.parametrize("N,bc", [(3, "periodic"), (6, "periodic"), (8, "dirichlet"), (12, "periodic")])
def test_mass_constrained_shared_path_matches_the_oracle(B, N, bc):
    wl = W.c3_2d_const()
    wl.kx, wl.ky, wl.order, wl.samples, wl.dt = 4, 3, N, 4, 1e-4
    wl.phi0 = lambda x, y: np.exp(np.cos(2 * np.pi * x) + 0.5 * np.sin(2 * np.pi * (y - 0.2)))
    if bc == "dirichlet":
        wl.bc = "dirichlet"
        wl.ghost = lambda x, y, t: np.exp(np.cos(2 * np.pi * x) + 0.5 * np.sin(2 * np.pi * (y - 0.2))) + 0.01
    mesh = oracle_mesh(wl)
    mesh.mass = True
    mesh, f, phi0, a = oracle_inputs(wl, mesh)
    got = _run(B, wl, a, 3, shared=1)
    ref = sl.run(mesh, f, phi0, wl.dt, 3, wl.seed, np.arange(wl.samples))
    _check(got, ref, f"mass shared N={N} {bc}")


def _rot(kx, order, samples=3):
    wl = W.c4_2d_rotation(kx=kx, ky=kx, samples=samples, steps=3)
    wl.order = order
    wl.dt = 2e-4
    return wl


@pytest.mark.parametrize("order,bc", [(3, "periodic"), (6, "periodic"), (8, "dirichlet"), (12, "periodic"),
                                      ("mixed", "periodic"), (16, "periodic")])
def test_mass_constrained_general_2d_matches_the_oracle(B, order, bc):
    """The reference solver's remap with the mass row (rotation: a non-uniform
    displacement, so the bubble iteration runs), against the oracle; the
    constraint must change the result and keep every element's integral of p0."""
    if order == "mixed":
        order = np.array([6, 8, 10, 4, 12, 3, 8, 6, 16], dtype=np.int32)
    wl = _rot(3, order)
    if bc == "dirichlet":
        wl.bc = "dirichlet"
        wl.ghost = lambda x, y, t: 0.2 + 0.1 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    mesh = oracle_mesh(wl)
    mesh.mass = True
    mesh, f, phi0, a = oracle_inputs(wl, mesh)
    got = _run(B, wl, a, 3, solver="reference")
    ref = sl.run(mesh, f, phi0, wl.dt, 3, wl.seed, np.arange(wl.samples))
    _check(got, ref, f"mass general 2-D order {order} {bc}")
    plain = sl.run(oracle_mesh(wl), f, phi0, wl.dt, 3, wl.seed, np.arange(wl.samples))
    assert np.max(np.abs(plain - ref)) > 1e-14


def test_mass_constrained_general_2d_vector_and_batch(B):
    """Two components (each its own mass row on the shared moves) against the oracle,
    and the same handle stepped in a batch with an unconstrained one: bitwise equal
    to each stepped alone."""
    wl = _rot(3, np.array([6, 8, 10, 6, 8, 10, 6, 8, 10], dtype=np.int32), samples=2)
    mesh = oracle_mesh(wl)
    mesh.mass = True
    mesh, f, phi0, a = oracle_inputs(wl, mesh)
    got = _run(B, wl, a, 2, solver="reference", ncomp=2)
    nodes = mesh.total_nodes
    for c in range(2):
        ref = sl.run(mesh, f, phi0 * (1.0 + 0.1 * c), wl.dt, 2, wl.seed, np.arange(wl.samples))
        _check(got[:, c * nodes:(c + 1) * nodes], ref, f"mass general 2-D component {c}")
    order = wl.order_array()

    def make(mass):
        h = B.sl_init_mesh(B.make_desc(2, wl.kx, wl.ky, wl.box, order, samples=wl.samples, seed=wl.seed,
                                       mass=mass, solver="reference"))
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], None, a["phi0"])
        return h
    alone = []
    for mass in (True, False):
        h = make(mass)
        try:
            B.sl_step(h, wl.dt, 2)
            alone.append(B.sl_get_samples(h, 0, wl.samples))
        finally:
            B.sl_destroy(h)
    hs = [make(True), make(False)]
    try:
        B.sl_step_batch(hs, [wl.dt, wl.dt], 2)
        for h, want in zip(hs, alone):
            assert np.array_equal(B.sl_get_samples(h, 0, wl.samples), want)
    finally:
        for h in hs:
            B.sl_destroy(h)


def test_mass_constraint_with_the_factorisation_solver_is_refused(B):
    wl = W.c4_2d_rotation(kx=2, ky=2, samples=2, steps=1)
    wl.order = 6
    mesh, f, phi0, a = oracle_inputs(wl)
    h = B.sl_init_mesh(B.make_desc(2, 2, 2, wl.box, 6, samples=2, seed=1, mass=True, solver="factor"))
    try:
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], None, a["phi0"])
        with pytest.raises(B.SLError) as ei:
            B.sl_step(h, wl.dt, 1)
        assert ei.value.code == B.SL_EUNSUPPORTED
    finally:
        B.sl_destroy(h)
