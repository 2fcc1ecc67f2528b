"""The mass-conservation constraint (descriptor constraints = boundary + mass) on the
GPU against the oracle's constrained fit with the mass row, through the C ABI: 1-D
(both fit forms, resident and tiled) and the 2-D shared-geometry path.  The fit
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


def _run(B, wl, a, steps, shared=0):
    order = wl.order if np.isscalar(wl.order) else wl.order_array()
    desc = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=wl.samples, seed=wl.seed, mass=True)
    h = B.sl_init_mesh(desc)
    try:
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], a["phi0"])
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


def test_mass_constraint_on_the_general_2d_path_is_refused(B):
    wl = W.c4_2d_rotation(kx=2, ky=2, samples=2, steps=1)
    wl.order = 6
    mesh, f, phi0, a = oracle_inputs(wl)
    order = wl.order
    h = B.sl_init_mesh(B.make_desc(2, 2, 2, wl.box, order, samples=2, seed=1, mass=True))
    try:
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], None, a["phi0"])
        with pytest.raises(B.SLError) as ei:
            B.sl_step(h, wl.dt, 1)
        assert ei.value.code == B.SL_EUNSUPPORTED
    finally:
        B.sl_destroy(h)
