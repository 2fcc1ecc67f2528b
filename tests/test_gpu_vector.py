"""Vector-valued phi* (Sec. 5.3, last paragraph: every component is defined on the
same advected points), through the C ABI: each component of a handle with
ncomp = 3 equals the oracle's scalar run of that component (the same Wiener
increments: the oracle draws them per sample and step) and, bit for bit, a
scalar handle run on that component alone -- on every path: 1-D resident and
tiled, 2-D reference solver (which shares each fit's geometry, constraint
matrix and its inverse across the components), 2-D factorisation, and the
shared-geometry path."""
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


def _fields(xy, dim):
    x = xy[:, 0]
    y = xy[:, 1] if dim == 2 else 0.0 * x
    return [np.exp(np.cos(2 * np.pi * x) + 0.5 * np.sin(2 * np.pi * (y - 0.2))),
            1.0 + 0.3 * np.sin(4 * np.pi * x) * np.cos(2 * np.pi * y),
            np.exp(-((x - 0.4) ** 2 + (y - 0.6) ** 2) / 0.02)]


def _run(B, wl, a, phi0, ncomp, steps, solver="auto", shared=0):
    order = wl.order if np.isscalar(wl.order) else wl.order_array()
    desc = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=wl.samples, seed=wl.seed,
                       solver=solver, ncomp=ncomp)
    h = B.sl_init_mesh(desc)
    try:
        B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], np.concatenate(phi0))
        if shared:
            B.sl_set_schedule(h, 0, 0, 0, 1)
        B.sl_step(h, wl.dt, steps)
        got = B.sl_get_samples(h, 0, wl.samples)
        mean = B.sl_mean(h)
        d = B.sl_diag(h)
    finally:
        B.sl_destroy(h)
    return got, mean, d


CASES = {
    "1d": lambda: (lambda wl: (setattr(wl, "kx", 24), setattr(wl, "order", 9), setattr(wl, "samples", 7),
                               setattr(wl, "dt", 2e-6), wl)[-1])(W.c2_1d_sine()),
    "1d_tiled": lambda: (lambda wl: (setattr(wl, "kx", 300), setattr(wl, "order", 5), setattr(wl, "samples", 3),
                                     setattr(wl, "dt", 2e-7), wl)[-1])(W.c2_1d_sine()),
    "2d": lambda: (lambda wl: (setattr(wl, "order", np.array([6, 8, 6, 8, 10, 6], dtype=np.int32)),
                               setattr(wl, "dt", 2e-4), wl)[-1])(W.c4_2d_rotation(kx=3, ky=2, samples=4, steps=3)),
    "2d_const": lambda: (lambda wl: (setattr(wl, "kx", 4), setattr(wl, "ky", 3), setattr(wl, "order", 7),
                                     setattr(wl, "samples", 4), setattr(wl, "dt", 1e-4), wl)[-1])(W.c3_2d_const()),
}


@pytest.mark.parametrize("case,solver,shared", [("1d", "auto", 0), ("1d_tiled", "auto", 0), ("2d", "reference", 0),
                                                ("2d", "factor", 0), ("2d_const", "auto", 1)])
def test_components_match_the_oracle_and_scalar_runs(B, case, solver, shared):
    wl = CASES[case]()
    mesh, f, _, a = oracle_inputs(wl)
    phi0 = _fields(mesh.node_coords(), wl.dim)
    steps = 3
    got, mean, d = _run(B, wl, a, phi0, 3, steps, solver=solver, shared=shared)
    assert d["ncomp"] == 3
    nodes = mesh.total_nodes
    got = got.reshape(wl.samples, 3, nodes)
    mean = mean.reshape(3, nodes)
    for c in range(3):
        ref = sl.run(mesh, f, phi0[c], wl.dt, steps, wl.seed, np.arange(wl.samples))
        err = rel_l2(got[:, c], ref)
        node = float(np.max(np.abs(got[:, c] - ref)) / np.max(np.abs(ref)))
        print(f"{case} {solver} shared={shared} component {c}: rel L2 {err:.2e}, max node {node:.2e}")
        assert err < TOL and node < TOL
        assert rel_l2(mean[c], sl.mean(got[:, c])) < 1e-14
        one, _, _ = _run(B, wl, a, [phi0[c]], 1, steps, solver=solver, shared=shared)
        assert np.array_equal(one, got[:, c]), (case, c)
    if wl.dim == 2 and solver != "factor" and not shared:
        assert d["solver_unconverged"] == [0, 0]
