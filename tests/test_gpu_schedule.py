"""Launch schedules of the step: per-order kernels, the persistent fused kernel,
hipGraph replay, batched steps of several problems and the autotuner.  The
method fixes the result, not the schedule, so every schedule must reproduce
the per-order direct launches bit for bit (and those match the oracle).  One
exception: the wide fit shape of the per-order kernels (twice the wavefronts a
fit up to order 12) orders its sums differently and must agree to rounding
(FUSED_TOL)."""
import numpy as np
import pytest

from oracle import sl
from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-11
FUSED_TOL = 1e-13


def _same(got, want, rounding):
    """Bitwise, or (rounding) within FUSED_TOL in relative L2 and per node."""
    if not rounding:
        return np.array_equal(got, want)
    scale = np.max(np.abs(want))
    return rel_l2(got, want) <= FUSED_TOL and np.max(np.abs(got - want)) <= FUSED_TOL * scale

MIXED = np.array([6, 8, 10, 6, 8, 6, 10, 8, 10, 2, 8, 3, 8, 10, 6, 4], dtype=np.int32)

# (fused, graph, grid, shared, wide)
SCHEDULES = [(0, 1, 0, 0, 0), (1, 0, 0, 0, 0), (1, 0, 5, 0, 0), (1, 1, 0, 0, 0), (1, 1, 7, 0, 0), (0, 0, 0, 0, 1),
             (0, 1, 0, 0, 1)]


@pytest.fixture(scope="module")
def B():
    from paper_2009_07340_amd import binding
    return binding


def _mixed_wl(samples=3):
    wl = W.c4_2d_rotation(kx=4, ky=4, samples=samples, steps=3)
    wl.order = MIXED.copy()
    wl.dt = 2e-4
    return wl


def _make(B, wl, precision="fp64", samples=None, ncomp=1, mass=False):
    mesh, f, phi0, a = oracle_inputs(wl)
    order = wl.order if np.isscalar(wl.order) else wl.order_array()
    desc = B.make_desc(wl.dim, wl.kx, wl.ky, wl.box, order, bc=wl.bc, samples=samples or wl.samples,
                       seed=wl.seed, precision=precision, ncomp=ncomp, mass=mass)
    h = B.sl_init_mesh(desc)
    p0 = np.concatenate([a["phi0"] * (1.0 + 0.1 * c) for c in range(ncomp)])
    B.sl_set_fields(h, a["u"], a["D"], a["divu"], a["un"], a["Dn"], a["ghost"], p0)
    return h, (mesh, f, phi0)


def _run(B, wl, sched, steps, precision="fp64", **kw):
    h, _ = _make(B, wl, precision, **kw)
    try:
        if sched is not None:
            B.sl_set_schedule(h, *sched)
        for n in steps:
            B.sl_step(h, wl.dt, n)
        out = B.sl_get_samples(h, 0, wl.samples)
        assert B.sl_get_step(h) == sum(steps)
        return out
    finally:
        B.sl_destroy(h)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine", "bf16split_refine"])
def test_every_schedule_is_bitwise_equal(B, precision):
    wl = _mixed_wl()
    ref = _run(B, wl, None, [3], precision)
    for sched in SCHEDULES:
        got = _run(B, wl, sched, [1, 2], precision)
        print(f"{precision} schedule {sched}: max |diff| {np.max(np.abs(got - ref)):.3e}", flush=True)
        # fp64 runs the reference solver (the automatic choice); the mixed modes the
        # factorisation, whose kernels have one fit shape
        assert _same(got, ref, precision == "fp64" and sched[4] == 1), (precision, sched)
    if precision == "fp64":
        mesh, f, phi0, a = oracle_inputs(wl)
        want = sl.run(mesh, f, phi0, wl.dt, 3, wl.seed, np.arange(wl.samples))
        assert rel_l2(ref, want) < TOL


@pytest.mark.parametrize("graph", [0, 1])
def test_wide_fit_shape_matches_the_default_and_the_oracle(B, graph):
    """Every order the wide shape changes (2..12: one wavefront a fit becomes two, two
    become four) and some it leaves alone (13, 16), direct and as a graph."""
    wl = W.c4_2d_rotation(kx=3, ky=3, samples=2, steps=3)
    wl.order = np.array([9, 11, 12, 13, 5, 7, 2, 16, 10], dtype=np.int32)
    wl.dt = 2e-4
    ref = _run(B, wl, None, [2])
    got = _run(B, wl, (0, graph, 0, 0, 1), [1, 1])
    print(f"wide graph={graph}: max |diff| {np.max(np.abs(got - ref)):.3e}", flush=True)
    assert _same(got, ref, True)
    mesh, f, phi0, a = oracle_inputs(wl)
    want = sl.run(mesh, f, phi0, wl.dt, 2, wl.seed, np.arange(wl.samples))
    assert rel_l2(got, want) < TOL
    assert np.max(np.abs(got - want)) <= TOL * np.max(np.abs(want))


@pytest.mark.parametrize("kw", [{"ncomp": 2}, {"mass": True}])
def test_wide_fit_shape_of_the_general_form(B, kw):
    """Several components, or the mass constraint: the full phase-1 form and the
    general phase-2 form in the wide shape agree with the default shape."""
    wl = _mixed_wl(samples=2)
    ref = _run(B, wl, None, [2], **kw)
    got = _run(B, wl, (0, 0, 0, 0, 1), [2], **kw)
    print(f"wide {kw}: max |diff| {np.max(np.abs(got - ref)):.3e}", flush=True)
    assert _same(got, ref, True)


def test_graph_follows_step_counter_and_dt(B):
    """A cached graph reads the device step counter and the current coefficients."""
    wl = _mixed_wl(samples=2)
    outs = []
    for sched in [None, (1, 1, 0), (0, 1, 0)]:
        h, _ = _make(B, wl)
        try:
            if sched:
                B.sl_set_schedule(h, *sched)
            B.sl_step(h, wl.dt, 2)
            B.sl_set_step(h, 40)
            B.sl_step(h, 0.5 * wl.dt, 1)
            B.sl_step(h, wl.dt, 1)
            assert B.sl_get_step(h) == 42
            outs.append(B.sl_get_samples(h, 0, wl.samples))
        finally:
            B.sl_destroy(h)
    assert np.array_equal(outs[1], outs[0])
    assert np.array_equal(outs[0], outs[2])


def _batch_members():
    """Problems of different dimension, size, order mix, sample count, boundary and precision."""
    a = _mixed_wl(samples=3)
    b = W.c3_2d_const()
    b.kx, b.ky, b.samples, b.order, b.bc = 3, 2, 5, 4, "dirichlet"
    b.ghost = lambda x, y, t: 0.25 + 0.0 * x
    c = W.c4_2d_rotation(kx=2, ky=3, samples=2, steps=3)
    c.order = 6
    d = W.c1_1d_const()
    d.samples = 8
    e = W.c1_1d_const()
    e.kx, e.order, e.samples, e.bc = 5, 3, 7, "dirichlet"
    e.ghost = lambda x, y, t: 0.1 + 0.0 * x
    f = W.c2_1d_sine()            # more than 256 elements: tiled steps
    f.kx, f.order, f.samples = 400, 6, 3
    g = W.c4_2d_rotation(kx=2, ky=2, samples=2, steps=3)
    g.order = np.array([12, 16, 14, 11], dtype=np.int32)
    return [(a, "fp64", 2e-4), (b, "fp64", 3e-4), (c, "fp32_refine", 1e-4), (d, "fp64", 1e-4), (e, "fp64", 2e-4),
            (f, "fp64", 2e-7), (g, "fp64", 5e-5)]


@pytest.mark.parametrize("fused,graph", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_batch_equals_each_problem_alone(B, fused, graph):
    members = _batch_members()
    alone = []
    for wl, prec, dt in members:
        h, _ = _make(B, wl, prec)
        try:
            B.sl_step(h, dt, 2)
            B.sl_step(h, dt, 1)
            alone.append(B.sl_get_samples(h, 0, wl.samples))
        finally:
            B.sl_destroy(h)
    hs = []
    try:
        for wl, prec, dt in members:
            h, _ = _make(B, wl, prec)
            B.sl_set_schedule(h, fused, graph, 0)
            hs.append(h)
        dts = [dt for _, _, dt in members]
        B.sl_step_batch(hs, dts, 2)
        B.sl_step_batch(hs, dts, 1)
        for (wl, prec, _), h, want in zip(members, hs, alone):
            assert B.sl_get_step(h) == 3
            got = B.sl_get_samples(h, 0, wl.samples)
            assert np.array_equal(got, want), wl.name
    finally:
        for h in hs:
            B.sl_destroy(h)


@pytest.mark.parametrize("fused", [0, 1])
def test_batch_of_many_problems_is_chunked(B, fused):
    """More problems than one launch takes: chunked launches, same results."""
    members = []
    for i in range(40):
        wl = W.c3_2d_const()
        wl.kx, wl.ky, wl.samples, wl.order = 1 + i % 3, 1 + (i // 3) % 2, 1 + i % 4, [2, 3, 4, 5][i % 4]
        members.append(wl)
    for i in range(36):
        wl = W.c1_1d_const()
        wl.kx, wl.order, wl.samples = 2 + i % 5, 4, 1 + i % 3
        members.append(wl)
    alone, hs = [], []
    try:
        for wl in members:
            h, _ = _make(B, wl)
            B.sl_step(h, wl.dt, 2)
            alone.append(B.sl_get_samples(h, 0, wl.samples))
            B.sl_destroy(h)
        for wl in members:
            h, _ = _make(B, wl)
            B.sl_set_schedule(h, fused, 1, 0)
            hs.append(h)
        B.sl_step_batch(hs, [wl.dt for wl in members], 2)
        for wl, h, want in zip(members, hs, alone):
            assert np.array_equal(B.sl_get_samples(h, 0, wl.samples), want)
    finally:
        for h in hs:
            B.sl_destroy(h)


def test_batch_argument_errors(B):
    wl = _mixed_wl(samples=1)
    h, _ = _make(B, wl)
    try:
        with pytest.raises(B.SLError) as ei:
            B.sl_step_batch([h, h], [wl.dt, wl.dt], 1)
        assert ei.value.code == B.SL_EINVAL
        with pytest.raises(B.SLError):
            B.sl_step_batch([h], [-1.0], 1)
        B.sl_step_batch([], [], 3)
        assert B.sl_get_step(h) == 0
    finally:
        B.sl_destroy(h)


def test_autotune_reads_cache_lines_without_a_fit_shape(B, tmp_path):
    """A cache line written before the fit shape was a choice (five fields) is a hit
    with the default shape."""
    wl = _mixed_wl(samples=2)
    cache = tmp_path / "tune.txt"
    h, _ = _make(B, wl)
    h2 = None
    try:
        B.sl_autotune(h, wl.dt, 1, cache)
        fields = cache.read_text().split()
        assert len(fields) == 6
        cache.write_text(" ".join(fields[:1] + ["0", "1", "0", "1.5"]) + "\n")   # per-order graph, no shape field
        h2, _ = _make(B, wl)
        s = B.sl_autotune(h2, wl.dt, 1, cache)
        assert (s["fused"], s["graph"], s["grid"], s["wide"]) == (0, 1, 0, 0)
        assert len(cache.read_text().splitlines()) == 1
    finally:
        B.sl_destroy(h)
        if h2 is not None:
            B.sl_destroy(h2)


def test_autotune_restores_state_and_uses_its_cache(B, tmp_path):
    wl = _mixed_wl(samples=4)
    cache = tmp_path / "tune.txt"
    h, _ = _make(B, wl)
    h2 = None
    try:
        B.sl_step(h, wl.dt, 1)
        before = B.sl_get_samples(h, 0, wl.samples)
        s = B.sl_autotune(h, wl.dt, 2, cache)
        assert s["fused"] in (0, 1) and s["graph"] in (0, 1) and s["wide"] in (0, 1) and s["ms_per_step"] > 0
        assert not (s["fused"] and s["wide"])
        assert B.sl_get_step(h) == 1
        assert np.array_equal(B.sl_get_samples(h, 0, wl.samples), before)
        assert len(cache.read_text().splitlines()) == 1
        B.sl_step(h, wl.dt, 2)
        tuned = B.sl_get_samples(h, 0, wl.samples)
        h2, _ = _make(B, wl)
        s2 = B.sl_autotune(h2, wl.dt, 2, cache)       # cache hit: no timing, same choice
        assert (s2["fused"], s2["graph"], s2["grid"], s2["wide"]) == (s["fused"], s["graph"], s["grid"], s["wide"])
        assert len(cache.read_text().splitlines()) == 1
        B.sl_set_schedule(h2, 0, 0, 0)
        B.sl_step(h2, wl.dt, 3)
        assert _same(B.sl_get_samples(h2, 0, wl.samples), tuned, s["wide"] == 1)
    finally:
        B.sl_destroy(h)
        if h2 is not None:
            B.sl_destroy(h2)
