"""The paper's validation cases (Sec. 6.1, 6.4, 6.7) on the oracle: spectral
P-convergence, measured per sample against its pathwise exact solution.

With constant u and D, Euler-Maruyama is exact, so sample s after n steps is the
initial field translated by its own Wiener path, sqrt(2 D) sum_k sqrt(dt) z_k;
giving Dirichlet boundaries that same translated field as ghost values leaves
only the spatial (polynomial) error, which must fall exponentially in P (the
paper: 'exponential convergence in P for even and odd order polynomials
separately').  The closed-form solutions are the workloads'; the paths come
straight from the Philox draws."""
import math

import numpy as np
import pytest

from oracle import sl
from paper_2009_07340_amd import workloads as W

from helpers import oracle_inputs


def _paths(mesh, wl, samples):
    """Cumulative displacement sqrt(2 D dt) sum z of every sample after each step: (steps, M, d)."""
    zs = np.array([sl.wiener_normals(mesh, wl.seed, k, samples) for k in range(wl.steps)])
    return math.sqrt(2.0 * 1.0 * wl.dt) * np.cumsum(zs, axis=0)


def _pathwise_error(wl, samples=(0, 1, 2)):
    """Max |oracle - exact| over nodes and samples after wl.steps steps, one sample at a
    time (each sample's Dirichlet ghost values follow its own path)."""
    mesh, f, phi0, a = oracle_inputs(wl)
    ex = wl.meta["exact"]
    t0 = wl.meta["t0"]
    xy = mesh.node_coords()
    exy = mesh.edge_coords()
    worst = 0.0
    for s in samples:
        sv = np.array([s])
        w = _paths(mesh, wl, sv)[:, 0, :]                       # (steps, d)
        phi = phi0[None].copy()
        for k in range(wl.steps):
            if wl.bc == "dirichlet":
                sh = exy - w[k][None, :]
                f.ghost = ex(sh[:, 0], sh[:, 1] if wl.dim == 2 else None, t0)
            z = sl.wiener_normals(mesh, wl.seed, k, sv)
            phi, _ = sl.step(mesh, f, phi, wl.dt, z)
        sh = xy - w[-1][None, :]
        want = ex(sh[:, 0], sh[:, 1] if wl.dim == 2 else None, t0)
        worst = max(worst, float(np.max(np.abs(phi[0] - want))))
    return worst


def _assert_spectral(errs, floor):
    """Exponential convergence in P: within each parity class of P the error falls with
    every increase of P by 2 (until it reaches `floor`), and over the upper half of the
    range it falls by at least 2x per unit of P on average.  An algebraic error P^-k
    falls by ((P + 1) / P)^k per unit, about 1.4 for k = 4 at P = 12, so the second
    condition separates the two over the range tested."""
    Ns = sorted(errs)
    for par in (0, 1):
        seq = [(N, errs[N]) for N in Ns if (N - 1) % 2 == par]
        for (n1, e1), (n2, e2) in zip(seq, seq[1:]):
            assert e2 < e1 or e2 < floor, (n1, e1, n2, e2, errs)
    lo, hi = Ns[len(Ns) // 2], Ns[-1]
    rate = (max(errs[lo], floor) / max(errs[hi], floor)) ** (1.0 / (hi - lo))
    assert rate >= 2.0, (lo, hi, rate, errs)


def test_sec_6_1_sine_p_convergence():
    """Sec. 6.1 (one periodic element, D = 1, dt = 1e-5, 50 steps): P = 2..15."""
    errs = {}
    for N in range(3, 17):
        wl = W.paper_sine_1d(N, samples=3)
        errs[N] = _pathwise_error(wl)
    print({N: f"{e:.1e}" for N, e in errs.items()})
    _assert_spectral(errs, 1e-11)
    assert errs[16] < 1e-3 * errs[3]          # three decades and more over the range


def test_sec_6_4_gaussian_p_convergence():
    """Sec. 6.4 (the heat kernel from t0 = 0.05 on one element of [-1, 1], Dirichlet, 100 steps)."""
    errs = {}
    for N in range(4, 17):
        wl = W.paper_gaussian_1d(N, samples=3)
        errs[N] = _pathwise_error(wl, samples=(0, 1))
    print({N: f"{e:.1e}" for N, e in errs.items()})
    _assert_spectral(errs, 1e-9)
    assert errs[16] < 1e-3 * errs[4]


@pytest.mark.slow
def test_sec_6_7_sine_2d_p_convergence():
    """Sec. 6.7 (one element of [0, 1]^2, Dirichlet, D = 1, dt = 1e-5, 50 steps): P = 2..9."""
    errs = {}
    for N in range(3, 11):
        wl = W.paper_sine_2d(N, samples=2)
        errs[N] = _pathwise_error(wl, samples=(0, 1))
    print({N: f"{e:.1e}" for N, e in errs.items()})
    _assert_spectral(errs, 1e-10)
    assert errs[10] < 1e-3 * errs[3]
