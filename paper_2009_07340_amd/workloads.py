"""Seeded synthetic workloads: mesh descriptions, analytic fields and initial data.

This module generates inputs only.  It holds none of the semi-Lagrangian
method's arithmetic (no nodes, no bases, no fits): the caller passes the
physical coordinates at which fields are wanted, and gets arrays back.  The
same arrays feed the GPU library and the CPU oracle.

The four fixed workloads and the request stream are the drift-diffusion
problems of the measurement plan; their shapes follow the paper's test cases
(Sec. 6): periodic boxes, Gaussian pulses carried by constant, sinusoidal or
solid-body-rotation drift, constant or sinusoidal diffusion.  The paper's
own cases use no dataset; nothing here stands in for one.

Time steps.  The paper keeps the step small enough that the nodes do not
leave their element (eq. 1d_timestep: |u|max dt + sqrt(2 Dmax dt) <= dx_min,
dx_min the smallest physical spacing of two nodes).  With the least-squares
remap read here the one-step map has a spectral radius slightly above 1 that
grows quickly with the displacement (see the design notes), so long runs need
the displacement well inside that bound.  Two plan workloads ask for more
than the scheme tolerates over their step counts: the 1-D sinusoidal one
(plan dt = 2e-5, a one-sigma move of 5x the node spacing) overflows within
100 steps, and still diverges after ~600 steps at the eq. 1d_timestep value
7.5e-7; in the mixed-order rotation the N = 10 elements diverge at the plan's
2e-5.  Both run with dt from eq. 1d_timestep with half the node spacing,
dx_min / 2 (1-D: 0.038722 h / 2 for N = 12 Gauss-Legendre nodes, giving
1.9e-7; 2-D: 0.054422 h / 2 for N = 10, giving 5.8e-6), with the plan's step
counts; the work per step does not depend on dt.  ``dt_specified`` records
the plan's value.  The other two keep the plan's dt (stable over their runs).
"""
from dataclasses import dataclass, field
import math

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class Workload:
    name: str
    dim: int
    kx: int
    ky: int
    order: object            # int, or np.ndarray of per-element N
    samples: int
    dt: float
    steps: int
    seed: int
    u: object                # (x, y) -> (ux, uy) arrays
    D: object                # (x, y) -> D array
    divu: object             # (x, y) -> div u array
    phi0: object             # (x, y) -> initial field
    box: tuple = (0.0, 1.0, 0.0, 1.0)
    bc: str = "periodic"
    ghost: object = None     # (x, y, t) -> Dirichlet value, when bc == "dirichlet"
    dt_specified: float = None  # the measurement plan's dt when the one used differs (see module doc)
    meta: dict = field(default_factory=dict)

    @property
    def K(self):
        return self.kx * self.ky

    def order_array(self):
        if np.isscalar(self.order):
            return np.full(self.K, int(self.order), dtype=np.int32)
        return np.asarray(self.order, dtype=np.int32)

    def sample_fields(self, node_xy, edge_xy, edge_axis, t=0.0):
        """Arrays for the library / oracle from coordinates.

        node_xy: (nodes, d); edge_xy: (edge points, d); edge_axis: (edge points,)
        0 for a point on an x-normal edge, 1 for a y-normal edge.
        Returns dict u (nodes, d), D, divu, phi0 (nodes,), un, Dn, ghost (edge points,).
        """
        node_xy = np.asarray(node_xy, dtype=np.float64).reshape(-1, self.dim)
        edge_xy = np.asarray(edge_xy, dtype=np.float64).reshape(-1, self.dim)
        xn = node_xy[:, 0]
        yn = node_xy[:, 1] if self.dim == 2 else np.zeros_like(xn)
        xe = edge_xy[:, 0]
        ye = edge_xy[:, 1] if self.dim == 2 else np.zeros_like(xe)
        ux, uy = self.u(xn, yn)
        u = np.stack([np.broadcast_to(ux, xn.shape), np.broadcast_to(uy, xn.shape)][:self.dim], 1)
        uex, uey = self.u(xe, ye)
        uex = np.broadcast_to(uex, xe.shape)
        uey = np.broadcast_to(uey, xe.shape)
        axis = np.asarray(edge_axis).reshape(-1)
        un = np.where(axis == 0, uex, uey)
        out = dict(u=np.ascontiguousarray(u, dtype=np.float64),
                   D=np.ascontiguousarray(np.broadcast_to(self.D(xn, yn), xn.shape), dtype=np.float64),
                   divu=np.ascontiguousarray(np.broadcast_to(self.divu(xn, yn), xn.shape), dtype=np.float64),
                   phi0=np.ascontiguousarray(np.broadcast_to(self.phi0(xn, yn), xn.shape), dtype=np.float64),
                   un=np.ascontiguousarray(un, dtype=np.float64),
                   Dn=np.ascontiguousarray(np.broadcast_to(self.D(xe, ye), xe.shape), dtype=np.float64),
                   ghost=None)
        if self.bc == "dirichlet":
            if self.ghost is None:
                raise ValueError("Dirichlet workload needs a ghost function")
            out["ghost"] = np.ascontiguousarray(np.broadcast_to(self.ghost(xe, ye, t), xe.shape), dtype=np.float64)
        return out


def gauss1(x, c, s, a=1.0):
    return a * np.exp(-((x - c) ** 2) / (2.0 * s * s))


def const(v):
    return lambda x, y: np.full(np.shape(x), float(v))


# --- the four fixed workloads -------------------------------------------------

def c1_1d_const():
    """1-D, K=16, N=8, M=64, u=1, D=0.01, Gaussian at 0.3 (sigma 0.05), dt=1e-4, 100 steps, seed 1."""
    return Workload("1d_const_K16_N8_M64", 1, 16, 1, 8, 64, 1e-4, 100, 1,
                    u=lambda x, y: (np.full(np.shape(x), 1.0), np.zeros(np.shape(x))),
                    D=const(0.01), divu=const(0.0),
                    phi0=lambda x, y: gauss1(x, 0.3, 0.05))


def c2_1d_sine():
    """1-D, K=256, N=12, M=1024, u=0.5+sin 2pi x, D=0.01(1+0.5 cos 2pi x), two Gaussians, 1000 steps, seed 7.

    dt = 1.9e-7 from eq. 1d_timestep with half the node spacing (the plan's 2e-5 diverges, see the module doc)."""
    return Workload("1d_sine_K256_N12_M1024", 1, 256, 1, 12, 1024, 1.9e-7, 1000, 7, dt_specified=2e-5,
                    u=lambda x, y: (0.5 + np.sin(TWO_PI * x), np.zeros(np.shape(x))),
                    D=lambda x, y: 0.01 * (1.0 + 0.5 * np.cos(TWO_PI * x)),
                    divu=lambda x, y: TWO_PI * np.cos(TWO_PI * x),
                    phi0=lambda x, y: gauss1(x, 0.25, 0.03, 1.0) + gauss1(x, 0.7, 0.05, 0.5))


def c3_2d_const():
    """2-D 64x64, N=8, M=256, u=(1,0.5), D=0.005, Gaussian at (0.3,0.3) sigma 0.05, dt=5e-5, 200 steps, seed 3."""
    return Workload("2d_const_64x64_N8_M256", 2, 64, 64, 8, 256, 5e-5, 200, 3,
                    u=lambda x, y: (np.full(np.shape(x), 1.0), np.full(np.shape(x), 0.5)),
                    D=const(0.005), divu=const(0.0),
                    phi0=lambda x, y: np.exp(-((x - 0.3) ** 2 + (y - 0.3) ** 2) / (2.0 * 0.05 ** 2)))


def c4_orders(kx=128, ky=128, seed=11, choices=(6, 8, 10)):
    """Per-element N drawn uniformly from ``choices`` with numpy PCG64(seed)."""
    return np.random.Generator(np.random.PCG64(seed)).choice(np.asarray(choices), size=kx * ky).astype(np.int32)


def c4_2d_rotation(kx=128, ky=128, samples=512, steps=500):
    """2-D 128x128, N~U{6,8,10}, M=512, solid-body rotation, D=0.002(1+0.5 sin sin), Gaussian at (0.5,0.75) sigma 0.04, 500 steps, seed 11.

    dt = 5.8e-6 from eq. 1d_timestep with half the node spacing (the plan's 2e-5 diverges for N = 10)."""
    return Workload("2d_rot_128x128_N6-10_M512", 2, kx, ky, c4_orders(kx, ky), samples, 5.8e-6, steps, 11,
                    dt_specified=2e-5,
                    u=lambda x, y: (-TWO_PI * (y - 0.5), TWO_PI * (x - 0.5)),
                    D=lambda x, y: 0.002 * (1.0 + 0.5 * np.sin(TWO_PI * x) * np.sin(TWO_PI * y)),
                    divu=const(0.0),
                    phi0=lambda x, y: np.exp(-((x - 0.5) ** 2 + (y - 0.75) ** 2) / (2.0 * 0.04 ** 2)))


WORKLOADS = {"c1": c1_1d_const, "c2": c2_1d_sine, "c3": c3_2d_const, "c4": c4_2d_rotation}


# --- request stream for the serving loop ---------------------------------------

def serving_requests(n=2000, rate=50.0, seed=2026, kmax=4096, mmax=2048):
    """Independent drift-diffusion requests with Poisson arrival times.

    60% 1-D / 40% 2-D; K log-uniform in [16, kmax] elements (2-D: a square
    kx = ky = round(sqrt(K))); N uniform in {4..16}; M log-uniform in
    [32, mmax]; drift and diffusion constant or sinusoidal with amplitudes in
    the ranges of the fixed workloads; 50-500 steps; per-request seed 1000+i.
    Each request's dt follows eq. 1d_timestep with the asymptotic smallest
    Gauss-Legendre node spacing 5.9 h / (N + 1/2)^2 (halved in 2-D):
    |u|max dt + sqrt(2 Dmax dt) = c * 5.9 h / (N + 1/2)^2, c = 1 (1-D), 1/2 (2-D).
    """
    g = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(g.exponential(1.0 / rate, size=n))
    reqs = []
    for i in range(n):
        dim = 1 if g.random() < 0.6 else 2
        K = int(round(math.exp(g.uniform(math.log(16), math.log(kmax)))))
        N = int(g.integers(4, 17))
        M = int(round(math.exp(g.uniform(math.log(32), math.log(mmax)))))
        steps = int(g.integers(50, 501))
        sinus = bool(g.random() < 0.5)
        u0 = float(g.uniform(0.5, 1.0))
        ua = float(g.uniform(0.0, 1.0)) if sinus else 0.0
        D0 = float(g.uniform(0.002, 0.01))
        Da = 0.5 if sinus else 0.0
        if dim == 1:
            kx, ky = K, 1
        else:
            kx = ky = max(1, int(round(math.sqrt(K))))
        h = 1.0 / kx
        umax, Dmax = u0 + ua, D0 * (1.0 + Da)
        # solve umax dt + sqrt(2 Dmax dt) = c' 5.9 h / (N + 1/2)^2 for dt (quadratic in sqrt(dt)):
        # eq. 1d_timestep with the asymptotic smallest node spacing, c' = 1 in 1-D, 1/2 in 2-D
        a, b, c = umax, math.sqrt(2.0 * Dmax), -(1.0 if dim == 1 else 0.5) * 5.9 * h / (N + 0.5) ** 2
        sdt = (-b + math.sqrt(b * b - 4 * a * c)) / (2 * a)
        dt = sdt * sdt
        reqs.append(dict(id=i, arrival=float(t[i]), dim=dim, kx=kx, ky=ky, N=N, M=M, steps=steps,
                         sinus=sinus, u0=u0, ua=ua, D0=D0, Da=Da, dt=dt, seed=1000 + i))
    return reqs


def request_workload(r):
    """Workload object for one serving request dict."""
    u0, ua, D0, Da = r["u0"], r["ua"], r["D0"], r["Da"]
    if r["dim"] == 1:
        u = lambda x, y: (u0 + ua * np.sin(TWO_PI * x), np.zeros(np.shape(x)))
        D = lambda x, y: D0 * (1.0 + Da * np.cos(TWO_PI * x))
        divu = lambda x, y: ua * TWO_PI * np.cos(TWO_PI * x)
        phi0 = lambda x, y: gauss1(x, 0.3, 0.05)
    else:
        u = lambda x, y: (u0 + ua * np.sin(TWO_PI * y), 0.5 * u0 + ua * np.sin(TWO_PI * x))
        D = lambda x, y: D0 * (1.0 + Da * np.sin(TWO_PI * x) * np.sin(TWO_PI * y))
        divu = const(0.0)
        phi0 = lambda x, y: np.exp(-((x - 0.3) ** 2 + (y - 0.3) ** 2) / (2.0 * 0.05 ** 2))
    return Workload(f"req{r['id']}", r["dim"], r["kx"], r["ky"], r["N"], r["M"], r["dt"], r["steps"],
                    r["seed"], u=u, D=D, divu=divu, phi0=phi0)


# --- the paper's validation cases (Sec. 6) ---------------------------------------
#
# Inputs at the paper's parameters.  `exact(x, y, t)` is the closed-form mean
# field of each case (a solution of the drift-diffusion equation, not part of
# the method), used for Dirichlet ghost values and by the validation checks;
# meta["t0"] is the time of the initial field.

def paper_sine_1d(N, samples=1_000_000, kx=1):
    """Sec. 6.1: [0, 1] periodic, u = 0, D = 1, phi0 = sin(2 pi x) + 2, dt = 1e-5, 50 steps, H = 1.
    Mean: exp(-4 pi^2 t) sin(2 pi x) + 2."""
    ex = lambda x, y, t: np.exp(-4.0 * math.pi ** 2 * t) * np.sin(TWO_PI * x) + 2.0
    return Workload("paper_6_1_sine", 1, kx, 1, N, samples, 1e-5, 50, 61,
                    u=lambda x, y: (np.zeros(np.shape(x)), np.zeros(np.shape(x))), D=const(1.0),
                    divu=const(0.0), phi0=lambda x, y: ex(x, y, 0.0), meta=dict(exact=ex, t0=0.0))


def paper_gaussian_1d(N, samples=1_000_000, kx=1):
    """Sec. 6.4: [-1, 1], u = 0, D = 1, phi = exp(-x^2 / (4 t)) / sqrt(4 pi t) from t0 = 0.05,
    Dirichlet ghost values from that solution, dt = 1e-5, 100 steps, H = 1."""
    ex = lambda x, y, t: np.exp(-np.asarray(x) ** 2 / (4.0 * t)) / math.sqrt(4.0 * math.pi * t)
    t0 = 0.05
    return Workload("paper_6_4_gaussian", 1, kx, 1, N, samples, 1e-5, 100, 64,
                    u=lambda x, y: (np.zeros(np.shape(x)), np.zeros(np.shape(x))), D=const(1.0),
                    divu=const(0.0), phi0=lambda x, y: ex(x, y, t0), box=(-1.0, 1.0, 0.0, 1.0),
                    bc="dirichlet", ghost=lambda x, y, t: ex(x, y, t0 + t), meta=dict(exact=ex, t0=t0))


def paper_ou_1d(N=16, samples=100, dt=1e-4, kx=1):
    """Sec. 6.5: Ornstein-Uhlenbeck, u = -alpha x (alpha = 1, div u = -1), D = 1, x0 = 2, on
    [-4, 6], Dirichlet ghost values from the density, from t = 0.25 to t = 1, re-seeded every
    100 steps, Ns = 100.  The paper runs P = 17; the library's largest order is N = 16 (P = 15).
    The paper does not give dt; 1e-4 keeps the move a tenth of the smallest node spacing.
    Density (tau = t, the process started from x0 at t = 0):
    sqrt(a / (2 pi D (1 - e^{-2 a t}))) exp(-a (x - x0 e^{-a t})^2 / (2 D (1 - e^{-2 a t})))."""
    a, D, x0, t0 = 1.0, 1.0, 2.0, 0.25

    def ex(x, y, t):
        v = 1.0 - math.exp(-2.0 * a * t)
        return math.sqrt(a / (2.0 * math.pi * D * v)) * np.exp(-a * (np.asarray(x) - x0 * math.exp(-a * t)) ** 2
                                                               / (2.0 * D * v))
    steps = int(round((1.0 - t0) / dt))
    return Workload("paper_6_5_ou", 1, kx, 1, N, samples, dt, steps, 65,
                    u=lambda x, y: (-a * np.asarray(x), np.zeros(np.shape(x))), D=const(D),
                    divu=const(-a), phi0=lambda x, y: ex(x, y, t0), box=(-4.0, 6.0, 0.0, 1.0),
                    bc="dirichlet", ghost=lambda x, y, t: ex(x, y, t0 + t),
                    meta=dict(exact=ex, t0=t0, reseed_every=100))


def paper_sine_2d(N, samples=10_000, kx=1):
    """Sec. 6.7: [0, 1]^2, u = 0, D = 1, phi0 = sin(2 pi x) sin(2 pi y) + 2, Dirichlet ghost
    values from the solution exp(-8 pi^2 t) sin(2 pi x) sin(2 pi y) + 2, dt = 1e-5, 50 steps, H = 1."""
    ex = lambda x, y, t: np.exp(-8.0 * math.pi ** 2 * t) * np.sin(TWO_PI * x) * np.sin(TWO_PI * y) + 2.0
    return Workload("paper_6_7_sine2d", 2, kx, kx, N, samples, 1e-5, 50, 67,
                    u=lambda x, y: (np.zeros(np.shape(x)), np.zeros(np.shape(x))), D=const(1.0),
                    divu=const(0.0), phi0=lambda x, y: ex(x, y, 0.0), bc="dirichlet",
                    ghost=lambda x, y, t: ex(x, y, t), meta=dict(exact=ex, t0=0.0))


PAPER_CASES = {"6.1": paper_sine_1d, "6.4": paper_gaussian_1d, "6.5": paper_ou_1d, "6.7": paper_sine_2d}
