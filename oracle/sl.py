"""The DSEM-SL Monte-Carlo step, restated plainly in float64 numpy.

TEST INFRASTRUCTURE (see the package doc): only tests/, the smoke check and
the CPU baseline of the benchmark call this module.

Notation follows Secs. 3 and 5 of the paper.  A mesh is a box split into
kx (x ky) equal affine elements; element e carries N_e Gauss nodes per
direction (n_e = N_e^d nodes).  One Monte-Carlo sample s is one polynomial
field; samples never interact.  One step of one sample, per element:

  1. Wiener increment dW = sqrt(dt) z with z from ``rng.normal_pair`` (one per
     sample, step and direction, shared by all nodes; Sec. 5.2).
  2. Move each node by Euler-Maruyama in physical coordinates (eq. def_dx),
     written in reference coordinates of the element:
        xi* = xi + (A + B z),  A = (u dt) / h,  B = sqrt((2 D) dt) / h.
  3. Carry the node value along with the composition-space source
     S = -psi div(u) (eq. advection_phi):  f = phi (1 - dt div u).
  4. The advected interpolant p0 in Q_{N-1} takes the value f at the moved
     nodes (eqs. phi_stardef, h_star).  Its values at the element's own edge
     points are the traces t (eq. remap_bnd).
  5. Upwinding (eq. bnd_update): at each edge point the displacement of the
     interface, disp = (un dt)/h + (sqrt((2 Dn) dt)/h) z, decides the source:
     disp > 0 takes the element on the negative side of the interface, else
     the one on the positive side; outside the domain a periodic image or the
     Dirichlet ghost value takes the neighbour's place (Sec. 5.3).
  6. Constrained least-squares remap (Sec. 5.3, last paragraphs; abstract):
        p = argmin_{q in Q_{N-1}} sum_i (q(xi*_i) - f_i)^2
            subject to q(edge points) = P g,
     P the orthogonal projector onto the edge-value vectors that polynomials
     of Q_{N-1} can take (rank 2 in 1-D, 4N-4 in 2-D).  With V the square
     basis matrix at the moved nodes and C at the edge points, the values of
     p at the moved nodes are a = f - pinv(C V^-1) (t - g).
  7. New node values phi = p(xi_i) at the Gauss nodes (eq. phi_star).

The mean over samples is eq. averaged; the norms are eqs. l2_error,
mass_cons and energy_cons.

Polynomials are written in the orthonormal Legendre basis centred on the
mean displacement dbar of the element's nodes: psi_k(xi - dbar).  This is a
conditioning choice only: Q_{N-1} is shift invariant, so p is unchanged.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from . import rng, tables

EDGE_W, EDGE_E, EDGE_S, EDGE_N = 0, 1, 2, 3
EDGE_L, EDGE_R = 0, 1


@dataclass
class Mesh:
    """Box of kx (x ky) equal elements; ``order`` holds N per element (e = ey*kx + ex)."""
    dim: int
    kx: int
    ky: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    order: np.ndarray = None
    family: str = "gl"
    bc: str = "periodic"
    mass: bool = False          # also keep each element's integral of p0 (see constrained_values)
    _cache: dict = field(default_factory=dict, repr=False)

    def __post_init__(self):
        if self.dim not in (1, 2):
            raise ValueError("dim must be 1 or 2")
        if self.dim == 1:
            self.ky = 1
        self.order = np.asarray(self.order, dtype=np.int64).reshape(-1)
        if self.order.size == 1:
            self.order = np.full(self.K, int(self.order[0]), dtype=np.int64)
        if self.order.size != self.K or np.any(self.order < 2):
            raise ValueError("order must give N >= 2 for every element")
        if self.bc not in ("periodic", "dirichlet"):
            raise ValueError("bc must be 'periodic' or 'dirichlet'")

    @property
    def K(self):
        return self.kx * self.ky

    @property
    def hx(self):
        return (self.x1 - self.x0) / self.kx

    @property
    def hy(self):
        return (self.y1 - self.y0) / self.ky

    @property
    def n_nodes(self):
        return self.order ** self.dim

    @property
    def n_edge(self):
        return np.full(self.K, 2) if self.dim == 1 else 4 * self.order

    @property
    def node_offset(self):
        return np.concatenate([[0], np.cumsum(self.n_nodes)])

    @property
    def edge_offset(self):
        return np.concatenate([[0], np.cumsum(self.n_edge)])

    @property
    def total_nodes(self):
        return int(self.node_offset[-1])

    @property
    def total_edge(self):
        return int(self.edge_offset[-1])

    def exy(self, e):
        return e % self.kx, e // self.kx

    def neighbour(self, e, edge):
        """Neighbour across ``edge`` of element e, or -1 at a Dirichlet boundary."""
        ex, ey = self.exy(e)
        if self.dim == 1:
            dx, dy = (-1, 0) if edge == EDGE_L else (1, 0)
        else:
            dx, dy = {EDGE_W: (-1, 0), EDGE_E: (1, 0), EDGE_S: (0, -1), EDGE_N: (0, 1)}[edge]
        nx, ny = ex + dx, ey + dy
        if self.bc == "periodic":
            nx %= self.kx
            ny %= self.ky
        elif not (0 <= nx < self.kx and 0 <= ny < self.ky):
            return -1
        return ny * self.kx + nx

    def ref_nodes(self, N):
        """Reference coordinates of the n = N^d nodes, node i = iy*N + ix: shape (n, d)."""
        xi = tables.nodes(int(N), self.family)
        if self.dim == 1:
            return xi[:, None].copy()
        ix = np.tile(np.arange(N), N)
        iy = np.repeat(np.arange(N), N)
        return np.stack([xi[ix], xi[iy]], axis=1)

    def ref_edge_points(self, N, edge, npts=None):
        """Reference coordinates of the edge points of an order-N element on ``edge``.

        ``npts`` selects the abscissae of another order (the receiving element's),
        used when evaluating a neighbour's polynomial at a receiver's points.
        """
        if self.dim == 1:
            return np.array([[0.0]]) if edge == EDGE_L else np.array([[1.0]])
        m = int(N if npts is None else npts)
        eta = np.asarray(tables.nodes(m, self.family))
        zero, one = np.zeros(m), np.ones(m)
        return {EDGE_W: np.stack([zero, eta], 1), EDGE_E: np.stack([one, eta], 1),
                EDGE_S: np.stack([eta, zero], 1), EDGE_N: np.stack([eta, one], 1)}[edge]

    def node_coords(self):
        """Physical node coordinates x = x0 + h (ex + xi): shape (total_nodes, d)."""
        out = np.empty((self.total_nodes, self.dim))
        off = self.node_offset
        for e in range(self.K):
            ex, ey = self.exy(e)
            r = self.ref_nodes(self.order[e])
            out[off[e]:off[e + 1], 0] = self.x0 + self.hx * (ex + r[:, 0])
            if self.dim == 2:
                out[off[e]:off[e + 1], 1] = self.y0 + self.hy * (ey + r[:, 1])
        return out

    def edge_coords(self):
        """Physical coordinates of every element's edge points: shape (total_edge, d)."""
        out = np.empty((self.total_edge, self.dim))
        off = self.edge_offset
        for e in range(self.K):
            ex, ey = self.exy(e)
            N = int(self.order[e])
            nedges = 2 if self.dim == 1 else 4
            per = 1 if self.dim == 1 else N
            for w in range(nedges):
                r = self.ref_edge_points(N, w)
                sl = slice(off[e] + w * per, off[e] + (w + 1) * per)
                out[sl, 0] = self.x0 + self.hx * (ex + r[:, 0])
                if self.dim == 2:
                    out[sl, 1] = self.y0 + self.hy * (ey + r[:, 1])
        return out

    def groups(self):
        """Elements grouped by order: {N: element index array}."""
        if "groups" not in self._cache:
            self._cache["groups"] = {int(N): np.nonzero(self.order == N)[0] for N in np.unique(self.order)}
        return self._cache["groups"]


@dataclass
class Fields:
    """Drift, diffusion and boundary data sampled where the mesh asks for them.

    u: (total_nodes, d) drift at the nodes; D: (total_nodes,) diffusion
    coefficient (sigma = sqrt(2D), eq. fokkerplanck); divu: (total_nodes,)
    physical divergence of u (0 when None); un: (total_edge,) normal component
    of u (along +x on W/E edges, +y on S/N edges); Dn: (total_edge,) D at the
    edge points; ghost: (total_edge,) Dirichlet ghost values at the edge points.
    """
    u: np.ndarray
    D: np.ndarray
    divu: np.ndarray = None
    un: np.ndarray = None
    Dn: np.ndarray = None
    ghost: np.ndarray = None


def _basis(pts, dbar, N, dim):
    """Rows psi_k(x - dbar_x) [psi_l(y - dbar_y)] at reference points.

    pts: (..., m, d); dbar: (..., d).  Returns (..., m, N^d), column p = l*N + k.
    """
    px = tables.legendre_basis(pts[..., 0] - dbar[..., None, 0], N)
    if dim == 1:
        return px
    py = tables.legendre_basis(pts[..., 1] - dbar[..., None, 1], N)
    out = py[..., :, :, None] * px[..., :, None, :]
    return out.reshape(out.shape[:-2] + (N * N,))


def wiener_normals(mesh, seed, step, samples, stream=0):
    """z for each sample: shape (M, d) (Sec. 5.2: one increment per sample and direction)."""
    za, zb = rng.normal_pair(seed, step, samples, stream)
    return za[:, None] if mesh.dim == 1 else np.stack([za, zb], 1)


def positions(mesh, fields, dt, z):
    """Moved reference coordinates xi* of every node, shape (M, total_nodes, d) (eq. def_dx)."""
    xi = np.concatenate([mesh.ref_nodes(N) for N in mesh.order], axis=0)
    h = np.array([mesh.hx, mesh.hy][:mesh.dim])
    u = np.asarray(fields.u, dtype=np.float64).reshape(mesh.total_nodes, mesh.dim)
    D = np.asarray(fields.D, dtype=np.float64).reshape(mesh.total_nodes)
    A = (u * dt) / h
    B = np.sqrt((2.0 * D) * dt)[:, None] / h
    return xi[None] + (A[None] + B[None] * z[:, None, :])


def source_factor(mesh, fields, dt):
    """1 - dt div(u) at every node (eq. advection_phi with S = -psi div u)."""
    if fields.divu is None:
        return np.ones(mesh.total_nodes)
    return 1.0 - dt * np.asarray(fields.divu, dtype=np.float64).reshape(mesh.total_nodes)


def edge_displacement(mesh, fields, dt, z):
    """disp = (un dt)/h + (sqrt((2 Dn) dt)/h) z at every edge point, shape (M, total_edge)."""
    un = np.asarray(fields.un, dtype=np.float64).reshape(mesh.total_edge)
    Dn = np.asarray(fields.Dn, dtype=np.float64).reshape(mesh.total_edge)
    hdir = np.empty(mesh.total_edge)
    zdir = np.empty((z.shape[0], mesh.total_edge))
    off = mesh.edge_offset
    for e in range(mesh.K):
        N = int(mesh.order[e])
        if mesh.dim == 1:
            hdir[off[e]:off[e + 1]] = mesh.hx
            zdir[:, off[e]:off[e + 1]] = z[:, 0:1]
        else:
            hdir[off[e]:off[e] + 2 * N] = mesh.hx
            hdir[off[e] + 2 * N:off[e + 1]] = mesh.hy
            zdir[:, off[e]:off[e] + 2 * N] = z[:, 0:1]
            zdir[:, off[e] + 2 * N:off[e + 1]] = z[:, 1:2]
    Af = (un * dt) / hdir
    Bf = np.sqrt((2.0 * Dn) * dt) / hdir
    return Af[None] + Bf[None] * zdir


def constraint_rank(N, dim):
    """Rank of the edge-evaluation map on Q_{N-1}: 2 in 1-D, 4N-4 in 2-D."""
    return 2 if dim == 1 else 4 * N - 4


def advected_interpolant(N, dim, xs, f, ref, family="gl"):
    """The advected interpolant p0 of a batch of fits (eqs. phi_stardef, h_star, remap_bnd).

    xs: (..., n, d) moved reference coordinates; f: (..., n) values carried to
    them; ref: (n, d) Gauss nodes.  Returns dbar (..., d), V (..., n, n) basis
    at the moved nodes, c0 (..., n) coefficients of p0, C (..., T, n) basis at
    the element's own edge points and t (..., T) the traces of p0 there.
    """
    dbar = np.mean(xs - ref, axis=-2)
    V = _basis(xs, dbar, N, dim)
    c0 = np.linalg.solve(V, f[..., None])[..., 0]
    own = own_edge_points(N, dim, family)
    C = _basis(np.broadcast_to(own, xs.shape[:-2] + own.shape), dbar, N, dim)
    t = np.einsum("...qp,...p->...q", C, c0)
    return dbar, V, c0, C, t


def own_edge_points(N, dim, family="gl"):
    """Reference edge points of an order-N element, edges in order L,R (1-D) or W,E,S,N (2-D)."""
    if dim == 1:
        return np.array([[0.0], [1.0]])
    eta = np.asarray(tables.nodes(int(N), family))
    zero, one = np.zeros(N), np.ones(N)
    return np.concatenate([np.stack([zero, eta], 1), np.stack([one, eta], 1),
                           np.stack([eta, zero], 1), np.stack([eta, one], 1)], 0)


def constrained_values(N, dim, V, C, f, t, g, m=None):
    """Values a at the moved nodes of the constrained least-squares fit (Sec. 5.3).

    The fit minimises sum_i (q(xi*_i) - f_i)^2 over q in Q_{N-1} subject to
    q(edge points) = P g.  In terms of the values a = V c at the moved nodes
    (V square and invertible) the constraint reads C* a = P g with
    C* = C V^-1, and the minimiser is a = f - pinv(C*) (C* f - g), where
    C* f = t.  pinv is the Moore-Penrose pseudo-inverse of rank
    ``constraint_rank`` (the trailing singular values of C* are zero).

    With the mass constraint (Introduction: a least-squares fit 'with boundary
    and mass conservation constraints'; the formulation itself is deferred to a
    reference not available) ``m`` holds, per fit, the coefficients-to-integral
    row of the element (integral over the element of the polynomial with
    coefficients c is m . c).  The fit must also keep the integral of p0: one
    more row m* = m V^-1 with right side m* f, whose residual is zero, so
    a = f - pinv([C*; m*]) [t - g; 0] with one more unit of rank (for N >= 3;
    for N = 2 the boundary values fix q and the row is left out).
    """
    r = constraint_rank(N, dim)
    rhs = t - g
    if m is not None and N >= 3:
        C = np.concatenate([C, m[..., None, :]], axis=-2)
        rhs = np.concatenate([rhs, np.zeros(rhs.shape[:-1] + (1,))], axis=-1)
        r += 1
    Vt = np.swapaxes(V, -1, -2)
    Cstar = np.swapaxes(np.linalg.solve(Vt, np.swapaxes(C, -1, -2)), -1, -2)
    U, sv, Wt = np.linalg.svd(Cstar, full_matrices=False)
    pinv = np.einsum("...rp,...r,...qr->...pq", Wt[..., :r, :], 1.0 / sv[..., :r], U[..., :, :r])
    return f - np.einsum("...pq,...q->...p", pinv, rhs)


def mass_row(N, dim, dbar, ref, family="gl"):
    """Row m with m . c = the integral over the (reference) element of the polynomial
    with coefficients c in the centred basis: the element's own quadrature (weights
    of its node family, exact on Q_{N-1}) applied to the basis at its Gauss nodes."""
    E = _basis(np.broadcast_to(ref, dbar.shape[:-1] + ref.shape), dbar, N, dim)     # (..., n, n)
    w1 = np.asarray(tables.weights(int(N), family))
    w = w1 if dim == 1 else np.kron(w1, w1)                                          # node i = iy N + ix
    return np.einsum("i,...ip->...p", w, E)


def values_at_nodes(N, dim, V, a, dbar, ref):
    """p(xi_i) at the Gauss nodes of the polynomial with values a at the moved nodes (eq. phi_star)."""
    c = np.linalg.solve(V, a[..., None])[..., 0]
    E = _basis(np.broadcast_to(ref, V.shape[:-2] + ref.shape), dbar, N, dim)
    return np.einsum("...ip,...p->...i", E, c)


def step(mesh, fields, phi, dt, z):
    """One DSEM-SL step of every sample in ``phi`` (shape (M, total_nodes)), given z (M, d).

    Returns the new phi and a dict of intermediates (positions, traces, g).
    """
    phi = np.asarray(phi, dtype=np.float64)
    M = phi.shape[0]
    d = mesh.dim
    xs_all = positions(mesh, fields, dt, z)                       # (M, Ntot, d)
    f_all = phi * source_factor(mesh, fields, dt)[None]           # (M, Ntot)
    noff, eoff = mesh.node_offset, mesh.edge_offset

    # --- per order group: moved nodes, interpolant p0 and its own traces
    per = {}
    for N, els in mesh.groups().items():
        n = N ** d
        ref = mesh.ref_nodes(N)
        idx = noff[els][:, None] + np.arange(n)[None, :]           # (K_N, n)
        f = f_all[:, idx]
        dbar, V, c0, C, t = advected_interpolant(N, d, xs_all[:, idx, :], f, ref, mesh.family)
        per[N] = dict(els=els, idx=idx, f=f, dbar=dbar, V=V, c0=c0, C=C, t=t, ref=ref)
    where = {}
    for N, g in per.items():
        for j, e in enumerate(g["els"]):
            where[int(e)] = (N, j)

    # --- upwinding (eq. bnd_update): g at every edge point of every element
    disp = edge_displacement(mesh, fields, dt, z)                 # (M, Etot)
    ghost = None if fields.ghost is None else np.asarray(fields.ghost, dtype=np.float64)
    gvals = np.empty((M, mesh.total_edge))
    tvals = np.empty((M, mesh.total_edge))
    nedges = 2 if d == 1 else 4
    opposite = {EDGE_L: EDGE_R, EDGE_R: EDGE_L} if d == 1 else \
        {EDGE_W: EDGE_E, EDGE_E: EDGE_W, EDGE_S: EDGE_N, EDGE_N: EDGE_S}
    # edges whose neighbour lies on the negative side of the interface
    neg_is_nbr = {EDGE_L: True, EDGE_R: False} if d == 1 else \
        {EDGE_W: True, EDGE_E: False, EDGE_S: True, EDGE_N: False}
    for e in range(mesh.K):
        N, j = where[e]
        g = per[N]
        per_edge = 1 if d == 1 else N
        for w in range(nedges):
            sl = slice(eoff[e] + w * per_edge, eoff[e] + (w + 1) * per_edge)
            own_t = g["t"][:, j, w * per_edge:(w + 1) * per_edge]  # (M, per_edge)
            tvals[:, sl] = own_t
            nb = mesh.neighbour(e, w)
            if nb < 0:
                if ghost is None:
                    raise ValueError("Dirichlet boundary needs ghost values")
                other = np.broadcast_to(ghost[sl], own_t.shape)
            else:
                Nn, jn = where[nb]
                gn = per[Nn]
                # neighbour's p0 at this element's edge points, in the neighbour's frame
                pts = mesh.ref_edge_points(Nn, opposite[w], npts=N if d == 2 else None)
                Cn = _basis(np.broadcast_to(pts, (M,) + pts.shape), gn["dbar"][:, jn], Nn, d)
                other = np.einsum("sqp,sp->sq", Cn, gn["c0"][:, jn])
            take_nbr = (disp[:, sl] > 0.0) if neg_is_nbr[w] else ~(disp[:, sl] > 0.0)
            gvals[:, sl] = np.where(take_nbr, other, own_t)

    # --- constrained least-squares remap and evaluation at the Gauss nodes
    new = np.empty_like(phi)
    for N, g in per.items():
        els = g["els"]
        T = eoff[els][:, None] + np.arange(mesh.n_edge[els[0]])[None, :]   # (K_N, T)
        m = mass_row(N, d, g["dbar"], g["ref"], mesh.family) if mesh.mass else None
        a = constrained_values(N, d, g["V"], g["C"], g["f"], g["t"], gvals[:, T], m)
        new[:, g["idx"]] = values_at_nodes(N, d, g["V"], a, g["dbar"], g["ref"])
    info = dict(positions=xs_all, traces=tvals, g=gvals, f=f_all)
    return new, info


def run(mesh, fields, phi0, dt, nsteps, seed, samples, stream=0, step0=0, reseed_every=0):
    """Advance ``len(samples)`` samples from phi0 (broadcast or (M, total_nodes)) nsteps steps.

    ``samples`` are global sample indices (they select the Philox counters), so a
    subset of samples gives exactly the rows a full run would give.
    ``reseed_every`` > 0 sets every sample to the mean after each such number of
    steps (eq. re-seed); it needs all samples of the run.
    """
    samples = np.asarray(samples, dtype=np.uint64)
    phi = np.broadcast_to(np.asarray(phi0, dtype=np.float64), (len(samples), mesh.total_nodes)).copy()
    for k in range(nsteps):
        z = wiener_normals(mesh, seed, step0 + k, samples, stream)
        phi, _ = step(mesh, fields, phi, dt, z)
        if reseed_every and (k + 1) % reseed_every == 0:
            phi[:] = mean(phi)[None]
    return phi


def mean(phi):
    """Sample mean at every node (eq. averaged): plain sum over samples in order, then / M."""
    phi = np.asarray(phi, dtype=np.float64)
    acc = np.zeros(phi.shape[1])
    for s in range(phi.shape[0]):
        acc = acc + phi[s]
    return acc / phi.shape[0]


def pdf_counts(phi, lo, hi, nbins):
    """Per-node histogram of the samples (Sec. 5.4: the PDF at each grid point by
    binning the samples): counts (nodes, nbins + 2), column 0 the values below lo,
    columns 1..nbins the bins of width w = (hi - lo) / nbins, column nbins + 1 the
    values at or above hi.  A value v in [lo, hi) goes to bin floor((v - lo) / w),
    capped at nbins - 1 (rounding can reach nbins just below hi).  Non-finite
    values are not counted.  Plain loops over samples and nodes."""
    phi = np.asarray(phi, dtype=np.float64)
    w = (hi - lo) / nbins
    M, nodes = phi.shape
    counts = np.zeros((nodes, nbins + 2), dtype=np.int64)
    for s in range(M):
        for i in range(nodes):
            v = phi[s, i]
            if not np.isfinite(v):
                continue
            if v < lo:
                counts[i, 0] += 1
            elif v >= hi:
                counts[i, nbins + 1] += 1
            else:
                b = int(math.floor((v - lo) / w))
                counts[i, 1 + min(b, nbins - 1)] += 1
    return counts


def _quad(mesh):
    """Per-node quadrature weights on the reference element (sum 1 per element)."""
    w = np.empty(mesh.total_nodes)
    off = mesh.node_offset
    for e in range(mesh.K):
        N = int(mesh.order[e])
        w1 = np.asarray(tables.weights(N, mesh.family))
        w[off[e]:off[e + 1]] = w1 if mesh.dim == 1 else np.kron(w1, w1)
    return w


def jacobian(mesh):
    return mesh.hx if mesh.dim == 1 else mesh.hx * mesh.hy


def l2_error(mesh, phi, exact):
    """Eq. l2_error: sum over elements of sqrt(int (phi - exact)^2 J dxi)."""
    w = _quad(mesh) * jacobian(mesh)
    off = mesh.node_offset
    err = (np.asarray(phi) - np.asarray(exact)) ** 2 * w
    return float(sum(np.sqrt(np.sum(err[off[e]:off[e + 1]])) for e in range(mesh.K)))


def mass_norm(mesh, phi, exact):
    """Eq. mass_cons: sum over elements of int phi dxi / int exact dxi."""
    w = _quad(mesh)
    off = mesh.node_offset
    return float(sum(np.sum((w * phi)[off[e]:off[e + 1]]) / np.sum((w * exact)[off[e]:off[e + 1]])
                     for e in range(mesh.K)))


def energy_norm(mesh, phi, exact):
    """Eq. energy_cons: sum over elements of int phi^2 dxi / int exact^2 dxi."""
    w = _quad(mesh)
    off = mesh.node_offset
    p2, x2 = w * np.asarray(phi) ** 2, w * np.asarray(exact) ** 2
    return float(sum(np.sum(p2[off[e]:off[e + 1]]) / np.sum(x2[off[e]:off[e + 1]]) for e in range(mesh.K)))


def integral(mesh, phi):
    """Quadrature of phi over the domain (GL weights times the Jacobian)."""
    return float(np.sum(_quad(mesh) * jacobian(mesh) * np.asarray(phi)))
