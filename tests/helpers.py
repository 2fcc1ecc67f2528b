"""Shared test plumbing: oracle inputs from the seeded workloads."""
import numpy as np

from oracle import sl
from paper_2009_07340_amd import workloads as W


def edge_axis(mesh):
    """Normal axis of each edge point in the oracle/library layout (W,E: x; S,N: y)."""
    ax = []
    for e in range(mesh.K):
        N = int(mesh.order[e])
        ax += [0, 0] if mesh.dim == 1 else [0] * (2 * N) + [1] * (2 * N)
    return np.array(ax)


def oracle_mesh(wl, family="gl"):
    x0, x1, y0, y1 = wl.box
    return sl.Mesh(dim=wl.dim, kx=wl.kx, ky=wl.ky, x0=x0, x1=x1, y0=y0, y1=y1,
                   order=wl.order_array(), family=family, bc=wl.bc)


def oracle_inputs(wl, mesh=None, t=0.0):
    """(mesh, Fields, phi0, raw arrays) for a workload, sampled at the oracle's coordinates."""
    mesh = mesh or oracle_mesh(wl)
    a = wl.sample_fields(mesh.node_coords(), mesh.edge_coords(), edge_axis(mesh), t)
    f = sl.Fields(u=a["u"], D=a["D"], divu=a["divu"], un=a["un"], Dn=a["Dn"], ghost=a["ghost"])
    return mesh, f, a["phi0"], a


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))
