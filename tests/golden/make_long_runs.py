"""Write the oracle's values after long runs of the 2-D workloads, for the GPU
parity tests at the workloads' own lengths (tests/test_gpu_long.py).

Calls only the float64 oracle (oracle/) and the seeded input generators
(paper_2009_07340_amd/workloads.py, which hold none of the method's
arithmetic).  The oracle needs seconds per step of one sample on these meshes,
so the runs are made once, here, and stored: for each (workload, sample,
steps) the values at a fixed subset of the nodes (every `stride`-th node from a
seeded offset, per sample), with the steps, the dt and the sample index.

    python tests/golden/make_long_runs.py [c3|c4|all]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import sl  # noqa: E402
from paper_2009_07340_amd import workloads as W  # noqa: E402

# (workload key, sample, snapshot steps, node stride)
RUNS = {
    "c3": ("c3", 0, (50, 200), 8),
    "c4": ("c4", 0, (20,), 16),
}


def node_subset(total, stride, seed):
    off = int(np.random.default_rng(seed).integers(stride))
    return np.arange(off, total, stride)


def run(key):
    wkey, sample, snaps, stride = RUNS[key]
    wl = W.WORKLOADS[wkey]()
    x0, x1, y0, y1 = wl.box
    mesh = sl.Mesh(dim=wl.dim, kx=wl.kx, ky=wl.ky, x0=x0, x1=x1, y0=y0, y1=y1, order=wl.order_array(), bc=wl.bc)
    ax = []
    for e in range(mesh.K):
        N = int(mesh.order[e])
        ax += [0] * (2 * N) + [1] * (2 * N)
    a = wl.sample_fields(mesh.node_coords(), mesh.edge_coords(), np.array(ax))
    f = sl.Fields(u=a["u"], D=a["D"], divu=a["divu"], un=a["un"], Dn=a["Dn"], ghost=a["ghost"])
    idx = node_subset(mesh.total_nodes, stride, 1000 + sample)
    phi = a["phi0"][None].copy()
    t0 = time.time()
    for k in range(max(snaps)):
        z = sl.wiener_normals(mesh, wl.seed, k, np.array([sample], dtype=np.uint64))
        phi, _ = sl.step(mesh, f, phi, wl.dt, z)
        if k + 1 in snaps:
            out = os.path.join(HERE, f"long_{wl.name}_s{sample}_n{k + 1}.npz")
            np.savez(out, idx=idx, values=phi[0, idx], steps=k + 1, sample=sample, dt=wl.dt,
                     seed=wl.seed, workload=wl.name, l2_full=np.sqrt(np.sum(phi[0] ** 2)))
            print(f"{out}: {k + 1} steps in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    for key in (RUNS if which == "all" else [which]):
        run(key)
