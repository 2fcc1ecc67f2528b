"""FP64 CPU oracle for the DSEM-SL Monte-Carlo step (arXiv:2009.07340).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or call anything in this package.  The GPU library never routes through
it, and it imports nothing from the GPU package.

The oracle is a plain, slow, obviously-correct restatement of what one
semi-Lagrangian Monte-Carlo step computes (Sec. 5 of the paper): seed at the
Gauss nodes (Sec. 5.1, eq. soln_init), move every node by one Euler-Maruyama
step with one Wiener increment per sample (Sec. 5.2, eq. def_dx), carry the
composition-space source along (eq. advection_phi), remap the advected
interpolant to the Gauss nodes by a least-squares fit constrained by upwinded
boundary values (Sec. 5.3, eqs. phi_star, remap_bnd, bnd_update) and average
the samples at the nodes (Sec. 5.4, eq. averaged).

Everything is float64 numpy.  Library primitives used as single steps:
``numpy.linalg.solve``, ``numpy.linalg.svd``, ``numpy.polynomial.legendre``
and ``mpmath`` (node tables).  There is no blocking, fusion or reordering
beyond the definitions.

Modules
  tables  Gauss node/weight tables and the orthonormal Legendre basis.
  rng     Philox4x32-10 counter-based generator and the polar normal map.
  sl      Mesh, positions, the constrained remap, upwinding, mean and norms.

Readings where the paper is silent or garbled (all also listed in the design doc):
node family default Gauss-Legendre; the least-squares remap is the
equality-constrained least-squares problem with the residual at the moved
nodes; 2-D boundary data are first projected onto the traces that a
polynomial of the element space can take; the source of a boundary value is
the unconstrained advected interpolant; nodes may leave the element (no
clamping); the upwind test is strict (``disp > 0`` takes the negative-side
element).
"""
