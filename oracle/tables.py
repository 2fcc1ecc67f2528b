"""Node and basis tables for the oracle (test infrastructure, see package doc).

Sec. 3 of the paper places the solution at N Gauss points per direction on the
unit reference interval [0, 1] and represents it by the Lagrange interpolant of
degree N-1 through them (eqs. 3.4, 3.5).  The printed node formula (eq.
gaussquad) is garbled, so two families are offered:

* ``"gl"`` (default): the N roots of the shifted Legendre polynomial
  P_N(2 xi - 1), i.e. Gauss-Legendre points mapped to [0, 1];
* ``"cg"``: Chebyshev-Gauss points xi_i = (1 - cos((2i+1) pi / (2N))) / 2.

Nodes are computed with mpmath at 50 significant digits and rounded once to
float64, so every entry is the correctly rounded value.

The polynomial space Q_{N-1} is spanned here by the orthonormal shifted
Legendre polynomials psi_k(t) = sqrt(2k+1) P_k(2t - 1), k < N (a basis
choice; the remapped polynomial does not depend on it).
"""
from functools import lru_cache

import mpmath
import numpy as np
from numpy.polynomial import legendre as npleg

_DPS = 50


@lru_cache(maxsize=None)
def _gl_nodes_weights_mp(n):
    """Roots of P_n on [-1, 1] and Gauss weights, mpmath at _DPS digits."""
    with mpmath.workdps(_DPS + 10):
        xs, ws = [], []
        for i in range(n):
            # asymptotic first guess for the i-th largest root, then Newton
            x = mpmath.cos(mpmath.pi * (i + mpmath.mpf(3) / 4) / (n + mpmath.mpf(1) / 2))
            for _ in range(100):
                p = mpmath.legendre(n, x)
                dp = n * (x * p - mpmath.legendre(n - 1, x)) / (x * x - 1)
                dx = p / dp
                x -= dx
                if abs(dx) < mpmath.mpf(10) ** (-(_DPS + 5)):
                    break
            p = mpmath.legendre(n, x)
            dp = n * (x * p - mpmath.legendre(n - 1, x)) / (x * x - 1)
            xs.append(x)
            ws.append(2 / ((1 - x * x) * dp * dp))
        return xs, ws


@lru_cache(maxsize=None)
def nodes(n, family="gl"):
    """Reference nodes xi_i in (0, 1), increasing, correctly rounded float64."""
    if n < 1:
        raise ValueError("n >= 1 required")
    with mpmath.workdps(_DPS):
        if family == "gl":
            xs, _ = _gl_nodes_weights_mp(n)
            vals = [(1 - x) / 2 for x in xs]       # largest root -> smallest xi
        elif family == "cg":
            vals = [(1 - mpmath.cos((2 * i + 1) * mpmath.pi / (2 * n))) / 2 for i in range(n)]
        else:
            raise ValueError(f"unknown node family {family!r}")
        out = np.array([float(v) for v in vals], dtype=np.float64)
    out.setflags(write=False)
    return out


@lru_cache(maxsize=None)
def weights(n, family="gl"):
    """Quadrature weights on [0, 1] (sum 1) for the interpolatory rule at nodes()."""
    with mpmath.workdps(_DPS):
        if family == "gl":
            _, ws = _gl_nodes_weights_mp(n)
            vals = [w / 2 for w in ws]
        else:
            # interpolatory weights: sum_i w_i xi_i^k = 1/(k+1), k < n (mpmath solve)
            xs = [(1 - mpmath.cos((2 * i + 1) * mpmath.pi / (2 * n))) / 2 for i in range(n)]
            A = mpmath.matrix(n, n)
            b = mpmath.matrix(n, 1)
            for k in range(n):
                for i in range(n):
                    A[k, i] = xs[i] ** k
                b[k] = mpmath.mpf(1) / (k + 1)
            sol = mpmath.lu_solve(A, b)
            vals = [sol[i] for i in range(n)]
        out = np.array([float(v) for v in vals], dtype=np.float64)
    out.setflags(write=False)
    return out


def legendre_basis(t, n):
    """psi_k(t) = sqrt(2k+1) P_k(2t-1) for k < n; shape t.shape + (n,)."""
    t = np.asarray(t, dtype=np.float64)
    v = npleg.legvander(2.0 * t - 1.0, n - 1)
    return v * np.sqrt(2.0 * np.arange(n) + 1.0)
