// Host-side tables (see tables.cpp).
#pragma once
#include <vector>
#include "sl_internal.hpp"

namespace sl {

// Gauss nodes of order n on [0, 1], increasing, correctly rounded to float64:
// family 0 = roots of P_n(2 xi - 1) (Gauss-Legendre), 1 = Chebyshev-Gauss.
std::vector<double> gauss_nodes(int n, int family);
LegendreRec legendre_recurrence();
double min_node_spacing(const std::vector<double>& xi);
// Lagrange interpolation matrix (to.size() x from.size(), row-major).
std::vector<double> lagrange_matrix(const std::vector<double>& from, const std::vector<double>& to);
// Orthonormal basis of the edge-value vectors of Q_{N-1} (4N x (4N-4)), column-major.
std::vector<double> edge_range_basis(int N, const std::vector<double>& xi);
// Weights of the interpolatory quadrature on [0, 1] at the nodes (exact on degree < n).
std::vector<double> quadrature_weights(const std::vector<double>& xi);
// Barycentric weights 1 / prod_{m != i} (xi_i - xi_m) of the nodes, in long double.
std::vector<double> barycentric_weights(const std::vector<double>& xi);
// Inverses of the reference Gram matrix Gx = Vx^T Vx and of the reference basis
// matrix Vx[i][k] = psi_k(xi_i) of the orthonormal Legendre basis at the nodes
// xi (each N x N, row-major, Gx^-1 first), computed in long double.
std::vector<double> reference_inverses(const std::vector<double>& xi);
// Null-space tables of order N (nsp_doubles(N) doubles, layout in sl_internal.hpp).
std::vector<double> nullspace_tables(int N, const std::vector<double>& xi);

}  // namespace sl
