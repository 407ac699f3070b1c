// Host-side construction of the reference-element and collocation tables.
#pragma once
#include <vector>

namespace sisdc {

// Gauss-Lobatto-Legendre nodes (ascending) and weights for degree P.
void gll(int P, std::vector<double>& x, std::vector<double>& w);
// Lagrange derivative matrix D[i*n+j] = l_j'(x_i) on the nodes x.
std::vector<double> derivative_matrix(const std::vector<double>& x);
// L[i*n_from+j] = l_j(t_i), Lagrange basis on x_from evaluated at t.
std::vector<double> lagrange(const std::vector<double>& x_from, const std::vector<double>& t);
// Radau-right collocation nodes on [0, 1] (last node = 1).
std::vector<double> radau_right(int M);
// Incremental weights w^nn[m*M+i] = int_{tau_{m-1}}^{tau_m} l_i (tau_0 = 0).
std::vector<double> nn_weights(const std::vector<double>& tau);

}  // namespace sisdc
