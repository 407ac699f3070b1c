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

// Discrete Legendre transform on the GLL nodes x (weights w) of degree P:
// A[k*n + i] = w_i phi_k(x_i) / sum_j w_j phi_k(x_j)^2, phi_k the Legendre
// polynomial of degree k scaled to unit L2 norm on [-1, 1].  Applied along an
// axis, A maps nodal values to the coefficients in the phi_k basis (the
// quadrature is exact for every product phi_j phi_k with j != k, so the
// basis is orthogonal in it and the transform inverts the nodal
// evaluation).
std::vector<double> legendre_analysis(int P, const std::vector<double>& x, const std::vector<double>& w);

// Fast diagonalisation of one axis of an element's diagonal block of the
// isotropic Helmholtz operator.  Per unit of J w_a w_b nu (the weights of the
// other axes, the Jacobian and the diffusivity), the axis contributes the
// symmetric n x n matrix
//   K = rh^2 [D^T W D - 1/2 sum_s sgn_s (D^T e_s e_s^T + e_s e_s^T D) + pen/2 sum_s e_s e_s^T],
// s over the element's two end nodes (sgn -1 at node 0, +1 at node P), rh =
// 2 / h, pen = C_tau (P + 1)^2: the volume term and the face terms of the
// interior-penalty form that couple the element with itself.  With the
// mass W = diag(w), this returns S (n x n, row-major S[i*n + k]) and lam (n)
// with S^T W S = I and S^T K S = diag(lam) (the generalised eigenproblem
// K s = lam W s, by Jacobi rotations on W^-1/2 K W^-1/2).
void fds_axis(const std::vector<double>& w, const std::vector<double>& D, double rh, double pen,
              std::vector<double>& S, std::vector<double>& lam);

}  // namespace sisdc
