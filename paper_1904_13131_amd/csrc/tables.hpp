// Host-side 1-D tables and transfer matrices.
#pragma once

#include <vector>

#include "common.hpp"

namespace mfh {

struct BandHost {
  int nout = 0, nin = 0, K = 0;
  std::vector<int> start;
  std::vector<double> vals;
};

// q-point Gauss-Legendre rule on [0, 1] (weights sum to 1).
std::vector<double> gauss_points(int q, std::vector<double>& w);
// Degree-p Gauss-Lobatto-Legendre points on [0, 1].
std::vector<double> gll_points(int p);
// Lagrange polynomials through nodes, values V and derivatives D (may be null) at x.
void lagrange(const std::vector<double>& nodes, double x, double* V, double* D);
// S, D, w, xg for degree p with p+1 Gauss points.
Tables<double> make_tables(int p);
Tables<float> to_float(const Tables<double>& t);
// Coordinates of the L = pN+1 lattice points of one axis.
std::vector<double> lattice_coords(int N, int p);
// M[k][I] = global 1-D basis function of lattice index I (N cells, degree p) at X[k].
std::vector<double> eval_global_1d(int N, int p, const std::vector<double>& X);
// Band storage of a dense nout x nin matrix.
BandHost make_band(const std::vector<double>& M, int nout, int nin);
// Largest eigenvalue of a symmetric tridiagonal matrix.
double tridiag_max_eig(const std::vector<double>& d, const std::vector<double>& e);
double tridiag_min_eig(const std::vector<double>& d, const std::vector<double>& e);

}  // namespace mfh
