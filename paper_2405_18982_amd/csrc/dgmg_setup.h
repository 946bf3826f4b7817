// Host-side FP64 construction of the reference 1-D tables (dgmg_setup.cpp).
#pragma once
#include <vector>

namespace dgmg {

// Reference data of Q_k on [0,1] and of the two-cell patch (h = 1, kappa = 1).
struct HostTables {
  int k = 0, n = 0, E = 0;
  double sigma = 0;
  std::vector<double> nodes;   // Gauss-Lobatto points, n
  std::vector<double> M, K;    // n x n, row-major
  std::vector<double> d0, d1;  // phi'(0), phi'(1)
  std::vector<double> Lc;      // interior-type SIPG cell block, n x n
  std::vector<double> P;       // stacked prolongation, E x n
  // fast diagonalisation on the Dirichlet local space per patch type t = 0..3,
  // padded to E:
  // S[t][p*E + q], lam[t][q] (+inf in unused slots)
  std::vector<double> S[4];
  std::vector<double> lam[4];
  // the same on the whole two-cell patch (Full kernel; every slot used)
  std::vector<double> Sf[4];
  std::vector<double> lamf[4];
  // clamped space (basis C): C S padded to E x E, eigenvalues (+inf unused)
  std::vector<double> Sc[4];
  std::vector<double> lamc[4];
};

// Builds every table; returns false (with a message) if a factorisation fails,
// e.g. when sigma is too small for the patch matrices to be positive definite.
bool build_host_tables(int k, double sigma, HostTables& out, const char** err);

// Gauss-Lobatto points on [0,1] and the Lagrange basis on them (exported for
// the node-coordinate query).
std::vector<double> gll_nodes01(int k);

}  // namespace dgmg
