// Host-side setup arithmetic of the library (see gmg_setup_math.cpp).
#pragma once

#include <cstdint>
#include <vector>

#include "gmg_kernels.h"

namespace gmg {

// Per-level tables of a uniform periodic mesh with n elements of order q.
struct LevelTables {
  OpTab stiff;                             // stiffness apply (and D^-1 by class)
  OpTab mass;                              // consistent mass apply
  double diag[kMaxQ * kMaxQ * kMaxQ];      // A_ii by node class
  double dinv_sqrt[kMaxQ * kMaxQ * kMaxQ]; // A_ii^-1/2
  double dsqrt[kMaxQ * kMaxQ * kMaxQ];     // A_ii^1/2
  double wint[kMaxQ * kMaxQ * kMaxQ];      // int phi_i dx (row sums of M) by class
};

// Tables of a level of an order without a specialised kernel (see GenOp): the banded
// rows of the stiffness and of the mass passes (6 q (2q+1) values each) and the node-class
// tables (q^3 values each).
struct GenTables {
  int q = 0;
  std::vector<double> stiff_rows, mass_rows;
  std::vector<double> diag, dinv, dsqrt, dinv_sqrt, wint;
};
GenTables make_generic_tables(int q, int n);
// P1 (2q x (q+1)) and P1^T (q x (4q+1)) weights, as in TransferTab
void make_generic_transfer(int q, std::vector<double>* p, std::vector<double>* r);

std::vector<double> lgl_nodes01(int q);
void gauss01(int m, std::vector<double>* pts, std::vector<double>* wts);
double lagrange_at(const std::vector<double>& xi, int a, double t);
double lagrange_deriv_at(const std::vector<double>& xi, int a, double t);
void reference_matrices(int q, std::vector<double>* khat, std::vector<double>* mhat);
LevelTables make_level_tables(int q, int n);
void make_transfer_table(int q, TransferTab* tab);
// (A_0 + 1 1^T / N0)^-1 of the coarsest level, dense, symmetric, row-major: by a dense
// factorisation up to 512 DoFs, from the eigenpairs of the 1D matrices above (up to 4096).
std::vector<double> coarse_pseudo_inverse(int q, int n);
// (A + 1 1^T / n0)^-1 of any dense symmetric n0 x n0 matrix A with null space 1 (row-major).
std::vector<double> dense_pseudo_inverse(std::vector<double> A, int n0);
uint64_t splitmix64_at(uint64_t key, uint64_t i);
void lanczos_start_vector(uint64_t seed, int level, int64_t count, double* out);
double tridiag_max_eig(const std::vector<double>& alpha, const std::vector<double>& beta);

}  // namespace gmg
