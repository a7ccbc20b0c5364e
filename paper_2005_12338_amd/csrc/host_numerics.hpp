// Host FP64 numerics of the set-up steps (eigen.cpp).  Plain C++ with
// OpenMP and no HIP, so the file is compiled by the host compiler.
#pragma once

#include <cstdint>

// Eigen-decomposition of the symmetric matrix a [n][n] (row-major, destroyed):
// eigenvalues ascending in e [n], eigenvectors as the columns of v [n][n].
void sym_eigen(int64_t n, double* a, double* e, double* v);

// Gauss-Legendre nodes (ascending) and weights on [-1, 1].
void gauss_legendre(int64_t n, double* x, double* w);
