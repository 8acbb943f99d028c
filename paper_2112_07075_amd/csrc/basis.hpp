// 1-D rules and Lagrange tables built by the library itself.
#pragma once
#include <vector>

namespace fepa {

void gauss_legendre01(int n, double *t, double *w);
void gauss_lobatto01(int p, double *t);
// Table of one (p, Q) pair in the layout B[Q][D] | G[Q][D] | Bl[Q][Dl] | W[Q].
std::vector<double> build_table(int p, int Q);
// BF16 form operand buffer of (p, Q): FP32 copy of the table, then the MFMA
// fragments of the dense reference-gradient matrix (layout: mfma_layout).
std::vector<unsigned char> build_mfma_table(int p, int Q, const std::vector<double> &tab);

}  // namespace fepa
