// 1-D rules and Lagrange tables built by the library itself.
#pragma once
#include <vector>

namespace fepa {

void gauss_legendre01(int n, double *t, double *w);
void gauss_lobatto01(int p, double *t);
// Table of one (p, Q) pair in the layout B[Q][D] | G[Q][D] | Bl[Q][Dl] | W[Q].
std::vector<double> build_table(int p, int Q);

}  // namespace fepa
