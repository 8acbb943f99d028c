// Launchers of the per-point mass kernels (kern_mm.hip): material masses and
// a density given point by point.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepa {

// mqk[i] = rho0 * (B_l^3 eta0)(point i) * dw[i] over the E elements of a unit
// (patch order; eta0 read at perm[el] * p^3)
void launch_mat_mass(int p, int Q, const double *dw, const double *eta0, const int32_t *perm,
                     double rho0, double *mqk, long long E, const double *tab, hipStream_t st);
// out[i] = sum over k < K of in[k * stride + i], for i < n
void launch_sum_blocks(const double *in, int K, long long stride, double *out, long long n,
                       hipStream_t st);

// m_q[i] *= rho0_q of point i: rho0q is the caller's [E][Q^3] array of one
// mesh, read at ((perm[el] - perm_base) * Q3 + q); *bad = 1 where a value is
// not a positive finite number
void launch_point_density(double *mq, const double *rho0q, const int32_t *perm, int perm_base,
                          int Q3, long long E, int *bad, hipStream_t st);

}  // namespace fepa
