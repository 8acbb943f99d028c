// Host-visible launch interface of the Lagrange-step kernels (kern_step.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepa {

// M_E^-1 of the E elements of one mesh: mq in patch order, perm[k] - perm_base
// the caller index of patch-order element k, minv [E][p^3][p^3] of the mesh.
void launch_l2_mass_inv(int p, int Q, const double *mq, const int32_t *perm, int perm_base, int E,
                        const double *tab, double *minv, hipStream_t st);
// out[0] = min(dt_max, cfl * key_value(key[1])), out[1] = key_value(key[1])
void launch_step_dt(const long long *key, double cfl, double dt_max, double *out, hipStream_t st);
// v = vs - h acc, x = xs + h (vbar ? (vs + v)/2 -> vbar : vs), h = frac * dt[0]
void launch_rk_h1(const double *vs, const double *xs, const double *acc, double *v, double *x,
                  double *vbar, long long n, const double *dt, double frac, hipStream_t st);
// e[r] = es[r] + frac * dt[0] * sum_k minv[r][k] z[r / N][k] for r < rows
void launch_rk_l2(const double *es, const double *minv, const double *z, double *e, long long rows,
                  int N, const double *dt, double frac, hipStream_t st);

}  // namespace fepa
