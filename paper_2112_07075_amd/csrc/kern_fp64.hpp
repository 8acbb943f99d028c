// Host-visible launch interface of the FP64 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepa {

// Scalars of the quadrature-data update.
struct QParams {
    double rho0;       // initial density (setup pass)
    double gamma;      // ratio of specific heats
    double gm1;        // gamma - 1
    double q1, q2;     // viscosity coefficients
    double inv_order;  // 1/p (length scale l = detJ^(1/3) / p)
};

// Launchers of one (p, Q) instance. Pointers are device pointers already
// offset to the mesh; ncomp is the component stride of H1 vectors.
struct KernelSet {
    void (*force)(const double *S, const double *e, const int32_t *map, double *y, int E,
                  long long ncomp, const double *tab, hipStream_t st);
    void (*force_t)(const double *S, const double *v, const int32_t *map, double *z, int E,
                    long long ncomp, const double *tab, hipStream_t st);
    void (*mass)(const double *mq, const double *x, const int32_t *map, double *y, int E,
                 long long ncomp, const double *tab, double *part, const int *skip,
                 hipStream_t st);
    void (*qdata)(const double *x, const double *v, const double *e, const int32_t *map,
                  long long ncomp, int node_off, double *mq, double *S, int E,
                  const double *tab, QParams prm, long long *min_key, int *nonfinite, bool init,
                  hipStream_t st);
    int (*mass_blocks)(int E);  // workgroups of one mass launch (for partial sums)
};

// nullptr when (p, Q) is not instantiated.
const KernelSet *fp64_kernels(int p, int Q);

void launch_fill(double *y, long long n, double val, hipStream_t st);
// *key = INT64_MAX (empty min of ordered detJ keys), *flag = 0; either may be NULL.
void launch_reset_diag(long long *key, int *flag, hipStream_t st);

}  // namespace fepa
