// Launchers of the stiffness (diffusion) operator kernels (kern_stiff.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kern_fp64.hpp"

namespace fepa {

struct StiffSet {
    // Dk [E][6][Q^3] (patch order) of the current positions x ([3][ncomp]);
    // kappa [caller element - kbase][Q^3] or null for 1
    void (*qdata)(const double *x, const PatchDev &pd, int E, long long ncomp,
                  const double *kappa, long long kbase, double *Dk, const double *tab,
                  hipStream_t st);
    // y = K u for the three components (patch kernel; shared nodes left as
    // partials in pd.part for launch_gather_shared); nw waves per workgroup
    void (*mult)(const double *Dk, const double *u, const PatchDev &pd, double *y,
                 long long ncomp, const double *tab, int nw, hipStream_t st);
};

// false when (p, Q) is not instantiated
bool stiff_kernels(int p, int Q, StiffSet *out);

}  // namespace fepa
