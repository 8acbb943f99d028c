// Launcher of the fully matrix-free force pair (kern_mf.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kern_fp64.hpp"

namespace fepa {

// y = F 1 (shared nodes left as partials in pd.part for launch_gather_shared)
// and z = F^T v of the state (x, v, e), the quadrature data formed on the fly
// from m_q (patch order) and never stored; min_key / nonfinite receive the
// smallest detJ and stable point step and the non-finite flag, as the qdata
// kernel does. nw: waves per workgroup (2 or 4).
using MfFn = void (*)(const double *x, const double *v, const double *e, const double *mq,
                      const PatchDev &pd, double *y, double *z, long long ncomp, const double *tab,
                      QParams prm, long long *min_key, int *nonfinite, int nw, hipStream_t st);
MfFn mf_kernel(int p, int Q);  // nullptr when (p, Q) is not instantiated

}  // namespace fepa
