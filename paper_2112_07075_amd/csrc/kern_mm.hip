// Multi-material kernels (Sec. 2.1's multi-material equations; Sec. 3.3's
// -sum_k F_k 1, M_E,k de_k/dt = F_k^T v and eta_k rho_k |J| = eta_k0 rho_k0
// |J0|). The material quadrature data S_k = w detJ eta_k sigma_k J^-T is the
// single-material qdata algebra with the material's mass per point
// m_qk = eta_k0 rho_k0 detJ0 w in place of m_q (rho = m_qk / (w detJ) is then
// eta_k rho_k, which makes p and mu those of eta_k sigma_k), so the library
// runs its qdata kernel once per material; this file holds the set-up of
// m_qk and the sums over materials.
#include "kern_common.hpp"
#include "kern_mm.hpp"

namespace fepa {

// m_qk = rho0_k * (B_l^3 eta0_k)(q) * dw[q], one thread per point; dw holds
// detJ0 w (patch order), eta0 the L2 coefficients of the element perm[el]
// (from the L2 base pointer of the unit).
template <int D, int Q>
__global__ void __launch_bounds__(256)
k_mat_mass(const double *__restrict__ dw, const double *__restrict__ eta0,
           const int32_t *__restrict__ perm, double rho0, double *__restrict__ mqk, long long n,
           const double *__restrict__ tab)
{
    constexpr int DL = D - 1, DL3 = DL * DL * DL, Q3 = Q * Q * Q;
    using T = Tab<D, Q>;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long el = i / Q3;
    const int q = (int)(i % Q3), qx = q % Q, qy = (q / Q) % Q, qz = q / (Q * Q);
    const double *__restrict__ et = eta0 + (long long)perm[el] * DL3;
    double s = 0.0;
    for (int j = 0; j < DL3; ++j) {
        const int jx = j % DL, jy = (j / DL) % DL, jz = j / (DL * DL);
        s += tab[T::BL + qx * DL + jx] * tab[T::BL + qy * DL + jy] * tab[T::BL + qz * DL + jz] * et[j];
    }
    mqk[i] = rho0 * s * dw[i];
}

// out[i] = sum_k in[k * stride + i], i < n (fixed order over k)
__global__ void k_sum_blocks(const double *__restrict__ in, int K, long long stride,
                             double *__restrict__ out, long long n)
{
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        double s = 0.0;
        for (int k = 0; k < K; ++k) s += in[k * stride + i];
        out[i] = s;
    }
}

// Initial density given point by point (Sec. 3.3's rho |J| = rho0 |J0| with
// rho0 varying over the mesh): m_q = rho0(q) detJ0 w from m_q = detJ0 w.
__global__ void k_point_density(double *__restrict__ mq, const double *__restrict__ rho0q,
                                const int32_t *__restrict__ perm, int perm_base, int Q3, long long n,
                                int *__restrict__ bad)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long el = i / Q3;
    const int q = (int)(i % Q3);
    const double r = rho0q[(long long)(perm[el] - perm_base) * Q3 + q];
    if (!(r > 0.0 && r < INFINITY)) *bad = 1;
    mq[i] *= r;
}

void launch_point_density(double *mq, const double *rho0q, const int32_t *perm, int perm_base,
                          int Q3, long long E, int *bad, hipStream_t st)
{
    const long long n = E * Q3;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_point_density, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, mq, rho0q,
                       perm, perm_base, Q3, n, bad);
}

void launch_mat_mass(int p, int Q, const double *dw, const double *eta0, const int32_t *perm,
                     double rho0, double *mqk, long long E, const double *tab, hipStream_t st)
{
    const long long n = E * Q * Q * Q;
    if (n <= 0) return;
#define FEPA_ENTRY(P, QQ)                                                                    \
    if (p == P && Q == QQ) {                                                                 \
        hipLaunchKernelGGL((k_mat_mass<P + 1, QQ>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, \
                           st, dw, eta0, perm, rho0, mqk, n, tab);                           \
        return;                                                                              \
    }
    FEPA_PQ_LIST(FEPA_ENTRY)
#undef FEPA_ENTRY
}

void launch_sum_blocks(const double *in, int K, long long stride, double *out, long long n,
                       hipStream_t st)
{
    if (n <= 0) return;
    long long b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    hipLaunchKernelGGL(k_sum_blocks, dim3((unsigned)b), dim3(256), 0, st, in, K, stride, out, n);
}

}  // namespace fepa
