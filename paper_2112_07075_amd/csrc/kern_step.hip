// Kernels of the full Lagrange step (the semi-discrete system of Sec. 3.3,
//   M_v dv/dt = -F 1,   M_E de/dt = F^T v,   dx/dt = v,
// advanced by a two-stage scheme): the inverse of every element's
// thermodynamic mass matrix M_E (built once, since rho |J| = rho0 |J0| keeps
// M_E fixed while the mesh moves), the stage updates of the kinematic and
// thermodynamic vectors, and the step size from the quadrature-point minimum.
#include "kern_common.hpp"
#include "kern_step.hpp"

namespace fepa {

// M_E^-1 of one element per workgroup. M_E[j][k] = sum_q m_q phi_j(q) phi_k(q)
// with phi the L2 basis (products of 1-D Lagrange values at the points), then
// Gauss-Jordan elimination on [M_E | I] in LDS. M_E is symmetric positive
// definite, so the elimination needs no pivoting. Elements are read in patch
// order (m_q's storage order) and written at their caller index perm - base.
template <int D, int Q>
__global__ void __launch_bounds__(256)
k_l2_mass_inv(const double *__restrict__ mq, const int32_t *__restrict__ perm, int perm_base,
              const double *__restrict__ tab, double *__restrict__ minv)
{
    constexpr int DL = D - 1, N = DL * DL * DL, Q3 = Q * Q * Q;
    using T = Tab<D, Q>;
    __shared__ double A[N][2 * N];
    __shared__ double sm[Q3];
    __shared__ double sBl[Q * DL];
    __shared__ double f[N];
    const int el = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    for (int q = tid; q < Q3; q += nt) sm[q] = mq[(long long)el * Q3 + q];
    for (int k = tid; k < Q * DL; k += nt) sBl[k] = tab[T::BL + k];
    __syncthreads();
    for (int k = tid; k < N * N; k += nt) {
        const int j = k / N, l = k % N;
        const int jx = j % DL, jy = (j / DL) % DL, jz = j / (DL * DL);
        const int lx = l % DL, ly = (l / DL) % DL, lz = l / (DL * DL);
        double s = 0.0;
        for (int qz = 0; qz < Q; ++qz)
            for (int qy = 0; qy < Q; ++qy) {
                const double yz = sBl[qz * DL + jz] * sBl[qz * DL + lz] * sBl[qy * DL + jy] *
                                  sBl[qy * DL + ly];
                for (int qx = 0; qx < Q; ++qx)
                    s += sm[(qz * Q + qy) * Q + qx] * yz * sBl[qx * DL + jx] * sBl[qx * DL + lx];
            }
        A[j][l] = s;
        A[j][N + l] = j == l ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        const double inv = 1.0 / A[k][k];
        __syncthreads();  // every thread has read the pivot before row k changes
        for (int c = tid; c < 2 * N; c += nt) A[k][c] *= inv;
        __syncthreads();
        for (int i = tid; i < N; i += nt) f[i] = A[i][k];
        __syncthreads();
        for (int idx = tid; idx < N * 2 * N; idx += nt) {
            const int i = idx / (2 * N), c = idx % (2 * N);
            if (i != k) A[i][c] -= f[i] * A[k][c];
        }
        __syncthreads();
    }
    double *__restrict__ out = minv + (long long)(perm[el] - perm_base) * N * N;
    for (int k = tid; k < N * N; k += nt) out[k] = A[k / N][N + k % N];
}

// dt = min(dt_max, cfl * smallest stable point step); out[0] = dt, out[1] = the
// smallest point step itself (the estimate before cfl).
__global__ void k_step_dt(const long long *__restrict__ key, double cfl, double dt_max,
                          double *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double est = key_value(key[1]);
        out[0] = fmin(dt_max, cfl * est);
        out[1] = est;
    }
}

// Kinematic update of a stage with h = frac * dt, a = -acc (acc solves
// M_v acc = F 1):
//   vbar == nullptr:  v = vs + h a,  x = xs + h vs
//   otherwise:        v = vs + h a,  vbar = (vs + v) / 2,  x = xs + h vbar
__global__ void k_rk_h1(const double *__restrict__ vs, const double *__restrict__ xs,
                        const double *__restrict__ acc, double *__restrict__ v,
                        double *__restrict__ x, double *__restrict__ vbar, long long n,
                        const double *__restrict__ dt, double frac)
{
    const double h = frac * dt[0];
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v0 = vs[i];
        const double v1 = v0 - h * acc[i];
        v[i] = v1;
        if (vbar) {
            const double vb = 0.5 * (v0 + v1);
            vbar[i] = vb;
            x[i] = xs[i] + h * vb;
        } else {
            x[i] = xs[i] + h * v0;
        }
    }
}

// Thermodynamic update of a stage for one mesh's rows (N = p^3 per element):
// e = es + h M_E^-1 z, h = frac * dt; minv holds M_E^-1 row by row.
__global__ void k_rk_l2(const double *__restrict__ es, const double *__restrict__ minv,
                        const double *__restrict__ z, double *__restrict__ e, long long rows, int N,
                        const double *__restrict__ dt, double frac)
{
    const double h = frac * dt[0];
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += stride) {
        const double *__restrict__ m = minv + r * N;
        const double *__restrict__ zz = z + (r / N) * N;
        double s = 0.0;
        for (int k = 0; k < N; ++k) s += m[k] * zz[k];
        e[r] = es[r] + h * s;
    }
}

void launch_l2_mass_inv(int p, int Q, const double *mq, const int32_t *perm, int perm_base, int E,
                        const double *tab, double *minv, hipStream_t st)
{
#define FEPA_ENTRY(P, QQ)                                                                          \
    if (p == P && Q == QQ) {                                                                       \
        hipLaunchKernelGGL((k_l2_mass_inv<P + 1, QQ>), dim3(E), dim3(P >= 3 ? 256 : 64), 0, st, mq, \
                           perm, perm_base, tab, minv);                                            \
        return;                                                                                    \
    }
    FEPA_PQ_LIST(FEPA_ENTRY)
#undef FEPA_ENTRY
}

void launch_step_dt(const long long *key, double cfl, double dt_max, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_step_dt, dim3(1), dim3(64), 0, st, key, cfl, dt_max, out);
}

static unsigned grid_for(long long n)
{
    long long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    return (unsigned)(b < 1 ? 1 : b);
}

void launch_rk_h1(const double *vs, const double *xs, const double *acc, double *v, double *x,
                  double *vbar, long long n, const double *dt, double frac, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rk_h1, dim3(grid_for(n)), dim3(256), 0, st, vs, xs, acc, v, x, vbar, n, dt,
                       frac);
}

void launch_rk_l2(const double *es, const double *minv, const double *z, double *e, long long rows,
                  int N, const double *dt, double frac, hipStream_t st)
{
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_rk_l2, dim3(grid_for(rows)), dim3(256), 0, st, es, minv, z, e, rows, N, dt,
                       frac);
}

}  // namespace fepa
