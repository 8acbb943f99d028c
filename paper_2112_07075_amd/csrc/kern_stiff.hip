// Stiffness (diffusion) operator of the hyper-viscosity term (Sec. 2.1 names
// the stiffness-matrix operator that shock capturing by hyper-viscosity
// needs; Sec. 6 the diffusion integrator used by the artificial-viscosity
// calculations): K[i][j] = int kappa grad w_i . grad w_j dx on the kinematic
// H1 space, one block per velocity component like M_v, by partial assembly
// (Sec. 3.1's A = P^T G^T B^T D B G P with B the reference gradient):
//   quadrature data  Dk_q = w_q kappa_q detJ_q J_q^-1 J_q^-T   (symmetric,
//                    6 values per point: xx yy zz xy xz yz)
//   action           y_c = R^T B^T Dk B R u_c, sum-factorised as the force
//                    kernels: three gradient stages of u_c, the pointwise
//                    3 x 3 product, three transposed gradient stages.
// Layouts as the force operator: Dk [E][6][Q^3] in patch order; one patch per
// workgroup, the patch's node values of u read once into LDS, element results
// summed into LDS slots, private nodes stored and shared nodes left as
// partials for k_gather_shared.
#include "kern_common.hpp"
#include "kern_stiff.hpp"

namespace fepa {

// One thread per quadrature point (pt_ne(Q) elements per workgroup): the
// Jacobian by three staged 1-D contractions of the gathered positions, then
// Dk = w kappa adj(J) adj(J)^T / detJ (J^-1 = adj(J) / detJ).
// kappa: [caller element][Q^3] or null for 1 (read at perm[el] - kbase).
template <int D, int Q>
__global__ void __launch_bounds__(pt_ne(Q) * Q * Q * Q)
k_stiff_qdata(const double *__restrict__ x, const int32_t *__restrict__ map,
              const int32_t *__restrict__ perm, long long ncomp, const double *__restrict__ kappa,
              long long kbase, double *__restrict__ Dk, int E, const double *__restrict__ tab)
{
    constexpr int NE = pt_ne(Q), QQ = Q * Q, Q3 = Q * Q * Q, D3 = D * D * D;
    using T = Tab<D, Q>;
    __shared__ double sTab[T::SIZE];
    __shared__ double sU[NE][3][D3];
    __shared__ double sX[NE][3][2][D * D * Q];
    __shared__ double sY[NE][3][3][D * QQ];

    const int tid = threadIdx.x, le = tid / Q3, q = tid % Q3;
    const int qx = q % Q, qy = (q / Q) % Q, qz = q / QQ;
    const long long el = (long long)xcd_block(blockIdx.x, gridDim.x) * NE + le;
    const bool act = el < E;

    for (int k = tid; k < T::SIZE; k += blockDim.x) sTab[k] = tab[k];
    for (int k = q; k < 3 * D3; k += Q3) {
        const int f = k / D3, i = k % D3;
        sU[le][f][i] = act ? x[f * ncomp + map[el * D3 + i]] : 0.0;
    }
    __syncthreads();
    // x-stage: items (f, iz, iy, qx')
    for (int k = q; k < 3 * D * D * Q; k += Q3) {
        const int f = k / (D * D * Q), r = k % (D * D * Q);
        const int iz = r / (D * Q), iy = (r / Q) % D, kx = r % Q;
        double ub = 0.0, ug = 0.0;
#pragma unroll
        for (int ix = 0; ix < D; ++ix) {
            const double u = sU[le][f][(iz * D + iy) * D + ix];
            ub += sTab[T::B + kx * D + ix] * u;
            ug += sTab[T::G + kx * D + ix] * u;
        }
        sX[le][f][0][r] = ub;
        sX[le][f][1][r] = ug;
    }
    __syncthreads();
    // y-stage: items (f, iz, qy', qx') -> (B_y G_x, G_y B_x, B_y B_x)
    for (int k = q; k < 3 * D * QQ; k += Q3) {
        const int f = k / (D * QQ), r = k % (D * QQ);
        const int iz = r / QQ, ky = (r / Q) % Q, kx = r % Q;
        double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
        for (int iy = 0; iy < D; ++iy) {
            const double ub = sX[le][f][0][(iz * D + iy) * Q + kx];
            const double ug = sX[le][f][1][(iz * D + iy) * Q + kx];
            const double by = sTab[T::B + ky * D + iy], gy = sTab[T::G + ky * D + iy];
            a += by * ug;
            b += gy * ub;
            c += by * ub;
        }
        sY[le][f][0][r] = a;
        sY[le][f][1][r] = b;
        sY[le][f][2][r] = c;
    }
    __syncthreads();
    double J[3][3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
        for (int iz = 0; iz < D; ++iz) {
            const double bz = sTab[T::B + qz * D + iz], gz = sTab[T::G + qz * D + iz];
            a += bz * sY[le][f][0][(iz * Q + qy) * Q + qx];
            b += bz * sY[le][f][1][(iz * Q + qy) * Q + qx];
            c += gz * sY[le][f][2][(iz * Q + qy) * Q + qx];
        }
        J[f][0] = a;
        J[f][1] = b;
        J[f][2] = c;
    }
    if (!act) return;
    // adjugate: J^-1 = A / detJ, A[d][k] the cofactor of J[k][d]
    double A[3][3];
    A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double detJ = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
    const double w = sTab[T::W + qx] * sTab[T::W + qy] * sTab[T::W + qz];
    const double kap = kappa ? kappa[((long long)perm[el] - kbase) * Q3 + q] : 1.0;
    const double f = w * kap / detJ;
    // (J^-1 J^-T)[a][b] detJ^2 = sum_k A[a][k] A[b][k]
    constexpr int PA[6] = {0, 1, 2, 0, 0, 1}, PB[6] = {0, 1, 2, 1, 2, 2};
    double *__restrict__ De = Dk + el * 6 * Q3 + q;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int a = PA[m], b = PB[m];
        De[m * Q3] = f * (A[a][0] * A[b][0] + A[a][1] * A[b][1] + A[a][2] * A[b][2]);
    }
}

// y = K u for the three components, one patch per workgroup, column layout
// (one thread per point column (qx, qy), qz in registers). Per element the six
// Dk values of the thread's column are loaded once and serve the three
// components. The y and x stages go through per-element LDS staging (the
// forward and the transposed stages share it: a wave fence separates them).
template <int D, int Q, int NW>
__global__ void __launch_bounds__(NW * 64)
k_stiff(const double *__restrict__ Dk, const double *__restrict__ u,
        const uint16_t *__restrict__ slot, const int32_t *__restrict__ pn,
        const int32_t *__restrict__ ptab, double *__restrict__ y, double *__restrict__ part,
        long long ncomp, const double *__restrict__ tab)
{
    constexpr int NE = NW * wave_ne(Q), UMAX = patch_umax(D);
    constexpr int QQ = Q * Q, Q3 = Q * Q * Q, D3 = D * D * D;
    constexpr int NX = 2 * D * D * Q, NA = 3 * D * QQ, NW_ = NA + NX;  // staging per element
    using T = Tab<D, Q>;
    __shared__ double us[3 * UMAX];
    __shared__ double acc[3 * UMAX];
    __shared__ int sSl[NE + 1][D3];
    __shared__ double sW[NE + 1][NW_];

    const Lane L = lane_map<Q, NE>();
    const int tid = threadIdx.x, le = L.le, t = L.t, qx = t % Q, qy = t / Q;
    const PatchRow pr = load_patch(ptab, xcd_block(blockIdx.x, gridDim.x));
    for (int k = tid; k < pr.U; k += blockDim.x) {
        const long long g = pn[pr.pno + k];
        us[3 * k] = u[g];
        us[3 * k + 1] = u[ncomp + g];
        us[3 * k + 2] = u[2 * ncomp + g];
        acc[3 * k] = acc[3 * k + 1] = acc[3 * k + 2] = 0.0;
    }
    // idle lanes (spare element row NE) read slots from the spare row: keep it valid
    for (int i = tid; i < D3; i += blockDim.x) sSl[NE][i] = 0;
    double rBx[D], rGx[D], rBy[D], rGy[D], cBy[Q], cGy[Q], cBx[Q], cGx[Q];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        rBx[i] = tab[T::B + qx * D + i];
        rGx[i] = tab[T::G + qx * D + i];
        rBy[i] = tab[T::B + qy * D + i];
        rGy[i] = tab[T::G + qy * D + i];
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        cBy[k] = qy < D ? tab[T::B + k * D + qy] : 0.0;
        cGy[k] = qy < D ? tab[T::G + k * D + qy] : 0.0;
        cBx[k] = qx < D ? tab[T::B + k * D + qx] : 0.0;
        cGx[k] = qx < D ? tab[T::G + k * D + qx] : 0.0;
    }
    __syncthreads();

    // one staging area per element, used in turn by the forward and the
    // transposed stages (so no restrict: sX and sA alias)
    double *sX = sW[le];       // forward x-stage [2][D][D*Q]
    double *sA = sW[le];       // transposed z-stage [3][D][QQ]
    double *sC = sW[le] + NA;  // transposed y-stage [2][D][D*Q]
#pragma unroll 1
    for (int base = 0; base < pr.cnt; base += NE) {
        const int idx = base + le;
        const bool act = L.valid && idx < pr.cnt;
        const long long el = pr.eb + (act ? idx : 0);
        const double *__restrict__ De = Dk + el * 6 * Q3 + t;
        double dk[6][Q];
#pragma unroll
        for (int m = 0; m < 6; ++m)
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) dk[m][qz] = __builtin_nontemporal_load(De + m * Q3 + qz * QQ);
        for (int i = t; i < D3; i += QQ) sSl[le][i] = slot[el * D3 + i];
        wave_sync();
        int sl[D];
        {
            const int qxc = qx < D ? qx : D - 1, qyc = qy < D ? qy : D - 1;
#pragma unroll
            for (int iz = 0; iz < D; ++iz) sl[iz] = sSl[le][(iz * D + qyc) * D + qxc];
        }
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            // forward: x-stage, thread (qx, iy = qy), from the node values
            if (qy < D) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    double ub = 0.0, ug = 0.0;
#pragma unroll
                    for (int ix = 0; ix < D; ++ix) {
                        const double uu = us[3 * sSl[le][(iz * D + qy) * D + ix] + c];
                        ub += rBx[ix] * uu;
                        ug += rGx[ix] * uu;
                    }
                    sX[(0 * D + iz) * D * Q + qy * Q + qx] = ub;
                    sX[(1 * D + iz) * D * Q + qy * Q + qx] = ug;
                }
            }
            wave_sync();
            double vx[D], vy[D], vz[D];
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                double a = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
                for (int iy = 0; iy < D; ++iy) {
                    const double ub = sX[(0 * D + iz) * D * Q + iy * Q + qx];
                    const double ug = sX[(1 * D + iz) * D * Q + iy * Q + qx];
                    a += rBy[iy] * ug;
                    b += rGy[iy] * ub;
                    cc += rBy[iy] * ub;
                }
                vx[iz] = a;
                vy[iz] = b;
                vz[iz] = cc;
            }
            wave_sync();  // sX is overwritten by the transposed stages below
            // z-stage, pointwise Dk grad_xi u, and the transposed z-stage
            double a0[D], a1[D], a2[D];
#pragma unroll
            for (int i = 0; i < D; ++i) a0[i] = a1[i] = a2[i] = 0.0;
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                double dx = 0.0, dy = 0.0, dz = 0.0;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const double bb = tab[T::B + qz * D + iz], gg = tab[T::G + qz * D + iz];
                    dx += bb * vx[iz];
                    dy += bb * vy[iz];
                    dz += gg * vz[iz];
                }
                const double g0 = dk[0][qz] * dx + dk[3][qz] * dy + dk[4][qz] * dz;
                const double g1 = dk[3][qz] * dx + dk[1][qz] * dy + dk[5][qz] * dz;
                const double g2 = dk[4][qz] * dx + dk[5][qz] * dy + dk[2][qz] * dz;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const double b = tab[T::B + qz * D + iz], g = tab[T::G + qz * D + iz];
                    a0[iz] += b * g0;
                    a1[iz] += b * g1;
                    a2[iz] += g * g2;
                }
            }
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                sA[(0 * D + iz) * QQ + t] = a0[iz];
                sA[(1 * D + iz) * QQ + t] = a1[iz];
                sA[(2 * D + iz) * QQ + t] = a2[iz];
            }
            wave_sync();
            if (qy < D) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    double c0 = 0.0, c1 = 0.0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) {
                        c0 += cBy[k] * sA[(0 * D + iz) * QQ + k * Q + qx];
                        c1 += cGy[k] * sA[(1 * D + iz) * QQ + k * Q + qx] +
                              cBy[k] * sA[(2 * D + iz) * QQ + k * Q + qx];
                    }
                    sC[(0 * D + iz) * D * Q + qy * Q + qx] = c0;
                    sC[(1 * D + iz) * D * Q + qy * Q + qx] = c1;
                }
            }
            wave_sync();
            if (act && qx < D && qy < D) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    double r = 0.0;
#pragma unroll
                    for (int k = 0; k < Q; ++k)
                        r += cGx[k] * sC[(0 * D + iz) * D * Q + qy * Q + k] +
                             cBx[k] * sC[(1 * D + iz) * D * Q + qy * Q + k];
                    atomicAdd(&acc[3 * sl[iz] + c], r);
                }
            }
            wave_sync();  // the staging is rewritten by the next component
        }
    }
    __syncthreads();
    patch_write<UMAX>(acc, pr, pn, y, part, ncomp);
}

// LDS bytes of k_stiff with NW waves per workgroup
__host__ __device__ constexpr int stiff_lds(int D, int Q, int NW)
{
    return 6 * 8 * patch_umax(D) +
           (NW * wave_ne(Q) + 1) * (4 * D * D * D + 8 * (3 * D * Q * Q + 2 * D * D * Q));
}

template <int D, int Q>
struct StiffLaunch {
    static void qdata(const double *x, const PatchDev &pd, int E, long long ncomp,
                      const double *kappa, long long kbase, double *Dk, const double *tab,
                      hipStream_t st)
    {
        const int ne = pt_ne(Q);
        hipLaunchKernelGGL((k_stiff_qdata<D, Q>), dim3((E + ne - 1) / ne), dim3(ne * Q * Q * Q), 0,
                           st, x, pd.map, pd.perm, ncomp, kappa, kbase, Dk, E, tab);
    }
    template <int NW>
    static void mult_nw(const double *Dk, const double *u, const PatchDev &pd, double *y,
                        long long ncomp, const double *tab, hipStream_t st)
    {
        hipLaunchKernelGGL((k_stiff<D, Q, NW>), dim3(pd.n_patch), dim3(NW * 64), 0, st, Dk, u,
                           pd.slot, pd.pn, pd.ptab, y, pd.part, ncomp, tab);
    }
    static void mult(const double *Dk, const double *u, const PatchDev &pd, double *y,
                     long long ncomp, const double *tab, int nw, hipStream_t st)
    {
        if constexpr (stiff_lds(D, Q, 4) <= kLdsMax)
            if (nw >= 4) return mult_nw<4>(Dk, u, pd, y, ncomp, tab, st);
        static_assert(stiff_lds(D, Q, 2) <= kLdsMax, "the 2-wave stiffness kernel must fit LDS");
        return mult_nw<2>(Dk, u, pd, y, ncomp, tab, st);
    }
};

bool stiff_kernels(int p, int Q, StiffSet *out)
{
#define FEPA_ENTRY(P, QQ)                                                     \
    if (p == P && Q == QQ) {                                                  \
        *out = StiffSet{StiffLaunch<P + 1, QQ>::qdata, StiffLaunch<P + 1, QQ>::mult}; \
        return true;                                                          \
    }
    FEPA_PQ_LIST(FEPA_ENTRY)
#undef FEPA_ENTRY
    return false;
}

}  // namespace fepa
