// Fully matrix-free force pair: y = F 1 and z = F^T v of the state (x, v, e)
// with the quadrature data formed on the fly and never stored (the
// on-the-fly quadrature-data style the paper uses for its mesh-optimisation
// kernels, Sec. 3.4, applied to the Lagrange force operator of Sec. 3.3).
// Per element, in one pass: the reference gradients of the positions and of
// the velocity by sum factorisation (Sec. 3.2), then at every point J, detJ,
// J^-1, rho = m_q / (w detJ), e_q, the ideal-gas pressure, the viscosity and
// S = w detJ sigma J^-T (the algebra of the qdata kernel), then the two force
// contractions of that S: its transposed gradient stages for F 1 and its
// S : grad_xi v with the L2 test functions for F^T v.
//
// Layout: one patch per workgroup (the element restriction R and its
// scatter-add R^T as in the PA kernels: the patch's node values of x and v
// read once into LDS, F 1 summed into LDS slots, private nodes stored and
// shared nodes left as partials for k_gather_shared); column layout, one
// thread per point column (qx, qy) with qz in registers; the 1-D stages of
// every direction but z go through per-element LDS staging, which the
// forward, transposed and L2 stages use in turn (wave fences between them).
#include "kern_common.hpp"
#include "kern_mf.hpp"

namespace fepa {

template <int D, int Q, int NW>
__global__ void __launch_bounds__(NW * 64)
k_force_mf(const double *__restrict__ x, const double *__restrict__ v,
           const double *__restrict__ e, const double *__restrict__ mq,
           const int32_t *__restrict__ perm, const uint16_t *__restrict__ slot,
           const int32_t *__restrict__ pn, const int32_t *__restrict__ ptab,
           double *__restrict__ y, double *__restrict__ part, double *__restrict__ z,
           long long ncomp, const double *__restrict__ tab, QParams prm,
           long long *__restrict__ min_key, int *__restrict__ nonfinite)
{
    constexpr int NE = NW * wave_ne(Q), UMAX = patch_umax(D);
    constexpr int DL = D - 1, QQ = Q * Q, Q3 = Q * Q * Q, D3 = D * D * D, DL3 = DL * DL * DL;
    constexpr int NX = 2 * D * D * Q, NA = 3 * D * QQ, NT = DL * QQ + DL * DL * Q;
    constexpr int NSW = (NA + NX > NT ? NA + NX : NT);  // staging per element
    using T = Tab<D, Q>;
    __shared__ double xs[3 * UMAX];
    __shared__ double vs[3 * UMAX];
    __shared__ double acc[3 * UMAX];
    __shared__ int sSl[NE + 1][D3];
    __shared__ double sW[NE + 1][NSW];
    __shared__ long long sMin, sDt;
    __shared__ int sBad;

    const Lane L = lane_map<Q, NE>();
    const int tid = threadIdx.x, le = L.le, t = L.t, qx = t % Q, qy = t / Q;
    const PatchRow pr = load_patch(ptab, xcd_block(blockIdx.x, gridDim.x));
    for (int k = tid; k < pr.U; k += blockDim.x) {
        const long long g = pn[pr.pno + k];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xs[3 * k + c] = x[c * ncomp + g];
            vs[3 * k + c] = v[c * ncomp + g];
            acc[3 * k + c] = 0.0;
        }
    }
    if (tid == 0) {
        sMin = sDt = 0x7fffffffffffffffLL;
        sBad = 0;
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
    const double wxy = tab[T::W + qx] * tab[T::W + qy];
    __syncthreads();

    // the element's staging, used in turn by the stages below (no restrict:
    // the views alias)
    double *sX = sW[le];       // forward x-stage [2][D][D*Q]
    double *sA = sW[le];       // transposed z-stage [3][D][QQ]
    double *sC = sW[le] + NA;  // transposed y-stage [2][D][D*Q]
    double *sT = sW[le];       // L2 z-stage [DL][QQ]
    double *sT2 = sW[le] + DL * QQ;  // L2 y-stage [DL][DL*Q]
    long long kMin = 0x7fffffffffffffffLL, kDt = 0x7fffffffffffffffLL;
    bool bad = false;

#pragma unroll 1
    for (int base = 0; base < pr.cnt; base += NE) {
        const int idx = base + le;
        const bool act = L.valid && idx < pr.cnt;
        const long long el = pr.eb + (act ? idx : 0);
        for (int i = t; i < D3; i += QQ) sSl[le][i] = slot[el * D3 + i];
        double mqv[Q], eq[Q];
#pragma unroll
        for (int qz = 0; qz < Q; ++qz) mqv[qz] = mq[el * Q3 + qz * QQ + t];
        {
            const double *__restrict__ ee = e + (long long)perm[el] * DL3;
            double tz[DL];
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                double s = 0.0;
#pragma unroll
                for (int jy = 0; jy < DL; ++jy) {
                    double u = 0.0;
#pragma unroll
                    for (int jx = 0; jx < DL; ++jx) u += tab[T::BL + qx * DL + jx] * ee[(jz * DL + jy) * DL + jx];
                    s += tab[T::BL + qy * DL + jy] * u;
                }
                tz[jz] = s;
            }
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                double s = 0.0;
#pragma unroll
                for (int jz = 0; jz < DL; ++jz) s += tab[T::BL + qz * DL + jz] * tz[jz];
                eq[qz] = s;
            }
        }
        wave_sync();
        // forward x and y stages of the six fields (x_c, then v_c): the
        // y-stage results (B_y G_x, G_y B_x, B_y B_x) stay in registers
        double yf[6][3][D];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const double *__restrict__ src = f < 3 ? xs : vs;
            const int c = f % 3;
            if (qy < D) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    double ub = 0.0, ug = 0.0;
#pragma unroll
                    for (int ix = 0; ix < D; ++ix) {
                        const double uu = src[3 * sSl[le][(iz * D + qy) * D + ix] + c];
                        ub += rBx[ix] * uu;
                        ug += rGx[ix] * uu;
                    }
                    sX[(0 * D + iz) * D * Q + qy * Q + qx] = ub;
                    sX[(1 * D + iz) * D * Q + qy * Q + qx] = ug;
                }
            }
            wave_sync();
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
                yf[f][0][iz] = a;
                yf[f][1][iz] = b;
                yf[f][2][iz] = cc;
            }
            wave_sync();  // sX is rewritten by the next field
        }
        // per point: z-stage, the quadrature-data algebra, the F^T v integrand
        // and the z-stage of the transposed gradient (all three components)
        double a0[3][D], a1[3][D], a2[3][D], st[Q];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int i = 0; i < D; ++i) a0[c][i] = a1[c][i] = a2[c][i] = 0.0;
#pragma unroll
        for (int qz = 0; qz < Q; ++qz) {
            double g[6][3];
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                double a = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const double bb = tab[T::B + qz * D + iz], gg = tab[T::G + qz * D + iz];
                    a += bb * yf[f][0][iz];
                    b += bb * yf[f][1][iz];
                    cc += gg * yf[f][2][iz];
                }
                g[f][0] = a;
                g[f][1] = b;
                g[f][2] = cc;
            }
            // J[c][d] = g[c][d]; grad_xi v = g[3 + c][d]
            const double A00 = g[1][1] * g[2][2] - g[1][2] * g[2][1], A01 = g[0][2] * g[2][1] - g[0][1] * g[2][2];
            const double A02 = g[0][1] * g[1][2] - g[0][2] * g[1][1], A10 = g[1][2] * g[2][0] - g[1][0] * g[2][2];
            const double A11 = g[0][0] * g[2][2] - g[0][2] * g[2][0], A12 = g[0][2] * g[1][0] - g[0][0] * g[1][2];
            const double A20 = g[1][0] * g[2][1] - g[1][1] * g[2][0], A21 = g[0][1] * g[2][0] - g[0][0] * g[2][1];
            const double A22 = g[0][0] * g[1][1] - g[0][1] * g[1][0];
            const double detJ = g[0][0] * A00 + g[0][1] * A10 + g[0][2] * A20;
            const double id = 1.0 / detJ;
            const double Ji[3][3] = {{A00 * id, A01 * id, A02 * id},
                                     {A10 * id, A11 * id, A12 * id},
                                     {A20 * id, A21 * id, A22 * id}};
            const double w = wxy * tab[T::W + qz];
            const double rho = mqv[qz] / (w * detJ);
            const double pres = prm.gm1 * rho * eq[qz];
            const double cs = sqrt(prm.gamma * prm.gm1 * fmax(eq[qz], 0.0));
            double Lg[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    Lg[c][k] = g[3 + c][0] * Ji[0][k] + g[3 + c][1] * Ji[1][k] + g[3 + c][2] * Ji[2][k];
            double eps[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) eps[a][b] = 0.5 * (Lg[a][b] + Lg[b][a]);
            const double tr = eps[0][0] + eps[1][1] + eps[2][2];
            const double ell = cbrt(detJ) * prm.inv_order;
            const double mu = rho * ell * (prm.q1 * cs + prm.q2 * ell * fmax(-tr, 0.0));
            if (act) {
                const double speed = cs + mu / (rho * ell);
                const long long kd = ordered_key(speed > 0.0 ? ell / speed : INFINITY);
                const long long km = ordered_key(detJ);
                kDt = kd < kDt ? kd : kDt;
                kMin = km < kMin ? km : kMin;
                if (!isfinite(detJ)) bad = true;
            }
            const double wd = w * detJ;
            double sdot = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double S[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    double sv = 0.0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) sv += (mu * eps[c][k] - (c == k ? pres : 0.0)) * Ji[d][k];
                    S[d] = sv * wd;
                }
                sdot += S[0] * g[3 + c][0] + S[1] * g[3 + c][1] + S[2] * g[3 + c][2];
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const double b = tab[T::B + qz * D + iz], gg = tab[T::G + qz * D + iz];
                    a0[c][iz] += b * S[0];
                    a1[c][iz] += b * S[1];
                    a2[c][iz] += gg * S[2];
                }
            }
            st[qz] = sdot;
        }
        // F 1: transposed y and x stages per component into the patch slots
        int sl[D];
        {
            const int qxc = qx < D ? qx : D - 1, qyc = qy < D ? qy : D - 1;
#pragma unroll
            for (int iz = 0; iz < D; ++iz) sl[iz] = sSl[le][(iz * D + qyc) * D + qxc];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                sA[(0 * D + iz) * QQ + t] = a0[c][iz];
                sA[(1 * D + iz) * QQ + t] = a1[c][iz];
                sA[(2 * D + iz) * QQ + t] = a2[c][iz];
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
            wave_sync();  // the staging is rewritten next
        }
        // F^T v: B_l^T in z (registers), y and x through the staging
#pragma unroll
        for (int jz = 0; jz < DL; ++jz) {
            double a = 0.0;
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) a += tab[T::BL + qz * DL + jz] * st[qz];
            sT[jz * QQ + t] = a;
        }
        wave_sync();
        if (qy < DL) {
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                double a = 0.0;
#pragma unroll
                for (int k = 0; k < Q; ++k) a += tab[T::BL + k * DL + qy] * sT[jz * QQ + k * Q + qx];
                sT2[jz * DL * Q + qy * Q + qx] = a;
            }
        }
        wave_sync();
        if (act && qx < DL && qy < DL) {
            double *__restrict__ zr = z + (long long)perm[el] * DL3;
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                double a = 0.0;
#pragma unroll
                for (int k = 0; k < Q; ++k) a += tab[T::BL + k * DL + qx] * sT2[jz * DL * Q + qy * Q + k];
                zr[(jz * DL + qy) * DL + qx] = a;
            }
        }
        wave_sync();  // sSl and the staging are rewritten by the next pass
    }
    // minima over the wave first: one LDS atomic per wave
    kMin = wave_min_key(kMin);
    kDt = wave_min_key(kDt);
    const bool anyBad = __any(bad);
    if ((tid & 63) == 0) {
        atomicMin(&sMin, kMin);
        atomicMin(&sDt, kDt);
        if (anyBad) atomicOr(&sBad, 1);
    }
    __syncthreads();
    patch_write<UMAX>(acc, pr, pn, y, part, ncomp);
    if (tid == 0) {
        atomicMin(min_key, sMin);
        atomicMin(min_key + 1, sDt);
        if (sBad) atomicOr(nonfinite, 1);
    }
}

// LDS bytes of k_force_mf with NW waves per workgroup
__host__ __device__ constexpr int force_mf_lds(int D, int Q, int NW)
{
    const int na = 3 * D * Q * Q + 2 * D * D * Q, nt = (D - 1) * Q * Q + (D - 1) * (D - 1) * Q;
    return 9 * 8 * patch_umax(D) + (NW * wave_ne(Q) + 1) * (4 * D * D * D + 8 * (na > nt ? na : nt)) + 32;
}

template <int D, int Q>
struct MfLaunch {
    template <int NW>
    static void run_nw(const double *x, const double *v, const double *e, const double *mq,
                       const PatchDev &pd, double *y, double *z, long long ncomp, const double *tab,
                       QParams prm, long long *min_key, int *nonfinite, hipStream_t st)
    {
        hipLaunchKernelGGL((k_force_mf<D, Q, NW>), dim3(pd.n_patch), dim3(NW * 64), 0, st, x, v, e, mq,
                           pd.perm, pd.slot, pd.pn, pd.ptab, y, pd.part, z, ncomp, tab, prm, min_key,
                           nonfinite);
    }
    static void run(const double *x, const double *v, const double *e, const double *mq,
                    const PatchDev &pd, double *y, double *z, long long ncomp, const double *tab,
                    QParams prm, long long *min_key, int *nonfinite, int nw, hipStream_t st)
    {
        if constexpr (force_mf_lds(D, Q, 4) <= kLdsMax)
            if (nw >= 4) return run_nw<4>(x, v, e, mq, pd, y, z, ncomp, tab, prm, min_key, nonfinite, st);
        static_assert(force_mf_lds(D, Q, 2) <= kLdsMax, "the 2-wave matrix-free kernel must fit LDS");
        return run_nw<2>(x, v, e, mq, pd, y, z, ncomp, tab, prm, min_key, nonfinite, st);
    }
};

// The pairs whose kernel keeps every value in registers (VGPRs and AGPRs, no
// scratch): p = 1, 2 at every Q and p = 3 at Q = 4. At larger p and Q the
// per-point algebra plus the stage results of six fields exceed the register
// file, and those pairs are not built (FE_EUNSUPPORTED).
#define FEPA_MF_LIST(X) X(1, 2) X(1, 3) X(1, 4) X(2, 3) X(2, 4) X(2, 5) X(3, 4)

MfFn mf_kernel(int p, int Q)
{
#define FEPA_ENTRY(P, QQ) \
    if (p == P && Q == QQ) return MfLaunch<P + 1, QQ>::run;
    FEPA_MF_LIST(FEPA_ENTRY)
#undef FEPA_ENTRY
    return nullptr;
}

}  // namespace fepa
