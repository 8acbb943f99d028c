// FP64 partial-assembly kernels for gfx950: quadrature data, force actions
// F e / F 1 and F^T v, and the H1 mass action (paper Sec. 3.1 operator
// decomposition, Sec. 3.2 sum factorisation, Sec. 3.3 Lagrange operators).
//
// Thread layouts
//   column layout (force, force^T, mass): one thread per quadrature column
//     (qx, qy) of an element, walking qz in registers; NE = 256/Q^2 elements
//     per workgroup. The qz contraction runs in registers with coefficients
//     that are uniform across the wave (scalar loads); the qy and qx
//     contractions go through LDS.
//   point layout (qdata): one thread per quadrature point, Q^3 per element,
//     all three 1-D stages staged through LDS.
// Element data (S, m_q) is stored element-slowest, quadrature-point-fastest,
// so every load instruction of a wave reads whole 128-byte lines.
#include "kern_common.hpp"
#include "kern_fp64.hpp"

namespace fepa {

template <typename RS>
__device__ __forceinline__ RS cvt(double v) { return (RS)v; }
template <>
__device__ __forceinline__ __bf16 cvt<__bf16>(double v) { return (__bf16)(float)v; }

// ---------------------------------------------------------------- helpers
__global__ void k_fill(double *__restrict__ y, long long n, double val)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) y[i] = val;
}

// ------------------------------------------------------------------ force F e
// y[c][g] = sum_E sum_q sum_d S[c][d](q) dw_i/dxi_d(q) (B_l e)(q), one patch
// per workgroup. Three H1 contraction stages per component with the three
// derivative terms fused: z-stage -> (B, B, G), y-stage -> (B | G + B),
// x-stage -> (G + B); element results are summed into the patch's LDS slots.
template <int D, int Q, bool ONE, typename R, int NW, typename RS = R>
__global__ void __launch_bounds__(NW * 64)
k_force(const RS *__restrict__ S, const double *__restrict__ e,
        const int32_t *__restrict__ perm, const uint16_t *__restrict__ slot,
        const int32_t *__restrict__ pn, const int32_t *__restrict__ ptab,
        double *__restrict__ y, double *__restrict__ part, long long ncomp,
        const R *__restrict__ tab)
{
    constexpr int NE = NW * wave_ne(Q), UMAX = patch_umax(D);
    constexpr int DL = D - 1, QQ = Q * Q, D3 = D * D * D, DL3 = DL * DL * DL;
    constexpr int SQ = s_stride<RS>(Q);  // points per stored (c, d) row
    using T = Tab<D, Q>;
    __shared__ R acc[3 * UMAX];
    __shared__ R sA[NE + 1][3][D][QQ];
    __shared__ R sC[NE + 1][2][D][D * Q];

    const Lane L = lane_map<Q, NE>();
    const int tid = threadIdx.x, le = L.le, t = L.t, qx = t % Q, qy = t / Q;
    const PatchRow pr = load_patch(ptab, xcd_block(blockIdx.x, gridDim.x));
    for (int k = tid; k < 3 * pr.U; k += blockDim.x) acc[k] = 0.0;

    R cBy[Q], cGy[Q], cBx[Q], cGx[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        cBy[k] = qy < D ? tab[T::B + k * D + qy] : 0.0;
        cGy[k] = qy < D ? tab[T::G + k * D + qy] : 0.0;
        cBx[k] = qx < D ? tab[T::B + k * D + qx] : 0.0;
        cGx[k] = qx < D ? tab[T::G + k * D + qx] : 0.0;
    }
    __syncthreads();

    // S by component: sv holds component c of this pass while sn loads the next
    // component (or component 0 of the next pass); loads never branch (lanes
    // without an element read a valid one and store nothing)
    R sv[3][Q], sn[3][Q];
    {
        const bool act0 = L.valid && le < pr.cnt;
        const RS *__restrict__ S0 = S + (long long)(pr.eb + (act0 ? le : 0)) * 9 * SQ + t;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) sv[d][qz] = (R)__builtin_nontemporal_load(S0 + d * SQ + qz * QQ);
    }
#pragma unroll 1
    for (int base = 0; base < pr.cnt; base += NE) {
        const int idx = base + le;
        const bool act = L.valid && idx < pr.cnt;
        const long long el = pr.eb + (act ? idx : 0);
        const bool actn = L.valid && idx + NE < pr.cnt;
        const RS *__restrict__ Sc = S + el * 9 * SQ + t;
        const RS *__restrict__ Sn = S + (long long)(pr.eb + (actn ? idx + NE : 0)) * 9 * SQ + t;
        int sl[D];
        const int qxc = qx < D ? qx : D - 1, qyc = qy < D ? qy : D - 1;
#pragma unroll
        for (int iz = 0; iz < D; ++iz) sl[iz] = slot[el * D3 + iz * D * D + qyc * D + qxc];
        R eq[Q];
        if (ONE) {
#pragma unroll
            for (int k = 0; k < Q; ++k) eq[k] = 1.0;
        } else {
            const double *__restrict__ ee = e + (long long)perm[el] * DL3;
            R tz[DL];
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                R s = 0.0;
#pragma unroll
                for (int jy = 0; jy < DL; ++jy) {
                    R u = 0.0;
#pragma unroll
                    for (int jx = 0; jx < DL; ++jx)
                        u += tab[T::BL + qx * DL + jx] * (R)ee[(jz * DL + jy) * DL + jx];
                    s += tab[T::BL + qy * DL + jy] * u;
                }
                tz[jz] = s;
            }
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                R s = 0.0;
#pragma unroll
                for (int jz = 0; jz < DL; ++jz) s += tab[T::BL + qz * DL + jz] * tz[jz];
                eq[qz] = s;
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int qz = 0; qz < Q; ++qz)
                    sn[d][qz] = (R)__builtin_nontemporal_load((c < 2 ? Sc + (c + 1) * 3 * SQ : Sn) + d * SQ + qz * QQ);
            R a0[D], a1[D], a2[D];
#pragma unroll
            for (int i = 0; i < D; ++i) a0[i] = a1[i] = a2[i] = 0.0;
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                const R s0 = sv[0][qz] * eq[qz];
                const R s1 = sv[1][qz] * eq[qz];
                const R s2 = sv[2][qz] * eq[qz];
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const R b = tab[T::B + qz * D + iz], g = tab[T::G + qz * D + iz];
                    a0[iz] += b * s0;
                    a1[iz] += b * s1;
                    a2[iz] += g * s2;
                }
            }
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                sA[le][0][iz][t] = a0[iz];
                sA[le][1][iz][t] = a1[iz];
                sA[le][2][iz][t] = a2[iz];
            }
            wave_sync();
            if (qy < D) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    R c0 = 0.0, c1 = 0.0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) {
                        c0 += cBy[k] * sA[le][0][iz][k * Q + qx];
                        c1 += cGy[k] * sA[le][1][iz][k * Q + qx] + cBy[k] * sA[le][2][iz][k * Q + qx];
                    }
                    sC[le][0][iz][qy * Q + qx] = c0;
                    sC[le][1][iz][qy * Q + qx] = c1;
                }
            }
            wave_sync();
            if (act && qx < D && qy < D) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    R r = 0.0;
#pragma unroll
                    for (int k = 0; k < Q; ++k)
                        r += cGx[k] * sC[le][0][iz][qy * Q + k] + cBx[k] * sC[le][1][iz][qy * Q + k];
                    atomicAdd(&acc[3 * sl[iz] + c], r);
                }
            }
            wave_sync();  // sA and sC are rewritten by the next component
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int qz = 0; qz < Q; ++qz) sv[d][qz] = sn[d][qz];
        }
    }
    __syncthreads();
    patch_write<UMAX>(acc, pr, pn, y, part, ncomp);
}

// ------------------------------------------------- force F e, F 1 at Q = 4
// The same action for four points per direction with the y and x contractions
// done across lanes instead of through LDS. An element's 16 point columns are
// one 16-lane DPP row, laid out qy-fastest: each quad holds the four qy of one
// qx, so a quad broadcast (quad_perm) hands every lane the four values it
// contracts in y, and rotations of the row by 4, 8 and 12 lanes hand it the
// four values it contracts in x. LDS then only holds the patch accumulator.
// S streams one component (3Q values per thread) at a time: the next
// component's loads are issued before the current one is contracted.

// value of the lane selected by a DPP control (row-local), for 32/64-bit types;
// every control used here reads a lane of the same row, so no lane keeps an
// old value and no initialisation of the destination is needed
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_r(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)(b & 0xffffffffLL)), hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_r(float v)
{
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
constexpr int kQuadBcast0 = 0x00, kQuadBcast1 = 0x55, kQuadBcast2 = 0xAA, kQuadBcast3 = 0xFF;
constexpr int kRowRor4 = 0x124, kRowRor8 = 0x128, kRowRor12 = 0x12C;
constexpr int kGatherK = 2;  // patch nodes per thread and round of the node gathers

template <int D, bool ONE, typename R, int NW, typename RS = R>
__global__ void __launch_bounds__(NW * 64)
k_force_q4(const RS *__restrict__ S, const double *__restrict__ e,
           const int32_t *__restrict__ perm, const uint16_t *__restrict__ slot,
           const int32_t *__restrict__ pn, const int32_t *__restrict__ ptab,
           double *__restrict__ y, double *__restrict__ part, long long ncomp,
           const R *__restrict__ tab)
{
    constexpr int Q = 4, NE = NW * 4, UMAX = patch_umax(D);
    constexpr int DL = D - 1, QQ = 16, D3 = D * D * D, DL3 = DL * DL * DL;
    constexpr int SQ = s_stride<RS>(Q);  // points per stored (c, d) row
    using T = Tab<D, Q>;
    __shared__ R acc[3 * UMAX];

    const int tid = threadIdx.x, lane = tid & 63;
    const int le = (tid >> 6) * 4 + (lane >> 4);  // element slot of the lane's row
    const int r = lane & 15, qy = r & 3, qx = r >> 2, t = qx + Q * qy;

    // y: the quad broadcast of lane k brings point row k of column qx
    R cBy[Q], cGy[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        cBy[k] = qy < D ? tab[T::B + k * D + qy] : (R)0;
        cGy[k] = qy < D ? tab[T::G + k * D + qy] : (R)0;
    }
    // x: the row rotation by 4j brings the column of the source lane
    int kx[Q];
    kx[0] = qx;
    kx[1] = dpp_i<kRowRor4>(qx);
    kx[2] = dpp_i<kRowRor8>(qx);
    kx[3] = dpp_i<kRowRor12>(qx);
    R cBx[Q], cGx[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        cBx[j] = qx < D ? tab[T::B + kx[j] * D + qx] : (R)0;
        cGx[j] = qx < D ? tab[T::G + kx[j] * D + qx] : (R)0;
    }

    const PatchRow pr = load_patch(ptab, xcd_block(blockIdx.x, gridDim.x));
    for (int k = tid; k < 3 * pr.U; k += blockDim.x) acc[k] = 0.0;
    __syncthreads();

    // S by component: sv holds component c of this pass while sn loads the next
    // component (or component 0 of the next pass)
    R sv[3][Q], sn[3][Q];
    {
        const bool act0 = le < pr.cnt;
        const RS *__restrict__ S0 = S + (long long)(pr.eb + (act0 ? le : 0)) * 9 * SQ + t;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) sv[d][qz] = (R)__builtin_nontemporal_load(S0 + d * SQ + qz * QQ);
    }
#pragma unroll 1
    for (int base = 0; base < pr.cnt; base += NE) {
        const int idx = base + le;
        const bool act = idx < pr.cnt;
        const long long el = pr.eb + (act ? idx : 0);
        const bool actn = idx + NE < pr.cnt;
        const RS *__restrict__ Sc = S + el * 9 * SQ + t;
        const RS *__restrict__ Sn = S + (long long)(pr.eb + (actn ? idx + NE : 0)) * 9 * SQ + t;
        // lanes past the element count or outside the D x D node columns load a
        // valid neighbour's data and never store (loads without branches)
        int sl[D];
        const int qxc = qx < D ? qx : D - 1, qyc = qy < D ? qy : D - 1;
#pragma unroll
        for (int iz = 0; iz < D; ++iz) sl[iz] = slot[el * D3 + iz * D * D + qyc * D + qxc];
        R eq[Q];
        if (ONE) {
#pragma unroll
            for (int k = 0; k < Q; ++k) eq[k] = 1.0;
        } else {
            const double *__restrict__ ee = e + (long long)perm[el] * DL3;
            R tz[DL];
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                R s = 0.0;
#pragma unroll
                for (int jy = 0; jy < DL; ++jy) {
                    R u = 0.0;
#pragma unroll
                    for (int jx = 0; jx < DL; ++jx)
                        u += tab[T::BL + qx * DL + jx] * (R)ee[(jz * DL + jy) * DL + jx];
                    s += tab[T::BL + qy * DL + jy] * u;
                }
                tz[jz] = s;
            }
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                R s = 0.0;
#pragma unroll
                for (int jz = 0; jz < DL; ++jz) s += tab[T::BL + qz * DL + jz] * tz[jz];
                eq[qz] = s;
            }
        }
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int qz = 0; qz < Q; ++qz)
                    sn[d][qz] = (R)__builtin_nontemporal_load((c < 2 ? Sc + (c + 1) * 3 * SQ : Sn) + d * SQ + qz * QQ);
            // z in registers
            R a0[D], a1[D], a2[D];
#pragma unroll
            for (int i = 0; i < D; ++i) a0[i] = a1[i] = a2[i] = 0.0;
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                const R s0 = sv[0][qz] * eq[qz];
                const R s1 = sv[1][qz] * eq[qz];
                const R s2 = sv[2][qz] * eq[qz];
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const R b = tab[T::B + qz * D + iz], g = tab[T::G + qz * D + iz];
                    a0[iz] += b * s0;
                    a1[iz] += b * s1;
                    a2[iz] += g * s2;
                }
            }
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                // y: thread (qx, iy = qy)
                const R u0[Q] = {dpp_r<kQuadBcast0>(a0[iz]), dpp_r<kQuadBcast1>(a0[iz]),
                                 dpp_r<kQuadBcast2>(a0[iz]), dpp_r<kQuadBcast3>(a0[iz])};
                const R u1[Q] = {dpp_r<kQuadBcast0>(a1[iz]), dpp_r<kQuadBcast1>(a1[iz]),
                                 dpp_r<kQuadBcast2>(a1[iz]), dpp_r<kQuadBcast3>(a1[iz])};
                const R u2[Q] = {dpp_r<kQuadBcast0>(a2[iz]), dpp_r<kQuadBcast1>(a2[iz]),
                                 dpp_r<kQuadBcast2>(a2[iz]), dpp_r<kQuadBcast3>(a2[iz])};
                R c0 = 0.0, c1 = 0.0;
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    c0 += cBy[k] * u0[k];
                    c1 += cGy[k] * u1[k] + cBy[k] * u2[k];
                }
                // x: thread (ix = qx, iy = qy)
                const R w0[Q] = {c0, dpp_r<kRowRor4>(c0), dpp_r<kRowRor8>(c0), dpp_r<kRowRor12>(c0)};
                const R w1[Q] = {c1, dpp_r<kRowRor4>(c1), dpp_r<kRowRor8>(c1), dpp_r<kRowRor12>(c1)};
                R rr = 0.0;
#pragma unroll
                for (int j = 0; j < Q; ++j) rr += cGx[j] * w0[j] + cBx[j] * w1[j];
                if (act && qx < D && qy < D) atomicAdd(&acc[3 * sl[iz] + c], rr);
            }
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int qz = 0; qz < Q; ++qz) sv[d][qz] = sn[d][qz];
        }
    }
    __syncthreads();
    patch_write<UMAX>(acc, pr, pn, y, part, ncomp);
}

// ---------------------------------------------------------- force^T F^T v
// z[E][j] = sum_q phi_j(q) sum_{c,d} S[c][d](q) (grad_xi v_c)_d(q), one patch per
// workgroup: the patch's distinct nodes of v are read once into LDS; rows of z
// are written in caller element order.

template <int D, int Q, typename R, typename RS, int NW>
__global__ void __launch_bounds__(NW * 64)
k_force_t(const RS *__restrict__ S, const double *__restrict__ v,
          const int32_t *__restrict__ perm, const uint16_t *__restrict__ slot,
          const int32_t *__restrict__ pn, const int32_t *__restrict__ ptab,
          double *__restrict__ z, long long ncomp, const R *__restrict__ tab)
{
    constexpr int NE = NW * wave_ne(Q), UMAX = patch_umax(D);
    constexpr int DL = D - 1, QQ = Q * Q, D3 = D * D * D, DL3 = DL * DL * DL;
    using T = Tab<D, Q>;
    constexpr bool LANES = Q == 4;          // y, x stages across lanes
    constexpr int NA = LANES ? 1 : NE + 1;  // staging of the LDS-staged stages
    __shared__ R vs[3 * UMAX];
    __shared__ int sSl[NE + 1][D3];
    __shared__ R sX[NA][2][D][D * Q];
    __shared__ R sT[NA][DL][QQ];
    __shared__ R sT2[NA][DL][DL * Q];

    const int tid = threadIdx.x;
    int le, t, qx, qy;
    bool valid;
    if constexpr (LANES) {
        // an element is one 16-lane row, point row qy fastest (quads share qx)
        const int lane = tid & 63, r = lane & 15;
        le = (tid >> 6) * 4 + (lane >> 4);
        qy = r & 3;
        qx = r >> 2;
        t = qx + Q * qy;
        valid = true;
    } else {
        const Lane L = lane_map<Q, NE>();
        le = L.le;
        t = L.t;
        qx = t % Q;
        qy = t / Q;
        valid = L.valid;
    }
    const PatchRow pr = load_patch(ptab, xcd_block(blockIdx.x, gridDim.x));
    patch_gather<kGatherK>(vs, pr, pn, v, nullptr, 0.0, ncomp);
    R rBx[D], rGx[D], rBy[D], rGy[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        rBx[i] = tab[T::B + qx * D + i];
        rGx[i] = tab[T::G + qx * D + i];
        rBy[i] = tab[T::B + qy * D + i];
        rGy[i] = tab[T::G + qy * D + i];
    }
    // across lanes: L2 weights of the point row qy, and of the rotated source
    // columns of the x stage
    R cLy[LANES ? Q : 1], cLx[LANES ? Q : 1];
    if constexpr (LANES) {
        const int kx[Q] = {qx, dpp_i<kRowRor4>(qx), dpp_i<kRowRor8>(qx), dpp_i<kRowRor12>(qx)};
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            cLx[j] = qx < DL ? tab[T::BL + kx[j] * DL + qx] : (R)0;
            cLy[j] = qy < DL ? tab[T::BL + j * DL + qy] : (R)0;
        }
    }
    // idle lanes (spare element row NE) read slots from the spare row: keep it valid
    for (int i = tid; i < D3; i += blockDim.x) sSl[NE][i] = 0;

    __syncthreads();

    // At Q = 4 a pass loads its element's 9 Q values of S at once. For Q >= 5
    // (registers) S streams by component: sv holds component c while sn
    // loads the next component (or component 0 of the next pass).
    constexpr bool STREAM = !LANES;
    constexpr int SQ = s_stride<RS>(Q);
    R sv[STREAM ? 3 : 9][Q], sn[STREAM ? 3 : 1][Q];
    if constexpr (STREAM) {
        const bool act0 = valid && le < pr.cnt;
        const RS *__restrict__ S0 = S + (long long)(pr.eb + (act0 ? le : 0)) * 9 * SQ + t;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) sv[d][qz] = (R)__builtin_nontemporal_load(S0 + d * SQ + qz * QQ);
    }
#pragma unroll 1
    for (int base = 0; base < pr.cnt; base += NE) {
        const int idx = base + le;
        const bool act = valid && idx < pr.cnt;
        const long long el = pr.eb + (act ? idx : 0);
        const RS *__restrict__ Se = S + el * 9 * SQ + t;
        const bool actn = valid && idx + NE < pr.cnt;
        const RS *__restrict__ Sn = S + (long long)(pr.eb + (actn ? idx + NE : 0)) * 9 * SQ + t;
        if constexpr (!STREAM) {
#pragma unroll
            for (int cd = 0; cd < 9; ++cd)
#pragma unroll
                for (int qz = 0; qz < Q; ++qz)
                    sv[cd][qz] = (R)__builtin_nontemporal_load(Se + cd * SQ + qz * QQ);
        }
        if constexpr (sizeof(R) == 8) {  // FP64 instances: the slot loads in flight together
            SlotPipe<D3, QQ> sp;
            sp.fetch(slot, el, t);
            sp.store(sSl[le], t);
        } else {
            for (int i = t; i < D3; i += QQ) sSl[le][i] = slot[el * D3 + i];
        }
        wave_sync();
        R s[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) s[k] = 0.0;
        constexpr int kCUnroll = STREAM ? 1 : 3;
#pragma unroll kCUnroll
        for (int c = 0; c < 3; ++c) {
            if constexpr (STREAM) {
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int qz = 0; qz < Q; ++qz)
                        sn[d][qz] = (R)__builtin_nontemporal_load((c < 2 ? Se + (c + 1) * 3 * SQ : Sn) +
                                                                  d * SQ + qz * QQ);
            }
            R vx[D], vy[D], vz[D];
            if constexpr (LANES) {
                // x-stage: thread (qx, iy = qy) from the node values; y-stage
                // over the quad's node rows
                const int qyc = qy < D ? qy : D - 1;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    R ub = 0.0, ug = 0.0;
#pragma unroll
                    for (int ix = 0; ix < D; ++ix) {
                        const R u = vs[3 * sSl[le][(iz * D + qyc) * D + ix] + c];
                        ub += rBx[ix] * u;
                        ug += rGx[ix] * u;
                    }
                    const R bb[Q] = {dpp_r<kQuadBcast0>(ub), dpp_r<kQuadBcast1>(ub),
                                     dpp_r<kQuadBcast2>(ub), dpp_r<kQuadBcast3>(ub)};
                    const R bg[Q] = {dpp_r<kQuadBcast0>(ug), dpp_r<kQuadBcast1>(ug),
                                     dpp_r<kQuadBcast2>(ug), dpp_r<kQuadBcast3>(ug)};
                    R a = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
                    for (int iy = 0; iy < D; ++iy) {
                        a += rBy[iy] * bg[iy];
                        b += rGy[iy] * bb[iy];
                        cc += rBy[iy] * bb[iy];
                    }
                    vx[iz] = a;
                    vy[iz] = b;
                    vz[iz] = cc;
                }
            } else {
                // x-stage: thread (qx, iy = qy)
                if (qy < D) {
#pragma unroll
                    for (int iz = 0; iz < D; ++iz) {
                        R ub = 0.0, ug = 0.0;
#pragma unroll
                        for (int ix = 0; ix < D; ++ix) {
                            const R u = vs[3 * sSl[le][(iz * D + qy) * D + ix] + c];
                            ub += rBx[ix] * u;
                            ug += rGx[ix] * u;
                        }
                        sX[le][0][iz][qy * Q + qx] = ub;
                        sX[le][1][iz][qy * Q + qx] = ug;
                    }
                }
                wave_sync();
                // y-stage into registers
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    R a = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
                    for (int iy = 0; iy < D; ++iy) {
                        const R ub = sX[le][0][iz][iy * Q + qx], ug = sX[le][1][iz][iy * Q + qx];
                        a += rBy[iy] * ug;
                        b += rGy[iy] * ub;
                        cc += rBy[iy] * ub;
                    }
                    vx[iz] = a;
                    vy[iz] = b;
                    vz[iz] = cc;
                }
                wave_sync();  // sX is rewritten by the next component
            }
            // z-stage and the pointwise S : grad v
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                R dx = 0.0, dy = 0.0, dz = 0.0;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const R bb = tab[T::B + qz * D + iz], gg = tab[T::G + qz * D + iz];
                    dx += bb * vx[iz];
                    dy += bb * vy[iz];
                    dz += gg * vz[iz];
                }
                const int r0 = STREAM ? 0 : c * 3;
                s[qz] += sv[r0][qz] * dx + sv[r0 + 1][qz] * dy + sv[r0 + 2][qz] * dz;
            }
            if constexpr (STREAM) {
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int qz = 0; qz < Q; ++qz) sv[d][qz] = sn[d][qz];
            }
        }
        // L2 test functions: B_l^T in z (registers), y and x (LDS, or across
        // lanes at Q = 4)
        if constexpr (LANES) {
            double *__restrict__ zr = z + (long long)perm[el] * DL3;
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                R a = 0.0;
#pragma unroll
                for (int qz = 0; qz < Q; ++qz) a += tab[T::BL + qz * DL + jz] * s[qz];
                const R u[Q] = {dpp_r<kQuadBcast0>(a), dpp_r<kQuadBcast1>(a), dpp_r<kQuadBcast2>(a),
                                dpp_r<kQuadBcast3>(a)};
                R b = 0.0;
#pragma unroll
                for (int k = 0; k < Q; ++k) b += cLy[k] * u[k];
                const R w[Q] = {b, dpp_r<kRowRor4>(b), dpp_r<kRowRor8>(b), dpp_r<kRowRor12>(b)};
                R o = 0.0;
#pragma unroll
                for (int j = 0; j < Q; ++j) o += cLx[j] * w[j];
                if (act && qx < DL && qy < DL) zr[(jz * DL + qy) * DL + qx] = (double)o;
            }
            wave_sync();  // sSl is rewritten by the next pass
        } else {
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                R a = 0.0;
#pragma unroll
                for (int qz = 0; qz < Q; ++qz) a += tab[T::BL + qz * DL + jz] * s[qz];
                sT[le][jz][t] = a;
            }
            wave_sync();
            if (qy < DL) {
#pragma unroll
                for (int jz = 0; jz < DL; ++jz) {
                    R a = 0.0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) a += tab[T::BL + k * DL + qy] * sT[le][jz][k * Q + qx];
                    sT2[le][jz][qy * Q + qx] = a;
                }
            }
            wave_sync();
            if (act && qx < DL && qy < DL) {
                double *__restrict__ zr = z + (long long)perm[el] * DL3;
#pragma unroll
                for (int jz = 0; jz < DL; ++jz) {
                    R a = 0.0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) a += tab[T::BL + k * DL + qx] * sT2[le][jz][qy * Q + k];
                    zr[(jz * DL + qy) * DL + qx] = (double)a;
                }
            }
        }
    }
}

// ------------------------------------------------ both force actions at once
// y = F e (or F 1) and z = F^T v in one pass over S: the two actions share S
// and the Lagrange step needs both at every stage (momentum and energy
// equations, Sec. 3.3), so one read of S serves both. Per component c a pass
// runs the F e contraction of c, then the F^T v contraction of c, while the
// next component's S loads. At Q = 4 the y and x stages of F e run across
// lanes as in k_force_q4.
template <int D, int Q, bool ONE, typename R, int NW, typename RS = R>
__global__ void __launch_bounds__(NW * 64)
k_force_pair(const RS *__restrict__ S, const double *__restrict__ e, const double *__restrict__ v,
             const int32_t *__restrict__ perm, const uint16_t *__restrict__ slot,
             const int32_t *__restrict__ pn, const int32_t *__restrict__ ptab,
             double *__restrict__ y, double *__restrict__ part, double *__restrict__ z,
             long long ncomp, const R *__restrict__ tab)
{
    constexpr int NE = NW * wave_ne(Q), UMAX = patch_umax(D);
    constexpr int DL = D - 1, QQ = Q * Q, D3 = D * D * D, DL3 = DL * DL * DL;
    constexpr bool LANES = Q == 4;
    constexpr int NA = LANES ? 1 : NE + 1;  // staging of the LDS-staged stages (unused across lanes)
    constexpr int SQ = s_stride<RS>(Q);  // points per stored (c, d) row
    using T = Tab<D, Q>;
    __shared__ R acc[3 * UMAX];
    __shared__ R vs[3 * UMAX];
    __shared__ int sSl[NE + 1][D3];
    __shared__ R sX[NA][2][D][D * Q];
    __shared__ R sT[NA][DL][QQ];
    __shared__ R sT2[NA][DL][DL * Q];
    __shared__ R sA[NA][3][D][QQ];
    __shared__ R sC[NA][2][D][D * Q];

    const int tid = threadIdx.x;
    int le, t, qx, qy;
    bool valid;
    if constexpr (LANES) {
        const int lane = tid & 63, r = lane & 15;
        le = (tid >> 6) * 4 + (lane >> 4);
        qy = r & 3;
        qx = r >> 2;
        t = qx + Q * qy;
        valid = true;
    } else {
        const Lane L = lane_map<Q, NE>();
        le = L.le;
        t = L.t;
        qx = t % Q;
        qy = t / Q;
        valid = L.valid;
    }
    const PatchRow pr = load_patch(ptab, xcd_block(blockIdx.x, gridDim.x));
    for (int k = tid; k < 3 * pr.U; k += blockDim.x) acc[k] = 0.0;
    patch_gather<kGatherK>(vs, pr, pn, v, nullptr, 0.0, ncomp);
    // F e: y weights (column qy), x weights (column qx, or the rotated source column)
    R cBy[Q], cGy[Q], cBx[Q], cGx[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        cBy[k] = qy < D ? tab[T::B + k * D + qy] : (R)0;
        cGy[k] = qy < D ? tab[T::G + k * D + qy] : (R)0;
    }
    // F^T v across lanes: L2 weights of the point row qy, and of the rotated
    // source columns for the x stage
    R cLy[LANES ? Q : 1], cLx[LANES ? Q : 1];
    if constexpr (LANES) {
        const int kx[Q] = {qx, dpp_i<kRowRor4>(qx), dpp_i<kRowRor8>(qx), dpp_i<kRowRor12>(qx)};
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            cBx[j] = qx < D ? tab[T::B + kx[j] * D + qx] : (R)0;
            cGx[j] = qx < D ? tab[T::G + kx[j] * D + qx] : (R)0;
            cLx[j] = qx < DL ? tab[T::BL + kx[j] * DL + qx] : (R)0;
            cLy[j] = qy < DL ? tab[T::BL + j * DL + qy] : (R)0;
        }
    } else {
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            cBx[k] = qx < D ? tab[T::B + k * D + qx] : (R)0;
            cGx[k] = qx < D ? tab[T::G + k * D + qx] : (R)0;
        }
    }
    // F^T v: interpolation weights of the point row qy / column qx
    R rBx[D], rGx[D], rBy[D], rGy[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        rBx[i] = tab[T::B + qx * D + i];
        rGx[i] = tab[T::G + qx * D + i];
        rBy[i] = tab[T::B + qy * D + i];
        rGy[i] = tab[T::G + qy * D + i];
    }
    // idle lanes (spare element row NE) read slots from the spare row: keep it valid
    for (int i = tid; i < D3; i += blockDim.x) sSl[NE][i] = 0;
    __syncthreads();

    // S by component: sv holds component c of this pass while sn loads the next
    // component (or component 0 of the next pass)
    R sv[3][Q], sn[3][Q];
    {
        const bool act0 = valid && le < pr.cnt;
        const RS *__restrict__ S0 = S + (long long)(pr.eb + (act0 ? le : 0)) * 9 * SQ + t;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int qz = 0; qz < Q; ++qz)
                sv[d][qz] = (R)__builtin_nontemporal_load(S0 + d * SQ + qz * QQ);
    }
    SlotPipe<D3, QQ> sp;
    if constexpr (sizeof(R) == 8) sp.fetch(slot, pr.eb + (valid && le < pr.cnt ? le : 0), t);
#pragma unroll 1
    for (int base = 0; base < pr.cnt; base += NE) {
        const int idx = base + le;
        const bool act = valid && idx < pr.cnt;
        const long long el = pr.eb + (act ? idx : 0);
        const bool actn = valid && idx + NE < pr.cnt;
        const RS *__restrict__ Sc = S + el * 9 * SQ + t;
        const RS *__restrict__ Sn = S + (long long)(pr.eb + (actn ? idx + NE : 0)) * 9 * SQ + t;
        if constexpr (sizeof(R) == 8) {  // FP64 instances: slots fetched a pass ahead
            sp.store(sSl[le], t);
            sp.fetch(slot, pr.eb + (actn ? idx + NE : 0), t);
        } else {
            for (int i = t; i < D3; i += QQ) sSl[le][i] = slot[el * D3 + i];
        }
        R eq[Q];
        if (ONE) {
#pragma unroll
            for (int k = 0; k < Q; ++k) eq[k] = 1.0;
        } else {
            const double *__restrict__ ee = e + (long long)perm[el] * DL3;
            R tz[DL];
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                R s = 0.0;
#pragma unroll
                for (int jy = 0; jy < DL; ++jy) {
                    R u = 0.0;
#pragma unroll
                    for (int jx = 0; jx < DL; ++jx)
                        u += tab[T::BL + qx * DL + jx] * (R)ee[(jz * DL + jy) * DL + jx];
                    s += tab[T::BL + qy * DL + jy] * u;
                }
                tz[jz] = s;
            }
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                R s = 0.0;
#pragma unroll
                for (int jz = 0; jz < DL; ++jz) s += tab[T::BL + qz * DL + jz] * tz[jz];
                eq[qz] = s;
            }
        }
        wave_sync();  // the element's slots are in LDS
        // across lanes: 3 x the LDS slots this thread reads (nodes (ix, row
        // qy, iz)) and adds to (node (qx, qy, iz)), for all three components
        int sx[LANES ? D * D : 1], so[LANES ? D : 1];
        if constexpr (LANES) {
            const int qyc = qy < D ? qy : D - 1, qxc = qx < D ? qx : D - 1;
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
#pragma unroll
                for (int ix = 0; ix < D; ++ix) sx[iz * D + ix] = 3 * sSl[le][(iz * D + qyc) * D + ix];
                so[iz] = 3 * sSl[le][(iz * D + qyc) * D + qxc];
            }
        }
        R sf[Q];      // F^T v: S : grad v at the column's points
#pragma unroll
        for (int k = 0; k < Q; ++k) sf[k] = 0.0;
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            // next component's S: this pass's c+1, or the next pass's component 0
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int qz = 0; qz < Q; ++qz)
                    sn[d][qz] = (R)__builtin_nontemporal_load((c < 2 ? Sc + (c + 1) * 3 * SQ : Sn) + d * SQ + qz * QQ);
            // ---- F e, component c: z in registers
            R a0[D], a1[D], a2[D];
#pragma unroll
            for (int i = 0; i < D; ++i) a0[i] = a1[i] = a2[i] = 0.0;
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                const R s0 = sv[0][qz] * eq[qz];
                const R s1 = sv[1][qz] * eq[qz];
                const R s2 = sv[2][qz] * eq[qz];
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const R b = tab[T::B + qz * D + iz], g = tab[T::G + qz * D + iz];
                    a0[iz] += b * s0;
                    a1[iz] += b * s1;
                    a2[iz] += g * s2;
                }
            }
            if constexpr (LANES) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const R u0[Q] = {dpp_r<kQuadBcast0>(a0[iz]), dpp_r<kQuadBcast1>(a0[iz]),
                                     dpp_r<kQuadBcast2>(a0[iz]), dpp_r<kQuadBcast3>(a0[iz])};
                    const R u1[Q] = {dpp_r<kQuadBcast0>(a1[iz]), dpp_r<kQuadBcast1>(a1[iz]),
                                     dpp_r<kQuadBcast2>(a1[iz]), dpp_r<kQuadBcast3>(a1[iz])};
                    const R u2[Q] = {dpp_r<kQuadBcast0>(a2[iz]), dpp_r<kQuadBcast1>(a2[iz]),
                                     dpp_r<kQuadBcast2>(a2[iz]), dpp_r<kQuadBcast3>(a2[iz])};
                    R c0 = 0.0, c1 = 0.0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) {
                        c0 += cBy[k] * u0[k];
                        c1 += cGy[k] * u1[k] + cBy[k] * u2[k];
                    }
                    const R w0[Q] = {c0, dpp_r<kRowRor4>(c0), dpp_r<kRowRor8>(c0), dpp_r<kRowRor12>(c0)};
                    const R w1[Q] = {c1, dpp_r<kRowRor4>(c1), dpp_r<kRowRor8>(c1), dpp_r<kRowRor12>(c1)};
                    R rr = 0.0;
#pragma unroll
                    for (int j = 0; j < Q; ++j) rr += cGx[j] * w0[j] + cBx[j] * w1[j];
                    if (act && qx < D && qy < D) atomicAdd(&acc[so[iz] + c], rr);
                }
            } else {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    sA[le][0][iz][t] = a0[iz];
                    sA[le][1][iz][t] = a1[iz];
                    sA[le][2][iz][t] = a2[iz];
                }
                wave_sync();
                if (qy < D) {
#pragma unroll
                    for (int iz = 0; iz < D; ++iz) {
                        R c0 = 0.0, c1 = 0.0;
#pragma unroll
                        for (int k = 0; k < Q; ++k) {
                            c0 += cBy[k] * sA[le][0][iz][k * Q + qx];
                            c1 += cGy[k] * sA[le][1][iz][k * Q + qx] + cBy[k] * sA[le][2][iz][k * Q + qx];
                        }
                        sC[le][0][iz][qy * Q + qx] = c0;
                        sC[le][1][iz][qy * Q + qx] = c1;
                    }
                }
                wave_sync();
                if (act && qx < D && qy < D) {
#pragma unroll
                    for (int iz = 0; iz < D; ++iz) {
                        R rr = 0.0;
#pragma unroll
                        for (int k = 0; k < Q; ++k)
                            rr += cGx[k] * sC[le][0][iz][qy * Q + k] + cBx[k] * sC[le][1][iz][qy * Q + k];
                        atomicAdd(&acc[3 * sSl[le][(iz * D + qy) * D + qx] + c], rr);
                    }
                }
            }
            // ---- F^T v, component c
            R vx[D], vy[D], vz[D];
            if constexpr (LANES) {
                // x-stage: thread (qx, iy = qy) from the node values; y-stage
                // over the quad's node rows
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    R ub = 0.0, ug = 0.0;
#pragma unroll
                    for (int ix = 0; ix < D; ++ix) {
                        const R u = vs[sx[iz * D + ix] + c];
                        ub += rBx[ix] * u;
                        ug += rGx[ix] * u;
                    }
                    const R bb[Q] = {dpp_r<kQuadBcast0>(ub), dpp_r<kQuadBcast1>(ub),
                                     dpp_r<kQuadBcast2>(ub), dpp_r<kQuadBcast3>(ub)};
                    const R bg[Q] = {dpp_r<kQuadBcast0>(ug), dpp_r<kQuadBcast1>(ug),
                                     dpp_r<kQuadBcast2>(ug), dpp_r<kQuadBcast3>(ug)};
                    R a = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
                    for (int iy = 0; iy < D; ++iy) {
                        a += rBy[iy] * bg[iy];
                        b += rGy[iy] * bb[iy];
                        cc += rBy[iy] * bb[iy];
                    }
                    vx[iz] = a;
                    vy[iz] = b;
                    vz[iz] = cc;
                }
            } else {
                // x-stage, thread (qx, iy = qy)
                if (qy < D) {
#pragma unroll
                    for (int iz = 0; iz < D; ++iz) {
                        R ub = 0.0, ug = 0.0;
#pragma unroll
                        for (int ix = 0; ix < D; ++ix) {
                            const R u = vs[3 * sSl[le][(iz * D + qy) * D + ix] + c];
                            ub += rBx[ix] * u;
                            ug += rGx[ix] * u;
                        }
                        sX[le][0][iz][qy * Q + qx] = ub;
                        sX[le][1][iz][qy * Q + qx] = ug;
                    }
                }
                wave_sync();
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    R a = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
                    for (int iy = 0; iy < D; ++iy) {
                        const R ub = sX[le][0][iz][iy * Q + qx], ug = sX[le][1][iz][iy * Q + qx];
                        a += rBy[iy] * ug;
                        b += rGy[iy] * ub;
                        cc += rBy[iy] * ub;
                    }
                    vx[iz] = a;
                    vy[iz] = b;
                    vz[iz] = cc;
                }
                wave_sync();  // sX (and sA, sC) are rewritten by the next component
            }
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                R dx = 0.0, dy = 0.0, dz = 0.0;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const R bb = tab[T::B + qz * D + iz], gg = tab[T::G + qz * D + iz];
                    dx += bb * vx[iz];
                    dy += bb * vy[iz];
                    dz += gg * vz[iz];
                }
                sf[qz] += sv[0][qz] * dx + sv[1][qz] * dy + sv[2][qz] * dz;
            }
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int qz = 0; qz < Q; ++qz) sv[d][qz] = sn[d][qz];
        }
        // F^T v: L2 test functions, B_l^T in z (registers), y and x (LDS, or
        // across lanes at Q = 4)
        if constexpr (LANES) {
            double *__restrict__ zr = z + (long long)perm[el] * DL3;
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                R a = 0.0;
#pragma unroll
                for (int qz = 0; qz < Q; ++qz) a += tab[T::BL + qz * DL + jz] * sf[qz];
                const R u[Q] = {dpp_r<kQuadBcast0>(a), dpp_r<kQuadBcast1>(a), dpp_r<kQuadBcast2>(a),
                                dpp_r<kQuadBcast3>(a)};
                R b = 0.0;
#pragma unroll
                for (int k = 0; k < Q; ++k) b += cLy[k] * u[k];
                const R w[Q] = {b, dpp_r<kRowRor4>(b), dpp_r<kRowRor8>(b), dpp_r<kRowRor12>(b)};
                R o = 0.0;
#pragma unroll
                for (int j = 0; j < Q; ++j) o += cLx[j] * w[j];
                if (act && qx < DL && qy < DL) zr[(jz * DL + qy) * DL + qx] = (double)o;
            }
        } else {
#pragma unroll
            for (int jz = 0; jz < DL; ++jz) {
                R a = 0.0;
#pragma unroll
                for (int qz = 0; qz < Q; ++qz) a += tab[T::BL + qz * DL + jz] * sf[qz];
                sT[le][jz][t] = a;
            }
            wave_sync();
            if (qy < DL) {
#pragma unroll
                for (int jz = 0; jz < DL; ++jz) {
                    R a = 0.0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) a += tab[T::BL + k * DL + qy] * sT[le][jz][k * Q + qx];
                    sT2[le][jz][qy * Q + qx] = a;
                }
            }
            wave_sync();
            if (act && qx < DL && qy < DL) {
                double *__restrict__ zr = z + (long long)perm[el] * DL3;
#pragma unroll
                for (int jz = 0; jz < DL; ++jz) {
                    R a = 0.0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) a += tab[T::BL + k * DL + qx] * sT2[le][jz][qy * Q + k];
                    zr[(jz * DL + qy) * DL + qx] = (double)a;
                }
            }
        }
        wave_sync();  // sSl (and sT, sT2) are rewritten by the next pass
    }
    __syncthreads();
    patch_write<UMAX>(acc, pr, pn, y, part, ncomp);
}

// -------------------------------------------------------------- mass M_v x
// y_c = R^T B^T diag(m_q) B R x_c, one patch per workgroup: the patch's
// distinct-node values of the three components are read once into LDS, each
// wave works through its own elements (m_q read once for the three) and sums
// into the patch's LDS slots, then the patch is written out. With DOT, the
// workgroup also writes sum_E x_E^T (M_E x_E) (= x^T M x over its elements).
// With x2 the operand is x + beta x2, formed during the gather (a CG
// iteration's new direction r + beta p, never stored by this kernel).

template <int D, int Q, bool DOT, typename R, int NW>
__global__ void __launch_bounds__(NW * 64)
k_mass(const R *__restrict__ mq, const double *__restrict__ x,
       const int32_t *__restrict__ map, const uint16_t *__restrict__ slot,
       const int32_t *__restrict__ pn, const int32_t *__restrict__ ptab,
       double *__restrict__ y, double *__restrict__ part, long long ncomp,
       const R *__restrict__ tab, double *__restrict__ part_dot,
       const int *__restrict__ skip, const double *__restrict__ x2,
       const double *__restrict__ beta, const int *__restrict__ pmesh, int sstride)
{
    constexpr int NE = NW * wave_ne(Q), UMAX = patch_umax(D);
    constexpr int QQ = Q * Q, Q3 = Q * Q * Q, D3 = D * D * D;
    using T = Tab<D, Q>;
    const int pi = xcd_block(blockIdx.x, gridDim.x);
    // CG flags and beta: one of each, or (with pmesh) one per mesh, sstride bytes apart
    const size_t soff = pmesh ? (size_t)pmesh[pi] * sstride : 0;
    if (skip && *(const int *)((const char *)skip + soff)) return;  // a finished CG solve
    __shared__ R acc[3 * UMAX];
    __shared__ R xs[3 * UMAX];
    __shared__ int sSl[NE + 1][D3];
    __shared__ R sX[NE + 1][D][D * Q];  // x-stage out, then y^T out
    __shared__ R sZ[NE + 1][D][QQ];
    __shared__ double sred[8];
    (void)map;

    const Lane L = lane_map<Q, NE>();
    const int tid = threadIdx.x, le = L.le, t = L.t, qx = t % Q, qy = t / Q;
    const PatchRow pr = load_patch(ptab, pi);
    const double bt = x2 ? *(const double *)((const char *)beta + soff) : 0.0;
    // the three components together: one gather, one pass over the elements
    // (m_q and the slots read once), one write-out
    for (int k = tid; k < 3 * pr.U; k += blockDim.x) acc[k] = (R)0;
    patch_gather<kGatherK>(xs, pr, pn, x, x2, bt, ncomp);
    R rBx[D], rBy[D], cBy[Q], cBx[Q];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        rBx[i] = tab[T::B + qx * D + i];
        rBy[i] = tab[T::B + qy * D + i];
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        cBy[k] = qy < D ? tab[T::B + k * D + qy] : (R)0;
        cBx[k] = qx < D ? tab[T::B + k * D + qx] : (R)0;
    }
    double dot = 0.0;
    // idle lanes (spare element row NE) read slots from the spare row: keep it valid
    for (int i = tid; i < D3; i += blockDim.x) sSl[NE][i] = 0;
    __syncthreads();
    SlotPipe<D3, QQ> sp;
    if constexpr (sizeof(R) == 8) sp.fetch(slot, pr.eb + (L.valid && le < pr.cnt ? le : 0), t);
#pragma unroll 1
    for (int base = 0; base < pr.cnt; base += NE) {
        const int idx = base + le;
        const bool act = L.valid && idx < pr.cnt;
        const long long el = pr.eb + (act ? idx : 0);
        R m[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) m[k] = mq[el * Q3 + k * QQ + t];
        // the slots fetched a pass ahead; the FP32 instances keep their waves
        // per SIMD with one load at a time
        if constexpr (sizeof(R) == 8) {
            sp.store(sSl[le], t);
            sp.fetch(slot, pr.eb + (L.valid && idx + NE < pr.cnt ? idx + NE : 0), t);
        } else {
            for (int i = t; i < D3; i += QQ) sSl[le][i] = slot[el * D3 + i];
        }
        wave_sync();
        // p <= 3: the LDS slots of the nodes this thread reads in the x stage
        // (node row iy = qy) and adds to in the x^T stage (node (qx, qy, iz)),
        // read once for the three components; at p = 4 (25 slots) they are
        // read per component, which keeps more waves per SIMD
        constexpr bool HOIST = D <= 4;
        const int qyc = qy < D ? qy : D - 1, qxc = qx < D ? qx : D - 1;
        int sl[HOIST ? D : 1][D], so[HOIST ? D : 1];
        if constexpr (HOIST) {
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
#pragma unroll
                for (int ix = 0; ix < D; ++ix) sl[iz][ix] = 3 * sSl[le][(iz * D + qyc) * D + ix];
                so[iz] = 3 * sSl[le][(iz * D + qyc) * D + qxc];
            }
        }
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            // x-stage: thread (qx, iy = qy)
            if (qy < D) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    R a = 0;
#pragma unroll
                    for (int ix = 0; ix < D; ++ix)
                        a += rBx[ix] * xs[(HOIST ? sl[HOIST ? iz : 0][ix] : 3 * sSl[le][(iz * D + qy) * D + ix]) + c];
                    sX[le][iz][qy * Q + qx] = a;
                }
            }
            wave_sync();
            // y-stage, z-stage, weights, z^T in registers of thread (qx, qy)
            R w[D];
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                R a = 0;
#pragma unroll
                for (int iy = 0; iy < D; ++iy) a += rBy[iy] * sX[le][iz][iy * Q + qx];
                w[iz] = a;
            }
            R a[D];
#pragma unroll
            for (int iz = 0; iz < D; ++iz) a[iz] = 0;
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                R u = 0;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) u += tab[T::B + qz * D + iz] * w[iz];
                u *= m[qz];
#pragma unroll
                for (int iz = 0; iz < D; ++iz) a[iz] += tab[T::B + qz * D + iz] * u;
            }
#pragma unroll
            for (int iz = 0; iz < D; ++iz) sZ[le][iz][t] = a[iz];
            wave_sync();
            // y^T: thread (qx, iy = qy), into sX
            if (qy < D) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    R b = 0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) b += cBy[k] * sZ[le][iz][k * Q + qx];
                    sX[le][iz][qy * Q + qx] = b;
                }
            }
            wave_sync();
            // x^T: thread (ix = qx, iy = qy), summed into the patch slots
            if (act && qx < D && qy < D) {
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const int s = (HOIST ? so[HOIST ? iz : 0] : 3 * sSl[le][(iz * D + qy) * D + qx]) + c;
                    R r = 0;
#pragma unroll
                    for (int k = 0; k < Q; ++k) r += cBx[k] * sX[le][iz][qy * Q + k];
                    atomicAdd(&acc[s], r);
                    if (DOT) dot += (double)r * (double)xs[s];
                }
            }
            wave_sync();  // sX is rewritten by the next component
        }
    }
    __syncthreads();
    patch_write<UMAX>(acc, pr, pn, y, part, ncomp);
    if (DOT) {
        for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off);
        const int lane = tid & 63, wv = tid >> 6;
        if (lane == 0) sred[wv] = dot;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int k = 0; k < (int)((blockDim.x + 63) >> 6); ++k) s += sred[k];
            part_dot[pi] = s;  // at the patch index: partial ranges per mesh follow patches
        }
    }
}

// The mass action at Q = 4 with the y, y^T and x^T contractions across lanes
// (quad broadcasts and row rotations as in k_force_q4): LDS holds only the
// patch's node values, its accumulator and the element slots, so all three
// components fit at once and a patch needs one gather, one pass over its
// elements and one write-out.
template <int D, bool DOT, typename R, int NW>
__global__ void __launch_bounds__(NW * 64)
k_mass_q4(const R *__restrict__ mq, const double *__restrict__ x,
          const int32_t *__restrict__ map, const uint16_t *__restrict__ slot,
          const int32_t *__restrict__ pn, const int32_t *__restrict__ ptab,
          double *__restrict__ y, double *__restrict__ part, long long ncomp,
          const R *__restrict__ tab, double *__restrict__ part_dot,
          const int *__restrict__ skip, const double *__restrict__ x2,
          const double *__restrict__ beta, const int *__restrict__ pmesh, int sstride)
{
    constexpr int Q = 4, NE = NW * 4, UMAX = patch_umax(D);
    constexpr int QQ = 16, Q3 = 64, D3 = D * D * D;
    using T = Tab<D, Q>;
    const int pi = xcd_block(blockIdx.x, gridDim.x);
    const size_t soff = pmesh ? (size_t)pmesh[pi] * sstride : 0;
    if (skip && *(const int *)((const char *)skip + soff)) return;  // a finished CG solve
    __shared__ R acc[3 * UMAX];
    __shared__ R xs[3 * UMAX];
    __shared__ int sSl[NE][D3];
    __shared__ double sred[8];
    (void)map;

    const int tid = threadIdx.x, lane = tid & 63;
    const int le = (tid >> 6) * 4 + (lane >> 4);
    const int r = lane & 15, qy = r & 3, qx = r >> 2, t = qx + Q * qy;
    const PatchRow pr = load_patch(ptab, pi);
    const double bt = x2 ? *(const double *)((const char *)beta + soff) : 0.0;
    // the three components together: one gather of the patch's node values, one
    // pass over the elements (m_q and the slots read once), one write-out
    for (int k = tid; k < 3 * pr.U; k += blockDim.x) acc[k] = (R)0;
    patch_gather<kGatherK>(xs, pr, pn, x, x2, bt, ncomp);
    // x: interpolation weights of column qx; y: weights of row qy (broadcast lane k
    // brings node row k); y^T: weights of node row qy over the quad's points;
    // x^T: weights over the rotated source columns
    R rBx[D], rBy[D], cBy[Q], cBx[Q];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        rBx[i] = tab[T::B + qx * D + i];
        rBy[i] = tab[T::B + qy * D + i];
    }
    const int kx[Q] = {qx, dpp_i<kRowRor4>(qx), dpp_i<kRowRor8>(qx), dpp_i<kRowRor12>(qx)};
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        cBy[k] = qy < D ? tab[T::B + k * D + qy] : (R)0;
        cBx[k] = qx < D ? tab[T::B + kx[k] * D + qx] : (R)0;
    }
    const int qyc = qy < D ? qy : D - 1;
    double dot = 0.0;
    __syncthreads();
    SlotPipe<D3, QQ> sp;  // FP64: the slots fetched a pass ahead
    if constexpr (sizeof(R) == 8) sp.fetch(slot, pr.eb + (le < pr.cnt ? le : 0), r);
#pragma unroll 1
    for (int base = 0; base < pr.cnt; base += NE) {
        const int idx = base + le;
        const bool act = idx < pr.cnt;
        const long long el = pr.eb + (act ? idx : 0);
        R m[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k) m[k] = mq[el * Q3 + k * QQ + t];
        if constexpr (sizeof(R) == 8) {
            sp.store(sSl[le], r);
            sp.fetch(slot, pr.eb + (idx + NE < pr.cnt ? idx + NE : 0), r);
        } else {  // FP32: fetched here (a pass ahead costs a wave per SIMD at p = 3)
            sp.fetch(slot, el, r);
            sp.store(sSl[le], r);
        }
        wave_sync();
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            // x: thread (qx, iy = qy) from the node values in LDS
            R X[D];
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                R a = 0;
#pragma unroll
                for (int ix = 0; ix < D; ++ix) a += rBx[ix] * xs[3 * sSl[le][(iz * D + qyc) * D + ix] + c];
                X[iz] = a;
            }
            // y: thread (qx, qy) over the quad's node rows iy < D
            R w[D];
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                const R u[Q] = {dpp_r<kQuadBcast0>(X[iz]), dpp_r<kQuadBcast1>(X[iz]),
                                dpp_r<kQuadBcast2>(X[iz]), dpp_r<kQuadBcast3>(X[iz])};
                R a = 0;
#pragma unroll
                for (int iy = 0; iy < D; ++iy) a += rBy[iy] * u[iy];
                w[iz] = a;
            }
            // z, weights, z^T in registers
            R a[D];
#pragma unroll
            for (int iz = 0; iz < D; ++iz) a[iz] = 0;
#pragma unroll
            for (int qz = 0; qz < Q; ++qz) {
                R u = 0;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) u += tab[T::B + qz * D + iz] * w[iz];
                u *= m[qz];
#pragma unroll
                for (int iz = 0; iz < D; ++iz) a[iz] += tab[T::B + qz * D + iz] * u;
            }
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                // y^T: thread (qx, iy = qy) over the quad's points
                const R u[Q] = {dpp_r<kQuadBcast0>(a[iz]), dpp_r<kQuadBcast1>(a[iz]),
                                dpp_r<kQuadBcast2>(a[iz]), dpp_r<kQuadBcast3>(a[iz])};
                R b = 0;
#pragma unroll
                for (int k = 0; k < Q; ++k) b += cBy[k] * u[k];
                // x^T: thread (ix = qx, iy = qy) over the row's point columns
                const R v4[Q] = {b, dpp_r<kRowRor4>(b), dpp_r<kRowRor8>(b), dpp_r<kRowRor12>(b)};
                R rr = 0;
#pragma unroll
                for (int j = 0; j < Q; ++j) rr += cBx[j] * v4[j];
                if (act && qx < D && qy < D) {
                    const int s = 3 * sSl[le][(iz * D + qy) * D + qx] + c;
                    atomicAdd(&acc[s], rr);
                    if (DOT) dot += (double)rr * (double)xs[s];
                }
            }
        }
        wave_sync();  // sSl is rewritten by the next pass
    }
    __syncthreads();
    patch_write<UMAX>(acc, pr, pn, y, part, ncomp);
    if (DOT) {
        for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off);
        const int wl = tid & 63, wv = tid >> 6;
        if (wl == 0) sred[wv] = dot;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int k = 0; k < (int)((blockDim.x + 63) >> 6); ++k) sum += sred[k];
            part_dot[pi] = sum;  // at the patch index: partial ranges per mesh follow patches
        }
    }
}

// Shared nodes: y[c][g] = sum of the patch partials of g, in ascending patch order.
__global__ void k_gather_shared(const double *__restrict__ part, const int32_t *__restrict__ sh_node,
                                const int32_t *__restrict__ sh_ptr,
                                const int32_t *__restrict__ sh_idx, int n_shared,
                                double *__restrict__ y, long long ncomp,
                                const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_shared) return;
    const long long g = sh_node[s];
    double a[3];
    sum_partials(part, sh_idx, sh_ptr[s], sh_ptr[s + 1], a);
    y[g] = a[0];
    y[ncomp + g] = a[1];
    y[2 * ncomp + g] = a[2];
}

// y[c][g] = 0 for nodes that no element references
__global__ void k_zero_nodes(const int32_t *__restrict__ nodes, int n, double *__restrict__ y,
                             long long ncomp, const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const long long g = nodes[s];
    y[g] = 0.0;
    y[ncomp + g] = 0.0;
    y[2 * ncomp + g] = 0.0;
}

// out[perm[k]][:] = in[k][:] (patch order -> caller order), widened to FP64
template <typename R>
__global__ void k_unpermute_rows(const R *__restrict__ in, const int32_t *__restrict__ perm,
                                 long long rows, int len, double *__restrict__ out)
{
    const long long n = rows * len;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const long long r = i / len, j = i % len;
        out[(long long)perm[r] * len + j] = (double)in[i];
    }
}

// ----------------------------------------------------------------- qdata
// One thread per quadrature point. Gathers x and v (INIT: x0 only), forms the
// reference gradients of the 6 (or 3) fields by three staged 1-D
// contractions, then the pointwise algebra:
//   J, detJ, J^-1; rho = m_q / (w detJ); e_q = (B_l^3 e)(q); p = (gamma-1) rho e_q;
//   grad v = (grad_xi v) J^-1; eps = sym grad v; l = detJ^(1/3)/p;
//   mu = rho l (q1 c_s + q2 l max(0, -tr eps)); sigma = -p I + mu eps;
//   S = w detJ sigma J^-T.
// min_key[0] receives the smallest detJ and min_key[1] the smallest stable
// explicit step of a point, l / (c_s + mu / (rho l)): the time a signal at
// the sound speed plus the viscous speed needs to cross the point's length l.
// INIT mode writes m_q = rho0 detJ0 w instead of S (and no step).
template <int D, int Q, bool INIT, typename RS>
__global__ void __launch_bounds__(pt_ne(Q) * Q * Q * Q)
k_qdata(const double *__restrict__ x, const double *__restrict__ v,
        const double *__restrict__ e, const int32_t *__restrict__ map,
        const int32_t *__restrict__ perm, long long ncomp,
        int node_off, double *__restrict__ mq, RS *__restrict__ S, int E,
        const double *__restrict__ tab, QParams prm, long long *__restrict__ min_key,
        int *__restrict__ nonfinite)
{
    constexpr int NE = pt_ne(Q), DL = D - 1, QQ = Q * Q, Q3 = Q * Q * Q, D3 = D * D * D;
    constexpr int DL3 = DL * DL * DL;
    constexpr int NF = INIT ? 3 : 6;
    using T = Tab<D, Q>;
    __shared__ double sTab[T::SIZE];
    __shared__ double sU[NE][NF][D3];
    __shared__ double sX[NE][NF][2][D * D * Q];
    __shared__ double sY[NE][NF][3][D * QQ];
    __shared__ double sE[NE][DL3 > 0 ? DL3 : 1];
    __shared__ long long sKey[2][pt_ne(Q) * Q * Q * Q];
    __shared__ int sBad;

    const int tid = threadIdx.x, le = tid / Q3, q = tid % Q3;
    const int qx = q % Q, qy = (q / Q) % Q, qz = q / QQ;
    const long long el = (long long)xcd_block(blockIdx.x, gridDim.x) * NE + le;
    const bool act = el < E;

    for (int k = tid; k < T::SIZE; k += blockDim.x) sTab[k] = tab[k];
    if (tid == 0) sBad = 0;
    for (int k = q; k < NF * D3; k += Q3) {
        const int f = k / D3, i = k % D3;
        double val = 0.0;
        if (act) {
            const long long g = (long long)map[el * D3 + i] - node_off;
            val = f < 3 ? x[f * ncomp + g] : v[(f - 3) * ncomp + g];
        }
        sU[le][f][i] = val;
    }
    if (!INIT)
        for (int k = q; k < DL3; k += Q3) sE[le][k] = act ? e[(long long)perm[el] * DL3 + k] : 0.0;
    __syncthreads();

    // x-stage: items (f, iz, iy, qx')
    for (int k = q; k < NF * D * D * Q; k += Q3) {
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
    for (int k = q; k < NF * D * QQ; k += Q3) {
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
    // z-stage at this thread's point: grad[f][d] = d(field f)/d(xi_d)
    double grad[NF][3];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
        for (int iz = 0; iz < D; ++iz) {
            const double bz = sTab[T::B + qz * D + iz], gz = sTab[T::G + qz * D + iz];
            a += bz * sY[le][f][0][(iz * Q + qy) * Q + qx];
            b += bz * sY[le][f][1][(iz * Q + qy) * Q + qx];
            c += gz * sY[le][f][2][(iz * Q + qy) * Q + qx];
        }
        grad[f][0] = a;
        grad[f][1] = b;
        grad[f][2] = c;
    }
    const double w = sTab[T::W + qx] * sTab[T::W + qy] * sTab[T::W + qz];
    // J[c][d] = grad[c][d]
    const double J00 = grad[0][0], J01 = grad[0][1], J02 = grad[0][2];
    const double J10 = grad[1][0], J11 = grad[1][1], J12 = grad[1][2];
    const double J20 = grad[2][0], J21 = grad[2][1], J22 = grad[2][2];
    const double A00 = J11 * J22 - J12 * J21, A01 = J02 * J21 - J01 * J22, A02 = J01 * J12 - J02 * J11;
    const double A10 = J12 * J20 - J10 * J22, A11 = J00 * J22 - J02 * J20, A12 = J02 * J10 - J00 * J12;
    const double A20 = J10 * J21 - J11 * J20, A21 = J01 * J20 - J00 * J21, A22 = J00 * J11 - J01 * J10;
    const double detJ = J00 * A00 + J01 * A10 + J02 * A20;
    bool nf = !isfinite(detJ);
    long long kDt = 0x7fffffffffffffffLL;  // this point's stable-step key (none: largest)

    if (INIT) {
        if (act) mq[el * Q3 + q] = prm.rho0 * detJ * w;
    } else if (act) {
        const double id = 1.0 / detJ;
        const double Ji[3][3] = {{A00 * id, A01 * id, A02 * id},
                                 {A10 * id, A11 * id, A12 * id},
                                 {A20 * id, A21 * id, A22 * id}};
        const double m = mq[el * Q3 + q];
        const double rho = m / (w * detJ);
        double eqv = 0.0;
        for (int j = 0; j < DL3; ++j) {
            const int jx = j % DL, jy = (j / DL) % DL, jz = j / (DL * DL);
            eqv += sTab[T::BL + qx * DL + jx] * sTab[T::BL + qy * DL + jy] *
                   sTab[T::BL + qz * DL + jz] * sE[le][j];
        }
        const double pres = prm.gm1 * rho * eqv;
        const double cs = sqrt(prm.gamma * prm.gm1 * fmax(eqv, 0.0));
        double L[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                L[c][k] = grad[3 + c][0] * Ji[0][k] + grad[3 + c][1] * Ji[1][k] +
                          grad[3 + c][2] * Ji[2][k];
        double eps[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) eps[a][b] = 0.5 * (L[a][b] + L[b][a]);
        const double tr = eps[0][0] + eps[1][1] + eps[2][2];
        const double ell = cbrt(detJ) * prm.inv_order;
        const double mu = rho * ell * (prm.q1 * cs + prm.q2 * ell * fmax(-tr, 0.0));
        const double speed = cs + mu / (rho * ell);
        kDt = ordered_key(speed > 0.0 ? ell / speed : INFINITY);
        const double wd = w * detJ;
        constexpr int SQ = s_stride<RS>(Q);
        RS *__restrict__ Se = S + el * 9 * SQ;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                double sv = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double sig = mu * eps[c][k] - (c == k ? pres : 0.0);
                    sv += sig * Ji[d][k];
                }
                sv *= wd;
                if (!isfinite(sv)) nf = true;
                Se[(c * 3 + d) * SQ + q] = cvt<RS>(sv);
            }
    }
    // minima over the workgroup without a per-point atomic: every point
    // leaves its keys in LDS, the first wave (always a full one) takes the
    // minima of a strided share each, then across its lanes
    sKey[0][tid] = act ? ordered_key(detJ) : 0x7fffffffffffffffLL;
    sKey[1][tid] = kDt;
    if (act && nf) sBad = 1;
    __syncthreads();
    if (tid < 64) {
        long long a = 0x7fffffffffffffffLL, b = 0x7fffffffffffffffLL;
        for (int k = tid; k < (int)blockDim.x; k += 64) {
            a = sKey[0][k] < a ? sKey[0][k] : a;
            b = sKey[1][k] < b ? sKey[1][k] : b;
        }
        a = wave_min_key(a);
        b = wave_min_key(b);
        if (tid == 0) {
            atomicMin(min_key, a);
            if (!INIT) atomicMin(min_key + 1, b);
            if (sBad) atomicOr(nonfinite, 1);
        }
    }
}

// Quadrature data at Q = 4 in the column layout of the force kernels: one
// patch per workgroup (its node values of x and v read once into LDS), an
// element's 16 point columns on one 16-lane row (point row qy fastest), qz in
// registers. Per field (x_c, then v_c) the x stage runs on the lane's column
// from LDS and the y stage over the quad's node rows by quad broadcasts; the z
// stage and the point algebra (that of k_qdata) run per qz, and each (c, d) row
// of S is written by the row's 16 lanes as 128 contiguous bytes. Minima of
// detJ and of the stable step go over the wave, then one atomic per workgroup.
constexpr int kQdataQ4Waves = 4;  // waves per workgroup of k_qdata_q4
template <int D, typename RS, int NW>
__global__ void __launch_bounds__(NW * 64)
k_qdata_q4(const double *__restrict__ x, const double *__restrict__ v,
           const double *__restrict__ e, const int32_t *__restrict__ perm,
           const uint16_t *__restrict__ slot, const int32_t *__restrict__ pn,
           const int32_t *__restrict__ ptab, long long ncomp, const double *__restrict__ mq,
           RS *__restrict__ S, const double *__restrict__ tab, QParams prm,
           long long *__restrict__ min_key, int *__restrict__ nonfinite)
{
    constexpr int Q = 4, NE = NW * 4, UMAX = patch_umax(D);
    constexpr int DL = D - 1, QQ = 16, Q3 = 64, D3 = D * D * D, DL3 = DL * DL * DL;
    constexpr int SQ = s_stride<RS>(Q);
    using T = Tab<D, Q>;
    __shared__ double xs[3 * UMAX];
    __shared__ double vs[3 * UMAX];
    __shared__ int sSl[NE][D3];
    __shared__ long long sKey[2][NW];
    __shared__ int sBad;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int le = wv * 4 + (lane >> 4);
    const int r = lane & 15, qy = r & 3, qx = r >> 2, t = qx + Q * qy;
    const PatchRow pr = load_patch(ptab, xcd_block(blockIdx.x, gridDim.x));
    for (int u = tid; u < pr.U; u += blockDim.x) {
        const long long g = pn[pr.pno + u];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xs[3 * u + c] = x[c * ncomp + g];
            vs[3 * u + c] = v[c * ncomp + g];
        }
    }
    if (tid == 0) sBad = 0;
    double rBx[D], rGx[D], rBy[D], rGy[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        rBx[i] = tab[T::B + qx * D + i];
        rGx[i] = tab[T::G + qx * D + i];
        rBy[i] = tab[T::B + qy * D + i];
        rGy[i] = tab[T::G + qy * D + i];
    }
    const double wxy = tab[T::W + qx] * tab[T::W + qy];
    // 1/w per point as (1/(w_x w_y)) (1/w_z): rho = m_q / (w detJ) without a
    // division per point
    const double iwxy = 1.0 / wxy;
    double iwz[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) iwz[k] = 1.0 / tab[T::W + k];
    const int qyc = qy < D ? qy : D - 1;
    long long kMin = 0x7fffffffffffffffLL, kDt = 0x7fffffffffffffffLL;
    bool bad = false;
    __syncthreads();

#pragma unroll 1
    for (int base = 0; base < pr.cnt; base += NE) {
        const int idx = base + le;
        const bool act = idx < pr.cnt;
        const long long el = pr.eb + (act ? idx : 0);
        for (int i = r; i < D3; i += QQ) sSl[le][i] = slot[el * D3 + i];
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
        int sl[D][D];  // slots of the nodes (iz, qyc, ix) this lane's x stage reads
#pragma unroll
        for (int iz = 0; iz < D; ++iz)
#pragma unroll
            for (int ix = 0; ix < D; ++ix) sl[iz][ix] = sSl[le][(iz * D + qyc) * D + ix];
        // x and y stages of the six fields: yf[f][0] = B_y G_x, [1] = G_y B_x, [2] = B_y B_x
        double yf[6][3][D];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const double *__restrict__ src = f < 3 ? xs : vs;
            const int c = f % 3;
#pragma unroll
            for (int iz = 0; iz < D; ++iz) {
                double ub = 0.0, ug = 0.0;
#pragma unroll
                for (int ix = 0; ix < D; ++ix) {
                    const double u = src[3 * sl[iz][ix] + c];
                    ub += rBx[ix] * u;
                    ug += rGx[ix] * u;
                }
                const double bb[Q] = {dpp_r<kQuadBcast0>(ub), dpp_r<kQuadBcast1>(ub),
                                      dpp_r<kQuadBcast2>(ub), dpp_r<kQuadBcast3>(ub)};
                const double bg[Q] = {dpp_r<kQuadBcast0>(ug), dpp_r<kQuadBcast1>(ug),
                                      dpp_r<kQuadBcast2>(ug), dpp_r<kQuadBcast3>(ug)};
                double a = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
                for (int iy = 0; iy < D; ++iy) {
                    a += rBy[iy] * bg[iy];
                    b += rGy[iy] * bb[iy];
                    cc += rBy[iy] * bb[iy];
                }
                yf[f][0][iz] = a;
                yf[f][1][iz] = b;
                yf[f][2][iz] = cc;
            }
        }
        RS *__restrict__ Se = S + el * 9 * SQ + t;
#pragma unroll
        for (int qz = 0; qz < Q; ++qz) {
            double g[6][3];
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                double a = 0.0, b = 0.0, cc = 0.0;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    const double bz = tab[T::B + qz * D + iz], gz = tab[T::G + qz * D + iz];
                    a += bz * yf[f][0][iz];
                    b += bz * yf[f][1][iz];
                    cc += gz * yf[f][2][iz];
                }
                g[f][0] = a;
                g[f][1] = b;
                g[f][2] = cc;
            }
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
            const double rho = mqv[qz] * id * (iwxy * iwz[qz]);
            const double pres = prm.gm1 * rho * eq[qz];
            const double cs = sqrt(prm.gamma * prm.gm1 * fmax(eq[qz], 0.0));
            double L[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    L[c][k] = g[3 + c][0] * Ji[0][k] + g[3 + c][1] * Ji[1][k] + g[3 + c][2] * Ji[2][k];
            double eps[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) eps[a][b] = 0.5 * (L[a][b] + L[b][a]);
            const double tr = eps[0][0] + eps[1][1] + eps[2][2];
            const double ell = cbrt(detJ) * prm.inv_order;
            // mu = rho l visc, and the viscous speed mu / (rho l) is visc itself
            const double visc = prm.q1 * cs + prm.q2 * ell * fmax(-tr, 0.0);
            const double mu = rho * ell * visc;
            const double speed = cs + visc;
            const double wd = w * detJ;
            double ssum = detJ;  // a non-finite S entry (or detJ) makes the sum non-finite
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    double sv = 0.0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) sv += (mu * eps[c][k] - (c == k ? pres : 0.0)) * Ji[d][k];
                    sv *= wd;
                    ssum += sv;
                    if (act) __builtin_nontemporal_store(cvt<RS>(sv), Se + (c * 3 + d) * SQ + qz * QQ);
                }
            const bool nf = !isfinite(ssum);
            if (act) {
                const long long kd = ordered_key(speed > 0.0 ? ell / speed : INFINITY);
                const long long km = ordered_key(detJ);
                kDt = kd < kDt ? kd : kDt;
                kMin = km < kMin ? km : kMin;
                bad = bad || nf;
            }
        }
        wave_sync();  // sSl is rewritten by the next pass
    }
    kMin = wave_min_key(kMin);
    kDt = wave_min_key(kDt);
    const bool anyBad = __any(bad);
    if (lane == 0) {
        sKey[0][wv] = kMin;
        sKey[1][wv] = kDt;
        if (anyBad) sBad = 1;
    }
    __syncthreads();
    if (tid == 0) {
        long long a = sKey[0][0], b = sKey[1][0];
        for (int k = 1; k < NW; ++k) {
            a = sKey[0][k] < a ? sKey[0][k] : a;
            b = sKey[1][k] < b ? sKey[1][k] : b;
        }
        atomicMin(min_key, a);
        atomicMin(min_key + 1, b);
        if (sBad) atomicOr(nonfinite, 1);
    }
}

// ---------------------------------------------------------------- launchers
// R: real type of S, m_q and the contractions (double, or float in the
// FP32 precision form); the quadrature-data algebra always runs in FP64.
template <int D, int Q, typename R>
struct Launch {
    static constexpr int NEp = pt_ne(Q);

    template <int NW>
    static void force_nw(const void *S, const double *e, const PatchDev &pd, double *y,
                         long long ncomp, const void *tab, hipStream_t st)
    {
        const dim3 grid(pd.n_patch), block(NW * 64);
        if constexpr (Q == 4) {
            if (e)
                hipLaunchKernelGGL((k_force_q4<D, false, R, NW>), grid, block, 0, st, (const R *)S, e,
                                   pd.perm, pd.slot, pd.pn, pd.ptab, y, pd.part, ncomp, (const R *)tab);
            else
                hipLaunchKernelGGL((k_force_q4<D, true, R, NW>), grid, block, 0, st, (const R *)S, e,
                                   pd.perm, pd.slot, pd.pn, pd.ptab, y, pd.part, ncomp, (const R *)tab);
        } else {
            if (e)
                hipLaunchKernelGGL((k_force<D, Q, false, R, NW>), grid, block, 0, st, (const R *)S, e,
                                   pd.perm, pd.slot, pd.pn, pd.ptab, y, pd.part, ncomp, (const R *)tab);
            else
                hipLaunchKernelGGL((k_force<D, Q, true, R, NW>), grid, block, 0, st, (const R *)S, e,
                                   pd.perm, pd.slot, pd.pn, pd.ptab, y, pd.part, ncomp, (const R *)tab);
        }
    }
    static void force(const void *S, const double *e, const PatchDev &pd, double *y,
                      long long ncomp, const void *tab, int nw, hipStream_t st)
    {
        constexpr int rs = sizeof(R);
        if (nw >= 8 && force_lds(D, Q, rs, 8) <= kLdsMax) return force_nw<8>(S, e, pd, y, ncomp, tab, st);
        if (nw >= 4 && force_lds(D, Q, rs, 4) <= kLdsMax) return force_nw<4>(S, e, pd, y, ncomp, tab, st);
        return force_nw<2>(S, e, pd, y, ncomp, tab, st);
    }
    template <int NW>
    static void force_pair_nw(const void *S, const double *e, const double *v, const PatchDev &pd,
                              double *y, double *z, long long ncomp, const void *tab, hipStream_t st)
    {
        const dim3 grid(pd.n_patch), block(NW * 64);
        if (e)
            hipLaunchKernelGGL((k_force_pair<D, Q, false, R, NW>), grid, block, 0, st, (const R *)S, e, v,
                               pd.perm, pd.slot, pd.pn, pd.ptab, y, pd.part, z, ncomp, (const R *)tab);
        else
            hipLaunchKernelGGL((k_force_pair<D, Q, true, R, NW>), grid, block, 0, st, (const R *)S, e, v,
                               pd.perm, pd.slot, pd.pn, pd.ptab, y, pd.part, z, ncomp, (const R *)tab);
    }
    static void force_pair(const void *S, const double *e, const double *v, const PatchDev &pd,
                           double *y, double *z, long long ncomp, const void *tab, int nw,
                           hipStream_t st)
    {
        constexpr int rs = sizeof(R);
        if constexpr (force_pair_lds(D, Q, rs, 8) <= kLdsMax)
            if (nw >= 8) return force_pair_nw<8>(S, e, v, pd, y, z, ncomp, tab, st);
        if constexpr (force_pair_lds(D, Q, rs, 4) <= kLdsMax)
            if (nw >= 4) return force_pair_nw<4>(S, e, v, pd, y, z, ncomp, tab, st);
        static_assert(force_pair_lds(D, Q, rs, 2) <= kLdsMax, "the 2-wave pair kernel must fit LDS");
        return force_pair_nw<2>(S, e, v, pd, y, z, ncomp, tab, st);
    }
    template <int NW>
    static void force_t_nw(const void *S, const double *v, const PatchDev &pd, double *z,
                           long long ncomp, const void *tab, hipStream_t st)
    {
        hipLaunchKernelGGL((k_force_t<D, Q, R, R, NW>), dim3(pd.n_patch), dim3(NW * 64), 0, st,
                           (const R *)S, v, pd.perm, pd.slot, pd.pn, pd.ptab, z, ncomp,
                           (const R *)tab);
    }
    static void force_t(const void *S, const double *v, const PatchDev &pd, int E, double *z,
                        long long ncomp, const void *tab, int nw, hipStream_t st)
    {
        (void)E;
        constexpr int rs = sizeof(R);
        if (nw >= 8 && force_t_lds(D, Q, rs, 8) <= kLdsMax) return force_t_nw<8>(S, v, pd, z, ncomp, tab, st);
        if (nw >= 4 && force_t_lds(D, Q, rs, 4) <= kLdsMax) return force_t_nw<4>(S, v, pd, z, ncomp, tab, st);
        return force_t_nw<2>(S, v, pd, z, ncomp, tab, st);
    }
    template <int NW>
    static void mass_nw(const void *mq, const double *x, const PatchDev &pd, double *y,
                        long long ncomp, const void *tab, const MassCg &cg, hipStream_t st)
    {
        const dim3 grid(pd.n_patch), block(NW * 64);
        if constexpr (Q == 4) {
            if (cg.part_dot)
                hipLaunchKernelGGL((k_mass_q4<D, true, R, NW>), grid, block, 0, st, (const R *)mq, x,
                                   pd.map, pd.slot, pd.pn, pd.ptab, y, pd.part, ncomp, (const R *)tab,
                                   cg.part_dot, cg.skip, cg.x2, cg.beta, cg.pmesh, cg.sstride);
            else
                hipLaunchKernelGGL((k_mass_q4<D, false, R, NW>), grid, block, 0, st, (const R *)mq, x,
                                   pd.map, pd.slot, pd.pn, pd.ptab, y, pd.part, ncomp, (const R *)tab,
                                   cg.part_dot, cg.skip, cg.x2, cg.beta, cg.pmesh, cg.sstride);
        } else {
            if (cg.part_dot)
                hipLaunchKernelGGL((k_mass<D, Q, true, R, NW>), grid, block, 0, st, (const R *)mq, x,
                                   pd.map, pd.slot, pd.pn, pd.ptab, y, pd.part, ncomp, (const R *)tab,
                                   cg.part_dot, cg.skip, cg.x2, cg.beta, cg.pmesh, cg.sstride);
            else
                hipLaunchKernelGGL((k_mass<D, Q, false, R, NW>), grid, block, 0, st, (const R *)mq, x,
                                   pd.map, pd.slot, pd.pn, pd.ptab, y, pd.part, ncomp, (const R *)tab,
                                   cg.part_dot, cg.skip, cg.x2, cg.beta, cg.pmesh, cg.sstride);
        }
    }
    static void mass(const void *mq, const double *x, const PatchDev &pd, double *y,
                     long long ncomp, const void *tab, const MassCg &cg, int nw, hipStream_t st)
    {
        constexpr int rs = sizeof(R);
        if (nw >= 8 && mass_lds(D, Q, rs, 8) <= kLdsMax) return mass_nw<8>(mq, x, pd, y, ncomp, tab, cg, st);
        if (nw >= 4 && mass_lds(D, Q, rs, 4) <= kLdsMax) return mass_nw<4>(mq, x, pd, y, ncomp, tab, cg, st);
        return mass_nw<2>(mq, x, pd, y, ncomp, tab, cg, st);
    }
    // Largest waves per workgroup (8, 4, 2) of kernel kind (0 force, 1 force^T,
    // 2 mass) whose instances fit the LDS limit and keep every value in
    // registers (no private-segment spills).
    template <typename K>
    static bool no_spill(K kern)
    {
        hipFuncAttributes a{};
        return hipFuncGetAttributes(&a, (const void *)kern) == hipSuccess && a.localSizeBytes == 0;
    }
    template <int NW>
    static bool fits(int kind)
    {
        constexpr int rs = sizeof(R);
        if (kind == 0)
        {
            if constexpr (Q == 4)
                return force_lds(D, Q, rs, NW) <= kLdsMax && no_spill(k_force_q4<D, true, R, NW>) &&
                       no_spill(k_force_q4<D, false, R, NW>);
            else
                return force_lds(D, Q, rs, NW) <= kLdsMax && no_spill(k_force<D, Q, true, R, NW>) &&
                       no_spill(k_force<D, Q, false, R, NW>);
        }
        // the FP32 set's shapes also serve the BF16 form, whose F^T v and pair
        // kernels read BF16 S: their instances must not spill either
        if (kind == 1) {
            bool ok = force_t_lds(D, Q, rs, NW) <= kLdsMax && no_spill(k_force_t<D, Q, R, R, NW>);
            if constexpr (sizeof(R) == 4) ok = ok && no_spill(k_force_t<D, Q, R, __bf16, NW>);
            return ok;
        }
        if (kind == 3) {
            if constexpr (force_pair_lds(D, Q, rs, NW) <= kLdsMax) {
                bool ok = no_spill(k_force_pair<D, Q, true, R, NW>) && no_spill(k_force_pair<D, Q, false, R, NW>);
                if constexpr (sizeof(R) == 4)
                    ok = ok && no_spill(k_force_pair<D, Q, true, R, NW, __bf16>) &&
                         no_spill(k_force_pair<D, Q, false, R, NW, __bf16>);
                return ok;
            } else {
                return false;
            }
        }
        if constexpr (Q == 4)
            return mass_lds(D, Q, rs, NW) <= kLdsMax && no_spill(k_mass_q4<D, true, R, NW>) &&
                   no_spill(k_mass_q4<D, false, R, NW>);
        else
            return mass_lds(D, Q, rs, NW) <= kLdsMax && no_spill(k_mass<D, Q, true, R, NW>) &&
                   no_spill(k_mass<D, Q, false, R, NW>);
    }
    static int max_nw(int kind)
    {
        if (fits<8>(kind)) return 8;
        if (fits<4>(kind)) return 4;
        return 2;
    }
    // tab: the FP64 table (the algebra is FP64); S receives R values
    static void qdata(const double *x, const double *v, const double *e, const PatchDev &pd, int E,
                      long long ncomp, int node_off, double *mq, void *S, const double *tab,
                      QParams prm, long long *min_key, int *nonfinite, bool init, hipStream_t st)
    {
        const dim3 grid((E + NEp - 1) / NEp), block(NEp * Q * Q * Q);
        if constexpr (Q == 4) {
            if (!init) {  // column layout per patch (node_off is 0 on this path)
                hipLaunchKernelGGL((k_qdata_q4<D, R, kQdataQ4Waves>), dim3(pd.n_patch),
                                   dim3(kQdataQ4Waves * 64), 0, st, x, v, e, pd.perm, pd.slot, pd.pn,
                                   pd.ptab, ncomp, mq, (R *)S, tab, prm, min_key, nonfinite);
                return;
            }
        }
        if (init)
            hipLaunchKernelGGL((k_qdata<D, Q, true, R>), grid, block, 0, st, x, v, e, pd.map,
                               pd.perm, ncomp, node_off, mq, (R *)S, E, tab, prm, min_key,
                               nonfinite);
        else
            hipLaunchKernelGGL((k_qdata<D, Q, false, R>), grid, block, 0, st, x, v, e, pd.map,
                               pd.perm, ncomp, node_off, mq, (R *)S, E, tab, prm, min_key,
                               nonfinite);
    }
};

template <typename R>
static const KernelSet *kernels_for(int p, int Q)
{
#define FEPA_ENTRY(P, QQ)                                                                        \
    static const KernelSet ks_##P##_##QQ = {                                                     \
        Launch<P + 1, QQ, R>::force, Launch<P + 1, QQ, R>::force_t, Launch<P + 1, QQ, R>::mass, \
        Launch<P + 1, QQ, R>::qdata, patch_umax(P + 1), Launch<P + 1, QQ, R>::max_nw,           \
        Launch<P + 1, QQ, R>::force_pair};                                                       \
    if (p == P && Q == QQ) return &ks_##P##_##QQ;
    FEPA_PQ_LIST(FEPA_ENTRY)
#undef FEPA_ENTRY
    return nullptr;
}

const KernelSet *fp64_kernels(int p, int Q) { return kernels_for<double>(p, Q); }

// BF16 form: F^T v and the fused pair read BF16 S with FP32 contractions;
// qdata writes BF16 S. (The single F e runs on MFMA, kern_bf16.hip.)
template <int D, int Q>
struct LaunchBf16 {
    template <int NW>
    static void force_pair_nw(const void *S, const double *e, const double *v, const PatchDev &pd,
                              double *y, double *z, long long ncomp, const void *tab, hipStream_t st)
    {
        const dim3 grid(pd.n_patch), block(NW * 64);
        if (e)
            hipLaunchKernelGGL((k_force_pair<D, Q, false, float, NW, __bf16>), grid, block, 0, st,
                               (const __bf16 *)S, e, v, pd.perm, pd.slot, pd.pn, pd.ptab, y, pd.part, z,
                               ncomp, (const float *)tab);
        else
            hipLaunchKernelGGL((k_force_pair<D, Q, true, float, NW, __bf16>), grid, block, 0, st,
                               (const __bf16 *)S, e, v, pd.perm, pd.slot, pd.pn, pd.ptab, y, pd.part, z,
                               ncomp, (const float *)tab);
    }
    static void force_pair(const void *S, const double *e, const double *v, const PatchDev &pd,
                           double *y, double *z, long long ncomp, const void *tab, int nw,
                           hipStream_t st)
    {
        if constexpr (force_pair_lds(D, Q, 4, 8) <= kLdsMax)
            if (nw >= 8) return force_pair_nw<8>(S, e, v, pd, y, z, ncomp, tab, st);
        if constexpr (force_pair_lds(D, Q, 4, 4) <= kLdsMax)
            if (nw >= 4) return force_pair_nw<4>(S, e, v, pd, y, z, ncomp, tab, st);
        static_assert(force_pair_lds(D, Q, 4, 2) <= kLdsMax, "the 2-wave pair kernel must fit LDS");
        return force_pair_nw<2>(S, e, v, pd, y, z, ncomp, tab, st);
    }
    template <int NW>
    static void force_t_nw(const void *S, const double *v, const PatchDev &pd, double *z,
                           long long ncomp, const void *tab, hipStream_t st)
    {
        hipLaunchKernelGGL((k_force_t<D, Q, float, __bf16, NW>), dim3(pd.n_patch), dim3(NW * 64),
                           0, st, (const __bf16 *)S, v, pd.perm, pd.slot, pd.pn, pd.ptab, z, ncomp,
                           (const float *)tab);
    }
    static void force_t(const void *S, const double *v, const PatchDev &pd, int E, double *z,
                        long long ncomp, const void *tab, int nw, hipStream_t st)
    {
        (void)E;
        if (nw >= 8 && force_t_lds(D, Q, 4, 8) <= kLdsMax) return force_t_nw<8>(S, v, pd, z, ncomp, tab, st);
        if (nw >= 4 && force_t_lds(D, Q, 4, 4) <= kLdsMax) return force_t_nw<4>(S, v, pd, z, ncomp, tab, st);
        return force_t_nw<2>(S, v, pd, z, ncomp, tab, st);
    }
    static void qdata(const double *x, const double *v, const double *e, const PatchDev &pd, int E,
                      long long ncomp, int node_off, double *mq, void *S, const double *tab,
                      QParams prm, long long *min_key, int *nonfinite, bool init, hipStream_t st)
    {
        constexpr int NEp = pt_ne(Q);
        const dim3 grid((E + NEp - 1) / NEp), block(NEp * Q * Q * Q);
        (void)init;
        if constexpr (Q == 4) {
            hipLaunchKernelGGL((k_qdata_q4<D, __bf16, kQdataQ4Waves>), dim3(pd.n_patch),
                               dim3(kQdataQ4Waves * 64), 0, st, x, v, e, pd.perm, pd.slot, pd.pn,
                               pd.ptab, ncomp, mq, (__bf16 *)S, tab, prm, min_key, nonfinite);
            return;
        }
        hipLaunchKernelGGL((k_qdata<D, Q, false, __bf16>), grid, block, 0, st, x, v, e, pd.map,
                           pd.perm, ncomp, node_off, mq, (__bf16 *)S, E, tab, prm, min_key,
                           nonfinite);
    }
};

bool bf16_parts(int p, int Q, KernelSet *ks)
{
#define FEPA_ENTRY(P, QQ)                                   \
    if (p == P && Q == QQ) {                                \
        ks->force_t = LaunchBf16<P + 1, QQ>::force_t;       \
        ks->qdata = LaunchBf16<P + 1, QQ>::qdata;           \
        ks->force_pair = LaunchBf16<P + 1, QQ>::force_pair; \
        return true;                                        \
    }
    FEPA_PQ_LIST(FEPA_ENTRY)
#undef FEPA_ENTRY
    return false;
}
const KernelSet *fp32_kernels(int p, int Q) { return kernels_for<float>(p, Q); }

__global__ void k_f64_to_f32(const double *__restrict__ in, float *__restrict__ out, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (float)in[i];
}

void launch_f64_to_f32(const double *in, float *out, long long n, hipStream_t st)
{
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) return;
    hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)blocks), dim3(256), 0, st, in, out, n);
}

void launch_scatter_prepare(const PatchDev &pd, double *y, long long ncomp, const int *skip,
                            hipStream_t st)
{
    if (pd.part || pd.n_shared <= 0) return;  // partial mode: nothing to prepare
    hipLaunchKernelGGL(k_zero_nodes, dim3((pd.n_shared + 255) / 256), dim3(256), 0, st, pd.sh_node,
                       pd.n_shared, y, ncomp, skip);
}

void launch_gather_shared(const PatchDev &pd, double *y, long long ncomp, const int *skip,
                          hipStream_t st)
{
    if (!pd.part || pd.n_shared <= 0) return;  // atomic mode: the sums are in y
    hipLaunchKernelGGL(k_gather_shared, dim3((pd.n_shared + 255) / 256), dim3(256), 0, st, pd.part,
                       pd.sh_node, pd.sh_ptr, pd.sh_idx, pd.n_shared, y, ncomp, skip);
}

void launch_zero_nodes(const int32_t *nodes, int n, double *y, long long ncomp, const int *skip,
                       hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_nodes, dim3((n + 255) / 256), dim3(256), 0, st, nodes, n, y, ncomp,
                       skip);
}

void launch_unpermute_rows(const void *in, bool in_f32, const int32_t *perm, long long rows,
                           int len, double *out, hipStream_t st)
{
    long long blocks = (rows * len + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    if (blocks < 1) return;
    if (in_f32)
        hipLaunchKernelGGL(k_unpermute_rows<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const float *)in, perm, rows, len, out);
    else
        hipLaunchKernelGGL(k_unpermute_rows<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const double *)in, perm, rows, len, out);
}

__global__ void k_reset_diag(long long *__restrict__ key, int *__restrict__ flag)
{
    if (threadIdx.x == 0) {
        if (key) key[0] = key[1] = 0x7fffffffffffffffLL;
        if (flag) *flag = 0;
    }
}

void launch_reset_diag(long long *key, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_diag, dim3(1), dim3(64), 0, st, key, flag);
}

void launch_fill(double *y, long long n, double val, hipStream_t st)
{
    if (n <= 0) return;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, y, n, val);
}

}  // namespace fepa
