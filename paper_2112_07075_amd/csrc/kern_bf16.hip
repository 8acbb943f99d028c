// BF16 form of the force action F e / F 1 on matrix cores (gfx950 MFMA).
//
// Per element the action is a dense contraction over (d, q):
//   y[c][i] = sum_d sum_q S[c][d](q) e(q) G3[(d, q)][i],
// the same for every element, so a wave stacks 16 elements as the 16 rows of
// v_mfma_f32_16x16x32_bf16: A = S (BF16, rows = elements, K = (d, q)), B = the
// reference-gradient table G3 (BF16, LDS resident), FP32 accumulation. One wave
// handles one patch: its element results are summed in FP32 LDS slots and
// written like the FP64 path (private nodes stored, shared nodes as partials).
#include "kern_common.hpp"
#include "kern_fp64.hpp"

namespace fepa {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

template <int D, int Q>
__host__ __device__ constexpr int mfma_lds_bytes()
{
    return mfma_layout(D, Q).nfrag * 16 + 4 * 3 * patch_umax(D) * 4 +
           4 * 16 * (mfma_layout(D, Q).q3p + (D - 1) * (D - 1) * (D - 1)) * 4;
}

template <int D, int Q, bool ONE>
__global__ void __launch_bounds__(256)
k_force_mfma(const __bf16 *__restrict__ S, const double *__restrict__ e,
             const int32_t *__restrict__ perm, const uint16_t *__restrict__ slot,
             const int32_t *__restrict__ pn, const int32_t *__restrict__ ptab, int n_patch,
             double *__restrict__ y, double *__restrict__ part, long long ncomp,
             const float *__restrict__ tab)
{
    constexpr MfmaLayout M = mfma_layout(D, Q);
    constexpr int DL = D - 1, DL3 = DL * DL * DL, UMAX = patch_umax(D), QQ = Q * Q;
    constexpr int Q3 = M.q3, Q3P = M.q3p, NS = M.ns, NT = M.nt, D3 = M.d3;
    using T = Tab<D, Q>;
    __shared__ bf16x8 sB[M.nfrag];
    __shared__ float acc[4][3 * UMAX];
    __shared__ float sEq[4][ONE ? 1 : 16][ONE ? 1 : Q3P];  // e at the points of a tile
    __shared__ float sEv[4][ONE ? 1 : 16][DL3];            // e coefficients of a tile
    __shared__ float sBl[Q * DL];

    const bf16x8 *__restrict__ gB = (const bf16x8 *)(tab + M.tabf);
    for (int k = threadIdx.x; k < M.nfrag; k += blockDim.x) sB[k] = gB[k];
    for (int k = threadIdx.x; k < Q * DL; k += blockDim.x) sBl[k] = tab[T::BL + k];
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int pk = xcd_block(blockIdx.x, gridDim.x) * 4 + w;
    if (pk >= n_patch) return;  // no workgroup barrier below this point
    const PatchRow pr = load_patch(ptab, pk);
    float *A = acc[w];
    for (int k = l; k < 3 * pr.U; k += 64) A[k] = 0.f;
    wave_sync();
    const int row = l & 15, chunk = l >> 4;

#pragma unroll 1
    for (int tile = 0; tile * 16 < pr.cnt; ++tile) {
        const int er = tile * 16 + row;
        const bool act = er < pr.cnt;
        const long long el = pr.eb + (act ? er : 0);
        // energy at the points of the tile's 16 elements, (B_l x B_l x B_l) e, into LDS
        if (!ONE) {
            for (int k = l; k < 16 * DL3; k += 64) {
                const int r2 = k / DL3, j = k % DL3;
                const int e2 = tile * 16 + r2;
                sEv[w][r2][j] = e2 < pr.cnt ? (float)e[(long long)perm[pr.eb + e2] * DL3 + j] : 0.f;
            }
            wave_sync();
            for (int k = l; k < 16 * Q3P; k += 64) {
                const int r2 = k / Q3P, q = k % Q3P;
                float v = 0.f;
                if (q < Q3) {
                    const int qx = q % Q, qy = (q / Q) % Q, qz = q / QQ;
                    for (int j = 0; j < DL3; ++j) {
                        const int jx = j % DL, jy = (j / DL) % DL, jz = j / (DL * DL);
                        v += sBl[qx * DL + jx] * sBl[qy * DL + jy] * sBl[qz * DL + jz] * sEv[w][r2][j];
                    }
                }
                sEq[w][r2][q] = v;
            }
            wave_sync();
        }
#pragma unroll 1
        for (int c = 0; c < 3; ++c) {
            f32x4 yt[NT];
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) yt[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    bf16x8 a;
                    if (act) {
                        a = __builtin_nontemporal_load(
                            (const bf16x8 *)(S + (el * 9 + c * 3 + d) * Q3P + s * 32 + chunk * 8));
                    } else {
#pragma unroll
                        for (int j = 0; j < 8; ++j) a[j] = (__bf16)0.f;
                    }
                    if (!ONE) {
                        const float *eqp = &sEq[w][row][s * 32 + chunk * 8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) a[j] = (__bf16)((float)a[j] * eqp[j]);
                    }
#pragma unroll
                    for (int ct = 0; ct < NT; ++ct)
                        yt[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            a, sB[((ct * 3 + d) * NS + s) * 64 + l], yt[ct], 0, 0, 0);
                }
            // yt[ct][i] = y of element tile*16 + chunk*4 + i at node ct*16 + row
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                const int node = ct * 16 + row;
                if (node < D3) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int er2 = tile * 16 + chunk * 4 + i;
                        if (er2 < pr.cnt) {
                            const int sidx = slot[(long long)(pr.eb + er2) * D3 + node];
                            atomicAdd(&A[3 * sidx + c], yt[ct][i]);
                        }
                    }
                }
            }
        }
    }
    wave_sync();
    patch_write<UMAX>(A, pr, pn, y, part, ncomp, l, 64);
}

template <int D, int Q>
struct LaunchMfma {
    static void force(const void *S, const double *e, const PatchDev &pd, double *y,
                      long long ncomp, const void *tab, int nw, hipStream_t st)
    {
        (void)nw;  // one wave per patch, four per workgroup
        const dim3 grid((pd.n_patch + 3) / 4), block(256);
        if (e)
            hipLaunchKernelGGL((k_force_mfma<D, Q, false>), grid, block, 0, st, (const __bf16 *)S,
                               e, pd.perm, pd.slot, pd.pn, pd.ptab, pd.n_patch, y, pd.part, ncomp,
                               (const float *)tab);
        else
            hipLaunchKernelGGL((k_force_mfma<D, Q, true>), grid, block, 0, st, (const __bf16 *)S,
                               e, pd.perm, pd.slot, pd.pn, pd.ptab, pd.n_patch, y, pd.part, ncomp,
                               (const float *)tab);
    }
};

// (p, Q) pairs whose operand table and patch slots fit one workgroup's LDS
#define FEPA_MFMA_LIST(X) \
    X(1, 2) X(1, 3) X(1, 4) X(2, 3) X(2, 4) X(2, 5) X(3, 4) X(3, 5)

ForceFn bf16_force(int p, int Q)
{
#define FEPA_ENTRY(P, QQ)                                                     \
    static_assert(mfma_lds_bytes<P + 1, QQ>() <= 160 * 1024, "LDS budget");   \
    if (p == P && Q == QQ) return LaunchMfma<P + 1, QQ>::force;
    FEPA_MFMA_LIST(FEPA_ENTRY)
#undef FEPA_ENTRY
    return nullptr;
}

int mfma_btab_bytes(int p, int Q) { return bf16_force(p, Q) ? mfma_layout(p + 1, Q).bytes : 0; }

}  // namespace fepa

namespace fepa {

// out[perm[r]][cd][q] = in[r][cd][q] for q < Q^3 (BF16 S, padded rows of Q3P), widened to FP64
__global__ void k_unpermute_s_bf16(const __bf16 *__restrict__ in, const int32_t *__restrict__ perm,
                                   long long rows, int q3, int q3p, double *__restrict__ out)
{
    const long long n = rows * 9 * q3;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const long long r = i / (9 * q3);
        const int rem = (int)(i % (9 * q3)), cd = rem / q3, q = rem % q3;
        out[((long long)perm[r] * 9 + cd) * q3 + q] = (double)(float)in[(r * 9 + cd) * q3p + q];
    }
}

void launch_unpermute_s_bf16(const void *in, const int32_t *perm, long long rows, int q3, int q3p,
                             double *out, hipStream_t st)
{
    long long blocks = (rows * 9 * q3 + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    if (blocks < 1) return;
    hipLaunchKernelGGL(k_unpermute_s_bf16, dim3((unsigned)blocks), dim3(256), 0, st,
                       (const __bf16 *)in, perm, rows, q3, q3p, out);
}

}  // namespace fepa
