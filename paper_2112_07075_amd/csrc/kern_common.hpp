// Shared device-side helpers of the PA kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepa {

// The (order, points per direction) pairs the library instantiates: p = 1..4
// with Q = p+1 .. p+3.
#define FEPA_PQ_LIST(X) \
    X(1, 2) X(1, 3) X(1, 4) X(2, 3) X(2, 4) X(2, 5) X(3, 4) X(3, 5) X(3, 6) X(4, 5) X(4, 6) X(4, 7)

// Layout of one (p, Q) basis table block in device memory (FP64):
//   B [Q][D]  H1 Lagrange values at the Gauss-Legendre points
//   G [Q][D]  their derivatives
//   Bl[Q][Dl] L2 Lagrange values
//   W [Q]     Gauss-Legendre weights on [0,1]
template <int D, int Q>
struct Tab {
    static constexpr int DL = D - 1;
    static constexpr int B = 0;
    static constexpr int G = Q * D;
    static constexpr int BL = 2 * Q * D;
    static constexpr int W = 2 * Q * D + Q * DL;
    static constexpr int SIZE = W + Q;
};

// Workgroups are dealt round-robin to the 8 XCDs of an MI355X. Remap the
// hardware block id so that each XCD walks one contiguous range of logical
// blocks: neighbouring elements (which share nodes) then meet in one L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    constexpr int X = 8;
    const int q = nb / X, r = nb % X;
    const int x = b % X, k = b / X;
    return x * q + (x < r ? x : r) + k;
}

// Elements per workgroup of the column-layout kernels (Q*Q threads each).
__host__ __device__ constexpr int col_ne(int Q) { return 256 / (Q * Q) > 0 ? 256 / (Q * Q) : 1; }
// Elements per workgroup of the point-layout kernels (Q^3 threads each).
__host__ __device__ constexpr int pt_ne(int Q) { return 256 / (Q * Q * Q) > 0 ? 256 / (Q * Q * Q) : 1; }

// Stored quadrature data of the BF16 form pads Q^3 to a multiple of 32 (the K
// step of one MFMA); other forms store Q^3 points.
template <typename RS>
__host__ __device__ constexpr int s_stride(int Q)
{
    return sizeof(RS) == 2 ? (Q * Q * Q + 31) / 32 * 32 : Q * Q * Q;
}

// BF16 form operand table of one (p, Q): the FP32 1-D table (Tab layout,
// padded to 16 bytes) followed by the MFMA B-operand fragments of the dense
// reference-gradient matrix G3[(d, q)][i] = d w_i / d xi_d at point q, for
// v_mfma_f32_16x16x32_bf16: fragment ((ct*3 + d)*NS + s)*64 + lane holds the 8
// values k = s*32 + (lane/16)*8 + j, column i = ct*16 + lane%16.
struct MfmaLayout {
    int q3, q3p, ns, d3, nt, tabf, nfrag, bytes;
};
__host__ __device__ constexpr MfmaLayout mfma_layout(int D, int Q)
{
    const int q3 = Q * Q * Q, q3p = (q3 + 31) / 32 * 32, d3 = D * D * D;
    const int tsize = 2 * Q * D + Q * (D - 1) + Q;
    const int tabf = (tsize + 3) / 4 * 4;
    const int nt = (d3 + 15) / 16, ns = q3p / 32;
    const int nfrag = nt * 3 * ns * 64;
    return MfmaLayout{q3, q3p, ns, d3, nt, tabf, nfrag, tabf * 4 + nfrag * 16};
}

// Order-preserving map of a double onto int64 (for atomicMin of detJ), and back.
__device__ __forceinline__ long long ordered_key(double d)
{
    long long b = __double_as_longlong(d);
    return b >= 0 ? b : (b ^ 0x7fffffffffffffffLL);
}
__device__ __forceinline__ double key_value(long long k)
{
    return __longlong_as_double(k >= 0 ? k : (k ^ 0x7fffffffffffffffLL));
}

// Smallest of a 64-bit key over the wavefront (every lane receives it).
__device__ __forceinline__ long long wave_min_key(long long k)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const long long o = __shfl_xor(k, off);
        k = o < k ? o : k;
    }
    return k;
}

// ---------------------------------------------------------------- patches
// Distinct-node slots per patch (UMAX): 768 at p = 1, 2 (a 4x4x4 block of Q2
// elements has 729 nodes), 512 at p = 3 (a 2x2x2 block of Q3 elements: 343)
// and 768 at p = 4 (a 2x2x2 block of Q4 elements: 729). Larger p = 3 tables
// (640 nodes for 2x2x4 blocks, 1024 for about 27 elements) were measured
// slower in FP64 at Q = 5: the fused pair's two node tables then leave room
// for one workgroup per CU instead of two.
__host__ __device__ constexpr int patch_umax(int D) { return D == 4 ? 512 : 768; }


// Elements whose threads sit in one wave exchange data through LDS with only a
// wave-level fence: DS instructions of a wave execute in order, so a wave never
// waits for the other waves of its workgroup inside a patch.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave-local element layout: 64/Q^2 elements per wave, 4 waves per workgroup.
__host__ __device__ constexpr int wave_ne(int Q) { return 64 / (Q * Q); }
struct Lane {
    int le;      // element slot in the workgroup (valid lanes only)
    int t;       // point column qx + Q*qy
    bool valid;  // lane carries an element column
};
// Idle lanes (64 not a multiple of Q^2) point at a spare slot NE whose LDS
// scratch nobody reads.
template <int Q, int NE>
__device__ __forceinline__ Lane lane_map()
{
    constexpr int NW = wave_ne(Q), QQ = Q * Q;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Lane L;
    L.valid = lane < NW * QQ;
    L.le = L.valid ? w * NW + lane / QQ : NE;
    L.t = L.valid ? lane % QQ : 0;
    return L;
}
__host__ __device__ constexpr int fit_waves(int Q, int per_elem, int fixed)
{
    int w = 4;
    while (w > 1 && fixed + (w * wave_ne(Q) + 1) * per_elem > 60 * 1024) --w;
    return w;
}

// Static LDS bytes of the patch kernels with NW waves per workgroup; rs =
// bytes of the real type of the stored data and the contractions. Instances
// above kLdsMax are not launched (gfx950: 160 KiB per workgroup).
constexpr int kLdsMax = 160 * 1024;
__host__ __device__ constexpr int force_lds(int D, int Q, int rs, int NW)
{
    // at Q = 4 the y and x stages run across lanes: only the accumulator
    return Q == 4 ? 3 * rs * patch_umax(D)
                  : 3 * rs * patch_umax(D) + (NW * wave_ne(Q) + 1) * rs * (3 * D * Q * Q + 2 * D * D * Q);
}
// F e and F^T v in one kernel: both accumulator/node tables, the element
// slots and (except at Q = 4, where the stages run across lanes) both stagings
__host__ __device__ constexpr int force_pair_lds(int D, int Q, int rs, int NW)
{
    return 6 * rs * patch_umax(D) + (NW * wave_ne(Q) + 1) * 4 * D * D * D +
           (Q == 4 ? 1 : NW * wave_ne(Q) + 1) *
               rs * (2 * D * D * Q + (D - 1) * Q * Q + (D - 1) * (D - 1) * Q + 3 * D * Q * Q + 2 * D * D * Q);
}
// F^T v: node table, element slots and (except at Q = 4, where the stages run
// across lanes) the stagings
__host__ __device__ constexpr int force_t_lds(int D, int Q, int rs, int NW)
{
    return 3 * rs * patch_umax(D) + (NW * wave_ne(Q) + 1) * 4 * D * D * D +
           (Q == 4 ? 1 : NW * wave_ne(Q) + 1) * rs * (2 * D * D * Q + (D - 1) * Q * Q + (D - 1) * (D - 1) * Q);
}
__host__ __device__ constexpr int mass_lds(int D, int Q, int rs, int NW)
{
    // at Q = 4 only the node values, the accumulator and the element slots
    return Q == 4 ? 6 * rs * patch_umax(D) + NW * 4 * 4 * D * D * D + 64
                  : 6 * rs * patch_umax(D) + (NW * wave_ne(Q) + 1) * (4 * D * D * D + rs * (D * D * Q + D * Q * Q)) + 64;
}

// One row of the patch table: first element, element count, offset of the
// distinct-node list, distinct nodes U, private nodes P, shared-partial offset.
struct PatchRow {
    int eb, cnt, pno, U, P, sho;
};
__device__ __forceinline__ PatchRow load_patch(const int32_t *__restrict__ ptab, int k)
{
    const int32_t *r = ptab + 6 * (long long)k;
    return PatchRow{r[0], r[1], r[2], r[3], r[4], r[5]};
}

// a[c] = sum of the partials part[3 * sh_idx[j] + c], j = j0 .. j1-1, added in
// ascending j. Four entries at a time: their index loads, then their partial
// loads, are all in flight together (a slot past j1 reads entry j0 again and
// its terms are not added), instead of one dependent pair of loads per entry.
__device__ __forceinline__ void sum_partials(const double *__restrict__ part,
                                             const int32_t *__restrict__ sh_idx, long long j0,
                                             long long j1, double a[3])
{
    a[0] = a[1] = a[2] = 0.0;
    for (long long j = j0; j < j1; j += 4) {
        int id[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) id[k] = sh_idx[j + k < j1 ? j + k : j0];
        double v[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double *src = part + 3 * (long long)id[k];
            v[k][0] = src[0];
            v[k][1] = src[1];
            v[k][2] = src[2];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (j + k < j1) {
                a[0] += v[k][0];
                a[1] += v[k][1];
                a[2] += v[k][2];
            }
    }
}

// The LDS node slots of one element, fetched one element pass ahead: lanes
// t = 0 .. NT-1 of the element share its D3 entries; fetch() issues the next
// pass's loads into registers, store() writes this pass's into the LDS row,
// so the loads' latency is covered by a pass of work.
template <int D3, int NT>
struct SlotPipe {
    static constexpr int NS = (D3 + NT - 1) / NT;
    int v[NS];
    __device__ __forceinline__ void fetch(const uint16_t *__restrict__ slot, long long el, int t)
    {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int i = t + k * NT;
            v[k] = i < D3 ? (int)slot[el * D3 + i] : 0;
        }
    }
    __device__ __forceinline__ void store(int *row, int t) const
    {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int i = t + k * NT;
            if (i < D3) row[i] = v[k];
        }
    }
};

// The patch's distinct-node values of the three components into LDS:
// dst[3u + c] = x[c][pn[u]], or x + bt * x2 there when x2 is given. Each
// thread takes up to K nodes a round: their node-number loads, then all their
// value loads, are in flight together.
template <int K, typename R>
__device__ __forceinline__ void patch_gather(R *dst, const PatchRow &pr,
                                             const int32_t *__restrict__ pn,
                                             const double *__restrict__ x,
                                             const double *__restrict__ x2, double bt,
                                             long long ncomp)
{
    const int st = blockDim.x;
    for (int u0 = threadIdx.x; u0 < pr.U; u0 += K * st) {
        long long g[K];
        bool h[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            h[k] = u0 + k * st < pr.U;
            g[k] = h[k] ? pn[pr.pno + u0 + k * st] : 0;
        }
        double a[K][3];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) a[k][c] = h[k] ? x[c * ncomp + g[k]] : 0.0;
        if (x2) {
            double b[K][3];
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) b[k][c] = h[k] ? x2[c * ncomp + g[k]] : 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) a[k][c] += bt * b[k][c];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (h[k]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) dst[3 * (u0 + k * st) + c] = (R)a[k][c];
            }
        }
    }
}

// R^T of one patch: private nodes are stored, shared nodes leave a partial
// (part != nullptr) or, in the atomic scatter mode (part == nullptr), are
// added to y with device-scope atomics (y zeroed there beforehand).
// Threads first, first + stride, ... of the caller share the work.
template <int UMAX, typename R>
__device__ __forceinline__ void patch_write(const R *acc, const PatchRow &pr,
                                            const int32_t *__restrict__ pn,
                                            double *__restrict__ y, double *__restrict__ part,
                                            long long ncomp, int first = -1, int stride = 0)
{
    if (first < 0) {
        first = threadIdx.x;
        stride = blockDim.x;
    }
    for (int u = first; u < pr.U; u += stride) {
        const double a0 = (double)acc[3 * u], a1 = (double)acc[3 * u + 1], a2 = (double)acc[3 * u + 2];
        if (u < pr.P) {
            const long long g = pn[pr.pno + u];
            y[g] = a0;
            y[ncomp + g] = a1;
            y[2 * ncomp + g] = a2;
        } else if (part) {
            double *dst = part + 3 * (long long)(pr.sho + u - pr.P);
            dst[0] = a0;
            dst[1] = a1;
            dst[2] = a2;
        } else {
            const long long g = pn[pr.pno + u];
            atomicAdd(&y[g], a0);
            atomicAdd(&y[ncomp + g], a1);
            atomicAdd(&y[2 * ncomp + g], a2);
        }
    }
}

}  // namespace fepa
