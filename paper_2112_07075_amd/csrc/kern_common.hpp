// Shared device-side helpers of the PA kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepa {

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

// Order-preserving map of a double onto int64 (for atomicMin of detJ).
__device__ __forceinline__ long long ordered_key(double d)
{
    long long b = __double_as_longlong(d);
    return b >= 0 ? b : (b ^ 0x7fffffffffffffffLL);
}

}  // namespace fepa
