// Vector kernels of the mass conjugate-gradient solve (the CG inversion of the
// kinematic mass matrix, paper Sec. 3.3 and Sec. 6): masked residual set-up,
// one fused step kernel per iteration (direction, axpys and r.r) plus a
// one-workgroup kernel for beta, and
// deterministic two-level FP64 reductions (per-workgroup partials, then one
// workgroup, always summed in the same order). The iteration state
// lives on the device; every kernel leaves at once when the solve is done, so
// the host can enqueue batches of iterations and poll rarely.
#include "kern_cg.hpp"
#include "kern_common.hpp"

namespace fepa {

__device__ __forceinline__ double block_sum(double v, double *sred)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sred[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)((blockDim.x + 63) >> 6); ++k) s += sred[k];
    __syncthreads();
    return s;  // valid in thread 0
}

// This thread's share of part[0 .. n) (threads stride blockDim.x), four
// independent running sums so that four loads are in flight at once; the
// order is fixed, so the result is the same at every call.
__device__ __forceinline__ double thread_parts(const double *__restrict__ part, int n)
{
    const int st = blockDim.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int k = threadIdx.x;
    for (; k + 3 * st < n; k += 4 * st) {
        a0 += part[k];
        a1 += part[k + st];
        a2 += part[k + 2 * st];
        a3 += part[k + 3 * st];
    }
    for (; k < n; k += st) a0 += part[k];
    return (a0 + a1) + (a2 + a3);
}

__global__ void k_mask_build(unsigned char *__restrict__ fr, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        fr[i] = 1;
}

__global__ void k_mask_ess(unsigned char *__restrict__ fr, long long n,
                           const int32_t *__restrict__ ess, int n_ess, int *__restrict__ bad)
{
    const int stride = gridDim.x * blockDim.x;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_ess; k += stride) {
        const long long i = ess[k];
        if (i >= 0 && i < n)
            fr[i] = 0;
        else
            atomicOr(bad, 1);
    }
}

// x_ess = 0
__global__ void k_mask_apply(double *__restrict__ x, const unsigned char *__restrict__ fr,
                             long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (!fr[i]) x[i] = 0.0;
}

// r = (b - Ax) on free DOFs (0 elsewhere); p = r; partials of r.r and b_free.b_free
__global__ void k_cg_start(const double *__restrict__ b, const double *__restrict__ Ax,
                           double *__restrict__ r, double *__restrict__ p,
                           const unsigned char *__restrict__ fr, long long n,
                           double *__restrict__ part_rr, double *__restrict__ part_bb)
{
    __shared__ double sred[16];
    double rr = 0.0, bb = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double bi = fr[i] ? b[i] : 0.0;
        const double ri = fr[i] ? bi - Ax[i] : 0.0;
        r[i] = ri;
        p[i] = ri;
        rr += ri * ri;
        bb += bi * bi;
    }
    rr = block_sum(rr, sred);
    bb = block_sum(bb, sred);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = rr;
        part_bb[blockIdx.x] = bb;
    }
}

// one workgroup: finish the start-up sums and decide whether any iteration is needed
__global__ void k_cg_start_final(const double *__restrict__ part_rr,
                                 const double *__restrict__ part_bb, int nparts,
                                 CgState *__restrict__ st, double rel_tol, int max_iter)
{
    __shared__ double sred[16];
    double rr = 0.0, bb = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) {
        rr += part_rr[k];
        bb += part_bb[k];
    }
    rr = block_sum(rr, sred);
    bb = block_sum(bb, sred);
    if (threadIdx.x == 0) {
        st->rr = rr;
        st->bb = bb;
        st->stop = rel_tol * rel_tol * bb;
        st->iter = 0;
        st->max_iter = max_iter;
        st->done = (rr <= st->stop) ? 1 : (max_iter <= 0 ? 2 : 0);
        if (bb == 0.0) {  // b_free = 0: x = 0 is the solution (k_cg_zero_rhs sets it)
            st->rr = 0.0;
            st->done = 1;
        }
        st->alpha = st->beta = st->pAp = st->alpha_p = 0.0;
        st->pend = 0;
    }
}

// b_free = 0: the solution is x = 0 whatever the first guess (a relative
// stopping test could never be met from a non-zero guess)
__global__ void k_cg_zero_rhs(double *__restrict__ x, long long n, const CgState *__restrict__ st)
{
    if (st->bb != 0.0) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = 0.0;
}

// One step of a one-mesh solve, after Ap = M p' with p' = r + beta p (the
// mass kernel forms p' during its gather, leaves partials of p'.Ap and leaves
// the shared nodes of Ap as patch partials, no gather pass) and alpha = rr /
// (p'.Ap) from k_cg_alpha: p = p', r -= alpha Ap on free DOFs, x += alpha p
// every second step, partials of the new r.r (one per workgroup). One node
// per thread (its three components), so that the dependent loads of many
// nodes are in flight at once. Ap of a shared node is the sum of its partials
// in ascending patch order (the order of the gather it replaces).
// One workgroup: alpha = rr / (p'.Ap) from the mass kernel's partials.
__global__ void k_cg_alpha(const double *__restrict__ part_pap, int n_pap, CgState *__restrict__ st)
{
    __shared__ double sred[16];
    if (st->done) return;
    const double s = block_sum(thread_parts(part_pap, n_pap), sred);
    if (threadIdx.x == 0) st->alpha = st->rr / s;
}

__global__ void k_cg_step_sh(double *__restrict__ x, double *__restrict__ r, double *__restrict__ p,
                             const double *__restrict__ Ap, const unsigned char *__restrict__ fr,
                             long long nn, CgState *__restrict__ st, double *__restrict__ part,
                             const long long *__restrict__ node_sh,
                             const int32_t *__restrict__ sh_idx, const double *__restrict__ shpart)
{
    __shared__ double sred[16];
    if (st->done) return;
    const double alpha = st->alpha, beta = st->beta;
    // x takes the directions of two iterations at once: after an even
    // iteration alpha is left pending, after an odd one both are added
    const bool flush = (st->iter & 1) != 0;
    const double alpha_p = st->alpha_p;
    double rr = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < nn; g += stride) {
        const long long code = node_sh[g];
        double ap[3];
        if (code < 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) ap[c] = Ap[c * nn + g];
        } else {
            const long long j0 = code >> 16;
            sum_partials(shpart, sh_idx, j0, j0 + (code & 0xffff), ap);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long long i = c * nn + g;
            const double ri = r[i], po = p[i];
            const double pi = ri + beta * po;
            p[i] = pi;
            if (flush) x[i] += alpha_p * po + alpha * pi;
            const double rn = fr[i] ? ri - alpha * ap[c] : 0.0;
            r[i] = rn;
            rr += rn * rn;
        }
    }
    rr = block_sum(rr, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = rr;
    // the pending alpha is read by every workgroup of a flushing step only, and
    // written (by one) only in the steps that do not flush
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!flush) st->alpha_p = alpha;
        st->pend = flush ? 0 : 1;
    }
}

__global__ void k_cg_finish(double *__restrict__ x, const double *__restrict__ p, long long n,
                            const CgState *__restrict__ st)
{
    if (!st->pend) return;
    const double a = st->alpha_p;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] += a * p[i];
}

// One workgroup: the new r.r, beta = rr_new / rr, convergence and limit checks.
__global__ void k_cg_beta(const double *__restrict__ part, int nparts, CgState *__restrict__ st)
{
    __shared__ double sred[16];
    if (st->done) return;
    const double s = block_sum(thread_parts(part, nparts), sred);
    if (threadIdx.x == 0) {
        st->iter += 1;
        st->beta = s / st->rr;
        st->rr = s;
        if (s <= st->stop)
            st->done = 1;
        else if (st->iter >= st->max_iter)
            st->done = 2;
    }
}

// ---------------------------------------------------------------- several meshes
// One workgroup per chunk: r = b - Ax (free DOFs), p = r, partials of r.r and b.b.
__global__ void k_cgm_start(const double *__restrict__ b, const double *__restrict__ Ax,
                            double *__restrict__ r, double *__restrict__ p,
                            const unsigned char *__restrict__ fr, const CgChunk *__restrict__ chunk,
                            double *__restrict__ part_rr, double *__restrict__ part_bb,
                            CgGlobal *__restrict__ glob)
{
    __shared__ double sred[16];
    const CgChunk ck = chunk[blockIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        glob->running = 0;
        glob->done = 0;
    }
    double rr = 0.0, bb = 0.0;
    for (int k = threadIdx.x; k < ck.len; k += blockDim.x) {
        const long long i = (long long)ck.start + k;
        const double bi = fr[i] ? b[i] : 0.0;
        const double ri = fr[i] ? bi - Ax[i] : 0.0;
        r[i] = ri;
        p[i] = ri;
        rr += ri * ri;
        bb += bi * bi;
    }
    rr = block_sum(rr, sred);
    bb = block_sum(bb, sred);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = rr;
        part_bb[blockIdx.x] = bb;
    }
}

// One workgroup per mesh: its start-up sums and whether it needs any iteration.
__global__ void k_cgm_start_final(const double *__restrict__ part_rr,
                                  const double *__restrict__ part_bb, const int *__restrict__ cbeg,
                                  CgState *__restrict__ state, CgGlobal *__restrict__ glob,
                                  double rel_tol, int max_iter)
{
    __shared__ double sred[16];
    const int m = blockIdx.x;
    double rr = 0.0, bb = 0.0;
    for (int k = cbeg[m] + threadIdx.x; k < cbeg[m + 1]; k += blockDim.x) {
        rr += part_rr[k];
        bb += part_bb[k];
    }
    rr = block_sum(rr, sred);
    bb = block_sum(bb, sred);
    if (threadIdx.x == 0) {
        CgState &st = state[m];
        st.rr = rr;
        st.bb = bb;
        st.stop = rel_tol * rel_tol * bb;
        st.iter = 0;
        st.max_iter = max_iter;
        st.done = (rr <= st.stop) ? 1 : (max_iter <= 0 ? 2 : 0);
        if (bb == 0.0) {  // b_free = 0 on this mesh: x = 0 (k_cgm_zero_rhs sets it)
            st.rr = 0.0;
            st.done = 1;
        }
        st.alpha = st.beta = st.pAp = st.alpha_p = 0.0;
        st.pend = 0;
        if (!st.done) atomicAdd(&glob->running, 1);
    }
}

// one thread: done when no mesh needs an iteration
__global__ void k_cgm_glob(CgGlobal *__restrict__ glob)
{
    if (threadIdx.x == 0) glob->done = glob->running == 0;
}

// One workgroup per mesh: alpha = rr / (p'.Ap) from the mesh's mass partials.
__global__ void k_cgm_alpha(const double *__restrict__ part, const int *__restrict__ prange,
                            CgState *__restrict__ state, const CgGlobal *__restrict__ glob)
{
    __shared__ double sred[16];
    const int m = blockIdx.x;
    if (glob->done || state[m].done) return;
    double s = 0.0;
    for (int k = prange[2 * m] + threadIdx.x; k < prange[2 * m + 1]; k += blockDim.x) s += part[k];
    s = block_sum(s, sred);
    if (threadIdx.x == 0) {
        // x takes two iterations' directions every second step: keep the
        // previous alpha for an odd iteration; an even one leaves its own pending
        CgState &st = state[m];
        const bool odd = (st.iter & 1) != 0;
        if (odd) st.alpha_p = st.alpha;
        st.pend = odd ? 0 : 1;
        st.pAp = s;
        st.alpha = st.rr / s;
    }
}

// One workgroup per chunk: p = r + beta p, r -= alpha Ap with the chunk's
// mesh scalars, x += alpha_(k-1) p_(k-1) + alpha_k p_k after odd iterations k;
// partial of the new r.r.
__global__ void k_cgm_step(double *__restrict__ x, double *__restrict__ r, double *__restrict__ p,
                           const double *__restrict__ Ap, const unsigned char *__restrict__ fr,
                           const CgChunk *__restrict__ chunk, const CgState *__restrict__ state,
                           const CgGlobal *__restrict__ glob, double *__restrict__ part)
{
    __shared__ double sred[16];
    if (glob->done) return;
    const CgChunk ck = chunk[blockIdx.x];
    const CgState &st = state[ck.mesh];
    if (st.done) return;
    const double alpha = st.alpha, beta = st.beta, alpha_p = st.alpha_p;
    const bool flush = (st.iter & 1) != 0;  // odd iteration: both directions into x
    double rr = 0.0;
    for (int k = threadIdx.x; k < ck.len; k += blockDim.x) {
        const long long i = (long long)ck.start + k;
        const double ri = r[i], po = p[i];
        const double pi = ri + beta * po;
        p[i] = pi;
        if (flush) x[i] += alpha_p * po + alpha * pi;
        const double rn = fr[i] ? ri - alpha * Ap[i] : 0.0;
        r[i] = rn;
        rr += rn * rn;
    }
    rr = block_sum(rr, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = rr;
}

// After the iterations: x += alpha p in the chunks of every mesh whose last
// (even) iteration left its direction pending.
__global__ void k_cgm_finish(double *__restrict__ x, const double *__restrict__ p,
                             const CgChunk *__restrict__ chunk, const CgState *__restrict__ state)
{
    const CgChunk ck = chunk[blockIdx.x];
    const CgState &st = state[ck.mesh];
    if (!st.pend) return;
    const double a = st.alpha;
    for (int k = threadIdx.x; k < ck.len; k += blockDim.x) {
        const long long i = (long long)ck.start + k;
        x[i] += a * p[i];
    }
}

// One workgroup per mesh: new r.r, beta, iteration count, convergence; the
// workgroup that finishes the last running mesh sets the global done flag.
__global__ void k_cgm_beta(const double *__restrict__ part, const int *__restrict__ cbeg,
                           CgState *__restrict__ state, CgGlobal *__restrict__ glob)
{
    __shared__ double sred[16];
    const int m = blockIdx.x;
    if (glob->done || state[m].done) return;
    double s = 0.0;
    for (int k = cbeg[m] + threadIdx.x; k < cbeg[m + 1]; k += blockDim.x) s += part[k];
    s = block_sum(s, sred);
    if (threadIdx.x == 0) {
        CgState &st = state[m];
        st.iter += 1;
        st.beta = s / st.rr;
        st.rr = s;
        if (s <= st.stop)
            st.done = 1;
        else if (st.iter >= st.max_iter)
            st.done = 2;
        if (st.done && atomicSub(&glob->running, 1) == 1) glob->done = 1;
    }
}

// One workgroup per chunk: partial of ||b - Ax||^2 over free DOFs.
__global__ void k_cgm_resid(const double *__restrict__ b, const double *__restrict__ Ax,
                            const unsigned char *__restrict__ fr, const CgChunk *__restrict__ chunk,
                            double *__restrict__ part)
{
    __shared__ double sred[16];
    const CgChunk ck = chunk[blockIdx.x];
    double s = 0.0;
    for (int k = threadIdx.x; k < ck.len; k += blockDim.x) {
        const long long i = (long long)ck.start + k;
        if (fr[i]) {
            const double d = b[i] - Ax[i];
            s += d * d;
        }
    }
    s = block_sum(s, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_cgm_sum(const double *__restrict__ part, const int *__restrict__ cbeg,
                          double *__restrict__ out)
{
    __shared__ double sred[16];
    const int m = blockIdx.x;
    double s = 0.0;
    for (int k = cbeg[m] + threadIdx.x; k < cbeg[m + 1]; k += blockDim.x) s += part[k];
    s = block_sum(s, sred);
    if (threadIdx.x == 0) out[m] = s;
}

// partials of the free-DOF residual norm ||b - Ax||^2
__global__ void k_resid_norm(const double *__restrict__ b, const double *__restrict__ Ax,
                             const unsigned char *__restrict__ fr, long long n,
                             double *__restrict__ part)
{
    __shared__ double sred[16];
    double s = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (fr[i]) {
            const double d = b[i] - Ax[i];
            s += d * d;
        }
    s = block_sum(s, sred);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_final(const double *__restrict__ part, int nparts, double *__restrict__ out)
{
    __shared__ double sred[16];
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) s += part[k];
    s = block_sum(s, sred);
    if (threadIdx.x == 0) *out = s;
}

// out = (b - Ax) on free DOFs, 0 elsewhere
__global__ void k_sub_masked(const double *__restrict__ b, const double *__restrict__ Ax,
                             const unsigned char *__restrict__ fr, double *__restrict__ out,
                             long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = fr[i] ? b[i] - Ax[i] : 0.0;
}

// x += d
__global__ void k_add(double *__restrict__ x, const double *__restrict__ d, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] += d[i];
}

void vec_sub_masked(const double *b, const double *Ax, const unsigned char *fr, double *out,
                    long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_sub_masked, dim3(kVecBlocks), dim3(256), 0, st, b, Ax, fr, out, n);
}

void vec_add(double *x, const double *d, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_add, dim3(kVecBlocks), dim3(256), 0, st, x, d, n);
}

void cg_mask(unsigned char *fr, long long n, const int32_t *ess, int n_ess, int *bad,
             hipStream_t st)
{
    hipLaunchKernelGGL(k_mask_build, dim3(kVecBlocks), dim3(256), 0, st, fr, n);
    if (n_ess > 0 && ess)
        hipLaunchKernelGGL(k_mask_ess, dim3(256), dim3(256), 0, st, fr, n, ess, n_ess, bad);
}

void cg_mask_apply(double *x, const unsigned char *fr, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_mask_apply, dim3(kVecBlocks), dim3(256), 0, st, x, fr, n);
}

void cg_start(double *x, const double *b, const double *Ax, double *r, double *p,
              const unsigned char *fr, long long n, double *part_a, double *part_b,
              CgState *state, double rel_tol, int max_iter, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_start, dim3(kVecBlocks), dim3(256), 0, st, b, Ax, r, p, fr, n, part_a,
                       part_b);
    hipLaunchKernelGGL(k_cg_start_final, dim3(1), dim3(1024), 0, st, part_a, part_b, kVecBlocks,
                       state, rel_tol, max_iter);
    hipLaunchKernelGGL(k_cg_zero_rhs, dim3(kVecBlocks), dim3(256), 0, st, x, n, state);
}

int cg_step_blocks(long long nn)
{
    const long long b = (nn + 255) / 256;
    return (int)(b < 1 ? 1 : (b > kStepBlocks ? kStepBlocks : b));
}

void cg_step_shared(double *x, double *r, double *p, const double *Ap, const unsigned char *fr,
                    long long nn, const double *part_pap, int n_pap, CgState *state, double *part,
                    const long long *node_sh, const int32_t *sh_idx, const double *shpart,
                    hipStream_t st)
{
    const int nb = cg_step_blocks(nn);
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(1024), 0, st, part_pap, n_pap, state);
    hipLaunchKernelGGL(k_cg_step_sh, dim3(nb), dim3(256), 0, st, x, r, p, Ap, fr, nn, state, part,
                       node_sh, sh_idx, shpart);
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(1024), 0, st, part, nb, state);
}

void cg_finish(double *x, const double *p, long long n, const CgState *state, hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_finish, dim3(kVecBlocks), dim3(256), 0, st, x, p, n, state);
}

void resid_norm2(const double *b, const double *Ax, const unsigned char *fr, long long n,
                 double *part, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_resid_norm, dim3(kVecBlocks), dim3(256), 0, st, b, Ax, fr, n, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(1024), 0, st, part, kVecBlocks, out);
}

// a mesh with b_free = 0: its chunks of x are set to the solution 0
__global__ void k_cgm_zero_rhs(double *__restrict__ x, const CgChunk *__restrict__ chunk,
                               const CgState *__restrict__ state)
{
    const CgChunk ck = chunk[blockIdx.x];
    if (state[ck.mesh].bb != 0.0) return;
    for (int k = threadIdx.x; k < ck.len; k += blockDim.x) x[(long long)ck.start + k] = 0.0;
}

void cgm_start(double *x, const double *b, const double *Ax, double *r, double *p,
               const unsigned char *fr, const CgMulti &cm, double *part_a, double *part_b,
               double rel_tol, int max_iter, hipStream_t st)
{
    hipLaunchKernelGGL(k_cgm_start, dim3(cm.n_chunk), dim3(256), 0, st, b, Ax, r, p, fr, cm.chunk,
                       part_a, part_b, cm.glob);
    hipLaunchKernelGGL(k_cgm_start_final, dim3(cm.n_mesh), dim3(256), 0, st, part_a, part_b, cm.cbeg,
                       cm.state, cm.glob, rel_tol, max_iter);
    hipLaunchKernelGGL(k_cgm_glob, dim3(1), dim3(64), 0, st, cm.glob);
    hipLaunchKernelGGL(k_cgm_zero_rhs, dim3(cm.n_chunk), dim3(256), 0, st, x, cm.chunk, cm.state);
}

void cgm_finish(double *x, const double *p, const CgMulti &cm, hipStream_t st)
{
    hipLaunchKernelGGL(k_cgm_finish, dim3(cm.n_chunk), dim3(256), 0, st, x, p, cm.chunk, cm.state);
}

void cgm_iterate(double *x, double *r, double *p, const double *Ap, const unsigned char *fr,
                 const CgMulti &cm, const double *part_pap, double *part, hipStream_t st)
{
    hipLaunchKernelGGL(k_cgm_alpha, dim3(cm.n_mesh), dim3(256), 0, st, part_pap, cm.prange, cm.state,
                       cm.glob);
    hipLaunchKernelGGL(k_cgm_step, dim3(cm.n_chunk), dim3(256), 0, st, x, r, p, Ap, fr, cm.chunk,
                       cm.state, cm.glob, part);
    hipLaunchKernelGGL(k_cgm_beta, dim3(cm.n_mesh), dim3(256), 0, st, part, cm.cbeg, cm.state,
                       cm.glob);
}

void cgm_resid(const double *b, const double *Ax, const unsigned char *fr, const CgMulti &cm,
               double *part, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_cgm_resid, dim3(cm.n_chunk), dim3(256), 0, st, b, Ax, fr, cm.chunk, part);
    hipLaunchKernelGGL(k_cgm_sum, dim3(cm.n_mesh), dim3(256), 0, st, part, cm.cbeg, out);
}

}  // namespace fepa
