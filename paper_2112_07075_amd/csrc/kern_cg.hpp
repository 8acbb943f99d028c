// Host-visible launch interface of the CG vector kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepa {

// Device-resident state of one CG solve. done: 0 running, 1 converged,
// 2 iteration limit reached. The step adds alpha p to x every second
// iteration (two directions at once); pend = 1 while x still lacks the last
// iteration's alpha p (cg_finish / cgm_finish apply it).
struct CgState {
    double rr, alpha, beta, bb, stop, pAp, alpha_p;
    int iter, done, max_iter, pend;
};

constexpr int kVecBlocks = 1024;  // workgroups of the vector kernels (partials per pass)
constexpr int kStepBlocks = 16384;  // most workgroups (and r.r partials) of the one-mesh CG step
// workgroups of the one-mesh CG step for nn nodes (one node per thread up to kStepBlocks)
int cg_step_blocks(long long nn);

// Several meshes solved at once, each with its own CG scalars (state[m]): the
// DOF vector is cut into chunks that never straddle two meshes, and the
// mass kernel's partials of mesh m are part_dot[prange[2m] .. prange[2m+1]).
struct CgChunk {
    int start, len, mesh, pad;
};
constexpr int kChunk = 2048;  // DOFs per chunk (one workgroup of 256 threads)
// running: meshes still iterating; done: set once running reaches zero
struct CgGlobal {
    int running, done;
};
struct CgMulti {
    const CgChunk *chunk = nullptr;
    int n_chunk = 0;
    const int *cbeg = nullptr;   // [n_mesh + 1] chunk ranges per mesh
    const int *prange = nullptr; // [n_mesh][2] mass-partial ranges per mesh
    int n_mesh = 0;
    CgState *state = nullptr;    // [n_mesh]
    CgGlobal *glob = nullptr;
};
// (x: the first guess; a mesh whose b_free is 0 gets x = 0 and counts as converged)
void cgm_start(double *x, const double *b, const double *Ax, double *r, double *p,
               const unsigned char *fr, const CgMulti &cm, double *part_a, double *part_b,
               double rel_tol, int max_iter, hipStream_t st);
void cgm_iterate(double *x, double *r, double *p, const double *Ap, const unsigned char *fr,
                 const CgMulti &cm, const double *part_pap, double *part, hipStream_t st);
// After the iterations: the pending last direction of every mesh whose step
// left one (x += alpha p in that mesh's chunks).
void cgm_finish(double *x, const double *p, const CgMulti &cm, hipStream_t st);
// out[m] = ||b_m - (Ax)_m||^2 over free DOFs
void cgm_resid(const double *b, const double *Ax, const unsigned char *fr, const CgMulti &cm,
               double *part, double *out, hipStream_t st);

void cg_mask(unsigned char *fr, long long n, const int32_t *ess, int n_ess, int *bad,
             hipStream_t st);
void cg_mask_apply(double *x, const unsigned char *fr, long long n, hipStream_t st);
// r = b - Ax, p = r and the start-up sums; b_free = 0 gives x = 0, converged
void cg_start(double *x, const double *b, const double *Ax, double *r, double *p,
              const unsigned char *fr, long long n, double *part_a, double *part_b,
              CgState *state, double rel_tol, int max_iter, hipStream_t st);
// One CG step of a one-mesh solve after Ap = M p' with p' = r + beta p (the
// mass kernel forms p' during its gather, leaves partials of p'.Ap in part_pap
// and skips the shared-node gather): one workgroup sets alpha = rr / (p.Ap);
// p = p', r -= alpha Ap on free DOFs, x += alpha p every second step
// (cg_finish adds a pending last one); then one workgroup finishes r.r (part
// holds cg_step_blocks(nn) partials) and sets beta, the iteration count and
// done. Ap of a shared node is the sum of its patch partials: node_sh[g] is
// (first << 16) | count of its entries sh_idx[first .. first + count) into
// shpart, or -1 for a node of one patch; nn = nodes.
void cg_step_shared(double *x, double *r, double *p, const double *Ap, const unsigned char *fr,
                    long long nn, const double *part_pap, int n_pap, CgState *state, double *part,
                    const long long *node_sh, const int32_t *sh_idx, const double *shpart,
                    hipStream_t st);
// After the iterations of a one-mesh solve: x += alpha_p p if the last
// iteration's direction is still pending.
void cg_finish(double *x, const double *p, long long n, const CgState *state, hipStream_t st);
void vec_sub_masked(const double *b, const double *Ax, const unsigned char *fr, double *out,
                    long long n, hipStream_t st);
void vec_add(double *x, const double *d, long long n, hipStream_t st);
void resid_norm2(const double *b, const double *Ax, const unsigned char *fr, long long n,
                 double *part, double *out, hipStream_t st);

}  // namespace fepa
