// Host-visible launch interface of the CG vector kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepa {

// Device-resident state of one CG solve. done: 0 running, 1 converged,
// 2 iteration limit reached.
struct CgState {
    double rr, alpha, beta, bb, stop, pAp;
    int iter, done, max_iter, pad;
};

constexpr int kVecBlocks = 1024;  // workgroups of the vector kernels (partials per pass)

void cg_mask(unsigned char *fr, long long n, const int32_t *ess, int n_ess, int *bad,
             hipStream_t st);
void cg_mask_apply(double *x, const unsigned char *fr, long long n, hipStream_t st);
void cg_start(const double *b, const double *Ax, double *r, double *p, const unsigned char *fr,
              long long n, double *part_a, double *part_b, CgState *state, double rel_tol,
              int max_iter, hipStream_t st);
// One CG step after Ap = M p' with p' = r + beta p (the mass kernel forms p'
// during its gather and leaves partials of p'.Ap in part_pap): p = p',
// alpha = rr / (p.Ap), x += alpha p, r -= alpha Ap on free DOFs; then one
// workgroup finishes r.r and sets beta, the iteration count and done.
void cg_step(double *x, double *r, double *p, const double *Ap, const unsigned char *fr,
             long long n, const double *part_pap, int n_pap, CgState *state, double *part,
             hipStream_t st);
void vec_sub_masked(const double *b, const double *Ax, const unsigned char *fr, double *out,
                    long long n, hipStream_t st);
void vec_add(double *x, const double *d, long long n, hipStream_t st);
void resid_norm2(const double *b, const double *Ax, const unsigned char *fr, long long n,
                 double *part, double *out, hipStream_t st);

}  // namespace fepa
