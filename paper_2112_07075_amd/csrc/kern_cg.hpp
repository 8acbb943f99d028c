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
void cg_alpha(const double *part, int nparts, CgState *state, hipStream_t st);
void cg_update(double *x, double *r, const double *p, const double *Ap, const unsigned char *fr,
               long long n, const CgState *state, double *part, hipStream_t st);
void cg_beta(const double *part, CgState *state, hipStream_t st);
void cg_direction(double *p, const double *r, long long n, const CgState *state, hipStream_t st);
void vec_sub_masked(const double *b, const double *Ax, const unsigned char *fr, double *out,
                    long long n, hipStream_t st);
void vec_add(double *x, const double *d, long long n, hipStream_t st);
void resid_norm2(const double *b, const double *Ax, const unsigned char *fr, long long n,
                 double *part, double *out, hipStream_t st);

}  // namespace fepa
