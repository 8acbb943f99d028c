// Host-visible launch interface of the FP64 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fepa {

// Scalars of the quadrature-data update.
struct QParams {
    double rho0;       // initial density (setup pass)
    double gamma;      // ratio of specific heats
    double gm1;        // gamma - 1
    double q1, q2;     // viscosity coefficients
    double inv_order;  // 1/p (length scale l = detJ^(1/3) / p)
};

// Device arrays of one mesh's patch plan. Element indices are local to the
// mesh and in patch order; node ids are global (offset by the mesh's first node).
struct PatchDev {
    const int32_t *perm = nullptr;   // patch-order element -> caller element of the mesh
    const int32_t *map = nullptr;    // [E][D^3] node ids, patch order
    const uint16_t *slot = nullptr;  // [E][D^3] LDS slot of each element node
    const int32_t *pn = nullptr;     // distinct nodes of every patch
    const int32_t *ptab = nullptr;   // [n_patch][6] patch table
    int n_patch = 0;
    const int32_t *sh_node = nullptr, *sh_ptr = nullptr, *sh_idx = nullptr;
    int n_shared = 0;
    double *part = nullptr;          // [entries][3] shared-node partials
    long long n_entries = 0;         // rows of part (host-side size, not a kernel argument)
};

// CG extras of a mass launch: part_dot receives per-workgroup partials of
// x . M x; with x2 the operand is x + (*beta) x2; skip points at a device flag
// that makes the launch a no-op when set. With pmesh (the mesh of every patch)
// each patch takes its mesh's flag and beta, sstride bytes apart per mesh.
// All null for a plain action.
struct MassCg {
    double *part_dot = nullptr;
    const int *skip = nullptr;
    const double *x2 = nullptr;
    const double *beta = nullptr;
    const int *pmesh = nullptr;
    int sstride = 0;
};

// Launchers of one (p, Q) instance; ncomp is the component stride of H1 vectors.
// S, m_q and tab of force/force_t/mass are of the set's real type (double for
// fp64_kernels, float for fp32_kernels); qdata always takes the FP64 table and
// writes S in the set's real type.
// nw: waves per workgroup of the patch kernels (2, 4 or 8; the largest
// instance that fits the LDS limit is used when nw is too large).
struct KernelSet {
    void (*force)(const void *S, const double *e, const PatchDev &pd, double *y,
                  long long ncomp, const void *tab, int nw, hipStream_t st);
    void (*force_t)(const void *S, const double *v, const PatchDev &pd, int E, double *z,
                    long long ncomp, const void *tab, int nw, hipStream_t st);
    void (*mass)(const void *mq, const double *x, const PatchDev &pd, double *y,
                 long long ncomp, const void *tab, const MassCg &cg, int nw, hipStream_t st);
    void (*qdata)(const double *x, const double *v, const double *e, const PatchDev &pd, int E,
                  long long ncomp, int node_off, double *mq, void *S, const double *tab,
                  QParams prm, long long *min_key, int *nonfinite, bool init, hipStream_t st);
    int umax;  // distinct-node capacity of a patch for this order
    // largest waves per workgroup of kind 0 (force), 1 (force^T), 2 (mass),
    // 3 (force pair) that fits the LDS limit without register spills
    int (*max_nw)(int kind);
    // y = F e (F 1 when e is null) and z = F^T v in one pass over S; nullptr
    // where the form has none (the BF16 form runs the two actions)
    void (*force_pair)(const void *S, const double *e, const double *v, const PatchDev &pd,
                       double *y, double *z, long long ncomp, const void *tab, int nw,
                       hipStream_t st);
};

// nullptr when (p, Q) is not instantiated.
const KernelSet *fp64_kernels(int p, int Q);
const KernelSet *fp32_kernels(int p, int Q);
// BF16 form: fills force_t (BF16 S, FP32 contractions) and qdata (writes BF16 S).
bool bf16_parts(int p, int Q, KernelSet *ks);
// BF16 form: MFMA force launcher (nullptr when (p, Q) has no MFMA instance).
using ForceFn = void (*)(const void *S, const double *e, const PatchDev &pd, double *y,
                         long long ncomp, const void *tab, int nw, hipStream_t st);
ForceFn bf16_force(int p, int Q);
// Size in bytes of the MFMA operand table of (p, Q) (0 when unsupported).
int mfma_btab_bytes(int p, int Q);
// BF16 S (rows of 9 x Q3P) -> caller-ordered FP64 [rows][9][Q^3]
void launch_unpermute_s_bf16(const void *in, const int32_t *perm, long long rows, int q3, int q3p,
                             double *out, hipStream_t st);
void launch_f64_to_f32(const double *in, float *out, long long n, hipStream_t st);

// y[c][g] for the shared nodes of a patch plan (after force or mass patches);
// nothing in the atomic scatter mode (pd.part == nullptr).
void launch_gather_shared(const PatchDev &pd, double *y, long long ncomp, const int *skip,
                          hipStream_t st);
// Before a patch kernel writes y in the atomic scatter mode: y = 0 at the
// plan's shared nodes (nothing in the partial mode).
void launch_scatter_prepare(const PatchDev &pd, double *y, long long ncomp, const int *skip,
                            hipStream_t st);
// y[c][g] = 0 for the listed nodes
void launch_zero_nodes(const int32_t *nodes, int n, double *y, long long ncomp, const int *skip,
                       hipStream_t st);
// out[perm[k]][:] = in[k][:] (in is float when in_f32, else double)
void launch_unpermute_rows(const void *in, bool in_f32, const int32_t *perm, long long rows,
                           int len, double *out, hipStream_t st);
void launch_fill(double *y, long long n, double val, hipStream_t st);
// key[0] = key[1] = INT64_MAX (empty minima of ordered detJ and time-step
// keys), *flag = 0; either pointer may be NULL.
void launch_reset_diag(long long *key, int *flag, hipStream_t st);

}  // namespace fepa
