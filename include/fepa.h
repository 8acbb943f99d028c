/*
 * fepa.h -- C ABI of the MI355X partial-assembly (PA) operator library for
 * high-order Lagrangian hydrodynamics on curved hexahedral meshes.
 *
 * The operators are those of the semi-discrete Lagrange system of the paper
 * (Sec. 3.3, equations semiDiscreteLagStart..semiDiscreteLagEnd):
 *
 *     M_v dv/dt = -F 1,      M_E de/dt = F^T v,      dx/dt = v,
 *     rho |J| = rho0 |J0|    (pointwise mass conservation),
 *
 * evaluated by partial assembly, A = P^T G^T B^T D B G P (Sec. 3.1), with the
 * basis operator B applied by sum factorisation (Sec. 3.2, eq. local_action).
 * Here G/G^T is the element restriction (gather through the element-to-node
 * map) and its scatter-add; P is the identity on one GPU; D is the stored
 * quadrature data (S for the force operator, m_q for the mass operator).
 *
 * Discretisation (the paper names the spaces, Sec. 2.1; the concrete choices
 * below are this library's):
 *   - reference element [0,1]^3;
 *   - kinematic H1 space Q_p, p = 1..4: nodal Lagrange at the p+1 Gauss-Lobatto
 *     points per axis (D = p+1);
 *   - thermodynamic L2 space Q_{p-1}: nodal Lagrange at the p Gauss-Legendre
 *     points per axis (Dl = p);
 *   - quadrature: tensor Gauss-Legendre with Q = q1d points per axis,
 *     p+1 <= Q <= p+3.
 *   - force matrix F[(i,c), j] = int sigma : grad(w_i e_c) phi_j dx, with
 *     sigma = -p I + mu eps(v) (ideal gas p = (gamma-1) rho e; scalar artificial
 *     viscosity mu = rho l (q1 c_s + q2 l max(0, -tr eps)), l = detJ^(1/3)/p,
 *     c_s = sqrt(gamma (gamma-1) max(e,0))), so the stored quadrature data is
 *     S_q = w_q detJ_q sigma_q J_q^{-T} (3x3 per point).
 *   - mass matrix M_v = block-diag over the 3 components of the scalar
 *     (M)_{ij} = sum_q m_q w_i(q) w_j(q), m_q = rho0 detJ0_q w_q (Sec. 3.2).
 *
 * Layouts (all device arrays contiguous, FP64 unless stated):
 *   - H1 vectors (x, v, forces): SoA by component, [3][N_tot]; entry (c, g)
 *     at c*N_tot + g, where g = node_offset[m] + local node id of mesh m.
 *   - L2 vectors (e, F^T v): [E_tot][Dl^3] with the mesh blocks concatenated
 *     (element offset elem_offset[m]); local j = jx + Dl*(jy + Dl*jz).
 *   - element-to-node map (host, given at setup): int32 [E][D^3], local
 *     i = ix + D*(iy + D*iz) (x fastest), values in [0, N) of that mesh.
 *   - exported quadrature data: S [E_tot][3][3][Q^3] (row c, column d,
 *     q = qx + Q*(qy + Q*qz)), m_q [E_tot][Q^3].
 *
 * Conventions:
 *   - Ownership: the caller owns every vector argument; the context owns maps,
 *     basis tables, S, m_q and all solver workspace, allocated once in
 *     fe_pa_setup. No other call allocates device memory.
 *   - Streams: all device work of a context is enqueued on the HIP stream given
 *     at setup. Calls are asynchronous except fe_pa_setup, fe_mass_cg,
 *     fe_get_diag, fe_export_qdata and fe_timer_read, which synchronise that
 *     stream.
 *   - Aliasing: inputs and outputs must not overlap (FE_EINVAL when an exact
 *     alias is seen).
 *   - Errors: functions return FE_OK (0) or a negative FE_E* code and never
 *     throw; fe_status_str() names a code and fe_last_error() gives the
 *     context's last detailed message. A context is not thread safe; distinct
 *     contexts are independent.
 */
#ifndef FEPA_H
#define FEPA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define FE_OK            0
#define FE_EINVAL       -1  /* bad argument: NULL pointer, size, alias, range  */
#define FE_ENOMEM       -2  /* device or host allocation failed during setup   */
#define FE_EDEVICE      -3  /* a HIP runtime call failed                        */
#define FE_EUNSUPPORTED -4  /* (p, Q) or precision not provided by this build   */
#define FE_EBADMESH     -5  /* non-positive Jacobian determinant at setup       */
#define FE_ENOTCONV     -6  /* CG reached max_iter before the tolerance         */

/* ------------------------------------------------------------ precisions */
#define FE_PREC_FP64 0  /* every contraction and stored value in FP64          */
#define FE_PREC_FP32 1  /* S, m_q stored FP32; contractions FP32 (precision form) */
#define FE_PREC_BF16 2  /* contractions BF16 x BF16 -> FP32 on MFMA (precision form) */

/* ------------------------------------------------------------ option flags */
#define FE_OPT_TIMERS   0x1  /* record HIP events around the main kernels     */
#define FE_OPT_BATCHED  0x2  /* multi-mesh: one launch per (order, Q) class of
                                meshes per action, over their joined patches */
#define FE_OPT_GRAPH    0x4  /* groups of CG iterations, and the actions of
                                a context with several launch units, replayed
                                from hipGraphs captured at first use (per
                                argument set), the units as parallel
                                branches; a one-unit action (two or three
                                kernels) is launched directly, which starts
                                sooner than a graph replay                  */
#define FE_OPT_STEP     0x8  /* also set up the full Lagrange step
                                (fe_lagrange_step): every element's inverse
                                thermodynamic mass M_E^-1 and the step's
                                workspace, allocated at setup              */

#define FE_OPT_STIFF    0x10 /* also set up the stiffness (diffusion) operator
                                of the hyper-viscosity term
                                (fe_stiffness_update / fe_stiffness_mult):
                                its quadrature data, 6 Q^3 FP64 values per
                                element, allocated at setup                */
#define FE_OPT_ATOMIC   0x20 /* scatter mode of R^T (the sum over elements,
                                Sec. 3.1's assembly of the element results):
                                a node shared by several patches receives
                                its patches' sums by device-scope FP64
                                atomic adds (after the node is zeroed)
                                instead of per-patch partials that a second
                                kernel sums in a fixed order. Either way the
                                elements of one patch are summed by LDS
                                atomics whose order is not fixed, so results
                                may differ in the last bits of the working
                                precision from run to run; the atomic mode
                                adds that freedom for the shared nodes     */

/* kernels timed under FE_OPT_TIMERS */
#define FE_TIMER_QDATA   0
#define FE_TIMER_FORCE   1
#define FE_TIMER_FORCE_T 2
#define FE_TIMER_MASS    3
#define FE_TIMER_PAIR    4  /* fe_force_mult_pair                          */
#define FE_TIMER_MF      5  /* fe_force_mult_pair_mf                       */
#define FE_TIMER_COUNT   6

typedef struct fe_ctx fe_ctx_t;

/* One mesh. elem_nodes is HOST memory, read during fe_pa_setup only.
 * x0 is DEVICE memory [3][n_nodes]: initial node positions, read during
 * fe_pa_setup only (to form m_q = rho0 detJ0 w, Sec. 3.3's rho |J| =
 * rho0 |J0| at every quadrature point). */
typedef struct fe_mesh_desc {
    int32_t n_elem;            /* E >= 1                                    */
    int32_t order;             /* p, 1..4                                   */
    int32_t q1d;               /* Q, order+1 .. order+3                     */
    int32_t n_nodes;           /* N >= 1 scalar H1 nodes                    */
    const int32_t *elem_nodes; /* host [E][(p+1)^3], entries in [0, N)      */
    const double *x0;          /* device [3][N]                             */
    double rho0;               /* initial density (> 0), uniform            */
    /* NULL, or the initial density at every quadrature point: device
     * [E][Q^3] (caller element order, q = qx + Q*(qy + Q*qz), all > 0),
     * read during fe_pa_setup only; then m_q = rho0_q detJ0 w and rho0 is
     * not used. A value that is not a positive finite number fails the
     * set-up with FE_EINVAL; with fe_opts_t.materials it is FE_EUNSUPPORTED
     * (each material has its own rho0). */
    const double *rho0_q;
} fe_mesh_desc_t;

/* Several materials in one context (Sec. 2.1's multi-material equations,
 * Sec. 3.3's semi-discrete system with sum_k F_k): material k has the
 * ideal-gas ratio gamma[k] (> 1), the initial density rho0[k] (> 0) and the
 * initial volume fraction eta0_k, an L2 field with the layout of e (for
 * every material a full L2 vector of l2_size_total entries, materials
 * concatenated: device [n_mat][L2_tot], read during fe_pa_setup only; for a
 * context of several meshes each mesh's block starts at a multiple of its
 * p^3, see fe_mesh_offsets). Without a closure model (volume-fraction
 * exchange and the energy exchange c_k are not modelled) eta_k stays eta0_k
 * along the motion, and eta_k rho_k |J| = eta_k0 rho_k0 |J0| fixes the
 * material's mass per point m_qk = eta0_k rho0[k] detJ0 w. gamma and rho0
 * are host arrays of n_mat entries, read during setup. */
#define FE_MAX_MATERIALS 8
typedef struct fe_materials {
    int32_t n_mat;             /* 1 .. FE_MAX_MATERIALS                     */
    const double *gamma;       /* host [n_mat]                              */
    const double *rho0;        /* host [n_mat]                              */
    const double *eta0;        /* device [n_mat][L2_tot]                    */
} fe_materials_t;

/* Tile shapes of the patch kernels. 0 selects, in order of precedence, the
 * matching line of the tuning table named by tune_table (or, when that is
 * NULL, by the environment variable FEPA_TUNE_TABLE; text lines "order q1d
 * precision nw_force nw_force_t nw_mass patch [nw_pair]", as written by the
 * package's autotuner), the library's built-in table (measured by the same
 * autotuner on MI355X), else the default rule. The scatter mode is a flag
 * (FE_OPT_ATOMIC; the default is the patch scatter with ordered partials). */
typedef struct fe_opts {
    int32_t precision;         /* FE_PREC_*                                 */
    int32_t flags;             /* FE_OPT_* bit set                          */
    double gamma;              /* ideal-gas ratio of specific heats (> 1)   */
    double q1, q2;             /* linear / quadratic viscosity coefficients */
    int32_t tune_nw_force;     /* waves per workgroup of F e (2, 4 or 8)    */
    int32_t tune_nw_force_t;   /* waves per workgroup of F^T v              */
    int32_t tune_nw_mass;      /* waves per workgroup of M x                */
    int32_t tune_patch;        /* elements per patch, 1..4096 (0: default)  */
    /* NULL, or the path of a tuning table (format above), read during
     * fe_pa_setup only, in place of FEPA_TUNE_TABLE; a file that cannot be
     * opened fails the set-up with FE_EINVAL. */
    const char *tune_table;
    /* NULL: one material (rho0 of the meshes, gamma above). Otherwise the
     * materials of a multi-material context (FE_PREC_FP64 only, not with
     * FE_OPT_STEP): the context's m_q (mass action and CG) becomes the
     * mixture's, sum_k m_qk, and fe_qdata_update_mm / fe_force_mult_T_mm
     * apply the material operators. */
    const fe_materials_t *materials;
} fe_opts_t;

typedef struct fe_info {
    int32_t n_mesh;
    int32_t nw_force, nw_force_t, nw_mass;  /* tile shapes in use for mesh 0 */
    int32_t patch;                          /* its elements per patch (cap)  */
    int64_t n_elem_total;      /* E_tot                                     */
    int64_t n_nodes_total;     /* N_tot (scalar); H1 vectors hold 3*N_tot    */
    int64_t l2_size_total;     /* L2 vector length: sum over meshes of E*p^3,
                                  each mesh's block starting at a multiple
                                  of its p^3 (see fe_mesh_offsets)          */
    int64_t qdata_bytes;       /* device bytes of S and m_q                 */
    int64_t workspace_bytes;   /* all other context-owned device bytes      */
    int32_t precision;
    int32_t flags;
} fe_info_t;

typedef struct fe_diag {
    double min_detj;           /* min detJ seen by the last fe_qdata_update */
    int32_t nonfinite;         /* 1 if the last qdata produced a NaN/Inf    */
    int32_t cg_iters;          /* iterations of the last fe_mass_cg         */
    double cg_rel_res;         /* its final true relative residual          */
    double dt_est;             /* smallest stable point step of the last
                                  fe_qdata_update: min over the points of
                                  l / (c_s + mu / (rho l)), l = detJ^(1/3)/p
                                  (+inf where no signal moves)             */
} fe_diag_t;

/* What one fe_lagrange_step did. */
typedef struct fe_step_info {
    double dt;                 /* step taken: min(dt_max, cfl * dt_est)     */
    double dt_est;             /* smallest stable point step of the state at
                                  the start of the step                    */
    int32_t cg_iters[2];       /* mass-CG iterations of the two stages      */
    double cg_rel_res[2];      /* and their true relative residuals         */
} fe_step_info_t;

/*
 * Build a context: validate the meshes, build the 1-D basis tables, upload the
 * maps, allocate S, m_q and the solver workspace, and compute m_q from x0
 * (Sec. 3.3's rho |J| = rho0 |J0|). n_mesh > 1 selects a multi-mesh context
 * whose vectors concatenate the meshes in order (offsets via fe_mesh_offsets).
 * hip_stream: a hipStream_t (NULL = the null stream).
 * Returns FE_EINVAL (bad sizes, NULL pointers, map out of range),
 * FE_EUNSUPPORTED ((p, Q) or precision not built), FE_EBADMESH (detJ0 <= 0
 * somewhere; the context is not created), FE_ENOMEM, FE_EDEVICE.
 * On success *out owns all resources until fe_destroy.
 */
int fe_pa_setup(const fe_mesh_desc_t *meshes, int32_t n_mesh, const fe_opts_t *opts,
                void *hip_stream, fe_ctx_t **out);

/* Release a context and all device memory it owns (synchronises its stream). NULL is ignored. */
void fe_destroy(fe_ctx_t *ctx);

/* Sizes and byte counts of a context (host only, no device work). */
int fe_query(const fe_ctx_t *ctx, fe_info_t *info);

/* Per-mesh offsets: node_offset[m], elem_offset[m], l2_offset[m] (host arrays of n_mesh int64; any may be NULL). */
int fe_mesh_offsets(const fe_ctx_t *ctx, int64_t *node_offset, int64_t *elem_offset,
                    int64_t *l2_offset);

/*
 * Quadrature-data update (the qdata step of the Lagrange phase; Sec. 2.1's
 * total stress of ideal-gas pressure plus artificial viscosity, Sec. 3.3's
 * rho |J| = rho0 |J0|, Sec. 6's quadrature-point data and viscosity
 * coefficients): from the
 * current positions x, velocities v ([3][N_tot], device) and specific internal
 * energy e ([E_tot][Dl^3], device), compute J, detJ, J^{-1}, rho = m_q/(w detJ),
 * e_q, the ideal-gas pressure, the viscosity and S_q = w detJ sigma J^{-T}
 * into the context. Also records min detJ and a non-finite flag (fe_get_diag).
 * Asynchronous. FE_EINVAL on NULL pointers.
 */
int fe_qdata_update(fe_ctx_t *ctx, const double *x, const double *v, const double *e);

/*
 * Force action y = F e ([3][N_tot], device, overwritten). e is [E_tot][Dl^3]
 * on the device, or NULL for e = 1 (the right side -F 1 of the momentum
 * equation, Sec. 3.3). Uses the S of the last fe_qdata_update. Asynchronous.
 */
int fe_force_mult(fe_ctx_t *ctx, const double *e, double *y);

/*
 * Transpose force action z = F^T v ([E_tot][Dl^3], device, overwritten) from
 * v ([3][N_tot], device): the right side of the energy equation (Sec. 3.3).
 * Element-local output, no scatter. Asynchronous.
 */
int fe_force_mult_T(fe_ctx_t *ctx, const double *v, double *z);

/*
 * Both force actions from one pass over the quadrature data: y = F e (e NULL:
 * y = F 1), as fe_force_mult, and z = F^T v, as fe_force_mult_T. The two share
 * S = w detJ sigma J^-T and the Lagrange step needs both at every stage (the
 * momentum and energy equations of Sec. 3.3), so the library reads S once.
 * Same layouts and ownership as the two single calls; y, z must not overlap
 * each other or the inputs (FE_EINVAL). Under FE_PREC_BF16 the fused kernel
 * reads the BF16 S and contracts in FP32 (y may then differ from the single
 * call's MFMA result by the BF16 rounding of the basis table). Where the tile
 * table measured the two single kernels faster, they run one after the
 * other. Asynchronous.
 */
int fe_force_mult_pair(fe_ctx_t *ctx, const double *e, double *y, const double *v, double *z);

/*
 * Quadrature data of the stiffness (diffusion) operator of the hyper-viscosity
 * term (Sec. 2.1: the stiffness-matrix operator that shock capturing by
 * hyper-viscosity needs; Sec. 6: the diffusion integrator of the
 * artificial-viscosity calculations),
 *     K[i][j] = int kappa grad w_i . grad w_j dx,
 * on the current mesh: from the positions x ([3][N_tot], device) and the
 * coefficient kappa at the quadrature points (device [E_tot][Q^3] in caller
 * element order, q = qx + Q*(qy + Q*qz); NULL for kappa = 1; only for
 * contexts whose meshes share one (order, q1d), FE_EINVAL otherwise), store
 * Dk_q = w_q kappa_q detJ_q J_q^-1 J_q^-T (symmetric, 6 values per point) in
 * the context, always in FP64. Needs FE_OPT_STIFF (FE_EINVAL otherwise).
 * Asynchronous.
 */
int fe_stiffness_update(fe_ctx_t *ctx, const double *x, const double *kappa);

/*
 * Stiffness action y = K u for each of the three components of u ([3][N_tot]
 * device in and out; y overwritten), block diagonal like M_v, with the data of
 * the last fe_stiffness_update. Constants are in its null space. FP64 in
 * every precision form. Needs FE_OPT_STIFF. Asynchronous.
 */
int fe_stiffness_mult(fe_ctx_t *ctx, const double *u, double *y);

/*
 * Quadrature data of a multi-material context (Sec. 3.3: F_k connects the
 * kinematic space to material k's energy; the momentum equation takes
 * sum_k F_k 1): from x, v ([3][N_tot]) and the material energies e
 * (device [n_mat][L2_tot], each material an L2 vector like e of
 * fe_qdata_update), for every material
 *     S_k = w detJ eta_k sigma_k J^-T,  sigma_k = -p_k I + mu_k eps(v),
 *     eta_k rho_k = m_qk / (w detJ),  p_k = (gamma_k - 1) rho_k e_k,
 *     mu_k = rho_k l (q1 c_s,k + q2 l max(0, -tr eps)),
 * and the context's S = sum_k S_k, so that fe_force_mult (e = NULL) and
 * fe_force_mult_pair then give sum_k F_k 1 (and sum_k F_k^T v). fe_get_diag
 * reports min detJ and the smallest stable point step over all materials.
 * FE_EINVAL without materials. Asynchronous.
 */
int fe_qdata_update_mm(fe_ctx_t *ctx, const double *x, const double *v, const double *e);

/*
 * Energy right sides of every material, z_k = F_k^T v (the M_E,k de_k/dt
 * equations of Sec. 3.3 without the closure term c_k): v [3][N_tot], z device
 * [n_mat][L2_tot] (overwritten), from the S_k of the last
 * fe_qdata_update_mm. FE_EINVAL without materials. Asynchronous.
 */
int fe_force_mult_T_mm(fe_ctx_t *ctx, const double *v, double *z);

/*
 * Fully matrix-free force pair: y = F 1 ([3][N_tot], as fe_force_mult with
 * e = NULL) and z = F^T v ([E_tot][Dl^3], as fe_force_mult_T) of the state
 * x, v ([3][N_tot]) and e ([E_tot][Dl^3]), with the quadrature data formed at
 * each point inside the kernel and never stored: what fe_qdata_update
 * followed by fe_force_mult_pair computes, without writing and reading S
 * (the on-the-fly quadrature-data style of the paper's mesh-optimisation
 * kernels, Sec. 3.4, applied to the force operator of Sec. 3.3). Also
 * records min detJ, the smallest stable point step and the non-finite flag
 * like fe_qdata_update (fe_get_diag); the context's stored S is not
 * touched. Built for p = 1, 2 (every Q) and p = 3 at Q = 4, where every
 * value stays in registers; FE_EUNSUPPORTED for other (order, q1d) and for
 * multi-material contexts. FP64 in every precision form. Asynchronous.
 */
int fe_force_mult_pair_mf(fe_ctx_t *ctx, const double *x, const double *v, const double *e,
                          double *y, double *z);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): fe_force_mult_pair with
 * the shared-node partials of the patch kernels held in a static device
 * array of this library (32 MiB per GPU, kept until the process ends)
 * instead of the context's own buffer. Same arguments, layouts, results and
 * errors as fe_force_mult_pair; the call allocates nothing and never builds
 * or replays a graph (its kernels are launched directly on the context
 * stream). Every partial it reads is written by the same call, so nothing
 * must start at zero. FE_EINVAL (with fe_last_error naming the size) when
 * one launch unit's partials (3 doubles per shared-node entry) exceed
 * 32 MiB; FE_EDEVICE if the array's device address could not be looked up
 * at set-up. All calls on one GPU share the array: calls that overlap in
 * time on one GPU (other streams, other contexts, other host threads) race
 * and must be ordered by the caller. Asynchronous.
 */
int fe_force_mult_pair_noalloc(fe_ctx_t *ctx, const double *e, double *y, const double *v,
                               double *z);

/* Mass action y = M_v x (the kinematic mass matrix of Sec. 3.3's momentum
 * equation, applied as Sec. 3.2's element mass matrices by sum factorisation;
 * [3][N_tot] device in and out; y overwritten). Asynchronous. */
int fe_mass_mult(fe_ctx_t *ctx, const double *x, double *y);

/*
 * Solve M_v x = b (Sec. 3.3's momentum equation; Sec. 6's inversion of the
 * global CG mass matrix) by unpreconditioned conjugate gradients on the free DOFs,
 * with x = 0 on the essential DOFs ess_dofs (device int32 indices into
 * [3][N_tot], sorted or not, no duplicates; NULL/n_ess = 0 for none).
 * x (device [3][N_tot]) holds the initial guess on entry and the solution on
 * exit; b (device) is not modified. Stops when ||r|| <= rel_tol ||b_free||
 * (recursive residual), then reports the true relative residual
 * ||b_free - (M x)_free|| / ||b_free|| in *rel_res and the iteration count in
 * *iters (either pointer may be NULL). Under FE_PREC_FP32/BF16 the solve is
 * iterative refinement: FP64 outer residuals with an inner low-precision CG.
 * A context of several meshes solves every mesh's (independent) system with
 * its own CG scalars and stopping test; *iters is then the largest iteration
 * count and *rel_res the largest relative residual over the meshes.
 * A (mesh's) zero right side b_free = 0 gives its exact solution x = 0 with
 * no iteration, whatever the first guess.
 * Synchronises the stream. Returns FE_ENOTCONV when max_iter iterations did
 * not reach rel_tol (x then holds the last iterate).
 */
int fe_mass_cg(fe_ctx_t *ctx, const double *b, double *x, const int32_t *ess_dofs,
               int32_t n_ess, double rel_tol, int32_t max_iter, int32_t *iters,
               double *rel_res);

/*
 * One step of the full Lagrange phase: the semi-discrete system of Sec. 3.3,
 *     M_v dv/dt = -F 1,   M_E de/dt = F^T v,   dx/dt = v,
 * (the right sides are Sec. 6's four computations: quadrature data and
 * viscosity, force actions, CG mass inversion) advanced by a two-stage scheme
 * from the state (x, v, e) at t to t + dt, in place:
 *   dt   = min(dt_max, cfl * dt_est), dt_est the smallest stable point step of
 *          the state at t (see fe_diag_t);
 *   stage 1, forces of the state at t:
 *          v_h = v + dt/2 a,  e_h = e + dt/2 M_E^-1 F^T v,  x_h = x + dt/2 v;
 *   stage 2, forces of the midpoint state:
 *          v' = v + dt a_h,  vbar = (v + v')/2,
 *          e' = e + dt M_E^-1 F_h^T vbar,  x' = x + dt vbar,
 * with a = M_v^-1 (-F 1) solved by fe_mass_cg on the free DOFs (a = 0 on
 * ess_dofs, rel_tol cg_tol, at most cg_max_iter iterations; the previous
 * stage's acceleration is the first guess). Averaging the velocity in both
 * the energy and the position update makes the kinetic energy lost,
 * vbar^T M_v (v' - v), equal the internal energy gained, 1^T M_E (e' - e),
 * up to the CG residual. M_E = sum_q m_q phi_j phi_k does not change while
 * the mesh moves (rho |J| = rho0 |J0|); its element inverses are built at
 * setup. x, v ([3][N_tot]) and e ([E_tot][Dl^3]) are device memory, updated
 * in place; v should be 0 on ess_dofs. One dt serves every mesh of the
 * context. Needs a context set up with FE_OPT_STEP (FE_EINVAL otherwise).
 * Synchronises the stream; FE_ENOTCONV if a CG solve hit cg_max_iter,
 * FE_EINVAL if no finite positive dt results (a still, pressureless state
 * with dt_max = +inf). info may be NULL.
 */
int fe_lagrange_step(fe_ctx_t *ctx, double *x, double *v, double *e, const int32_t *ess_dofs,
                     int32_t n_ess, double cfl, double dt_max, double cg_tol, int32_t cg_max_iter,
                     fe_step_info_t *info);

/*
 * Copy the element inverses M_E^-1 of an FE_OPT_STEP context to out (device,
 * FP64): for each mesh in order, [E][Dl^3][Dl^3] in caller element order.
 * Synchronises the stream. For tests.
 */
int fe_export_l2_mass_inv(fe_ctx_t *ctx, double *out);

/* Diagnostics of the last qdata update and CG solve. Synchronises the stream. */
int fe_get_diag(fe_ctx_t *ctx, fe_diag_t *diag);

/*
 * Copy the stored quadrature data to caller device buffers S_out
 * ([E_tot][3][3][Q^3], FP64) and mq_out ([E_tot][Q^3], FP64); either may be
 * NULL. Only for single-(p,Q) contexts (all meshes share Q); FE_EINVAL
 * otherwise. FP32-stored data is widened. Synchronises the stream.
 */
int fe_export_qdata(fe_ctx_t *ctx, double *S_out, double *mq_out);

/*
 * Per-kernel timers (FE_OPT_TIMERS): total milliseconds and launch count of
 * kernel class `which` (FE_TIMER_*) since setup or the last reset, measured
 * with HIP events recorded on the context stream around each launch.
 * Synchronises the stream. FE_EINVAL when timers are off.
 */
int fe_timer_read(fe_ctx_t *ctx, int32_t which, double *total_ms, int64_t *count);
int fe_timer_reset(fe_ctx_t *ctx);

/* Static name of a status code. */
const char *fe_status_str(int status);

/* Last detailed error message of a context ("" if none); NULL ctx gives the message of the last failed setup. */
const char *fe_last_error(const fe_ctx_t *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FEPA_H */
