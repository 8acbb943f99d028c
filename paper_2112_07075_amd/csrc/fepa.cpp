// Host side of the C ABI declared in include/fepa.h: context set-up and
// validation, device memory ownership (everything allocated once at set-up),
// dispatch of the (p, Q) kernel instances per mesh, the CG driver and the
// per-kernel event timers.
#include "fepa.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "basis.hpp"
#include "kern_cg.hpp"
#include "kern_common.hpp"
#include "kern_fp64.hpp"
#include "kern_step.hpp"
#include "kern_stiff.hpp"
#include "kern_mm.hpp"
#include "kern_mf.hpp"
#include "noalloc.hpp"
#include "patch.hpp"

using namespace fepa;

namespace {

thread_local std::string g_setup_error;

struct MeshRec {
    int E = 0, p = 0, Q = 0, N = 0;
    long long node_off = 0, elem_off = 0, l2_off = 0, S_off = 0, mq_off = 0;
    long long part_off = 0;  // into the CG dot-partial array (one per patch)
    long long minv_off = 0;  // FE_OPT_STEP: first entry of the mesh's M_E^-1 blocks
    long long Dk_off = 0;    // FE_OPT_STIFF: first entry of the mesh's stiffness data
    StiffSet sk{};           // stiffness kernels of (p, Q)
    MfFn mf = nullptr;       // matrix-free force pair of (p, Q), if built
    int tab_slot = 0;        // into the table buffer (doubles)
    const KernelSet *ks = nullptr;   // FP64 kernels
    KernelSet kl{};                  // kernels of the context's precision
    long long Sb_off = 0;            // offset of the mesh's S in the stored type
    int nw_force = 4, nw_force_t = 4, nw_mass = 4;  // waves per workgroup
    int nw_pair = 4;                                 // of the fused F e + F^T v kernel
    int nw_stiff = 4;                                // of the stiffness action
    int nw_mf = 4;                                   // of the matrix-free force pair
    bool pair_split = false;                         // the pair runs as the two actions
    int patch = 0;                                   // elements per patch (0: default)
    long long tabb_off = 0;          // BF16 form: byte offset of its operand buffer
    double rho0 = 1.0;
    PatchDev pd;             // device patch plan
    const int32_t *orphans = nullptr;
    int n_orphans = 0;
    // batched form: the class (launch unit) holding the mesh and the mesh's
    // first element in it; the mesh's pd then only views the class's perm/map
    int unit = -1;
    long long el_in_unit = 0;
    int patch_in_unit = 0, n_patch_mesh = 0;  // the mesh's rows of its unit's patch table
};

struct TimerPool {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    double folded_ms = 0.0;
    long long count = 0;
};

constexpr size_t kTimerPairs = 4096;

// A captured graph and what it was captured for: the action and the caller's
// pointers (a graph bakes its kernel arguments in).
struct GraphKey {
    int action = 0;
    const void *a = nullptr, *b = nullptr, *c = nullptr;
    int extra = 0;
    const void *d = nullptr, *f = nullptr;
    bool operator==(const GraphKey &o) const
    {
        return action == o.action && a == o.a && b == o.b && c == o.c && extra == o.extra && d == o.d &&
               f == o.f;
    }
};
struct GraphRec {
    GraphKey key;
    hipGraphExec_t exec = nullptr;
};
constexpr int kAuxStreams = 3;     // side streams of the unit branches in a graph
constexpr size_t kMaxGraphs = 32;  // cached graphs per context (oldest dropped)
constexpr int kGraphCgIters = 8;   // CG iterations per captured graph
enum { kActQdata = 1, kActForce, kActForceT, kActMass, kActCg, kActPair, kActStiffQ, kActStiff, kActQdataMm, kActForceTMm, kActPairMf };

}  // namespace

struct fe_ctx {
    std::vector<MeshRec> mesh;
    // batched form: one launch unit per (order, Q) class, covering all of the
    // class's meshes; otherwise every mesh is its own unit
    bool batched = false;
    bool atomic = false;  // FE_OPT_ATOMIC: shared nodes summed by device atomics
    std::vector<MeshRec> unit;
    const std::vector<MeshRec> &units() const { return batched ? unit : mesh; }
    fe_opts_t opts{};
    hipStream_t st = nullptr;
    int device = 0;
    long long E_tot = 0, N_tot = 0, L2_tot = 0, S_len = 0, mq_len = 0;
    long long Sb_len = 0;  // S entries in the stored layout
    bool uniform_pq = true;
    // device memory owned by the context
    bool lo = false;                  // FP32 storage and contractions (precision form)
    bool bf = false;                  // BF16 S, MFMA force contractions (precision form)
    void *S = nullptr;                // [E][9][Q^3] double / float, or [E][9][Q3P] BF16
    unsigned char *tabsb = nullptr;   // BF16 form operand buffers
    double *mq = nullptr, *tabs = nullptr;
    float *mq32 = nullptr, *tabs32 = nullptr;
    double *ref_r = nullptr, *ref_d = nullptr;  // refinement vectors
    std::vector<void *> plan_bufs;  // patch plan and CG chunk arrays
    long long *min_key = nullptr;
    int *nonfinite = nullptr;
    double *r = nullptr, *p = nullptr, *Ap = nullptr;
    double *part = nullptr, *part2 = nullptr, *scal = nullptr;
    unsigned char *fr = nullptr;
    CgState *cg = nullptr;
    int *bad = nullptr;
    long long n_parts = 0;
    // one mesh: the shared-node row of every node (-1: private or unreferenced),
    // so the CG step reads shared Ap from the patch partials (no gather pass)
    long long *node_sh = nullptr;  // one-mesh CG: (first << 16) | count of a node's partials, or -1
    // several meshes: one CG per mesh (chunked vectors, per-mesh scalars)
    bool multi = false;
    CgMulti cm;
    CgChunk *chunk = nullptr;
    int *cbeg = nullptr, *prange = nullptr, *pmesh = nullptr;
    CgState *cgm = nullptr;
    CgGlobal *glob = nullptr;
    double *part3 = nullptr, *mres = nullptr;
    // FE_OPT_STEP: element inverses of the L2 mass, the saved state of the
    // step (xs, vs, es), the stage acceleration (solution of M_v acc = F 1,
    // kept as the next solve's first guess), F 1, F^T w, the averaged
    // velocity and the device step size (dtv[0] = dt, dtv[1] = estimate)
    double *minv = nullptr, *xs = nullptr, *vs = nullptr, *es = nullptr, *acc = nullptr;
    double *sy = nullptr, *sz = nullptr, *vbar = nullptr, *dtv = nullptr, *h_dt = nullptr;
    long long minv_len = 0;
    // several materials (fe_opts_t.materials): per-material mass per point
    // [K][mq_len] and quadrature data [K][S_len] (patch order, FP64)
    int n_mat = 0;
    std::vector<double> mat_gamma;
    double *mqk = nullptr, *Sk = nullptr;
    // FE_OPT_STIFF: stiffness quadrature data w kappa detJ J^-1 J^-T, [E][6][Q^3]
    double *Dk = nullptr;
    long long Dk_len = 0;
    CgState *h_cgm = nullptr;
    CgGlobal *h_glob = nullptr;
    double *h_mres = nullptr;
    // pinned host staging
    CgState *h_cg = nullptr;
    double *h_scal = nullptr;
    long long *h_key = nullptr;
    int *h_flag = nullptr;
    // bookkeeping
    long long qdata_bytes = 0, work_bytes = 0;
    int last_iters = 0;
    double last_res = 0.0;
    // iterations of the last CG solve with the FP64 [0] and the FP32 [1]
    // operator: where the next solve's first poll of the device state goes
    int cg_hint[2] = {0, 0};
    std::string err;
    TimerPool timers[FE_TIMER_COUNT];
    // FE_OPT_GRAPH: captured action graphs, the private capture stream and the
    // side streams / events of the parallel unit branches
    std::vector<GraphRec> graphs;
    hipStream_t gst = nullptr;
    hipStream_t aux[kAuxStreams] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kAuxStreams] = {};
};

namespace {

int fail(fe_ctx *c, int code, const char *fmt, const char *detail = nullptr)
{
    char buf[512];
    std::snprintf(buf, sizeof(buf), fmt, detail ? detail : "");
    if (c)
        c->err = buf;
    else
        g_setup_error = buf;
    return code;
}

#define HIP_OK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) return fail(ctx, FE_EDEVICE, "%s", hipGetErrorString(e_)); \
    } while (0)

template <class T>
int dev_alloc(fe_ctx *ctx, T **ptr, long long count, long long *acc)
{
    const size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    if (hipMalloc((void **)ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
        return fail(ctx, FE_ENOMEM, "device allocation failed%s");
    }
    if (acc) *acc += (long long)bytes;
    return FE_OK;
}

void free_all(fe_ctx *c)
{
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    void *dptrs[] = {c->S, c->mq, c->tabs, c->mq32, c->tabs32, c->tabsb, c->ref_r, c->ref_d, c->min_key,
                     c->nonfinite, c->r, c->p, c->Ap, c->part, c->part2, c->scal, c->fr, c->cg,
                     c->bad, c->cgm, c->glob, c->part3, c->mres, c->minv, c->xs, c->vs, c->es,
                     c->acc, c->sy, c->sz, c->vbar, c->dtv, c->Dk, c->mqk, c->Sk};
    for (void *d : dptrs)
        if (d) (void)hipFree(d);
    for (void *d : c->plan_bufs)
        if (d) (void)hipFree(d);
    void *hptrs[] = {c->h_cg, c->h_scal, c->h_key, c->h_flag, c->h_cgm, c->h_glob, c->h_mres,
                     c->h_dt};
    for (void *h : hptrs)
        if (h) (void)hipHostFree(h);
    for (auto &tp : c->timers)
        for (auto &pr : tp.ev) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (GraphRec &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    for (hipStream_t s : c->aux)
        if (s) (void)hipStreamDestroy(s);
    if (c->gst) (void)hipStreamDestroy(c->gst);
    for (hipEvent_t e : c->ev_join)
        if (e) (void)hipEventDestroy(e);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
}

double key_to_double(long long k)
{
    long long b = k >= 0 ? k : (k ^ 0x7fffffffffffffffLL);
    double d;
    std::memcpy(&d, &b, sizeof(d));
    return d;
}

// ---- timers
struct ScopedTimer {
    fe_ctx *c;
    TimerPool *tp = nullptr;
    ScopedTimer(fe_ctx *ctx, int which) : c(ctx)
    {
        if (!(c->opts.flags & FE_OPT_TIMERS)) return;
        tp = &c->timers[which];
        if (tp->used == tp->ev.size()) {
            // pool exhausted: fold what was recorded so far
            (void)hipStreamSynchronize(c->st);
            for (auto &pr : tp->ev) {
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, pr.first, pr.second);
                tp->folded_ms += ms;
            }
            tp->used = 0;
        }
        (void)hipEventRecord(tp->ev[tp->used].first, c->st);
    }
    ~ScopedTimer()
    {
        if (!tp) return;
        (void)hipEventRecord(tp->ev[tp->used].second, c->st);
        tp->used++;
        tp->count++;
    }
};

bool supported_pq(int p, int Q) { return fp64_kernels(p, Q) != nullptr; }

struct TuneEntry {
    int p, Q, prec, nwf, nwt, nwm, patch, nwp;  // nwp: fused pair (0: as F e)
};

// Tile shapes measured by the autotuner (paper_2112_07075_amd/autotune.py,
// --builtin) on MI355X, one row per (p, Q, precision); ends with a zero row.
const TuneEntry kBuiltinTune[] = {
#include "tune_table.inc"
    {0, 0, 0, 0, 0, 0, 0, 0}};

// the built-in table followed by the one named by opt_path, else by
// FEPA_TUNE_TABLE (a missing file: none from the environment, *opened = false
// from opt_path); later rows take precedence
std::vector<TuneEntry> read_tune_table(const char *opt_path, bool *opened)
{
    std::vector<TuneEntry> t;
    for (const TuneEntry &e : kBuiltinTune)
        if (e.p) t.push_back(e);
    *opened = true;
    const char *path = opt_path ? opt_path : std::getenv("FEPA_TUNE_TABLE");
    if (!path || !*path) return t;
    FILE *f = std::fopen(path, "r");
    if (!f) {
        *opened = opt_path == nullptr;  // a missing file named by the environment is ignored
        return t;
    }
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        TuneEntry e{};
        if (line[0] == '#') continue;
        if (std::sscanf(line, "%d %d %d %d %d %d %d %d", &e.p, &e.Q, &e.prec, &e.nwf, &e.nwt, &e.nwm,
                        &e.patch, &e.nwp) >= 7)
            t.push_back(e);
    }
    std::fclose(f);
    return t;
}

// Waves per workgroup when no table row applies: the largest of `pref` or
// fewer whose LDS leaves room for two workgroups per CU (the force kernels run
// best at 4 waves, the mass kernel at 8, at the 48^3 Q2 workload).
int default_nw(int pref, int lds8, int lds4)
{
    if (pref >= 8 && lds8 <= 80 * 1024) return 8;
    if (pref >= 4 && lds4 <= 80 * 1024) return 4;
    return 2;
}

}  // namespace

// typed views of the context's stored data for one mesh
static void *S_of(fe_ctx *c, const MeshRec &r)
{
    if (c->bf) return (void *)((uint16_t *)c->S + r.Sb_off);
    return c->lo ? (void *)((float *)c->S + r.Sb_off) : (void *)((double *)c->S + r.Sb_off);
}
static const void *tab_of(fe_ctx *c, const MeshRec &r)
{
    if (c->bf) return (const void *)(c->tabsb + r.tabb_off);
    return c->lo ? (const void *)(c->tabs32 + r.tab_slot) : (const void *)(c->tabs + r.tab_slot);
}

// Enqueues per_unit(r, stream) for every launch unit after the work already on
// s. With branch set (graph capture) the units become independent branches,
// spread over the side streams and joined back on s: units own disjoint nodes
// and elements, so their outputs never overlap.
template <typename F>
static void enqueue_units(fe_ctx *ctx, hipStream_t s, bool branch, F &&per_unit)
{
    const std::vector<MeshRec> &U = ctx->units();
    if (!branch || U.size() < 2) {
        for (const MeshRec &r : U) per_unit(r, s);
        return;
    }
    const int naux = std::min<int>(kAuxStreams, (int)U.size() - 1);
    (void)hipEventRecord(ctx->ev_fork, s);
    for (int i = 0; i < naux; ++i) (void)hipStreamWaitEvent(ctx->aux[i], ctx->ev_fork, 0);
    for (size_t k = 0; k < U.size(); ++k) per_unit(U[k], k == 0 ? s : ctx->aux[(k - 1) % naux]);
    for (int i = 0; i < naux; ++i) {
        (void)hipEventRecord(ctx->ev_join[i], ctx->aux[i]);
        (void)hipStreamWaitEvent(s, ctx->ev_join[i], 0);
    }
}

// Runs enqueue(stream, branch) on the caller's stream; with FE_OPT_GRAPH it
// replays the graph captured from enqueue for the same key instead (captured
// on the context's private stream at first use, then launched on the caller's).
template <typename F>
static int run_graph(fe_ctx *ctx, const GraphKey &key, F &&enqueue)
{
    // A graph pays for itself where it replaces many launches: several launch
    // units as parallel branches, or the CG's groups of iterations. The two or
    // three kernels of a one-unit action start sooner as plain launches (C2:
    // F 1 118 vs 124 us, M x 55 vs 62 us per action).
    const bool worth = key.action == kActCg || ctx->units().size() > 1;
    if (!(ctx->opts.flags & FE_OPT_GRAPH) || !worth) {
        enqueue(ctx->st, false);
        HIP_OK(hipGetLastError());
        return FE_OK;
    }
    for (const GraphRec &g : ctx->graphs)
        if (g.key == key) {
            HIP_OK(hipGraphLaunch(g.exec, ctx->st));
            return FE_OK;
        }
    HIP_OK(hipStreamBeginCapture(ctx->gst, hipStreamCaptureModeThreadLocal));
    enqueue(ctx->gst, true);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->gst, &graph);
    if (ec != hipSuccess || !graph) {
        (void)hipGetLastError();
        return fail(ctx, FE_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, FE_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    if (ctx->graphs.size() >= kMaxGraphs) {
        HIP_OK(hipStreamSynchronize(ctx->st));  // the oldest graph may still run
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(GraphRec{key, exec});
    HIP_OK(hipGraphLaunch(exec, ctx->st));
    return FE_OK;
}

// ======================================================================= ABI
extern "C" {

const char *fe_status_str(int s)
{
    switch (s) {
    case FE_OK: return "ok";
    case FE_EINVAL: return "invalid argument";
    case FE_ENOMEM: return "out of memory";
    case FE_EDEVICE: return "HIP runtime error";
    case FE_EUNSUPPORTED: return "unsupported order/quadrature/precision";
    case FE_EBADMESH: return "non-positive Jacobian determinant";
    case FE_ENOTCONV: return "CG did not converge";
    default: return "unknown status";
    }
}

const char *fe_last_error(const fe_ctx_t *ctx)
{
    return ctx ? ctx->err.c_str() : g_setup_error.c_str();
}

int fe_pa_setup(const fe_mesh_desc_t *meshes, int32_t n_mesh, const fe_opts_t *opts,
                void *hip_stream, fe_ctx_t **out)
{
    fe_ctx *ctx = nullptr;
    g_setup_error.clear();
    if (!out) return fail(nullptr, FE_EINVAL, "out is NULL%s");
    *out = nullptr;
    if (!meshes || n_mesh < 1) return fail(nullptr, FE_EINVAL, "need at least one mesh%s");
    fe_opts_t o{};
    if (opts) {
        o = *opts;
    } else {
        o.precision = FE_PREC_FP64;
        o.gamma = 5.0 / 3.0;
        o.q1 = 0.5;
        o.q2 = 2.0;
    }
    if (!(o.gamma > 1.0) || !(o.q1 >= 0.0) || !(o.q2 >= 0.0))
        return fail(nullptr, FE_EINVAL, "gamma must be > 1 and q1, q2 >= 0%s");
    if (o.precision != FE_PREC_FP64 && o.precision != FE_PREC_FP32 && o.precision != FE_PREC_BF16)
        return fail(nullptr, FE_EUNSUPPORTED, "precision not provided by this build%s");
    if (o.flags & ~(FE_OPT_TIMERS | FE_OPT_BATCHED | FE_OPT_GRAPH | FE_OPT_STEP | FE_OPT_STIFF | FE_OPT_ATOMIC))
        return fail(nullptr, FE_EINVAL, "unknown option flags%s");
    if (o.materials) {
        const fe_materials_t &mt = *o.materials;
        if (mt.n_mat < 1 || mt.n_mat > FE_MAX_MATERIALS || !mt.gamma || !mt.rho0 || !mt.eta0)
            return fail(nullptr, FE_EINVAL, "materials: n_mat in [1, 8] and non-NULL arrays%s");
        for (int k = 0; k < mt.n_mat; ++k)
            if (!(mt.gamma[k] > 1.0) || !(mt.rho0[k] > 0.0))
                return fail(nullptr, FE_EINVAL, "materials: gamma must be > 1 and rho0 > 0%s");
        if (o.precision != FE_PREC_FP64)
            return fail(nullptr, FE_EUNSUPPORTED, "materials need FE_PREC_FP64%s");
        if (o.flags & FE_OPT_STEP)
            return fail(nullptr, FE_EUNSUPPORTED, "the Lagrange step is single-material%s");
    }
    for (int v : {o.tune_nw_force, o.tune_nw_force_t, o.tune_nw_mass})
        if (v != 0 && v != 2 && v != 4 && v != 8)
            return fail(nullptr, FE_EINVAL, "waves per workgroup must be 2, 4 or 8%s");
    if (o.tune_patch < 0 || o.tune_patch > 4096)
        return fail(nullptr, FE_EINVAL, "elements per patch must be in [1, 4096] (0: default)%s");
    // host-side validation of every mesh before any device work
    for (int m = 0; m < n_mesh; ++m) {
        const fe_mesh_desc_t &d = meshes[m];
        if (d.n_elem < 1 || d.n_nodes < 1 || d.order < 1 || d.order > 4)
            return fail(nullptr, FE_EINVAL, "mesh sizes or order out of range%s");
        if (d.q1d < d.order + 1 || d.q1d > d.order + 3)
            return fail(nullptr, FE_EUNSUPPORTED, "q1d must be in [order+1, order+3]%s");
        if (!supported_pq(d.order, d.q1d))
            return fail(nullptr, FE_EUNSUPPORTED, "(order, q1d) not built%s");
        if (o.precision == FE_PREC_BF16 && !bf16_force(d.order, d.q1d))
            return fail(nullptr, FE_EUNSUPPORTED, "(order, q1d) has no BF16 MFMA instance%s");
        if (!d.elem_nodes || !d.x0) return fail(nullptr, FE_EINVAL, "NULL mesh array%s");
        if (!d.rho0_q && !(d.rho0 > 0.0)) return fail(nullptr, FE_EINVAL, "rho0 must be > 0%s");
        if (d.rho0_q && o.materials)
            return fail(nullptr, FE_EUNSUPPORTED, "rho0_q with materials (each has its own rho0)%s");
        const long long D3 = (long long)(d.order + 1) * (d.order + 1) * (d.order + 1);
        const long long cnt = D3 * d.n_elem;
        for (long long k = 0; k < cnt; ++k)
            if (d.elem_nodes[k] < 0 || d.elem_nodes[k] >= d.n_nodes)
                return fail(nullptr, FE_EINVAL, "element-to-node map entry out of range%s");
    }

    ctx = new (std::nothrow) fe_ctx();
    if (!ctx) return fail(nullptr, FE_ENOMEM, "host allocation failed%s");
    ctx->opts = o;
    ctx->lo = o.precision != FE_PREC_FP64;
    ctx->bf = o.precision == FE_PREC_BF16;
    ctx->st = (hipStream_t)hip_stream;
    auto bail = [&](int code) {
        g_setup_error = ctx->err;
        free_all(ctx);
        delete ctx;
        return code;
    };
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        ctx->err = "no HIP device";
        return bail(FE_EDEVICE);
    }
    // device address of this GPU's static scratch (allocation-free entry
    // points), looked up once per device; a failure only disables those calls
    (void)static_scratch_init(ctx->device);

    // layout of the concatenated vectors and context arrays
    bool tune_opened = true;
    const std::vector<TuneEntry> tune = read_tune_table(o.tune_table, &tune_opened);
    if (!tune_opened) {
        ctx->err = "cannot open the tuning table named by tune_table";
        return bail(FE_EINVAL);
    }
    std::map<std::pair<int, int>, int> slot_of;
    std::vector<double> tab_host;
    for (int m = 0; m < n_mesh; ++m) {
        const fe_mesh_desc_t &d = meshes[m];
        MeshRec r;
        r.E = d.n_elem;
        r.p = d.order;
        r.Q = d.q1d;
        r.N = d.n_nodes;
        // with rho0_q the set-up forms detJ0 w and scales it point by point
        r.rho0 = d.rho0_q ? 1.0 : d.rho0;
        r.ks = fp64_kernels(r.p, r.Q);
        r.kl = ctx->lo ? *fp32_kernels(r.p, r.Q) : *r.ks;
        {
            const int D = r.p + 1, rs = ctx->lo ? 4 : 8;
            r.nw_force = default_nw(4, force_lds(D, r.Q, rs, 8), force_lds(D, r.Q, rs, 4));
            r.nw_force_t = default_nw(4, force_t_lds(D, r.Q, rs, 8), force_t_lds(D, r.Q, rs, 4));
            r.nw_mass = default_nw(8, mass_lds(D, r.Q, rs, 8), mass_lds(D, r.Q, rs, 4));
            r.patch = 0;
            r.nw_pair = 0;
            r.pair_split = false;
            for (const TuneEntry &te : tune)
                if (te.p == r.p && te.Q == r.Q && te.prec == o.precision) {
                    if (te.nwf) r.nw_force = te.nwf;
                    if (te.nwt) r.nw_force_t = te.nwt;
                    if (te.nwm) r.nw_mass = te.nwm;
                    if (te.patch) r.patch = te.patch;
                    r.nw_pair = te.nwp > 0 ? te.nwp : 0;
                    r.pair_split = te.nwp < 0;
                }
            if (o.tune_nw_force) r.nw_force = o.tune_nw_force;
            if (o.tune_nw_force_t) r.nw_force_t = o.tune_nw_force_t;
            if (o.tune_nw_mass) r.nw_mass = o.tune_nw_mass;
            if (o.tune_patch) r.patch = o.tune_patch;
            // never a tile shape whose kernels spill registers or overflow LDS
            const KernelSet &kc = ctx->lo ? *fp32_kernels(r.p, r.Q) : *r.ks;
            r.nw_force = std::min(r.nw_force, kc.max_nw(0));
            r.nw_force_t = std::min(r.nw_force_t, kc.max_nw(1));
            r.nw_mass = std::min(r.nw_mass, kc.max_nw(2));
            // explicit shapes: one wave count for both and the fused kernel (the
            // autotuner times the two single kernels on their own)
            if (o.tune_nw_force) r.pair_split = false;
            if (o.tune_nw_force || !r.nw_pair) r.nw_pair = r.nw_force;
            r.nw_pair = std::min(r.nw_pair, kc.max_nw(3));
        }
        r.mf = mf_kernel(r.p, r.Q);
        if (!stiff_kernels(r.p, r.Q, &r.sk)) {
            ctx->err = "no stiffness kernels for this (order, q1d)";
            return bail(FE_EUNSUPPORTED);
        }
        if (ctx->bf) {
            r.kl.force = bf16_force(r.p, r.Q);
            bf16_parts(r.p, r.Q, &r.kl);
        }
        // each mesh's L2 block starts at a multiple of p^3, so that an L2 element
        // index (offset / p^3) addresses it in every mesh of the same order
        const long long DL3 = (long long)r.p * r.p * r.p;
        ctx->L2_tot = (ctx->L2_tot + DL3 - 1) / DL3 * DL3;
        r.node_off = ctx->N_tot;
        r.elem_off = ctx->E_tot;
        r.l2_off = ctx->L2_tot;
        auto key = std::make_pair(r.p, r.Q);
        if (!slot_of.count(key)) {
            slot_of[key] = (int)tab_host.size();
            std::vector<double> t = build_table(r.p, r.Q);
            tab_host.insert(tab_host.end(), t.begin(), t.end());
            while (tab_host.size() % 32) tab_host.push_back(0.0);  // 256-byte aligned slots
        }
        r.tab_slot = slot_of[key];
        ctx->N_tot += r.N;
        ctx->E_tot += r.E;
        ctx->L2_tot += (long long)r.E * DL3;
        if (m > 0 && (r.p != ctx->mesh[0].p || r.Q != ctx->mesh[0].Q)) ctx->uniform_pq = false;
        ctx->mesh.push_back(r);
    }
    // storage of S and m_q: grouped by (order, Q) class in the batched form, so
    // that every class is one contiguous range; in caller order otherwise
    ctx->batched = (o.flags & FE_OPT_BATCHED) != 0;
    ctx->atomic = (o.flags & FE_OPT_ATOMIC) != 0;
    std::vector<int> order(n_mesh);
    for (int m = 0; m < n_mesh; ++m) order[m] = m;
    if (ctx->batched)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return std::make_pair(ctx->mesh[a].p, ctx->mesh[a].Q) <
                   std::make_pair(ctx->mesh[b].p, ctx->mesh[b].Q);
        });
    for (int m : order) {
        MeshRec &r = ctx->mesh[m];
        const long long Q3 = (long long)r.Q * r.Q * r.Q;
        r.S_off = ctx->S_len;
        r.Sb_off = ctx->Sb_len;
        r.mq_off = ctx->mq_len;
        r.Dk_off = ctx->Dk_len;
        ctx->Dk_len += 6 * Q3 * r.E;
        ctx->S_len += 9 * Q3 * r.E;
        ctx->Sb_len += 9 * (ctx->bf ? (Q3 + 31) / 32 * 32 : Q3) * r.E;
        ctx->mq_len += Q3 * r.E;
        if (ctx->batched) {
            if (ctx->unit.empty() || ctx->unit.back().p != r.p || ctx->unit.back().Q != r.Q) {
                MeshRec u = r;  // kernels, tables, tile shapes and storage start of the class
                u.E = 0;
                u.N = 0;
                u.node_off = u.elem_off = u.l2_off = 0;
                ctx->unit.push_back(u);
            }
            MeshRec &u = ctx->unit.back();
            r.unit = (int)ctx->unit.size() - 1;
            r.el_in_unit = u.E;
            u.E += r.E;
            u.N += r.N;
        }
    }
    if (ctx->E_tot > (1LL << 31) - 1 || ctx->L2_tot > (1LL << 31) - 1) {
        ctx->err = "too many elements for int32 element indices";
        return bail(FE_EINVAL);
    }
    if (ctx->N_tot * 3 > (1LL << 31) - 1) {
        ctx->err = "too many nodes for int32 DOF indices";
        return bail(FE_EINVAL);
    }

    long long qb = 0, wb = 0;
    int rc = FE_OK;
    if (ctx->lo) {
        void *S32 = nullptr;
        if ((rc = ctx->bf ? dev_alloc(ctx, (uint16_t **)&S32, ctx->Sb_len, &qb)
                          : dev_alloc(ctx, (float **)&S32, ctx->Sb_len, &qb)) ||
            (rc = dev_alloc(ctx, &ctx->mq32, ctx->mq_len, &qb)) ||
            (rc = dev_alloc(ctx, &ctx->tabs32, (long long)tab_host.size(), &wb)) ||
            (rc = dev_alloc(ctx, &ctx->ref_r, 3 * ctx->N_tot, &wb)) ||
            (rc = dev_alloc(ctx, &ctx->ref_d, 3 * ctx->N_tot, &wb))) {
            ctx->S = S32;
            return bail(rc);
        }
        ctx->S = S32;
    } else {
        double *S64 = nullptr;
        rc = dev_alloc(ctx, &S64, ctx->S_len, &qb);
        ctx->S = S64;
        if (rc) return bail(rc);
    }
    if ((rc = dev_alloc(ctx, &ctx->mq, ctx->mq_len, &qb)) ||
        (rc = dev_alloc(ctx, &ctx->tabs, (long long)tab_host.size(), &wb)) ||
        (rc = dev_alloc(ctx, &ctx->min_key, 2, &wb)) || (rc = dev_alloc(ctx, &ctx->nonfinite, 1, &wb)) ||
        (rc = dev_alloc(ctx, &ctx->r, 3 * ctx->N_tot, &wb)) || (rc = dev_alloc(ctx, &ctx->p, 3 * ctx->N_tot, &wb)) ||
        (rc = dev_alloc(ctx, &ctx->Ap, 3 * ctx->N_tot, &wb)) ||
        (rc = dev_alloc(ctx, &ctx->part2, std::max(kVecBlocks, kStepBlocks), &wb)) || (rc = dev_alloc(ctx, &ctx->scal, 8, &wb)) ||
        (rc = dev_alloc(ctx, &ctx->fr, 3 * ctx->N_tot, &wb)) || (rc = dev_alloc(ctx, &ctx->cg, 1, &wb)) ||
        (rc = dev_alloc(ctx, &ctx->bad, 1, &wb)))
        return bail(rc);
    if (hipMemsetAsync(ctx->cg, 0, sizeof(CgState), ctx->st) != hipSuccess) {
        ctx->err = "device memset failed";
        return bail(FE_EDEVICE);
    }
    if (o.flags & FE_OPT_GRAPH) {
        bool ok = hipStreamCreateWithFlags(&ctx->gst, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) == hipSuccess;
        for (int i = 0; ok && i < kAuxStreams; ++i)
            ok = hipStreamCreateWithFlags(&ctx->aux[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&ctx->ev_join[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            ctx->err = "stream or event creation failed";
            return bail(FE_EDEVICE);
        }
    }
    if ((o.flags & FE_OPT_STIFF) && (rc = dev_alloc(ctx, &ctx->Dk, ctx->Dk_len, &qb))) return bail(rc);
    if (o.materials) {
        ctx->n_mat = o.materials->n_mat;
        ctx->mat_gamma.assign(o.materials->gamma, o.materials->gamma + ctx->n_mat);
        if ((rc = dev_alloc(ctx, &ctx->mqk, ctx->n_mat * ctx->mq_len, &qb)) ||
            (rc = dev_alloc(ctx, &ctx->Sk, ctx->n_mat * ctx->S_len, &qb)))
            return bail(rc);
    }
    if (o.flags & FE_OPT_STEP) {
        for (MeshRec &r : ctx->mesh) {
            r.minv_off = ctx->minv_len;
            ctx->minv_len += (long long)r.E * r.p * r.p * r.p * r.p * r.p * r.p;
        }
        const long long n3 = 3 * ctx->N_tot;
        if ((rc = dev_alloc(ctx, &ctx->minv, ctx->minv_len, &wb)) || (rc = dev_alloc(ctx, &ctx->xs, n3, &wb)) ||
            (rc = dev_alloc(ctx, &ctx->vs, n3, &wb)) || (rc = dev_alloc(ctx, &ctx->es, ctx->L2_tot, &wb)) ||
            (rc = dev_alloc(ctx, &ctx->acc, n3, &wb)) || (rc = dev_alloc(ctx, &ctx->sy, n3, &wb)) ||
            (rc = dev_alloc(ctx, &ctx->sz, ctx->L2_tot, &wb)) || (rc = dev_alloc(ctx, &ctx->vbar, n3, &wb)) ||
            (rc = dev_alloc(ctx, &ctx->dtv, 2, &wb)))
            return bail(rc);
        launch_fill(ctx->acc, n3, 0.0, ctx->st);
        if (hipHostMalloc((void **)&ctx->h_dt, 2 * sizeof(double)) != hipSuccess) {
            ctx->err = "pinned host allocation failed";
            return bail(FE_ENOMEM);
        }
    }
    if (hipHostMalloc((void **)&ctx->h_cg, sizeof(CgState)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_scal, 8 * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_key, 2 * sizeof(long long)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_flag, sizeof(int)) != hipSuccess) {
        ctx->err = "pinned host allocation failed";
        return bail(FE_ENOMEM);
    }
    if (o.flags & FE_OPT_TIMERS)
        for (auto &tp : ctx->timers) {
            tp.ev.resize(kTimerPairs);
            for (auto &pr : tp.ev)
                if (hipEventCreate(&pr.first) != hipSuccess || hipEventCreate(&pr.second) != hipSuccess) {
                    ctx->err = "event creation failed";
                    return bail(FE_EDEVICE);
                }
        }
    if (hipMemcpyAsync(ctx->tabs, tab_host.data(), tab_host.size() * sizeof(double),
                       hipMemcpyHostToDevice, ctx->st) != hipSuccess) {
        ctx->err = "upload failed";
        return bail(FE_EDEVICE);
    }
    if (ctx->lo) launch_f64_to_f32(ctx->tabs, ctx->tabs32, (long long)tab_host.size(), ctx->st);
    if (ctx->bf) {
        std::vector<unsigned char> tb;
        std::map<std::pair<int, int>, long long> boff;
        for (MeshRec &r : ctx->mesh) {
            auto key = std::make_pair(r.p, r.Q);
            if (!boff.count(key)) {
                boff[key] = (long long)tb.size();
                std::vector<double> t = build_table(r.p, r.Q);
                std::vector<unsigned char> m = build_mfma_table(r.p, r.Q, t);
                tb.insert(tb.end(), m.begin(), m.end());
                while (tb.size() % 256) tb.push_back(0);
            }
            r.tabb_off = boff[key];
        }
        for (MeshRec &u : ctx->unit) u.tabb_off = boff[std::make_pair(u.p, u.Q)];
        if ((rc = dev_alloc(ctx, &ctx->tabsb, (long long)tb.size(), &wb))) return bail(rc);
        if (hipMemcpy(ctx->tabsb, tb.data(), tb.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemsetAsync(ctx->S, 0, 2 * (size_t)ctx->Sb_len, ctx->st) != hipSuccess) {
            ctx->err = "upload failed";
            return bail(FE_EDEVICE);
        }
    }

    // patch plans (element order, distinct nodes, shared-node gather) per mesh
    auto upload = [&](const void *src, size_t bytes, void **dst) -> int {
        void *d = nullptr;
        if (hipMalloc(&d, bytes ? bytes : 4) != hipSuccess) {
            (void)hipGetLastError();
            return FE_ENOMEM;
        }
        ctx->plan_bufs.push_back(d);
        wb += (long long)(bytes ? bytes : 4);
        *dst = d;
        if (src && bytes && hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
            return FE_EDEVICE;
        return FE_OK;
    };
    auto upload_plan = [&](const PatchPlan &pl, MeshRec &r) -> int {
        void *dp = nullptr;
        int urc = FE_OK;
        if ((urc = upload(pl.perm.data(), pl.perm.size() * 4, &dp)) == FE_OK) r.pd.perm = (const int32_t *)dp;
        if (!urc && (urc = upload(pl.map_int.data(), pl.map_int.size() * 4, &dp)) == FE_OK) r.pd.map = (const int32_t *)dp;
        if (!urc && (urc = upload(pl.slot.data(), pl.slot.size() * 2, &dp)) == FE_OK) r.pd.slot = (const uint16_t *)dp;
        if (!urc && (urc = upload(pl.pn.data(), pl.pn.size() * 4, &dp)) == FE_OK) r.pd.pn = (const int32_t *)dp;
        if (!urc && (urc = upload(pl.patch.data(), pl.patch.size() * sizeof(PatchRec), &dp)) == FE_OK) r.pd.ptab = (const int32_t *)dp;
        if (!urc && (urc = upload(pl.sh_node.data(), pl.sh_node.size() * 4, &dp)) == FE_OK) r.pd.sh_node = (const int32_t *)dp;
        if (!urc && (urc = upload(pl.sh_ptr.data(), pl.sh_ptr.size() * 4, &dp)) == FE_OK) r.pd.sh_ptr = (const int32_t *)dp;
        if (!urc && (urc = upload(pl.sh_idx.data(), pl.sh_idx.size() * 4, &dp)) == FE_OK) r.pd.sh_idx = (const int32_t *)dp;
        // shared-node partials (none in the atomic scatter mode: pd.part stays null)
        if (!urc && !ctx->atomic &&
            (urc = upload(nullptr, (size_t)pl.n_entries * 3 * sizeof(double), &dp)) == FE_OK)
            r.pd.part = (double *)dp;
        r.pd.n_entries = pl.n_entries;
        if (!urc && (urc = upload(pl.orphans.data(), pl.orphans.size() * 4, &dp)) == FE_OK) r.orphans = (const int32_t *)dp;
        static_assert(sizeof(PatchRec) == 6 * sizeof(int32_t), "patch table rows are 6 int32");
        r.pd.n_patch = (int)pl.patch.size();
        r.pd.n_shared = (int)pl.sh_node.size();
        r.n_orphans = (int)pl.orphans.size();
        return urc;
    };
    // patch size: the largest Morton block (512, 64, 8 elements) allowed for the
    // order that still leaves >= 1024 workgroups per launch (of the mesh, or of
    // its class in the batched form), unless the tuning sets it
    auto pick_patch = [](const MeshRec &r, long long E) {
        const int bmax = r.p == 1 ? 512 : (r.p == 2 ? 64 : 8);
        int B = 8;
        for (int cand : {512, 64, 8})
            if (cand <= bmax && E / cand >= 1024) { B = cand; break; }
        return r.patch ? r.patch : B;
    };
    for (MeshRec &u : ctx->unit) u.patch = pick_patch(u, u.E);
    std::vector<PatchPlan> cplan(ctx->unit.size());
    for (int m = 0; m < n_mesh; ++m) {
        MeshRec &r = ctx->mesh[m];
        std::vector<double> x0h(3 * (size_t)r.N);
        if (hipStreamSynchronize(ctx->st) != hipSuccess ||
            hipMemcpy(x0h.data(), meshes[m].x0, x0h.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            ctx->err = "cannot read x0";
            return bail(FE_EDEVICE);
        }
        r.patch = ctx->batched ? ctx->unit[r.unit].patch : pick_patch(r, r.E);
        PatchPlan pl = build_patch_plan(r.E, r.p, r.N, meshes[m].elem_nodes, x0h.data(), r.patch,
                                        r.ks->umax);
        for (auto &g : pl.map_int) g += (int32_t)r.node_off;
        for (auto &g : pl.pn) g += (int32_t)r.node_off;
        for (auto &g : pl.sh_node) g += (int32_t)r.node_off;
        for (auto &g : pl.orphans) g += (int32_t)r.node_off;
        if (ctx->batched) {
            // element ids of the class plan are L2 element indices of the whole vector
            const long long DL3 = (long long)r.p * r.p * r.p;
            r.patch_in_unit = (int)cplan[r.unit].patch.size();
            r.n_patch_mesh = (int)pl.patch.size();
            append_plan(cplan[r.unit], pl, (int32_t)(r.l2_off / DL3));
            continue;
        }
        if (upload_plan(pl, r)) {
            ctx->err = "patch plan upload failed";
            return bail(FE_ENOMEM);
        }
    }
    for (size_t k = 0; k < ctx->unit.size(); ++k)
        if (upload_plan(cplan[k], ctx->unit[k])) {
            ctx->err = "patch plan upload failed";
            return bail(FE_ENOMEM);
        }
    cplan.clear();
    for (MeshRec &r : ctx->mesh)
        if (ctx->batched) {  // the mesh's rows of its class plan (set-up and export kernels)
            const MeshRec &u = ctx->unit[r.unit];
            const long long D3 = (long long)(r.p + 1) * (r.p + 1) * (r.p + 1);
            r.pd = PatchDev{};
            r.pd.perm = u.pd.perm + r.el_in_unit;
            r.pd.map = u.pd.map + r.el_in_unit * D3;
        }
    for (MeshRec &r : ctx->batched ? ctx->unit : ctx->mesh) {
        r.part_off = ctx->n_parts;
        ctx->n_parts += r.pd.n_patch;
    }
    if ((rc = dev_alloc(ctx, &ctx->part, std::max<long long>(ctx->n_parts, kVecBlocks), &wb)))
        return bail(rc);
    // several meshes: chunks of at most kChunk DOFs inside one mesh and component,
    // ordered by mesh; each mesh's range of mass partials; the mesh of each partial
    ctx->multi = n_mesh > 1;
    if (!ctx->multi) {
        const MeshRec &r = ctx->units()[0];
        // a shared node's entry range in the gather lists, packed into one
        // word so that the step kernel reads it in one load
        std::vector<long long> nsh((size_t)ctx->N_tot, -1);
        std::vector<int32_t> shn((size_t)r.pd.n_shared), shp((size_t)r.pd.n_shared + 1);
        if (r.pd.n_shared &&
            (hipMemcpy(shn.data(), r.pd.sh_node, shn.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(shp.data(), r.pd.sh_ptr, shp.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)) {
            ctx->err = "cannot read the shared-node list";
            return bail(FE_EDEVICE);
        }
        // atomic scatter mode: the mass kernel leaves Ap complete at every node
        for (size_t k = 0; k < (ctx->atomic ? 0 : shn.size()); ++k) {
            const long long cnt = shp[k + 1] - shp[k];
            if (cnt >= 0x10000) {
                ctx->err = "a node is shared by 65536 or more patches";
                return bail(FE_EUNSUPPORTED);
            }
            nsh[(size_t)shn[k]] = ((long long)shp[k] << 16) | cnt;
        }
        void *dp = nullptr;
        if (upload(nsh.data(), nsh.size() * sizeof(long long), &dp)) {
            ctx->err = "CG workspace allocation failed";
            return bail(FE_ENOMEM);
        }
        ctx->node_sh = (long long *)dp;
    }
    if (ctx->multi) {
        std::vector<CgChunk> ch;
        std::vector<int> cbeg(n_mesh + 1), prange(2 * (size_t)n_mesh), pmesh((size_t)ctx->n_parts);
        for (int m = 0; m < n_mesh; ++m) {
            const MeshRec &r = ctx->mesh[m];
            cbeg[m] = (int)ch.size();
            for (int c = 0; c < 3; ++c)
                for (int off = 0; off < r.N; off += kChunk)
                    ch.push_back(CgChunk{(int)(c * ctx->N_tot + r.node_off + off),
                                         std::min(kChunk, r.N - off), m, 0});
            const long long pb = ctx->batched ? ctx->unit[r.unit].part_off + r.patch_in_unit : r.part_off;
            const long long pc = ctx->batched ? r.n_patch_mesh : r.pd.n_patch;
            prange[2 * m] = (int)pb;
            prange[2 * m + 1] = (int)(pb + pc);
            for (long long k = pb; k < pb + pc; ++k) pmesh[k] = m;
        }
        cbeg[n_mesh] = (int)ch.size();
        const long long nch = (long long)ch.size();
        void *dp = nullptr;
        int urc = upload(ch.data(), ch.size() * sizeof(CgChunk), &dp);
        ctx->chunk = (CgChunk *)dp;
        if (!urc && !(urc = upload(cbeg.data(), cbeg.size() * 4, &dp))) ctx->cbeg = (int *)dp;
        if (!urc && !(urc = upload(prange.data(), prange.size() * 4, &dp))) ctx->prange = (int *)dp;
        if (!urc && !(urc = upload(pmesh.data(), pmesh.size() * 4, &dp))) ctx->pmesh = (int *)dp;
        if (urc || (rc = dev_alloc(ctx, &ctx->cgm, n_mesh, &wb)) || (rc = dev_alloc(ctx, &ctx->glob, 1, &wb)) ||
            (rc = dev_alloc(ctx, &ctx->part3, std::max<long long>(nch, kVecBlocks), &wb)) ||
            (rc = dev_alloc(ctx, &ctx->mres, n_mesh, &wb))) {
            ctx->err = "CG workspace allocation failed";
            return bail(FE_ENOMEM);
        }
        if (nch > kVecBlocks) {
            (void)hipFree(ctx->part2);
            ctx->part2 = nullptr;
            if ((rc = dev_alloc(ctx, &ctx->part2, nch, &wb))) return bail(rc);
        }
        if (hipHostMalloc((void **)&ctx->h_cgm, n_mesh * sizeof(CgState)) != hipSuccess ||
            hipHostMalloc((void **)&ctx->h_glob, sizeof(CgGlobal)) != hipSuccess ||
            hipHostMalloc((void **)&ctx->h_mres, n_mesh * sizeof(double)) != hipSuccess) {
            ctx->err = "pinned host allocation failed";
            return bail(FE_ENOMEM);
        }
        ctx->cm.chunk = ctx->chunk;
        ctx->cm.n_chunk = (int)nch;
        ctx->cm.cbeg = ctx->cbeg;
        ctx->cm.prange = ctx->prange;
        ctx->cm.n_mesh = n_mesh;
        ctx->cm.state = ctx->cgm;
        ctx->cm.glob = ctx->glob;
    }
    ctx->qdata_bytes = qb;
    ctx->work_bytes = wb;

    // m_q = rho0 detJ0 w from x0 (qdata kernels in set-up mode)
    launch_reset_diag(ctx->min_key, ctx->nonfinite, ctx->st);
    for (int m = 0; m < n_mesh; ++m) {
        const MeshRec &r = ctx->mesh[m];
        QParams prm{r.rho0, o.gamma, o.gamma - 1.0, o.q1, o.q2, 1.0 / r.p};
        r.ks->qdata(meshes[m].x0, nullptr, nullptr, r.pd, r.E, r.N, (int)r.node_off,
                    ctx->mq + r.mq_off, nullptr, ctx->tabs + r.tab_slot, prm, ctx->min_key,
                    ctx->nonfinite, true, ctx->st);
    }
    launch_reset_diag(nullptr, ctx->bad, ctx->st);
    for (int m = 0; m < n_mesh; ++m) {
        if (!meshes[m].rho0_q) continue;
        const MeshRec &r = ctx->mesh[m];
        const int perm_base = ctx->batched ? (int)(r.l2_off / ((long long)r.p * r.p * r.p)) : 0;
        launch_point_density(ctx->mq + r.mq_off, meshes[m].rho0_q, r.pd.perm, perm_base,
                             r.Q * r.Q * r.Q, r.E, ctx->bad, ctx->st);
    }
    int bad_rho = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&bad_rho, ctx->bad, sizeof(int), hipMemcpyDeviceToHost, ctx->st) != hipSuccess ||
        hipMemcpyAsync(ctx->h_key, ctx->min_key, sizeof(long long), hipMemcpyDeviceToHost, ctx->st) != hipSuccess ||
        hipMemcpyAsync(ctx->h_flag, ctx->nonfinite, sizeof(int), hipMemcpyDeviceToHost, ctx->st) != hipSuccess ||
        hipStreamSynchronize(ctx->st) != hipSuccess) {
        ctx->err = "set-up kernels failed";
        return bail(FE_EDEVICE);
    }
    if (ctx->n_mat) {
        // m_qk = rho0_k eta0_k(q) detJ0 w = (rho0_k / rho0) eta0_k(q) m_q, then
        // the context's m_q becomes the mixture's, sum_k m_qk
        const fe_materials_t &mt = *o.materials;
        for (int k = 0; k < ctx->n_mat; ++k)
            for (const MeshRec &r : ctx->mesh) {
                const double *eta = mt.eta0 + k * ctx->L2_tot + (ctx->batched ? 0 : r.l2_off);
                launch_mat_mass(r.p, r.Q, ctx->mq + r.mq_off, eta, r.pd.perm, mt.rho0[k] / r.rho0,
                                ctx->mqk + k * ctx->mq_len + r.mq_off, r.E, ctx->tabs + r.tab_slot,
                                ctx->st);
            }
        launch_sum_blocks(ctx->mqk, ctx->n_mat, ctx->mq_len, ctx->mq, ctx->mq_len, ctx->st);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->st) != hipSuccess) {
            ctx->err = "set-up kernels failed";
            return bail(FE_EDEVICE);
        }
    }
    if (ctx->lo) {
        launch_f64_to_f32(ctx->mq, ctx->mq32, ctx->mq_len, ctx->st);
        if (hipStreamSynchronize(ctx->st) != hipSuccess) {
            ctx->err = "set-up kernels failed";
            return bail(FE_EDEVICE);
        }
    }
    if (bad_rho) {
        ctx->err = "rho0_q holds a value that is not a positive finite number";
        return bail(FE_EINVAL);
    }
    const double min0 = key_to_double(*ctx->h_key);
    if (!(min0 > 0.0) || *ctx->h_flag) {
        char buf[128];
        std::snprintf(buf, sizeof(buf), "initial mesh has min detJ = %.3e", min0);
        ctx->err = buf;
        return bail(FE_EBADMESH);
    }
    if (o.flags & FE_OPT_STEP) {
        // M_E^-1 of every element from m_q (fixed while the mesh moves)
        for (const MeshRec &r : ctx->mesh) {
            const int perm_base = ctx->batched ? (int)(r.l2_off / ((long long)r.p * r.p * r.p)) : 0;
            launch_l2_mass_inv(r.p, r.Q, ctx->mq + r.mq_off, r.pd.perm, perm_base, r.E,
                               ctx->tabs + r.tab_slot, ctx->minv + r.minv_off, ctx->st);
        }
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->st) != hipSuccess) {
            ctx->err = "set-up kernels failed";
            return bail(FE_EDEVICE);
        }
    }
    *out = ctx;
    return FE_OK;
}

void fe_destroy(fe_ctx_t *ctx)
{
    if (!ctx) return;
    free_all(ctx);
    delete ctx;
}

int fe_query(const fe_ctx_t *ctx, fe_info_t *info)
{
    if (!ctx || !info) return FE_EINVAL;
    info->n_mesh = (int32_t)ctx->mesh.size();
    info->nw_force = ctx->mesh[0].nw_force;
    info->nw_force_t = ctx->mesh[0].nw_force_t;
    info->nw_mass = ctx->mesh[0].nw_mass;
    info->patch = ctx->mesh[0].patch;
    info->n_elem_total = ctx->E_tot;
    info->n_nodes_total = ctx->N_tot;
    info->l2_size_total = ctx->L2_tot;
    info->qdata_bytes = ctx->qdata_bytes;
    info->workspace_bytes = ctx->work_bytes;
    info->precision = ctx->opts.precision;
    info->flags = ctx->opts.flags;
    return FE_OK;
}

int fe_mesh_offsets(const fe_ctx_t *ctx, int64_t *node_offset, int64_t *elem_offset,
                    int64_t *l2_offset)
{
    if (!ctx) return FE_EINVAL;
    for (size_t m = 0; m < ctx->mesh.size(); ++m) {
        if (node_offset) node_offset[m] = ctx->mesh[m].node_off;
        if (elem_offset) elem_offset[m] = ctx->mesh[m].elem_off;
        if (l2_offset) l2_offset[m] = ctx->mesh[m].l2_off;
    }
    return FE_OK;
}

int fe_qdata_update(fe_ctx_t *ctx, const double *x, const double *v, const double *e)
{
    if (!ctx) return FE_EINVAL;
    if (!x || !v || !e) return fail(ctx, FE_EINVAL, "NULL input%s");
    ScopedTimer tm(ctx, FE_TIMER_QDATA);
    return run_graph(ctx, GraphKey{kActQdata, x, v, e}, [&](hipStream_t s, bool branch) {
        launch_reset_diag(ctx->min_key, ctx->nonfinite, s);
        enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
            QParams prm{r.rho0, ctx->opts.gamma, ctx->opts.gamma - 1.0, ctx->opts.q1, ctx->opts.q2,
                        1.0 / r.p};
            r.kl.qdata(x, v, e + r.l2_off, r.pd, r.E, ctx->N_tot, 0, ctx->mq + r.mq_off,
                       S_of(ctx, r), ctx->tabs + r.tab_slot, prm, ctx->min_key, ctx->nonfinite,
                       false, su);
        });
    });
}

int fe_force_mult(fe_ctx_t *ctx, const double *e, double *y)
{
    if (!ctx) return FE_EINVAL;
    if (!y) return fail(ctx, FE_EINVAL, "NULL output%s");
    if ((const void *)e == (const void *)y) return fail(ctx, FE_EINVAL, "input aliases output%s");
    ScopedTimer tm(ctx, FE_TIMER_FORCE);
    return run_graph(ctx, GraphKey{kActForce, e, y}, [&](hipStream_t s, bool branch) {
        enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
            launch_scatter_prepare(r.pd, y, ctx->N_tot, nullptr, su);
            r.kl.force(S_of(ctx, r), e ? e + r.l2_off : nullptr, r.pd, y, ctx->N_tot,
                       tab_of(ctx, r), r.nw_force, su);
            launch_gather_shared(r.pd, y, ctx->N_tot, nullptr, su);
            launch_zero_nodes(r.orphans, r.n_orphans, y, ctx->N_tot, nullptr, su);
        });
    });
}

int fe_force_mult_T(fe_ctx_t *ctx, const double *v, double *z)
{
    if (!ctx) return FE_EINVAL;
    if (!v || !z) return fail(ctx, FE_EINVAL, "NULL argument%s");
    if ((const void *)v == (const void *)z) return fail(ctx, FE_EINVAL, "input aliases output%s");
    ScopedTimer tm(ctx, FE_TIMER_FORCE_T);
    return run_graph(ctx, GraphKey{kActForceT, v, z}, [&](hipStream_t s, bool branch) {
        enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
            r.kl.force_t(S_of(ctx, r), v, r.pd, r.E, z + r.l2_off, ctx->N_tot, tab_of(ctx, r),
                         r.nw_force_t, su);
        });
    });
}

int fe_force_mult_pair(fe_ctx_t *ctx, const double *e, double *y, const double *v, double *z)
{
    if (!ctx) return FE_EINVAL;
    if (!y || !v || !z) return fail(ctx, FE_EINVAL, "NULL argument%s");
    const void *in[] = {e, v}, *out[] = {y, z};
    if (out[0] == out[1]) return fail(ctx, FE_EINVAL, "outputs alias%s");
    for (const void *i : in)
        for (const void *o : out)
            if (i && i == o) return fail(ctx, FE_EINVAL, "input aliases output%s");
    ScopedTimer tm(ctx, FE_TIMER_PAIR);
    return run_graph(ctx, GraphKey{kActPair, e, y, v, 0, z}, [&](hipStream_t s, bool branch) {
        enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
            launch_scatter_prepare(r.pd, y, ctx->N_tot, nullptr, su);
            if (r.pair_split) {  // the tile table measured the two kernels faster here
                r.kl.force(S_of(ctx, r), e ? e + r.l2_off : nullptr, r.pd, y, ctx->N_tot,
                           tab_of(ctx, r), r.nw_force, su);
                r.kl.force_t(S_of(ctx, r), v, r.pd, r.E, z + r.l2_off, ctx->N_tot, tab_of(ctx, r),
                             r.nw_force_t, su);
            } else {
                r.kl.force_pair(S_of(ctx, r), e ? e + r.l2_off : nullptr, v, r.pd, y, z + r.l2_off,
                                ctx->N_tot, tab_of(ctx, r), r.nw_pair, su);
            }
            launch_gather_shared(r.pd, y, ctx->N_tot, nullptr, su);
            launch_zero_nodes(r.orphans, r.n_orphans, y, ctx->N_tot, nullptr, su);
        });
    });
}

int fe_force_mult_pair_noalloc(fe_ctx_t *ctx, const double *e, double *y, const double *v,
                               double *z)
{
    if (!ctx) return FE_EINVAL;
    if (!y || !v || !z) return fail(ctx, FE_EINVAL, "NULL argument%s");
    const void *in[] = {e, v}, *out[] = {y, z};
    if (out[0] == out[1]) return fail(ctx, FE_EINVAL, "outputs alias%s");
    for (const void *i : in)
        for (const void *o : out)
            if (i && i == o) return fail(ctx, FE_EINVAL, "input aliases output%s");
    double *scr = static_scratch(ctx->device);
    if (!scr) return fail(ctx, FE_EDEVICE, "static scratch of this device is not available%s");
    // the units run one after another on the context stream, so each reuses
    // the scratch from its start
    for (const MeshRec &r : ctx->units()) {
        const long long need = ctx->atomic ? 0 : r.pd.n_entries * 3 * (long long)sizeof(double);
        if (need > kStaticScratchBytes) {
            char buf[160];
            std::snprintf(buf, sizeof(buf),
                          "shared-node partials need %lld bytes, above the %lld-byte static scratch",
                          need, kStaticScratchBytes);
            ctx->err = buf;
            return FE_EINVAL;
        }
    }
    hipStream_t su = ctx->st;
    for (const MeshRec &r : ctx->units()) {
        PatchDev pd = r.pd;
        if (!ctx->atomic) pd.part = scr;
        launch_scatter_prepare(pd, y, ctx->N_tot, nullptr, su);
        if (r.pair_split) {
            r.kl.force(S_of(ctx, r), e ? e + r.l2_off : nullptr, pd, y, ctx->N_tot, tab_of(ctx, r),
                       r.nw_force, su);
            r.kl.force_t(S_of(ctx, r), v, pd, r.E, z + r.l2_off, ctx->N_tot, tab_of(ctx, r),
                         r.nw_force_t, su);
        } else {
            r.kl.force_pair(S_of(ctx, r), e ? e + r.l2_off : nullptr, v, pd, y, z + r.l2_off,
                            ctx->N_tot, tab_of(ctx, r), r.nw_pair, su);
        }
        launch_gather_shared(pd, y, ctx->N_tot, nullptr, su);
        launch_zero_nodes(r.orphans, r.n_orphans, y, ctx->N_tot, nullptr, su);
    }
    HIP_OK(hipGetLastError());
    return FE_OK;
}

int fe_stiffness_update(fe_ctx_t *ctx, const double *x, const double *kappa)
{
    if (!ctx) return FE_EINVAL;
    if (!(ctx->opts.flags & FE_OPT_STIFF)) return fail(ctx, FE_EINVAL, "context set up without FE_OPT_STIFF%s");
    if (!x) return fail(ctx, FE_EINVAL, "NULL positions%s");
    if (kappa && !ctx->uniform_pq)
        return fail(ctx, FE_EINVAL, "a point coefficient needs one (order, q1d) for all meshes%s");
    return run_graph(ctx, GraphKey{kActStiffQ, x, kappa}, [&](hipStream_t s, bool branch) {
        enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
            const long long Q3 = (long long)r.Q * r.Q * r.Q;
            r.sk.qdata(x, r.pd, r.E, ctx->N_tot, kappa ? kappa + r.elem_off * Q3 : nullptr, 0,
                       ctx->Dk + r.Dk_off, ctx->tabs + r.tab_slot, su);
        });
    });
}

int fe_stiffness_mult(fe_ctx_t *ctx, const double *u, double *y)
{
    if (!ctx) return FE_EINVAL;
    if (!(ctx->opts.flags & FE_OPT_STIFF)) return fail(ctx, FE_EINVAL, "context set up without FE_OPT_STIFF%s");
    if (!u || !y) return fail(ctx, FE_EINVAL, "NULL argument%s");
    if ((const void *)u == (const void *)y) return fail(ctx, FE_EINVAL, "input aliases output%s");
    return run_graph(ctx, GraphKey{kActStiff, u, y}, [&](hipStream_t s, bool branch) {
        enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
            launch_scatter_prepare(r.pd, y, ctx->N_tot, nullptr, su);
            r.sk.mult(ctx->Dk + r.Dk_off, u, r.pd, y, ctx->N_tot, ctx->tabs + r.tab_slot,
                      r.nw_stiff, su);
            launch_gather_shared(r.pd, y, ctx->N_tot, nullptr, su);
            launch_zero_nodes(r.orphans, r.n_orphans, y, ctx->N_tot, nullptr, su);
        });
    });
}

int fe_qdata_update_mm(fe_ctx_t *ctx, const double *x, const double *v, const double *e)
{
    if (!ctx) return FE_EINVAL;
    if (!ctx->n_mat) return fail(ctx, FE_EINVAL, "context set up without materials%s");
    if (!x || !v || !e) return fail(ctx, FE_EINVAL, "NULL input%s");
    ScopedTimer tm(ctx, FE_TIMER_QDATA);
    return run_graph(ctx, GraphKey{kActQdataMm, x, v, e}, [&](hipStream_t s, bool branch) {
        launch_reset_diag(ctx->min_key, ctx->nonfinite, s);
        enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
            for (int k = 0; k < ctx->n_mat; ++k) {
                const double g = ctx->mat_gamma[k];
                QParams prm{r.rho0, g, g - 1.0, ctx->opts.q1, ctx->opts.q2, 1.0 / r.p};
                r.kl.qdata(x, v, e + k * ctx->L2_tot + r.l2_off, r.pd, r.E, ctx->N_tot, 0,
                           ctx->mqk + k * ctx->mq_len + r.mq_off, ctx->Sk + k * ctx->S_len + r.S_off,
                           ctx->tabs + r.tab_slot, prm, ctx->min_key, ctx->nonfinite, false, su);
            }
            const long long Q3 = (long long)r.Q * r.Q * r.Q;
            launch_sum_blocks(ctx->Sk + r.S_off, ctx->n_mat, ctx->S_len, (double *)ctx->S + r.S_off,
                              9 * Q3 * r.E, su);
        });
    });
}

int fe_force_mult_T_mm(fe_ctx_t *ctx, const double *v, double *z)
{
    if (!ctx) return FE_EINVAL;
    if (!ctx->n_mat) return fail(ctx, FE_EINVAL, "context set up without materials%s");
    if (!v || !z) return fail(ctx, FE_EINVAL, "NULL argument%s");
    if ((const void *)v == (const void *)z) return fail(ctx, FE_EINVAL, "input aliases output%s");
    ScopedTimer tm(ctx, FE_TIMER_FORCE_T);
    return run_graph(ctx, GraphKey{kActForceTMm, v, z}, [&](hipStream_t s, bool branch) {
        enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
            for (int k = 0; k < ctx->n_mat; ++k)
                r.kl.force_t(ctx->Sk + k * ctx->S_len + r.S_off, v, r.pd, r.E,
                             z + k * ctx->L2_tot + r.l2_off, ctx->N_tot, tab_of(ctx, r),
                             r.nw_force_t, su);
        });
    });
}

int fe_force_mult_pair_mf(fe_ctx_t *ctx, const double *x, const double *v, const double *e,
                          double *y, double *z)
{
    if (!ctx) return FE_EINVAL;
    if (!x || !v || !e || !y || !z) return fail(ctx, FE_EINVAL, "NULL argument%s");
    const void *in[] = {x, v, e}, *out[] = {y, z};
    if (out[0] == out[1]) return fail(ctx, FE_EINVAL, "outputs alias%s");
    for (const void *i : in)
        for (const void *o : out)
            if (i == o) return fail(ctx, FE_EINVAL, "input aliases output%s");
    if (ctx->n_mat) return fail(ctx, FE_EUNSUPPORTED, "the matrix-free pair is single-material%s");
    for (const MeshRec &r : ctx->units())
        if (!r.mf) return fail(ctx, FE_EUNSUPPORTED, "no matrix-free kernel for this (order, q1d)%s");
    ScopedTimer tm(ctx, FE_TIMER_MF);
    return run_graph(ctx, GraphKey{kActPairMf, x, v, e, 0, y, z}, [&](hipStream_t s, bool branch) {
        launch_reset_diag(ctx->min_key, ctx->nonfinite, s);
        enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
            QParams prm{r.rho0, ctx->opts.gamma, ctx->opts.gamma - 1.0, ctx->opts.q1, ctx->opts.q2,
                        1.0 / r.p};
            launch_scatter_prepare(r.pd, y, ctx->N_tot, nullptr, su);
            r.mf(x, v, e + r.l2_off, ctx->mq + r.mq_off, r.pd, y, z + r.l2_off, ctx->N_tot,
                 ctx->tabs + r.tab_slot, prm, ctx->min_key, ctx->nonfinite, r.nw_mf, su);
            launch_gather_shared(r.pd, y, ctx->N_tot, nullptr, su);
            launch_zero_nodes(r.orphans, r.n_orphans, y, ctx->N_tot, nullptr, su);
        });
    });
}

// lo: the FP32 operator (precision form); otherwise the FP64 operator.
// With x2 set, the launch is a CG iteration's: the operand is x + beta x2
// (x = r, x2 = p; beta and the done flag from the device CG state) and the
// kernels leave partials of the operand's M-norm in ctx->part.
static void mass_enqueue(fe_ctx *ctx, const double *x, double *y, bool lo, const double *x2,
                         hipStream_t s, bool branch, bool gather = true)
{
    // one CG: its done flag; several meshes: all-done for the gathers, and each
    // patch's own mesh state in the mass kernel
    const int *skip = !x2 ? nullptr : (ctx->multi ? &ctx->glob->done : &ctx->cg->done);
    enqueue_units(ctx, s, branch, [&](const MeshRec &r, hipStream_t su) {
        MassCg cg;
        if (x2) {
            cg.part_dot = ctx->part + r.part_off;
            cg.x2 = x2;
            if (ctx->multi) {
                cg.skip = &ctx->cgm[0].done;
                cg.beta = &ctx->cgm[0].beta;
                cg.pmesh = ctx->pmesh + r.part_off;
                cg.sstride = (int)sizeof(CgState);
            } else {
                cg.skip = skip;
                cg.beta = &ctx->cg->beta;
            }
        }
        launch_scatter_prepare(r.pd, y, ctx->N_tot, skip, su);
        if (lo)
            r.kl.mass(ctx->mq32 + r.mq_off, x, r.pd, y, ctx->N_tot, ctx->tabs32 + r.tab_slot, cg,
                      r.nw_mass, su);
        else
            r.ks->mass(ctx->mq + r.mq_off, x, r.pd, y, ctx->N_tot, ctx->tabs + r.tab_slot, cg,
                       r.nw_mass, su);
        if (gather) launch_gather_shared(r.pd, y, ctx->N_tot, skip, su);
        launch_zero_nodes(r.orphans, r.n_orphans, y, ctx->N_tot, skip, su);
    });
}

static void mass_launch(fe_ctx *ctx, const double *x, double *y, bool lo)
{
    mass_enqueue(ctx, x, y, lo, nullptr, ctx->st, false);
}

int fe_mass_mult(fe_ctx_t *ctx, const double *x, double *y)
{
    if (!ctx) return FE_EINVAL;
    if (!x || !y) return fail(ctx, FE_EINVAL, "NULL argument%s");
    if ((const void *)x == (const void *)y) return fail(ctx, FE_EINVAL, "input aliases output%s");
    ScopedTimer tm(ctx, FE_TIMER_MASS);
    return run_graph(ctx, GraphKey{kActMass, x, y, nullptr, ctx->lo ? 1 : 0},
                     [&](hipStream_t s, bool branch) { mass_enqueue(ctx, x, y, ctx->lo, nullptr, s, branch); });
}

}  // extern "C"

// CG on the free DOFs (mask already built, x already zero on essential DOFs)
// with the FP64 operator, or the FP32 one when lo; one solve per mesh when the
// context holds several. On return out[m] holds mesh m's final device state
// (iterations, ||b_free||^2, done flag).
static int cg_run(fe_ctx *ctx, const double *b, double *x, double rel_tol, int max_iter, bool lo,
                  std::vector<CgState> &out)
{
    const long long n = 3 * ctx->N_tot;
    mass_launch(ctx, x, ctx->Ap, lo);
    if (ctx->multi)
        cgm_start(x, b, ctx->Ap, ctx->r, ctx->p, ctx->fr, ctx->cm, ctx->part2, ctx->part3, rel_tol,
                  max_iter, ctx->st);
    else
        cg_start(x, b, ctx->Ap, ctx->r, ctx->p, ctx->fr, n, ctx->part, ctx->part2, ctx->cg, rel_tol,
                 max_iter, ctx->st);
    HIP_OK(hipGetLastError());
    // one iteration: Ap = M (r + beta p) with partials of its M-norm, then the
    // step kernels (alpha, the axpys and the new r.r, beta)
    // one mesh: the step reads shared Ap from the partials, so the mass launch
    // of an iteration skips the gather
    const bool fused = !ctx->multi;
    auto step = [&](hipStream_t s) {
        if (ctx->multi) {
            cgm_iterate(x, ctx->r, ctx->p, ctx->Ap, ctx->fr, ctx->cm, ctx->part, ctx->part2, s);
        } else {
            const MeshRec &r = ctx->units()[0];
            cg_step_shared(x, ctx->r, ctx->p, ctx->Ap, ctx->fr, ctx->N_tot, ctx->part,
                           (int)ctx->n_parts, ctx->cg, ctx->part2, ctx->node_sh, r.pd.sh_idx,
                           r.pd.part, s);
        }
    };
    const bool graph = (ctx->opts.flags & FE_OPT_GRAPH) != 0;
    const int gi = graph ? kGraphCgIters : 4;  // iterations per graph replay / per poll at first
    int batch = gi;
    // A context solves with one mass matrix per mesh, so consecutive solves
    // take about as many iterations: the first poll of the device state goes
    // out at the last multiple of gi not past the previous solve's count, the
    // later ones after gi, 2 gi, 4 gi, ... (at most 32) more. Iterations past
    // convergence are launched but return at once.
    int &hint = ctx->cg_hint[lo ? 1 : 0];
    bool hinted = std::min(hint, max_iter) / gi * gi > batch;
    if (hinted) batch = std::min(hint, max_iter) / gi * gi;
    for (;;) {
        if (graph) {
            // kGraphCgIters iterations per replay; finished iterations are no-ops
            for (int k = 0; k < batch; k += kGraphCgIters) {
                const int rc = run_graph(ctx, GraphKey{kActCg, x, nullptr, nullptr, lo ? 1 : 0},
                                         [&](hipStream_t s, bool branch) {
                                             for (int i = 0; i < kGraphCgIters; ++i) {
                                                 mass_enqueue(ctx, ctx->r, ctx->Ap, lo, ctx->p, s, branch,
                                                              !fused);
                                                 step(s);
                                             }
                                         });
                if (rc) return rc;
            }
        } else {
            for (int k = 0; k < batch; ++k) {
                {
                    ScopedTimer tm(ctx, FE_TIMER_MASS);
                    mass_enqueue(ctx, ctx->r, ctx->Ap, lo, ctx->p, ctx->st, false, !fused);
                }
                step(ctx->st);
            }
        }
        HIP_OK(hipGetLastError());
        if (ctx->multi)
            HIP_OK(hipMemcpyAsync(ctx->h_glob, ctx->glob, sizeof(CgGlobal), hipMemcpyDeviceToHost, ctx->st));
        else
            HIP_OK(hipMemcpyAsync(ctx->h_cg, ctx->cg, sizeof(CgState), hipMemcpyDeviceToHost, ctx->st));
        HIP_OK(hipMemcpyAsync(ctx->h_flag, ctx->bad, sizeof(int), hipMemcpyDeviceToHost, ctx->st));
        HIP_OK(hipStreamSynchronize(ctx->st));
        if (*ctx->h_flag) return fail(ctx, FE_EINVAL, "essential DOF index out of range%s");
        if (ctx->multi ? ctx->h_glob->done : ctx->h_cg->done) break;
        if (hinted) {
            batch = gi;
            hinted = false;
        } else if (batch < 32) {
            batch *= 2;
        }
    }
    // the last direction, where the step left it pending
    if (ctx->multi)
        cgm_finish(x, ctx->p, ctx->cm, ctx->st);
    else
        cg_finish(x, ctx->p, n, ctx->cg, ctx->st);
    HIP_OK(hipGetLastError());
    if (ctx->multi) {
        const size_t nm = ctx->mesh.size();
        HIP_OK(hipMemcpyAsync(ctx->h_cgm, ctx->cgm, nm * sizeof(CgState), hipMemcpyDeviceToHost, ctx->st));
        HIP_OK(hipStreamSynchronize(ctx->st));
        out.assign(ctx->h_cgm, ctx->h_cgm + nm);
    } else {
        out.assign(1, *ctx->h_cg);
    }
    hint = 0;
    for (const CgState &c : out) hint = std::max(hint, c.iter);
    return FE_OK;
}

// per mesh (one value for a single-mesh context): ||b_free - Ax_free||^2 (synchronises)
static int resid2_of(fe_ctx *ctx, const double *b, const double *Ax, std::vector<double> &r2)
{
    const long long n = 3 * ctx->N_tot;
    if (ctx->multi) {
        const size_t nm = ctx->mesh.size();
        cgm_resid(b, Ax, ctx->fr, ctx->cm, ctx->part3, ctx->mres, ctx->st);
        HIP_OK(hipMemcpyAsync(ctx->h_mres, ctx->mres, nm * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
        HIP_OK(hipStreamSynchronize(ctx->st));
        r2.assign(ctx->h_mres, ctx->h_mres + nm);
        return FE_OK;
    }
    resid_norm2(b, Ax, ctx->fr, n, ctx->part2, ctx->scal, ctx->st);
    HIP_OK(hipMemcpyAsync(ctx->h_scal, ctx->scal, sizeof(double), hipMemcpyDeviceToHost, ctx->st));
    HIP_OK(hipStreamSynchronize(ctx->st));
    r2.assign(1, *ctx->h_scal);
    return FE_OK;
}

// the same with Ax = M x of the FP64 operator (leaves M x in ctx->Ap)
static int true_resid2(fe_ctx *ctx, const double *b, const double *x, std::vector<double> &r2)
{
    mass_launch(ctx, x, ctx->Ap, false);
    return resid2_of(ctx, b, ctx->Ap, r2);
}

// largest relative residual over the meshes
static double max_rel(const std::vector<double> &r2, const std::vector<double> &bb)
{
    double res = 0.0;
    for (size_t m = 0; m < r2.size(); ++m)
        res = std::max(res, std::sqrt(r2[m] / (bb[m] > 0.0 ? bb[m] : 1.0)));
    return res;
}

extern "C" {

int fe_mass_cg(fe_ctx_t *ctx, const double *b, double *x, const int32_t *ess_dofs, int32_t n_ess,
               double rel_tol, int32_t max_iter, int32_t *iters, double *rel_res)
{
    if (!ctx) return FE_EINVAL;
    if (!b || !x) return fail(ctx, FE_EINVAL, "NULL argument%s");
    if ((const void *)b == (const void *)x) return fail(ctx, FE_EINVAL, "b aliases x%s");
    if (n_ess < 0 || (n_ess > 0 && !ess_dofs)) return fail(ctx, FE_EINVAL, "bad essential DOF list%s");
    if (!(rel_tol >= 0.0) || max_iter < 0) return fail(ctx, FE_EINVAL, "bad tolerance or max_iter%s");
    const long long n = 3 * ctx->N_tot;
    launch_reset_diag(nullptr, ctx->bad, ctx->st);
    cg_mask(ctx->fr, n, ess_dofs, n_ess, ctx->bad, ctx->st);
    cg_mask_apply(x, ctx->fr, n, ctx->st);
    int rc = FE_OK, total = 0;
    bool limit = false;
    double res = 0.0;
    std::vector<CgState> st;
    std::vector<double> r2, bb;
    if (!ctx->lo) {
        if ((rc = cg_run(ctx, b, x, rel_tol, max_iter, false, st))) return rc;
        if ((rc = true_resid2(ctx, b, x, r2))) return rc;
        for (const CgState &s : st) {
            bb.push_back(s.bb);
            total = std::max(total, s.iter);
            limit = limit || s.done == 2;
        }
        res = max_rel(r2, bb);
    } else {
        // iterative refinement: FP64 residual r = b - M x, inner CG on the FP32
        // operator for M d = r to a relative 1e-5 (or rel_tol if looser), x += d
        const double inner_tol = rel_tol > 1e-5 ? rel_tol : 1e-5;
        launch_fill(ctx->ref_d, n, 0.0, ctx->st);
        if ((rc = resid2_of(ctx, b, ctx->ref_d, bb))) return rc;
        for (int sweep = 0;; ++sweep) {
            if ((rc = true_resid2(ctx, b, x, r2))) return rc;  // leaves Ap = M x
            res = max_rel(r2, bb);
            if (res <= rel_tol) break;
            if (total >= max_iter || sweep >= 60) {
                limit = true;
                break;
            }
            vec_sub_masked(b, ctx->Ap, ctx->fr, ctx->ref_r, n, ctx->st);
            launch_fill(ctx->ref_d, n, 0.0, ctx->st);
            if ((rc = cg_run(ctx, ctx->ref_r, ctx->ref_d, inner_tol, max_iter - total, true, st)))
                return rc;
            int inner = 0;
            for (const CgState &s : st) inner = std::max(inner, s.iter);
            total += inner;
            vec_add(x, ctx->ref_d, n, ctx->st);
        }
    }
    ctx->last_iters = total;
    ctx->last_res = res;
    if (iters) *iters = total;
    if (rel_res) *rel_res = res;
    if (limit) return fail(ctx, FE_ENOTCONV, "iteration limit reached%s");
    return FE_OK;
}

int fe_lagrange_step(fe_ctx_t *ctx, double *x, double *v, double *e, const int32_t *ess_dofs,
                     int32_t n_ess, double cfl, double dt_max, double cg_tol, int32_t cg_max_iter,
                     fe_step_info_t *info)
{
    if (!ctx) return FE_EINVAL;
    if (!(ctx->opts.flags & FE_OPT_STEP)) return fail(ctx, FE_EINVAL, "context set up without FE_OPT_STEP%s");
    if (!x || !v || !e) return fail(ctx, FE_EINVAL, "NULL state vector%s");
    if ((const void *)x == (const void *)v) return fail(ctx, FE_EINVAL, "x aliases v%s");
    if (!(cfl > 0.0) || !(dt_max > 0.0)) return fail(ctx, FE_EINVAL, "cfl and dt_max must be > 0%s");
    const long long n3 = 3 * ctx->N_tot;
    hipStream_t st = ctx->st;
    fe_step_info_t out{};
    // the state at the start of the step
    HIP_OK(hipMemcpyAsync(ctx->xs, x, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->vs, v, n3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(ctx->es, e, ctx->L2_tot * sizeof(double), hipMemcpyDeviceToDevice, st));
    auto l2_update = [&](double frac) {
        for (const MeshRec &r : ctx->mesh) {
            const int N = r.p * r.p * r.p;
            launch_rk_l2(ctx->es + r.l2_off, ctx->minv + r.minv_off, ctx->sz + r.l2_off, e + r.l2_off,
                         (long long)r.E * N, N, ctx->dtv, frac, st);
        }
    };
    // stage 1: forces of the state n; dt from its smallest stable point step
    int rc = fe_qdata_update(ctx, ctx->xs, ctx->vs, ctx->es);
    if (rc) return rc;
    launch_step_dt(ctx->min_key, cfl, dt_max, ctx->dtv, st);
    HIP_OK(hipMemcpyAsync(ctx->h_dt, ctx->dtv, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    if ((rc = fe_force_mult_pair(ctx, nullptr, ctx->sy, ctx->vs, ctx->sz))) return rc;
    // the step size is known before any solve: a state with no finite step
    // (still and pressureless, no dt_max) is refused before the CG runs
    HIP_OK(hipStreamSynchronize(st));
    out.dt = ctx->h_dt[0];
    out.dt_est = ctx->h_dt[1];
    if (!(out.dt > 0.0) || !std::isfinite(out.dt))
        return fail(ctx, FE_EINVAL, "no finite positive step (set dt_max)%s");
    int it = 0;
    double res = 0.0;
    rc = fe_mass_cg(ctx, ctx->sy, ctx->acc, ess_dofs, n_ess, cg_tol, cg_max_iter, &it, &res);
    out.cg_iters[0] = it;
    out.cg_rel_res[0] = res;
    if (rc) return rc;
    launch_rk_h1(ctx->vs, ctx->xs, ctx->acc, v, x, nullptr, n3, ctx->dtv, 0.5, st);
    l2_update(0.5);
    // stage 2: forces of the midpoint state; v' and vbar, then e' and x' with vbar
    if ((rc = fe_qdata_update(ctx, x, v, e))) return rc;
    if ((rc = fe_force_mult(ctx, nullptr, ctx->sy))) return rc;
    rc = fe_mass_cg(ctx, ctx->sy, ctx->acc, ess_dofs, n_ess, cg_tol, cg_max_iter, &it, &res);
    out.cg_iters[1] = it;
    out.cg_rel_res[1] = res;
    if (rc) return rc;
    launch_rk_h1(ctx->vs, ctx->xs, ctx->acc, v, x, ctx->vbar, n3, ctx->dtv, 1.0, st);
    if ((rc = fe_force_mult_T(ctx, ctx->vbar, ctx->sz))) return rc;
    l2_update(1.0);
    HIP_OK(hipGetLastError());
    if (info) *info = out;
    return FE_OK;
}

int fe_export_l2_mass_inv(fe_ctx_t *ctx, double *out)
{
    if (!ctx || !out) return FE_EINVAL;
    if (!(ctx->opts.flags & FE_OPT_STEP)) return fail(ctx, FE_EINVAL, "context set up without FE_OPT_STEP%s");
    HIP_OK(hipMemcpyAsync(out, ctx->minv, ctx->minv_len * sizeof(double), hipMemcpyDeviceToDevice, ctx->st));
    HIP_OK(hipStreamSynchronize(ctx->st));
    return FE_OK;
}

int fe_get_diag(fe_ctx_t *ctx, fe_diag_t *diag)
{
    if (!ctx || !diag) return FE_EINVAL;
    HIP_OK(hipMemcpyAsync(ctx->h_key, ctx->min_key, 2 * sizeof(long long), hipMemcpyDeviceToHost, ctx->st));
    HIP_OK(hipMemcpyAsync(ctx->h_flag, ctx->nonfinite, sizeof(int), hipMemcpyDeviceToHost, ctx->st));
    HIP_OK(hipStreamSynchronize(ctx->st));
    diag->min_detj = key_to_double(ctx->h_key[0]);
    diag->dt_est = key_to_double(ctx->h_key[1]);
    diag->nonfinite = *ctx->h_flag;
    diag->cg_iters = ctx->last_iters;
    diag->cg_rel_res = ctx->last_res;
    return FE_OK;
}

int fe_export_qdata(fe_ctx_t *ctx, double *S_out, double *mq_out)
{
    if (!ctx) return FE_EINVAL;
    if (!ctx->uniform_pq) return fail(ctx, FE_EINVAL, "export needs one (order, q1d) for all meshes%s");
    for (const MeshRec &r : ctx->mesh) {
        const int Q3 = r.Q * r.Q * r.Q;
        // batched form: the mesh's element ids are already global (one order, so
        // L2 element index = caller element index); otherwise mesh-local
        const long long e0 = ctx->batched ? 0 : r.elem_off;
        if (S_out && ctx->bf)
            launch_unpermute_s_bf16(S_of(ctx, r), r.pd.perm, r.E, Q3, (Q3 + 31) / 32 * 32,
                                    S_out + e0 * 9 * Q3, ctx->st);
        else if (S_out)
            launch_unpermute_rows(S_of(ctx, r), ctx->lo, r.pd.perm, r.E, 9 * Q3,
                                  S_out + e0 * 9 * Q3, ctx->st);
        if (mq_out)
            launch_unpermute_rows(ctx->mq + r.mq_off, false, r.pd.perm, r.E, Q3, mq_out + e0 * Q3,
                                  ctx->st);
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(ctx->st));
    return FE_OK;
}

int fe_timer_read(fe_ctx_t *ctx, int32_t which, double *total_ms, int64_t *count)
{
    if (!ctx || which < 0 || which >= FE_TIMER_COUNT) return FE_EINVAL;
    if (!(ctx->opts.flags & FE_OPT_TIMERS)) return fail(ctx, FE_EINVAL, "timers are off%s");
    HIP_OK(hipStreamSynchronize(ctx->st));
    TimerPool &tp = ctx->timers[which];
    double ms = tp.folded_ms;
    for (size_t k = 0; k < tp.used; ++k) {
        float t = 0.f;
        HIP_OK(hipEventElapsedTime(&t, tp.ev[k].first, tp.ev[k].second));
        ms += t;
    }
    if (total_ms) *total_ms = ms;
    if (count) *count = tp.count;
    return FE_OK;
}

int fe_timer_reset(fe_ctx_t *ctx)
{
    if (!ctx) return FE_EINVAL;
    HIP_OK(hipStreamSynchronize(ctx->st));
    for (auto &tp : ctx->timers) {
        tp.used = 0;
        tp.folded_ms = 0.0;
        tp.count = 0;
    }
    return FE_OK;
}

}  // extern "C"
