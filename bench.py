"""Benchmark of the PA Lagrange-phase hot path on one MI355X.

One step = the whole hot path over a Taylor-Green workload with inputs resident
in HBM: one quadrature-data update, 50 x (F.1 + F^T.v, both from one read of S
through fe_force_mult_pair), and one mass CG solve to a 1e-12 relative
residual (v.n = 0 on the boundary). The single actions are timed separately.

value = kinematic DOFs processed by force actions per second of the whole
step, 3N x 100 / t_step / 1e9 (GDOF/s; the CG and qdata time count against
it). The roofline object rates the dominant kernel (
the step's force work: the fused F.1 + F^T.v launch) by algorithmic bytes per
launch over its mean duration, measured with HIP events recorded by the
library on its own stream.

Workloads: c2 (default) 48^3 Q2-Q1; c3 24^3 Q4-Q3; c4 64^3 Q3-Q2 (with
--precision fp64|fp32|bf16, the precision form); c5 the 256-mesh uneven batch
(4^3..24^3 elements, p 1..4, Q = p+2) run as one batched, graph-replayed
context and, for comparison, as per-mesh launches of the plain path.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2|c3|c4|c5]
                       [--precision fp64|fp32|bf16]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

CONFIGS = {
    # name: (n, p, Q, label)
    "c2": (48, 2, 4, "48^3 hex, H1 Q2 / L2 Q1, 4^3 Gauss points, every node +-0.1h (seeded "
                     "uniform), Taylor-Green, seed 0"),
    "c3": (24, 4, 6, "24^3 hex, H1 Q4 / L2 Q3, 6^3 Gauss points, vertices +-0.05h (seeded uniform), "
                     "other nodes on the trilinear map plus +-0.025h, Taylor-Green, seed 0"),
    "c4": (64, 3, 5, "64^3 hex, H1 Q3 / L2 Q2, 5^3 Gauss points, every node +-0.05h (seeded "
                     "uniform), Taylor-Green, seed 0"),
    "c5": (None, None, None, "256 perturbed cubes, 4^3..24^3 elements, H1 Q1..Q4, Q = p+2, every "
                             "node +-0.1h (p <= 2), 0.05h (p = 3), 0.025h (p = 4), Taylor-Green, "
                             "seeds 1000..1255"),
}
# vertex perturbation (in h) of the workloads that perturb vertices and
# high-order nodes separately
VERTEX_AMP = {"c3": 0.05}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
N_PAIRS = 50
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes scaled by a plain 1 GiB copy (fetch x2, write x1), and the
# SHA-256 prefixes of the kernel sources and tile table they were taken with:
# reported only while those are unchanged (profiles/c2_fp64_step.md,
# profiles/c4_step.md).
TRAFFIC = {
    ("c2", "fp64"): {"action": "pair", "kernel": "k_force_pair<3,4,ONE,double,2>", "bytes": 614.8e6,
                     "src": {"kern_fp64.hip": "0eef1e45315ca80c", "kern_common.hpp": "81135cc579cad6ef",
                             "tune_table.inc": "971665e72d09a781"}},
    ("c4", "fp64"): {"action": "pair", "kernel": "k_force_pair<4,5,ONE,double,4>", "bytes": 3337.6e6,
                     "src": {"kern_fp64.hip": "0eef1e45315ca80c", "kern_common.hpp": "81135cc579cad6ef",
                             "tune_table.inc": "971665e72d09a781"}},
}


def measured_traffic(config, precision, action):
    import hashlib
    rec = TRAFFIC.get((config, precision))
    if rec is None or rec["action"] != action:
        return None
    src = os.path.join(HERE, "paper_2112_07075_amd", "csrc")
    for name, sha in rec["src"].items():
        with open(os.path.join(src, name), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest()[:16] != sha:
                return None
    return rec["bytes"] / 1e6


def algorithmic_bytes(E, N, p, Q):
    """Bytes the PA action must move (stored S, unique-DOF vectors, map)."""
    Q3, D3, Dl3 = Q ** 3, (p + 1) ** 3, p ** 3
    S = 9 * Q3 * E * 8
    return {
        "force_1": S + 3 * N * 8 + D3 * E * 4,
        "force_e": S + Dl3 * E * 8 + 3 * N * 8 + D3 * E * 4,
        "force_T": S + 3 * N * 8 + Dl3 * E * 8 + D3 * E * 4,
        # F.1 and F^T.v from one read of S: S, v in, y and z out, the map
        "pair": S + 2 * 3 * N * 8 + Dl3 * E * 8 + D3 * E * 4,
        "mass": Q3 * E * 8 + 2 * 3 * N * 8 + D3 * E * 4,
        "qdata": 2 * 3 * N * 8 + Dl3 * E * 8 + Q3 * E * 8 + D3 * E * 4 + S,
    }


def host_cpu():
    """CPU model name and logical core count of the host the bench runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline_allcore(meshes, qs, fields, threads, budget_s=10.0):
    """The same oracle calls on every thread at once: each thread applies F.1 and
    F^T.v over its own slice of an element sample into a private output (the
    oracle releases the GIL inside its C calls); the slices' outputs would be
    summed, which is not timed. Scaled per element to the whole workload."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor
    classes = {}
    for m, Q, f in zip(meshes, qs, fields):
        classes.setdefault((m.p, Q), (m, f))
    per_elem, notes = {}, []
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for (p, Q), (mesh, (v, e)) in classes.items():
            E, N = mesh.n_elem, mesh.n_nodes
            k = min(64 * threads, E)
            while True:
                el = np.arange(k, dtype=np.int32)
                S = O.qdata(mesh.elem_nodes, p, Q, N, mesh.x0, mesh.x0, v, e, elems=el,
                            want=("S",))["S"]
                parts = np.array_split(el, threads)

                def work(part, S=S, v=v, p=p, Q=Q, N=N, mesh=mesh):
                    O.force_mult(mesh.elem_nodes, p, Q, N, S, None, elems=part)
                    O.force_mult_T(mesh.elem_nodes, p, Q, N, S, v, elems=part)

                t1 = time.perf_counter()
                list(ex.map(work, parts))
                t2 = time.perf_counter()
                if (t2 - t1) > budget_s / (4 * len(classes)) or k * 2 > E:
                    break
                k *= 2
            per_elem[(p, Q)] = (t2 - t1) / k
            notes.append(f"p={p},Q={Q}: first {k} of {E} elements in {threads} slices, {t2 - t1:.2f} s")
    pair_s = sum(per_elem[(m.p, Q)] * m.n_elem for m, Q in zip(meshes, qs))
    dofs = sum(3 * m.n_nodes for m in meshes)
    return {"value": dofs * 2 / pair_s / 1e9, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
            "sample": "F.1 + F^T.v on " + "; ".join(notes) + ", scaled per element to the workload"}


def cpu_baseline(meshes, qs, fields, budget_s=12.0):
    """The plain oracle (single thread) on a bounded element sample: F.1 and F^T.v
    over the first k elements of the first mesh of every (p, Q) class, scaled to
    GDOF/s of the whole workload (qdata on the sample is timed but excluded)."""
    import oracle as O
    classes = {}
    for m, Q, f in zip(meshes, qs, fields):
        classes.setdefault((m.p, Q), (m, f))
    per_elem, notes, t_q = {}, [], 0.0
    for (p, Q), (mesh, (v, e)) in classes.items():
        E, N = mesh.n_elem, mesh.n_nodes
        k = min(64, E)
        while True:
            el = np.arange(k, dtype=np.int32)
            t0 = time.perf_counter()
            S = O.qdata(mesh.elem_nodes, p, Q, N, mesh.x0, mesh.x0, v, e, elems=el,
                        want=("S",))["S"]
            t1 = time.perf_counter()
            O.force_mult(mesh.elem_nodes, p, Q, N, S, None, elems=el)
            O.force_mult_T(mesh.elem_nodes, p, Q, N, S, v, elems=el)
            t2 = time.perf_counter()
            if (t2 - t0) > budget_s / (4 * len(classes)) or k * 2 > E:
                break
            k *= 2
        per_elem[(p, Q)] = (t2 - t1) / k
        t_q += t1 - t0
        notes.append(f"p={p},Q={Q}: first {k} of {E} elements, {t2 - t1:.2f} s")
    pair_s = sum(per_elem[(m.p, Q)] * m.n_elem for m, Q in zip(meshes, qs))
    dofs = sum(3 * m.n_nodes for m in meshes)
    return {"value": dofs * 2 / pair_s / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": "F.1 + F^T.v on " + "; ".join(notes) +
                      f" (qdata on the samples {t_q:.2f} s, excluded), scaled per element to "
                      "the whole workload"}


def precision_errors(torch, fe, run, meshes, qs, fields, W):
    """max |y_form - y_fp64| / max |y_fp64| for F.1, F.e, F^T.v, M x and the CG
    solution of the same right-hand side (the form's CG runs refinement to 1e-12).
    F^T.v of the divergence-free Taylor-Green velocity is a near cancellation, so
    its error is large relative to the output; the tests bound every output on
    the scale of the summed term magnitudes instead."""
    ref = Runner(torch, fe, W, meshes, qs, fields, fe.Opts(flags=0))
    outs = []
    for r in (run, ref):
        fe.fe_qdata_update(r.ctx, r.x0, r.v, r.e)
        o = {}
        fe.fe_force_mult(r.ctx, None, r.y)
        o["F.1"] = r.y.clone()
        fe.fe_force_mult(r.ctx, r.e, r.y)
        o["F.e"] = r.y.clone()
        fe.fe_force_mult_T(r.ctx, r.v, r.z)
        o["F^T.v"] = r.z.clone()
        fe.fe_mass_mult(r.ctx, r.v, r.y)
        o["M.x"] = r.y.clone()
        outs.append(o)
    # the solve on the same right-hand side (the FP64 path's -F.1) in both contexts
    b = -outs[1]["F.1"]
    for r, o in ((run, outs[0]), (ref, outs[1])):
        r.a.zero_()
        fe.fe_mass_cg(r.ctx, b, r.a, r.ess, rel_tol=1e-12, max_iter=5000)
        o["CG x (same b)"] = r.a.clone()
    err = {k: (outs[0][k] - outs[1][k]).abs().max().item() / outs[1][k].abs().max().item()
           for k in outs[1]}
    del ref
    return {k: float(f"{v:.3e}") for k, v in err.items()}


def mf_flops(p, Q):
    """FP64 operations per element of the matrix-free pair kernel as written:
    forward x, y, z stages of six fields, the per-point algebra (counted from
    the kernel: cofactors, inverse, velocity gradient, strain, viscosity,
    S = w detJ sigma J^-T, the F^T v integrand), the transposed stages of three
    components and the L2 stages of F^T v (multiply-add = 2)."""
    D, Dl = p + 1, p
    fwd = 2 * (2 * D ** 3 * Q + 3 * D ** 2 * Q ** 2 + 3 * D * Q ** 3)
    point = 27 + 9 + 5 + 45 + 18 + 4 + 8 + 9 * 8 + 3 + 18 + 9 * 3 * 2
    trans = 2 * (3 * D * Q ** 3 + 3 * D ** 2 * Q ** 2 // 1 + 2 * D ** 3 * Q)
    l2 = 2 * (Dl * Q ** 3 + Dl ** 2 * Q ** 2 + Dl ** 3 * Q)
    einterp = 2 * (Dl ** 3 * Q * Q + Dl * Q ** 3)
    return 6 * fwd + point * Q ** 3 + 3 * trans + l2 + einterp


def time_calls(torch, fn, reps=20, warm=3):
    """Mean milliseconds of fn() over reps calls on the current stream (HIP events)."""
    for _ in range(warm):
        fn()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def extra_rows(torch, fe, W, mesh, Q, fields):
    """The operators beyond the force pair, timed on the same single-mesh
    workload: the stiffness (diffusion) action of the hyper-viscosity term, the
    fully matrix-free force pair (against stored-S qdata + pair), two materials
    (their qdata and every material's F_k^T v), the full Lagrange step, and the
    pair, F 1 and M x in both scatter modes."""
    dev = torch.device("cuda:0")
    p, E, N = mesh.p, mesh.n_elem, mesh.n_nodes
    Q3, D3, Dl3 = Q ** 3, (p + 1) ** 3, p ** 3
    v = torch.from_numpy(fields[0]).to(dev)
    e = torch.from_numpy(fields[1].ravel()).to(dev)
    x0 = torch.from_numpy(mesh.x0).to(dev)
    x = x0 + (0.05 / mesh.n) * v
    y = torch.empty((3, N), dtype=torch.float64, device=dev)
    z = torch.empty(E * Dl3, dtype=torch.float64, device=dev)
    desc = fe.MeshDesc(mesh.elem_nodes, x0, p, Q)
    rows = {}

    def rate(bytes_, ms):
        gbs = bytes_ / (ms * 1e-3) / 1e9
        return {"us": round(ms * 1e3, 2), "algorithmic_MB": round(bytes_ / 1e6, 1),
                "GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}

    # stiffness: Dk (6 Q^3 per element) + u in + y out + map
    ctx = fe.fe_pa_setup(desc, fe.Opts(flags=fe.FE_OPT_STIFF))
    ms_q = time_calls(torch, lambda: fe.fe_stiffness_update(ctx, x))
    ms_k = time_calls(torch, lambda: fe.fe_stiffness_mult(ctx, v, y))
    rows["stiffness"] = {"action": rate(6 * Q3 * E * 8 + 2 * 3 * N * 8 + D3 * E * 4, ms_k),
                         "qdata": rate(3 * N * 8 + 6 * Q3 * E * 8 + D3 * E * 4, ms_q),
                         "gdof_s": round(3 * N / (ms_k * 1e-3) / 1e9, 2)}
    del ctx
    # matrix-free pair vs qdata + stored-S pair
    ctx = fe.fe_pa_setup(desc, fe.Opts())
    try:
        ms_mf = time_calls(torch, lambda: fe.fe_force_mult_pair_mf(ctx, x, v, e, y, z))
        ms_pa = time_calls(torch, lambda: (fe.fe_qdata_update(ctx, x, v, e),
                                           fe.fe_force_mult_pair(ctx, None, y, v, z)))
        b = 2 * 3 * N * 8 + Dl3 * E * 8 + Q3 * E * 8 + 3 * N * 8 + Dl3 * E * 8 + D3 * E * 4
        fl = mf_flops(p, Q) * E
        r = rate(b, ms_mf)
        r.update(gflops=round(fl / (ms_mf * 1e-3) / 1e9, 1), flop_per_elem=mf_flops(p, Q),
                 frac_fp64=round(fl / (ms_mf * 1e-3) / 78.6e12, 4),
                 pa_qdata_plus_pair_us=round(ms_pa * 1e3, 2),
                 speedup_vs_pa=round(ms_pa / ms_mf, 3),
                 gdof_s=round(3 * N * 2 / (ms_mf * 1e-3) / 1e9, 2))
        rows["matrix_free_pair"] = r
    except fe.FepaError as err:
        rows["matrix_free_pair"] = {"unsupported": str(err)}
    del ctx
    # two materials: fractions 0.3 / 0.7, energies e and 1.5 e
    eta = torch.cat([torch.full_like(e, 0.3), torch.full_like(e, 0.7)]).contiguous()
    ctx = fe.fe_pa_setup(desc, fe.Opts(materials=fe.Materials([5.0 / 3.0, 1.4], [1.0, 4.0], eta)))
    e2 = torch.cat([e, 1.5 * e]).contiguous()
    z2 = torch.empty(2 * E * Dl3, dtype=torch.float64, device=dev)
    ms_qm = time_calls(torch, lambda: fe.fe_qdata_update_mm(ctx, x, v, e2), reps=5)
    ms_zm = time_calls(torch, lambda: fe.fe_force_mult_T_mm(ctx, v, z2))
    ms_y = time_calls(torch, lambda: fe.fe_force_mult(ctx, None, y))
    S = 9 * Q3 * E * 8
    rows["multimaterial_2"] = {
        "qdata_mm": rate(2 * (2 * 3 * N * 8 + Dl3 * E * 8 + Q3 * E * 8 + D3 * E * 4 + S) + 3 * S, ms_qm),
        "force_T_mm": rate(2 * (S + 3 * N * 8 + Dl3 * E * 8 + D3 * E * 4), ms_zm),
        "force_1_sum": rate(S + 3 * N * 8 + D3 * E * 4, ms_y)}
    del ctx
    # the full Lagrange step (two stages: 2 qdata, pair + F 1 + F^T vbar, 2 CG)
    ctx = fe.fe_pa_setup(desc, fe.Opts(flags=fe.FE_OPT_STEP | fe.FE_OPT_GRAPH))
    ess = torch.from_numpy(W.boundary_normal_dofs(mesh).astype(np.int32)).to(dev)
    xs, vs, es = x0.clone(), v.clone(), e.clone()
    info = fe.fe_lagrange_step(ctx, xs, vs, es, ess, cfl=0.5, cg_tol=1e-12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nstep = 3
    for _ in range(nstep):
        info = fe.fe_lagrange_step(ctx, xs, vs, es, ess, cfl=0.5, cg_tol=1e-12)
    ms_step = (time.perf_counter() - t0) * 1e3 / nstep
    rows["lagrange_step"] = {"ms": round(ms_step, 3), "dt": info["dt"], "cg_iters": list(info["cg_iters"]),
                             "gdof_s": round(3 * N / (ms_step * 1e-3) / 1e9, 3)}
    del ctx
    # the two scatter modes of R^T: ordered patch partials (default) and
    # device-scope atomics (FE_OPT_ATOMIC), same tile shapes
    modes = {}
    for name, fl in (("partials", 0), ("atomic", fe.FE_OPT_ATOMIC)):
        ctx = fe.fe_pa_setup(desc, fe.Opts(flags=fl))
        fe.fe_qdata_update(ctx, x, v, e)
        ms_p = time_calls(torch, lambda: fe.fe_force_mult_pair(ctx, None, y, v, z))
        ms_f = time_calls(torch, lambda: fe.fe_force_mult(ctx, None, y))
        ms_m = time_calls(torch, lambda: fe.fe_mass_mult(ctx, v, y))
        modes[name] = {"pair_us": round(ms_p * 1e3, 2), "force_1_us": round(ms_f * 1e3, 2),
                       "mass_us": round(ms_m * 1e3, 2)}
        del ctx
    rows["scatter_modes"] = modes
    return rows


def finite(obj):
    """NaN (a timer with no launches, e.g. inside replayed graphs) -> null."""
    if isinstance(obj, dict):
        return {k: finite(v) for k, v in obj.items()}
    if isinstance(obj, (list, tuple)):
        return [finite(v) for v in obj]
    if isinstance(obj, float) and obj != obj:
        return None
    return obj


def build_workload(config, W):
    """(meshes, q1d per mesh, (v, e) per mesh, label)"""
    if config == "c5":
        items = W.batch_meshes(256)
        meshes = [b.mesh for b in items]
        qs = [b.q1d for b in items]
    else:
        n, p, Q, _ = CONFIGS[config]
        meshes = [W.cube_mesh(n, p, W.default_amp(p), seed=0, vertex_amp=VERTEX_AMP.get(config))]
        qs = [Q]
    fields = [W.taylor_green_fields(m) for m in meshes]
    return meshes, qs, fields, CONFIGS[config][3]


class Runner:
    """One context over the workload's meshes and the vectors of one step."""

    def __init__(self, torch, fe, W, meshes, qs, fields, opts):
        dev = torch.device("cuda:0")
        self.torch, self.fe = torch, fe
        noff = np.concatenate([[0], np.cumsum([m.n_nodes for m in meshes])]).astype(np.int64)
        self.Ntot = int(noff[-1])
        self.x0 = torch.from_numpy(np.concatenate([m.x0 for m in meshes], axis=1)).to(dev)
        descs = [fe.MeshDesc(m.elem_nodes, self.x0[:, noff[k]:noff[k + 1]].contiguous(), m.p, qs[k])
                 for k, m in enumerate(meshes)]
        self.ctx = fe.fe_pa_setup(descs, opts)
        del descs
        _, _, loff = fe.fe_mesh_offsets(self.ctx)
        self.L2 = fe.fe_query(self.ctx)["l2_size_total"]
        self.v = torch.from_numpy(np.concatenate([f[0] for f in fields], axis=1)).to(dev)
        eh = np.zeros(self.L2)
        ess = []
        for k, (m, f) in enumerate(zip(meshes, fields)):
            eh[loff[k]:loff[k] + f[1].size] = f[1].ravel()
            idx = W.boundary_normal_dofs(m)
            ess.append((idx // m.n_nodes) * self.Ntot + noff[k] + idx % m.n_nodes)
        self.e = torch.from_numpy(eh).to(dev)
        self.ess = torch.from_numpy(np.concatenate(ess).astype(np.int32)).to(dev)
        self.y = torch.empty((3, self.Ntot), dtype=torch.float64, device=dev)
        self.z = torch.empty(self.L2, dtype=torch.float64, device=dev)
        self.a = torch.zeros((3, self.Ntot), dtype=torch.float64, device=dev)
        self.cg = {}

    def step(self):
        fe, t = self.fe, self.torch
        fe.fe_qdata_update(self.ctx, self.x0, self.v, self.e)
        for _ in range(N_PAIRS):
            # F.1 (momentum) and F^T.v (energy) of one stage, from one read of S
            fe.fe_force_mult_pair(self.ctx, None, self.y, self.v, self.z)
        # momentum equation M_v a = -F.1, a = 0 on v.n = 0 DOFs
        t.neg(self.y, out=self.y)
        self.a.zero_()
        rc, it, rr = fe.fe_mass_cg(self.ctx, self.y, self.a, self.ess, rel_tol=1e-12, max_iter=5000)
        self.cg.update(iters=it, rel_res=rr)

    def time(self, steps, warmup):
        t, fe = self.torch, self.fe
        for _ in range(warmup):
            self.step()
        t.cuda.synchronize()
        fe.fe_timer_reset(self.ctx)
        t.cuda.synchronize()
        t0 = time.perf_counter()
        marks = []
        for _ in range(steps):
            self.step()  # ends in the CG solve, which synchronises the stream
            marks.append(time.perf_counter())
        t.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / steps
        self.step_times = np.diff(np.concatenate([[t0], marks]))
        per = {}
        for name, which in (("qdata", fe.FE_TIMER_QDATA), ("pair", fe.FE_TIMER_PAIR)):
            ms, cnt = fe.fe_timer_read(self.ctx, which)
            per[name] = (ms / cnt if cnt else float("nan"), ms)
        # the single actions and the mass action, timed after the steps (not part
        # of a step; inside the step the CG's mass launches run in graphs)
        fe.fe_timer_reset(self.ctx)
        for _ in range(10):
            fe.fe_force_mult(self.ctx, None, self.y)
            fe.fe_force_mult_T(self.ctx, self.v, self.z)
            fe.fe_mass_mult(self.ctx, self.v, self.a)
        t.cuda.synchronize()
        for name, which in (("force_1", fe.FE_TIMER_FORCE), ("force_T", fe.FE_TIMER_FORCE_T),
                            ("mass", fe.FE_TIMER_MASS)):
            ms, cnt = fe.fe_timer_read(self.ctx, which)
            per[name] = (ms / cnt if cnt else float("nan"), ms)
        # the CG solve of the step on its own (synchronous call): time per iteration
        rhs = -self.y
        fe.fe_force_mult(self.ctx, None, self.y)
        t.neg(self.y, out=rhs)
        solves = []
        for _ in range(3):
            self.a.zero_()
            t.cuda.synchronize()
            c0 = time.perf_counter()
            _, it, _ = fe.fe_mass_cg(self.ctx, rhs, self.a, self.ess, rel_tol=1e-12, max_iter=5000)
            solves.append(((time.perf_counter() - c0) * 1e3, it))
        ms_solve = float(np.median([a for a, _ in solves]))
        self.cg.update(ms_per_solve=round(ms_solve, 3),
                       us_per_iter=round(ms_solve * 1e3 / max(1, solves[0][1]), 2))
        return step_s, per


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--precision", default="fp64", choices=sorted(PRECISIONS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the timing of the stiffness, matrix-free, multi-material and step operators")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the PA path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2112_07075_amd as fe
    from paper_2112_07075_amd import workload as W

    if args.copy_calib:
        # reads 1 GiB and writes 1 GiB per launch: the reference for FETCH_SIZE/WRITE_SIZE
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        ev0.record()
        for _ in range(reps):
            dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        # a read-only pass: the sum streams 1 GiB
        s_ = src.sum()
        ev0.record()
        for _ in range(reps):
            s_ = src.sum()
        ev1.record()
        torch.cuda.synchronize()
        ms_r = ev0.elapsed_time(ev1) / reps
        print(json.dumps({"copy_calib_bytes_each_way": src.numel() * 8, "launches": 3 + reps,
                          "copy_GBps": 2 * src.numel() * 8 / (ms * 1e-3) / 1e9,
                          "read_GBps": src.numel() * 8 / (ms_r * 1e-3) / 1e9}))
        return

    if args.precision != "fp64" and args.config == "c5":
        print("the batch workload runs the plain FP64 path", file=sys.stderr)
        sys.exit(2)
    meshes, qs, fields, label = build_workload(args.config, W)
    E = sum(m.n_elem for m in meshes)
    N = sum(m.n_nodes for m in meshes)
    # groups of 8 CG iterations (launch-bound: three short kernels per iteration)
    # and the actions of several-unit contexts are replayed from captured hipGraphs;
    # the library launches a one-unit action directly
    base = fe.FE_OPT_TIMERS | fe.FE_OPT_GRAPH
    flags = base | (fe.FE_OPT_BATCHED if args.config == "c5" else 0)
    run = Runner(torch, fe, W, meshes, qs, fields,
                 fe.Opts(precision=PRECISIONS[args.precision], flags=flags))
    step_s, per = run.time(args.steps, args.warmup)
    ab = {}
    for m, Q in zip(meshes, qs):
        for k, b in algorithmic_bytes(m.n_elem, m.n_nodes, m.p, Q).items():
            ab[k] = ab.get(k, 0) + b
    if args.precision != "fp64":
        # S and m_q are stored in 4 (FP32) or 2 (BF16) bytes instead of 8
        rs = 4 if args.precision == "fp32" else 2
        for m, Q in zip(meshes, qs):
            S = 9 * Q ** 3 * m.n_elem
            for k in ("force_1", "force_e", "force_T", "pair", "qdata"):
                ab[k] -= S * (8 - rs)
            ab["mass"] -= Q ** 3 * m.n_elem * 4  # m_q in FP32 (both forms)
    if per["pair"][1] == 0.0:  # a form without the fused kernel runs the two actions
        per["pair"] = (per["force_1"][0] + per["force_T"][0], per["force_1"][1] + per["force_T"][1])
    dom = "pair"  # the force work of a step is the fused pair
    achieved = ab[dom] / (per[dom][0] * 1e-3) / 1e9
    diag = fe.fe_get_diag(run.ctx)
    order = meshes[0].p if len(meshes) == 1 else "1..4"
    out = {
        "metric": "F.1 + F^T.v action GDOF/s and % HBM roofline",
        "value": 3 * N * 2 * N_PAIRS / step_s / 1e9,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[args.precision],
        "data": "synthetic (seeded perturbed unit cubes, Taylor-Green fields)",
        "config": {
            "workload": f"{args.config.upper()}: {label}; step = qdata + {N_PAIRS} x (F.1 + F^T.v,"
                        f" fused) + mass CG to 1e-12",
            "meshes": len(meshes), "elements": E, "h1_dofs": 3 * N, "order": order,
            "precision": args.precision, "parallelism": "single GPU",
            "launch": ("batched, actions and CG groups replayed from hipGraphs" if args.config == "c5"
                       else "direct action launches, CG groups replayed from hipGraphs"),
        },
        "ms_per_step_median": round(float(np.median(run.step_times)) * 1e3, 3),
        "ms_per_step_min_max": [round(float(run.step_times.min()) * 1e3, 3),
                                round(float(run.step_times.max()) * 1e3, 3)],
        "kernels_us": {k: round(vv[0] * 1e3, 2) for k, vv in per.items()},
        "kernels_gbs": {k: round(ab[k] / (per[k][0] * 1e-3) / 1e9, 1) for k in per},
        "force_pair_gdof_s": 3 * N * 2 / (per["pair"][0] * 1e-3) / 1e9,
        "single_actions_gdof_s": 3 * N * 2 / ((per["force_1"][0] + per["force_T"][0]) * 1e-3) / 1e9,
        "cg": {"iters": run.cg.get("iters"), "true_rel_res": run.cg.get("rel_res"),
               "mass_us": round(per["mass"][0] * 1e3, 2), "ms_per_solve": run.cg.get("ms_per_solve"),
               "us_per_iter": run.cg.get("us_per_iter")},
        "min_detj": diag["min_detj"],
        "roofline": {"bound": "hbm", "kernel": dom,
                     "timed": "whole action: k_force_pair (or k_force + k_force_t) + k_gather_shared, "
                              "HIP events around every action of the timed steps",
                     "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.config, args.precision, dom),
                     "traffic_unit": "MB per launch", "algorithmic_MB": round(ab[dom] / 1e6, 1)},
    }
    if args.config == "c3":
        # the pair's working set (272.8 MB) is about the 256 MB Infinity Cache:
        # time the pair again over four contexts (four copies of S) in turn
        ctxs = [run] + [Runner(torch, fe, W, meshes, qs, fields, fe.Opts(flags=flags)) for _ in range(3)]
        for c in ctxs:
            fe.fe_qdata_update(c.ctx, c.x0, c.v, c.e)
        k = [0]

        def rotated_pair():
            c = ctxs[k[0] % 4]
            k[0] += 1
            fe.fe_force_mult_pair(c.ctx, None, c.y, c.v, c.z)

        ms_rot = time_calls(torch, rotated_pair, reps=40, warm=4)
        ach = ab[dom] / (ms_rot * 1e-3) / 1e9
        out["roofline_rotated_S_x4"] = {"kernel": dom, "us": round(ms_rot * 1e3, 2),
                                        "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                                        "timed": "HIP events around 40 pair actions cycling over four "
                                                 "contexts of the same mesh"}
        del ctxs
    if args.precision != "fp64":
        # the same outputs from the FP64 path (which matches the oracle to 1e-12):
        # error of every output of the precision form, relative to max |FP64 output|
        out["error_vs_fp64"] = precision_errors(torch, fe, run, meshes, qs, fields, W)
    if args.config == "c5":
        # the same step as per-mesh launches of the plain path (one context, no batching)
        del run
        torch.cuda.empty_cache()
        plain = Runner(torch, fe, W, meshes, qs, fields, fe.Opts(flags=fe.FE_OPT_TIMERS))
        p_step, p_per = plain.time(max(1, args.steps // 2), 1)
        out["per_mesh_plain"] = {"value": 3 * N * 2 * N_PAIRS / p_step / 1e9,
                                 "ms_per_step": p_step * 1e3,
                                 "kernels_us": {k: round(vv[0] * 1e3, 2) for k, vv in p_per.items()}}
        out["batched_speedup"] = round(p_step / step_s, 3)
        del plain
    if len(meshes) == 1 and args.precision == "fp64" and not args.no_rows:
        del run
        torch.cuda.empty_cache()
        out["rows"] = extra_rows(torch, fe, W, meshes[0], qs[0], fields[0])
    if not args.no_cpu_baseline:
        model, ncpu = host_cpu()
        out["cpu_baseline"] = cpu_baseline(meshes, qs, fields)
        out["cpu_baseline"].update(host_cpu=model, host_logical_cores=ncpu)
        # all host cores (at most 16: the CPU share of one GPU on the GPU machines)
        threads = max(1, min(16, ncpu))
        out["cpu_baseline_allcore"] = cpu_baseline_allcore(meshes, qs, fields, threads)
        out["cpu_baseline_allcore"].update(host_cpu=model, host_logical_cores=ncpu)
    print(json.dumps(finite(out)))


if __name__ == "__main__":
    main()
