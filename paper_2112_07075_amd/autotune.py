"""Autotuner of the patch-kernel tile shapes.

For one workload (order p, points Q, precision) it sweeps the elements per
patch and the waves per workgroup of the F.1, F^T.v, M x and fused F.1 + F^T.v
kernels, times each action with the library's event timers on the GPU, and
writes the fastest choice as one line "p Q precision nw_force nw_force_t
nw_mass patch nw_pair" of a tuning table. fe_pa_setup reads that table when the environment variable
FEPA_TUNE_TABLE names it (explicit fe_opts_t tune fields take precedence).

The --builtin mode tunes every (p, Q) pair in FP64 and the Q = p+2 pairs in
FP32 and BF16, each on a Taylor-Green cube of about 2.7M velocity DOFs (the
benchmark workloads' own sizes where they exist), and writes the rows as the
C++ initialiser file that the library compiles in as its default table
(paper_2112_07075_amd/csrc/tune_table.inc).

Usage: python -m paper_2112_07075_amd.autotune --n 48 --p 2 --q 4 --out tune.txt
       python -m paper_2112_07075_amd.autotune --builtin path/to/tune_table.inc
"""
from __future__ import annotations

import argparse
import functools
import json
import os
import sys

WAVES = (2, 4, 8)


def patch_choices(p: int):
    return {1: (32, 64, 128, 256), 2: (16, 32, 48, 64)}.get(p, (4, 6, 8))


def time_actions(fe, torch, mesh, p, Q, precision, nw, patch, reps=20):
    dev = torch.device("cuda:0")
    x0 = torch.from_numpy(mesh.x0).to(dev)
    from . import workload as W
    v_np, e_np = W.taylor_green_fields(mesh)
    v, e = torch.from_numpy(v_np).to(dev), torch.from_numpy(e_np).to(dev)
    ctx = fe.fe_pa_setup(fe.MeshDesc(mesh.elem_nodes, x0, p, Q),
                         fe.Opts(precision=precision, flags=fe.FE_OPT_TIMERS, tune_nw_force=nw,
                                 tune_nw_force_t=nw, tune_nw_mass=nw, tune_patch=patch))
    fe.fe_qdata_update(ctx, x0, v, e)
    y = torch.empty((3, mesh.n_nodes), dtype=torch.float64, device=dev)
    z = torch.empty((mesh.n_elem, p ** 3), dtype=torch.float64, device=dev)
    for _ in range(3):
        fe.fe_force_mult(ctx, None, y)
        fe.fe_force_mult_T(ctx, v, z)
        fe.fe_mass_mult(ctx, v, y)
        fe.fe_force_mult_pair(ctx, None, y, v, z)
    fe.fe_timer_reset(ctx)
    for _ in range(reps):
        fe.fe_force_mult(ctx, None, y)
        fe.fe_force_mult_T(ctx, v, z)
        fe.fe_mass_mult(ctx, v, y)
        fe.fe_force_mult_pair(ctx, None, y, v, z)
    out = {}
    for name, which in (("force", fe.FE_TIMER_FORCE), ("force_t", fe.FE_TIMER_FORCE_T),
                        ("mass", fe.FE_TIMER_MASS), ("pair", fe.FE_TIMER_PAIR)):
        ms, cnt = fe.fe_timer_read(ctx, which)
        out[name] = ms / cnt * 1e3 if cnt else float("nan")
    if out["pair"] != out["pair"]:  # a form without the fused kernel runs the two actions
        out["pair"] = out["force"] + out["force_t"]
    info = fe.fe_query(ctx)
    out["used"] = (info["nw_force"], info["nw_force_t"], info["nw_mass"], info["patch"])
    fe.fe_destroy(ctx)
    return out


@functools.lru_cache(maxsize=1)
def _mesh(n: int, p: int):
    # half the workload perturbation: timings do not depend on it, and the
    # higher point counts (Q = p+3) must not meet an inverted point
    from . import workload as W
    return W.cube_mesh(n, p, 0.5 * W.default_amp(p), seed=0)


def tune(n: int, p: int, Q: int, precision: int = 0, verbose: bool = True):
    import torch

    import paper_2112_07075_amd as fe
    from . import workload as W

    mesh = _mesh(n, p)
    best = {}
    trials = []
    for patch in patch_choices(p):
        for nw in WAVES:
            t = time_actions(fe, torch, mesh, p, Q, precision, nw, patch)
            trials.append({"patch": patch, "nw": nw,
                           **{k: t[k] for k in ("force", "force_t", "mass", "pair")},
                           "used": t["used"]})
            if verbose:
                print(f"patch {patch:3d} waves {nw}: F.1 {t['force']:8.1f} us  F^T.v "
                      f"{t['force_t']:8.1f} us  M x {t['mass']:8.1f} us  pair {t['pair']:8.1f} us"
                      f"  (in use {t['used']})", flush=True)
    # patches are shared by the three actions: choose the patch size minimising the sum
    # of the best times, then the waves per workgroup of each action for that patch size
    # the step runs the fused pair and the mass action; the single actions are
    # tuned too (they are called on their own)
    def best_for(patch):
        rows = [r for r in trials if r["patch"] == patch]
        pick = {k: min(rows, key=lambda r: r[k]) for k in ("force", "force_t", "mass", "pair")}
        return pick["pair"]["pair"] + pick["mass"]["mass"], pick

    total, pick, patch = min((best_for(pt) + (pt,) for pt in patch_choices(p)),
                             key=lambda x: x[0])
    best = {"p": p, "Q": Q, "precision": precision, "patch": patch,
            "nw_force": pick["force"]["used"][0], "nw_force_t": pick["force_t"]["used"][1],
            "nw_mass": pick["mass"]["used"][2],
            # -1: the two single kernels beat the fused one (the pair then runs them)
            "nw_pair": (pick["pair"]["nw"] if pick["pair"]["pair"] <= pick["force"]["force"] +
                        pick["force_t"]["force_t"] else -1),
            "us": {k: pick[k][k] for k in pick}, "trials": trials}
    return best


def builtin_cases():
    """(p, Q, precision, n) of the built-in table."""
    size = {1: 96, 2: 48, 3: 32, 4: 24}
    cases = []
    for p in range(1, 5):
        for Q in (p + 1, p + 2, p + 3):
            n = 64 if (p, Q) == (3, 5) else size[p]
            cases.append((p, Q, 0, n))
    for prec in (1, 2):
        for p in range(1, 5):
            cases.append((p, p + 2, prec, 64 if p == 3 else size[p]))
    return cases


def write_builtin(path: str):
    import paper_2112_07075_amd as fe
    rows = []
    for p, Q, prec, n in builtin_cases():
        print(f"== p={p} Q={Q} precision={prec} n={n}", flush=True)
        try:
            b = tune(n, p, Q, prec)
        except fe.FepaError as err:
            if err.status != fe.FE_EUNSUPPORTED:
                raise
            print("   unsupported, skipped", flush=True)
            continue
        rows.append(b)
        print("   best:", table_line(b), json.dumps(b["us"]), flush=True)
    with open(path, "w") as f:
        f.write("// Generated by paper_2112_07075_amd/autotune.py --builtin: {p, Q, precision,\n"
                "// waves F, waves F^T, waves M, elements per patch, waves F + F^T fused\n"
                "// (-1: the pair runs as the two single kernels)},\n"
                "// fastest measured on MI355X.\n")
        for b in rows:
            us = b["us"]
            f.write(f"{{{b['p']}, {b['Q']}, {b['precision']}, {b['nw_force']}, {b['nw_force_t']}, "
                    f"{b['nw_mass']}, {b['patch']}, {b['nw_pair']}}},  // F.1 {us['force']:.1f} us, "
                    f"F^T.v {us['force_t']:.1f} us, M x {us['mass']:.1f} us, pair {us['pair']:.1f} us\n")


def table_line(b) -> str:
    return (f"{b['p']} {b['Q']} {b['precision']} {b['nw_force']} {b['nw_force_t']} "
            f"{b['nw_mass']} {b['patch']} {b['nw_pair']}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=48)
    ap.add_argument("--p", type=int, default=2)
    ap.add_argument("--q", type=int, default=4)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--out", default="")
    ap.add_argument("--json", default="")
    ap.add_argument("--builtin", default="", help="tune the built-in set, write this .inc file")
    args = ap.parse_args()
    if args.builtin:
        write_builtin(args.builtin)
        return 0
    b = tune(args.n, args.p, args.q, args.precision)
    line = table_line(b)
    print("best:", line, json.dumps(b["us"]))
    if args.out:
        old = []
        if os.path.exists(args.out):
            key = line.split()[:3]
            old = [l for l in open(args.out) if l.split()[:3] != key]
        with open(args.out, "w") as f:
            f.writelines(old + [line + "\n"])
    if args.json:
        with open(args.json, "w") as f:
            json.dump(b, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
