"""Throughput benchmark of the cut-cell DVM step on one MI355X.

Workload: 2D reduced model, 512 x 256 cells on [0,1] x [0,0.5], 32^2
velocities on [-6,6]^2, fixed cylinder r = 0.05 at (0.5, 0.25), Kn 0.1,
inflow Mach 0.8, diffuse wall T_w = 1, CFL 0.5, force (drag) recorded every
step.  Inputs are synthetic (the flow set-up itself) and resident in HBM
before timing starts.

Prints one JSON line: whole-job cell-velocity updates per second, the
roofline position of the dominant kernel (k_step2d, regular-cell stencil) measured
with HIP events on the solver's stream, and the oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD_TEXT = {
    "cyl512": "cyl512: 2D 512x256 cells, 32x32 velocities on [-6,6]^2, cylinder r=0.05, "
              "Kn {kn}, Mach 0.8, T_w 1, CFL 0.5, drag every step",
    "ellipse256": "ellipse256: 2D 256x256 cells, 40x40 velocities on [-6,6]^2, ellipse 0.2x0.04 "
                  "free to rotate (J=0.01), Kn {kn}, Mach 0.5, geometry rebuilt every step, "
                  "torque every step",
    "cyl32": "cyl32: 2D 32x32 cells, 16x16 velocities, cylinder r=0.2, Kn {kn}, Mach 0.5",
    "sphere128": "sphere128: 3D 128x64x64 cells on [0,1]x[0,0.5]^2, 16^3 velocities on [-6,6]^3, "
                 "sphere r=0.1, Kn {kn}, Mach 0.5, T_w 1, CFL 0.5, force every step",
    "sphere_amr": "sphere_amr: 3D octree, 32x16x16 coarse cells on [0,1]x[0,0.5]^2 refined twice near "
                  "the sphere (1/128 there, as sphere128), 16^3 velocities, sphere r=0.1, Kn {kn}, "
                  "Mach 0.5, T_w 1, CFL 0.5, force every step",
    "vane_amr": "vane_amr: 3D octree, 32x32x16 coarse cells on [0,1]^2x[0,0.5] refined twice near a "
                "vane (plate 0.4x0.06x0.24 with rounded edges) turning freely about z (J=0.002, "
                "omega0=2, theta0=pi/8), mesh adapted every step, 16^3 velocities, Kn {kn}, Mach 0.5, "
                "T_w 1, CFL 0.5, torque every step",
}
# committed rocprofv3 counter summaries: workload -> (kernel source, summary);
# a summary holds for the kernel source and the headers it includes
TRAFFIC = {
    "cyl512": ("step2d.hip", "traffic_regular2d_cyl512.json"),
    "sphere128": ("step3d.hip", "traffic_regular3d_sphere128.json"),
}
KERNEL_HEADERS = ("ccdvm_impl.h", "equilibrium.h")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _code_only(text):
    """C/C++ source without comments and blank lines (so that a change of a
    comment does not invalidate a counter summary, a change of code does)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def src_hash(src):
    """sha256[:16] of the code of a kernel source file followed by the
    library headers it includes (csrc/ccdvm_impl.h, csrc/equilibrium.h,
    include/ccdvm.h), comments stripped."""
    csrc = os.path.join(ROOT, "paper_1503_04544_amd", "csrc")
    h = hashlib.sha256()
    for path in [os.path.join(csrc, src)] + [os.path.join(csrc, x) for x in KERNEL_HEADERS] + \
            [os.path.join(ROOT, "include", "ccdvm.h")]:
        with open(path, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the regular-cell kernel from the committed
    rocprofv3 counter summary, valid only for the kernel source it was taken on."""
    if workload not in TRAFFIC:
        return None
    src, summary = TRAFFIC[workload]
    try:
        with open(os.path.join(ROOT, "profiles", summary)) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256_16") != src_hash(src):
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(cfg, nsteps, threads=None):
    """The oracle as it stands, on the host cores (or `threads` of them):
    nsteps full steps of the same workload from the inflow-Maxwellian state."""
    import oracle
    prev = oracle.threads()
    if threads:
        oracle.set_threads(threads)
    try:
        o = oracle.Oracle2D(cfg)
        f, g = o.init()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            f, g, _ = o.step(f, g)
        dt = time.perf_counter() - t0
        used = oracle.threads()
    finally:
        if threads:
            oracle.set_threads(prev)
    geo = o.geometry()
    nupd = int((geo["type"] != 2).sum()) * cfg.nv ** 2 * nsteps
    return {"value": nupd / dt / 1e9, "unit": "G cell-velocity updates/s",
            "cores": used, "kind": "oracle",
            "sample": f"{nsteps} full steps of the 512x256x32^2 workload from the inflow "
                      f"Maxwellian ({dt:.1f} s)"}


def measure(cfg, name, steps, warmup, args):
    """Time `steps` steps of one workload after `warmup` untimed ones, then
    the same steps again with per-kernel HIP events on the solver's stream."""
    import torch
    from paper_1503_04544_amd.solver import Solver
    dev = torch.device("cuda:0")
    s = Solver(cfg, device=dev)
    n_irr, n_mem, n_solid = s.counts()
    active = s.ncell - n_solid   # cells, or the leaves of an octree
    ncell0 = s.ncell
    nvel = cfg.nv ** cfg.dim
    s.init_maxwellian()
    diag = torch.empty((max(steps, warmup, 1), 4), dtype=torch.float64, device=dev)
    log(f"bench {name}: warmup {warmup} steps")
    if warmup:
        s.step(warmup, diag=diag[:warmup])
    torch.cuda.synchronize()
    log(f"bench {name}: timing {steps} steps")
    t0 = time.perf_counter()
    s.step(steps, diag=diag[:steps])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / steps * 1e3
    value = active * nvel * steps / elapsed / 1e9
    drag_last = float(diag[steps - 1, 0].item())

    # live per-kernel durations (HIP events on the solver's stream), same steps
    log(f"bench {name}: per-kernel event timing")
    s.profile_enable(True)
    s.step(steps, diag=diag[:steps])
    reg_ms, reg_n = s.profile_read(0)
    cut_ms, cut_n = s.profile_read(1)
    red_ms, red_n = s.profile_read(2)
    mrg_ms, mrg_n = s.profile_read(3)
    mom_ms, mom_n = s.profile_read(4)
    rlx_ms, rlx_n = s.profile_read(5)
    plan_ms, plan_n = s.profile_read(6)
    adapt_ms, adapt_n = s.profile_read(7)
    build_ms, build_n = s.profile_read(8)
    s.profile_enable(False)
    amr = s.amr
    # the uniform kernels stream the regular cells (cut control volumes have
    # their own kernel); the octree kernel updates every control volume
    n_regular = active - n_mem if amr else active - n_irr - n_mem
    # read + write of the state, FP64: f,g in 2D (32 B), F in 3D (16 B)
    bytes_per_launch = n_regular * nvel * (32 if cfg.dim == 2 else 16)
    avg_s = reg_ms / max(reg_n, 1) / 1e3
    achieved = bytes_per_launch / avg_s / 1e9
    traffic = measured_traffic(name)

    # 2D semi-implicit with the direct equilibrium: the relaxation runs inside
    # the streaming kernel (its own instantiation) for up to 8 chunks per half
    im_fused = (cfg.dim == 2 and cfg.scheme == "imex" and cfg.maxwellian == "direct"
                and ((cfg.nv + 1) // 2 * cfg.nv + 63) // 64 <= 8)
    kernel_name = ("k_step2d_im" if im_fused else "k_step2d") if cfg.dim == 2 else \
        ("k_amr_step" if amr else "k_step3d")
    out = {
        "metric": "cell-velocity updates/s",
        "value": round(value, 3),
        "unit": "G cell-velocity updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[name].format(kn=cfg.kn),
                   "cells": ncell0, "active_cells": active, "velocities": nvel,
                   "cut_control_volumes": n_irr, "merged_cells": n_mem, "dt": s.dt,
                   "maxwellian": cfg.maxwellian, "scheme": cfg.scheme, "model": cfg.model,
                   "drag_last_step": drag_last, "positivity_number": s.cfl_number()},
        "roofline": {"bound": "hbm", "kernel": kernel_name,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "avg_launch_us": round(avg_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "cut_kernel_avg_us": round(cut_ms / max(cut_n, 1) * 1e3, 2),
                     "reduce_kernel_avg_us": round(red_ms / max(red_n, 1) * 1e3, 2),
                     "merge_kernel_avg_us": round(mrg_ms / max(mrg_n, 1) * 1e3, 2)},
    }
    if s.turning:
        # turning body: the host plans each step and adapts the mesh; the
        # remap kernel carries the state to the new mesh
        out["roofline"]["remap_kernel_avg_us"] = round(mom_ms / max(mom_n, 1) * 1e3, 2)
        out["host"] = {"plan_ms_per_step": round(plan_ms / max(plan_n, 1), 3),
                       "adapt_ms_per_step": round(adapt_ms / max(adapt_n, 1), 3),
                       "mesh_build_ms_per_step": round(build_ms / max(build_n, 1), 3),
                       "note": "cells and active_cells are those of the initial mesh"}
    elif cfg.dim == 2 and cfg.body.motion != "fixed":
        # moving 2D body: the geometry of t^{n+1} is rebuilt every step, beside
        # the streaming kernel of the step before (timed alone while profiling)
        geo_ms = mom_ms / max(mom_n, 1)
        out["roofline"]["geometry_rebuild_avg_us"] = round(geo_ms * 1e3, 2)
        out["roofline"]["general_cv_kernel_avg_us"] = round(cut_ms / max(cut_n, 1) * 1e3, 2)
        out["roofline"]["geometry_overlapped"] = True
    elif cfg.dim == 3 or cfg.maxwellian == "conservative":
        # 3D: moments from the chunk sums (and the Newton triplet);
        # 2D conservative: the Newton pass between steps
        out["roofline"]["between_steps_kernel_avg_us"] = round(mom_ms / max(mom_n, 1) * 1e3, 2)
    if cfg.scheme == "imex":
        out["roofline"]["relax_kernel_avg_us"] = round(rlx_ms / max(rlx_n, 1) * 1e3, 2)
    return s, out


def summary(line):
    """The figures of another workload's line carried in the headline line."""
    r = line["roofline"]
    keep = {"ms_per_step": line["ms_per_step"], "value": line["value"], "unit": line["unit"],
            "steps": line["steps"], "kernel": r["kernel"], "kernel_avg_us": r["avg_launch_us"],
            "achieved_GBs": r["achieved"], "frac": r["frac"], "traffic": r["traffic"],
            "workload": line["config"]["workload"]}
    for k in ("geometry_rebuild_avg_us", "general_cv_kernel_avg_us", "geometry_overlapped"):
        if k in r:
            keep[k] = r[k]
    return keep


def bench_batch(args, steps=None, warmup=None, quiet=False):
    """64 heterogeneous 2D fixed-cylinder instances (seeded recipe): batched
    step (one graph launch per step) against the same instances stepped one
    after the other with their own launches.  quiet: return the figures
    instead of printing a line."""
    import torch
    from ccdvm_inputs import batch_instances
    from paper_1503_04544_amd.solver import Batch, Solver
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    cfgs = batch_instances()
    solvers = []
    for c in cfgs:
        s = Solver(c, device=dev, stream=stream)
        s.init_maxwellian()
        solvers.append(s)
    upd = sum((c.ncell - s.counts()[2]) * c.nv ** 2 for c, s in zip(cfgs, solvers))
    log(f"bench batch: {len(cfgs)} instances, {upd / 1e6:.1f} M cell-velocity updates per step")
    for s in solvers:
        s.step(warmup)
    stream.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps)
    stream.synchronize()
    t_seq = time.perf_counter() - t0
    b = Batch(solvers)
    rows = b.autotune(5)
    b.step(warmup)
    stream.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    stream.synchronize()
    t_bat = time.perf_counter() - t0
    groups = b.groups()
    b.close()
    # forward + adjoint (drag of the final state, gradient w.r.t. T_w, Kn,
    # Ma) of a subset of the instances: every cc_adjoint in turn, then one
    # cc_batch_adjoint over the same instances
    nadj = min(args.batch_adjoint_instances, len(solvers))
    na, ka = args.batch_adjoint_steps, args.batch_adjoint_ckpt
    adj = None
    if nadj > 0 and na > 0:
        sub = solvers[:nadj]
        # the batched call holds every instance's checkpoint pool at once:
        # instances go in consecutive groups whose pools fit the budget
        budget = args.batch_adjoint_budget_gb * 1e9
        chunks, cur, cur_b = [], [], 0
        for s in sub:
            nb = s.adjoint_workspace_bytes(na, ka)
            if cur and cur_b + nb > budget:
                chunks.append(cur)
                cur, cur_b = [], 0
            cur.append(s)
            cur_b += nb
        chunks.append(cur)
        log(f"bench batch: adjoint of {nadj} instances, {na} steps, checkpoint every {ka}, "
            f"{len(chunks)} batched call(s)")
        # device pools allocated before the timed calls (one for the
        # sequential calls, one for the batched ones), as a caller that
        # repeats the gradient would keep them
        pool = torch.empty(max(s.adjoint_workspace_bytes(na, ka) for s in sub), dtype=torch.uint8, device=dev)
        sub[0].adjoint(na, ka, "drag", pool=pool)        # warm-up
        stream.synchronize()
        t0 = time.perf_counter()
        seq = [s.adjoint(na, ka, "drag", pool=pool) for s in sub]
        stream.synchronize()
        t_seq_adj = time.perf_counter() - t0
        del pool
        torch.cuda.empty_cache()
        batches = [Batch(ch) for ch in chunks]
        ws = torch.empty(max(b.adjoint_workspace_bytes(na, ka) for b in batches), dtype=torch.uint8, device=dev)
        batches[0].adjoint(na, ka, "drag", workspace=ws)  # warm-up
        stream.synchronize()
        J, G = [], []
        t0 = time.perf_counter()
        for b2 in batches:
            j, g = b2.adjoint(na, ka, "drag", workspace=ws)
            J.extend(j)
            G.extend(g)
        stream.synchronize()
        t_bat_adj = time.perf_counter() - t0
        for b2 in batches:
            b2.close()
        del ws
        torch.cuda.empty_cache()
        same = all(J[i] == seq[i][0] and (G[i] == seq[i][1]).all() for i in range(nadj))
        adj = {"instances": nadj, "steps": na, "ckpt_every": ka, "batched_calls": len(chunks),
               "sequential_s": round(t_seq_adj, 4), "batched_s": round(t_bat_adj, 4),
               "batched_over_sequential": round(t_seq_adj / t_bat_adj, 3),
               "bitwise_equal_to_sequential": bool(same)}
    fig = {"ms_per_step": round(t_bat / steps * 1e3, 4),
           "value": round(upd * steps / t_bat / 1e9, 3), "unit": "G cell-velocity updates/s",
           "steps": steps, "updates_per_step": upd,
           "achieved_GBs": round(upd * 32 * steps / t_bat / 1e9, 1),
           "frac": round(upd * 32 * steps / t_bat / 1e9 / HBM_PEAK_GBS, 4),
           "sequential_ms_per_step": round(t_seq / steps * 1e3, 4),
           "batched_over_sequential": round(t_seq / t_bat, 3),
           "groups_chunks_rows": groups, "autotuned_rows": rows,
           "forward_adjoint": adj,
           "workload": "batch: 64 2D fixed-cylinder instances, n in {64,128,256}^2, N in {16,24,32}^2, "
                       "Kn 10^U(-2,0), T_w U(0.5,2), Mach U(0.3,1), seed 20150316"}
    for s in solvers:
        s.close()
    if quiet:
        return fig
    out = {
        "metric": "cell-velocity updates/s", "value": fig["value"],
        "unit": "G cell-velocity updates/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": fig["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": fig["workload"], "updates_per_step": upd,
                   "sequential_ms_per_step": fig["sequential_ms_per_step"],
                   "batched_over_sequential": fig["batched_over_sequential"],
                   "groups_chunks_rows": fig["groups_chunks_rows"], "autotuned_rows": rows,
                   "forward_adjoint": adj},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kn", type=float, default=None)
    ap.add_argument("--workload", default="cyl512",
                    choices=["cyl512", "ellipse256", "cyl32", "sphere128", "sphere_amr", "vane_amr", "batch"],
                    help="cyl512 (default, the headline line) | ellipse256 (moving body) | cyl32 | "
                         "sphere128 (3D) | sphere_amr (3D octree) | vane_amr (3D octree, turning body)")
    ap.add_argument("--maxwellian", default="direct", choices=["direct", "conservative"],
                    help="equilibrium of the relaxation: direct moments (default) or the conservative "
                         "Newton triplet")
    ap.add_argument("--scheme", default="explicit", choices=["explicit", "imex"],
                    help="time scheme: explicit (default) or semi-implicit (transport explicit, "
                         "relaxation implicit)")
    ap.add_argument("--model", default="bgk", choices=["bgk", "shakhov"],
                    help="relaxation model: BGK (default) or Shakhov (Pr from --prandtl)")
    ap.add_argument("--prandtl", type=float, default=2.0 / 3.0)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=40,
                    help="steps of the adjoint/forward time ratio measurement (0: skip)")
    ap.add_argument("--adjoint-ckpt", type=int, default=8)
    ap.add_argument("--batch-adjoint-instances", type=int, default=32,
                    help="instances of the batch recipe whose forward + adjoint is timed (0: skip)")
    ap.add_argument("--batch-adjoint-steps", type=int, default=20)
    ap.add_argument("--batch-adjoint-ckpt", type=int, default=5)
    ap.add_argument("--batch-adjoint-budget-gb", type=float, default=120.0,
                    help="HBM for the checkpoint pools of one batched adjoint call")
    ap.add_argument("--extra-steps", type=int, default=20,
                    help="timed steps of each other workload carried in the cyl512 line")
    ap.add_argument("--no-extra", action="store_true",
                    help="cyl512 line without the other workloads")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy 10 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus 1); the step is not sharded across GPUs",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calib:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": a.numel() * 8,
                          "copy_bytes_written_per_launch": a.numel() * 8, "launches": 10}))
        return
    from ccdvm_inputs import workload
    from paper_1503_04544_amd.solver import Solver
    if args.workload == "batch":
        return bench_batch(args)

    cfg = workload(args.workload, kn=args.kn).with_(maxwellian=args.maxwellian,
                                                    scheme=args.scheme, model=args.model,
                                                    prandtl=args.prandtl)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s, out = measure(cfg, args.workload, args.steps, args.warmup, args)
    if (args.workload == "cyl512" and args.adjoint_steps > 0 and args.maxwellian == "direct"
            and args.scheme == "explicit" and args.model == "bgk"):
        # adjoint over the same workload: forward alone vs forward with
        # checkpoints + recomputation + adjoint sweep (cc_adjoint)
        na, ka = args.adjoint_steps, args.adjoint_ckpt
        log(f"bench: adjoint over {na} steps, checkpoint every {ka}")
        # the checkpoint pool is allocated before the timed call (a caller
        # that repeats the gradient keeps it), after one untimed call
        pool = torch.empty(s.adjoint_workspace_bytes(na, ka), dtype=torch.uint8, device=dev)
        s.adjoint(na, ka, "drag", pool=pool)
        s.init_maxwellian()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(na)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        J, grad = s.adjoint(na, ka, "drag", pool=pool)
        t_adj = time.perf_counter() - t0
        del pool
        out["adjoint"] = {"steps": na, "ckpt_every": ka, "forward_s": round(t_fwd, 4),
                          "adjoint_total_s": round(t_adj, 4),
                          "backward_over_forward": round((t_adj - t_fwd) / t_fwd, 3),
                          "adjoint_total_over_forward": round(t_adj / t_fwd, 3),
                          "drag": J, "d_drag_d_Tw_Kn_Ma": [float(x) for x in grad]}
    s.close()
    del s
    torch.cuda.empty_cache()
    if args.workload == "cyl512" and not args.no_extra:
        # the other full-size workloads, timed in the same run: 3D sphere,
        # moving ellipse (geometry rebuilt every step), the fixed sphere on
        # the octree, and the batch
        extra = {}
        for name, steps, warmup in (("sphere128", args.extra_steps, 3),
                                    ("ellipse256", 2 * args.extra_steps, 5),
                                    ("sphere_amr", 2 * args.extra_steps, 5)):
            s2, line = measure(workload(name), name, steps, warmup, args)
            s2.close()
            del s2
            torch.cuda.empty_cache()
            extra[name] = summary(line)
        extra["batch"] = bench_batch(args, steps=args.extra_steps, warmup=3, quiet=True)
        torch.cuda.empty_cache()
        out["other_workloads"] = extra
    if not args.no_cpu and args.workload == "cyl512":
        log(f"bench: oracle on the host, {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
        log("bench: oracle on one host thread, 1 step")
        out["cpu_baseline"]["one_thread"] = cpu_baseline(cfg, 1, threads=1)
        out["paper_context"] = {
            "note": "the paper reports no timing of this 2D step; its one figure is the 3D Crookes "
                    "radiometer on an octree (240 000 cells) in under 12 h on 240 MPI processes "
                    "(CPU model not stated), velocity grid and step count not stated",
            "implied_G_updates_per_s": ">= ~1.5 only if 30^3 velocities and 1e4 steps (assumed)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
