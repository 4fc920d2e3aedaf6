"""Benchmark of the MI355X tactile force field (one JSON line on stdout).

Workload: the roofline shape -- 8192 environments x 2 pads x 80x100 taxels
(1.31e8 taxel evaluations per step) against eight objects voxelized at 256^3
(FP32), seeded poses with ~70% of taxels in contact, velocities uniform in
[-0.1, 0.1] m/s.  A step is one pass of the whole path: per-pad prologue,
the per-taxel force field with SoA outputs, per-pad wrench.

Also reported:
* roofline of the dominant kernel (k_force_fwd): algorithmic bytes per launch
  / its average duration from HIP events recorded around it on its stream
  during the timed steps;
* cpu_baseline: the FP64 oracle on the host cores;
* batched_vs_plain: the uneven batch (4096 envs, pads {20x25, 40x50, 80x100},
  grids {64,128,256}^3 x 8 objects) as one persistent launch per substep vs
  one plain launch per (pad, grid) group, both captured as HIP graphs of 100
  substeps, with the per-taxel outputs of the two compared;
* differentiation: adjoint throughput on 1024 envs x 2 pads x 40x50;
* contact_impulse: the batched implicit soft-contact impulse at the contact
  count of the roofline batch (16384 pads x 64 contacts) and as a 33.5 M
  contact stream, against HBM bandwidth.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "taxel force evals/sec at 1 GPU + % HBM roofline; batched vs plain speedup at 1e-4 rel"
HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


FOOTPRINT = os.path.join(ROOT, "tests", "golden", "sdf_footprint.json")


# rocprofv3 summaries of the forward kernel on the roofline workload, one per profiled launch shape
PROFILE_GLOB = os.path.join(ROOT, "profiles", "k_force_fwd_roofline_8192x2x80x100_256*.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2408_06506_amd", "csrc", f)
                  for f in ("tacsl_kernels.hip", "tacsl_device.h", "tacsl_internal.h")]


def measured_traffic(tuning):
    """HBM bytes per launch of the forward kernel from a committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (copy-calibrated) taken with this tuning,
    or None when none matches the tuning and the current kernel sources."""
    import glob
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    sha = h.hexdigest()[:16]
    for path in sorted(glob.glob(PROFILE_GLOB)):
        try:
            rec = {}
            for line in open(path):
                if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "kernel_source_sha1", "tuning"):
                    k, v = line.split(":", 1)
                    rec[k] = v.strip()
            if rec.get("kernel_source_sha1") == sha and json.loads(rec["tuning"]) == dict(tuning):
                return float(rec["traffic_bytes_per_launch"])
        except (OSError, KeyError, ValueError):
            continue
    return None


def sdf_footprint_nodes(key, scene):
    """Distinct scalar SDF nodes touched by one step's taxel stencils, as
    counted once for the seeded workload and stored with the test fixtures."""
    with open(FOOTPRINT) as f:
        rec = json.load(f)["workloads"][key]
    if rec["n_taxels"] != scene.n_taxels or rec["n_inst"] != scene.n_inst:
        raise RuntimeError(f"stored SDF footprint of {key} does not describe this scene")
    return int(rec["nodes"])


def algorithmic_bytes(scene, footprint_nodes):
    """Compulsory bytes of one step: 40 B/taxel of outputs written once, 4 B
    per distinct scalar SDF node the stencils touch, the template read once,
    per-pad pose/twist in and wrench out, per-env pose, twist and parameters
    in."""
    T = scene.n_taxels
    tmpl = 12 * int(scene.tmpl_offset[-1])
    per_inst = (7 + 6 + 6) * 4
    per_env = (7 + 6 + 4) * 4
    return 40 * T + 4 * footprint_nodes + tmpl + per_inst * scene.n_inst + per_env * scene.n_env


def run_main(args, torch, api, wl, autotune):
    t0 = time.time()
    sc = wl.make_c3()
    log(f"c3 scene: {sc.n_env} envs, {sc.n_inst} pads, {sc.n_taxels} taxels ({time.time() - t0:.1f}s)")
    plan = api.Plan(sc)
    st = plan.state(sc.state())
    out = plan.new_outputs()
    tun = None
    if args.tuning:
        tun = json.loads(args.tuning)
        plan.set_tuning(tun)
    elif not args.no_tune:
        t1 = time.time()
        res = autotune.autotune(plan, sc, st, out, reps=5, tag="c3")
        tun = res["tuning"]
        log(f"autotune: {tun} {res['ms']:.4f} ms ({'cached' if res['cached'] else 'searched'}, {time.time() - t1:.1f}s)")
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        plan.forward(st, out)
    torch.cuda.synchronize()
    plan.timer_start(args.steps)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        plan.forward(st, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kms = plan.timer_read(args.steps)
    plan.timer_start(0)
    ms_step = wall * 1e3 / args.steps
    value = sc.n_taxels * args.steps / wall
    V = sdf_footprint_nodes("roofline_8192x2x80x100_256", sc)
    B = algorithmic_bytes(sc, V)
    k_avg = float(np.mean(kms))
    achieved = B / (k_avg * 1e-3)
    contact = float((out["depth"] > 0).float().mean().item())
    log(f"{ms_step:.4f} ms/step, kernel {k_avg:.4f} ms, {achieved / 1e9:.1f} GB/s, contact {contact:.3f}")
    return dict(scene=sc, plan=plan, state=st, out=out, tuning=plan.tuning, ms_step=ms_step,
                value=value, kernel_ms=k_avg, kernel_ms_all=kms, bytes=B, footprint=V, achieved=achieved,
                contact=contact)


def run_tiny(args, torch, api, wl):
    """The tiny ball case: 1 env, 1 pad of 20x25 taxels, sphere r = 10 mm at
    64^3 / 0.5 mm, 100 seeded steps (each step its own pose and velocity).
    Latency-bound: reported as microseconds per step, for one call per step
    (host launch included) and for the 100 steps captured in one HIP graph."""
    scenes = [wl.make_c1(step) for step in range(100)]
    plan = api.Plan(scenes[0])
    states = [plan.state(s.state()) for s in scenes]
    outs = [plan.new_outputs() for _ in states]
    # the launch shape: one workgroup of 128, 256 or 512 threads (the 500
    # taxels in 4, 2 or 1 iterations), chosen on graph replays of the 100 steps
    reps = 20
    best = None
    for tun in (dict(block=256), dict(block=512), dict(block=128)):
        plan.set_tuning(tun)
        g = api.SubstepGraph(plan, states, outs)
        g.launch()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        h0 = time.perf_counter()
        for _ in range(reps):
            g.launch()
        host_us = (time.perf_counter() - h0) * 1e6 / (reps * len(states))  # submission only
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / (reps * len(states))
        g.close()
        if best is None or us < best[1]:
            best = (tun, us, host_us)
    plan.set_tuning(best[0])
    us_graph, host_us = best[1], best[2]
    out = plan.new_outputs()
    for st in states[:10]:
        plan.forward(st, out)
    torch.cuda.synchronize()
    plan.timer_start(len(states))
    t0 = time.perf_counter()
    for st in states:
        plan.forward(st, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = plan.timer_read(len(states))
    plan.timer_start(0)
    tuning = plan.tuning
    plan.close()
    T = scenes[0].n_taxels
    res = {"workload": "tiny ball: 1 env x 1 pad 20x25 taxels, sphere r=10 mm at 64^3 / 0.5 mm, 100 seeded steps",
           "taxels_per_step": T, "tuning": tuning, "us_per_step_eager": wall * 1e6 / len(states),
           "us_per_step_graph": us_graph, "host_us_per_step_graph_submit": host_us,
           "kernel_avg_us": float(np.mean(kms)) * 1e3,
           "taxel_evals_per_s_graph": T / (us_graph * 1e-6)}
    log(f"tiny: {res['us_per_step_eager']:.1f} us/step eager, {us_graph:.2f} us/step in a graph, "
        f"kernel {res['kernel_avg_us']:.2f} us")
    return res, scenes


def run_scale(args, torch, api, wl, autotune):
    """The plain method at scale: 1024 envs x 2 pads x 40x50 taxels, five
    objects at 128^3, penetration U[0, 2] mm; autotuned; throughput and the
    forward kernel against the HBM roofline (same byte count as the main leg)."""
    sc = wl.make_c2()
    plan = api.Plan(sc)
    st = plan.state(sc.state())
    out = plan.new_outputs()
    if not args.no_tune:
        autotune.autotune(plan, sc, st, out, reps=5, tag="c2")
    for _ in range(args.warmup):
        plan.forward(st, out)
    steps = max(20, args.steps)
    plan.timer_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forward(st, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = float(np.mean(plan.timer_read(steps)))
    tun = plan.tuning
    plan.close()
    V = sdf_footprint_nodes("scale_1024x2x40x50_128", sc)
    B = algorithmic_bytes(sc, V)
    res = {"workload": "plain scale: 1024 envs x 2 pads x 40x50 taxels, 5 objects at 128^3",
           "taxels_per_step": sc.n_taxels, "ms_per_step": wall * 1e3 / steps,
           "taxel_evals_per_s": sc.n_taxels * steps / wall, "tuning": tun, "kernel": "k_force_fwd",
           "kernel_avg_ms": kms, "algorithmic_bytes_per_launch": B,
           "achieved_GBps": B / (kms * 1e-3) / 1e9, "frac_of_hbm_peak": B / (kms * 1e-3) / HBM_PEAK}
    log(f"scale: {res['ms_per_step']:.4f} ms/step, kernel {kms:.4f} ms, frac {res['frac_of_hbm_peak']:.3f}")
    return res, sc


def host_cores():
    """Host CPUs as the OS reports them: (os.cpu_count(), CPUs this process may run on)."""
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = os.cpu_count() or 1
    return os.cpu_count() or 1, aff


def oracle_timings(scenes, threads):
    """The oracle on the other workloads, each on `threads` threads (plus one
    thread for the tiny case): the tiny case and the plain scale in full, the
    differentiation workload's forward and its dual-number gradient (16
    directions) in full, the batched uneven workload at substeps 0, 1, 49, 99."""
    import oracle
    res = {}
    tiny = scenes.get("tiny")
    if tiny:
        for nt in (1, threads):
            t0 = time.perf_counter()
            for s in tiny:
                oracle.force_field(s, oracle.state64(s), nthreads=nt)
            dt = time.perf_counter() - t0
            n = sum(s.n_taxels for s in tiny)
            res[f"tiny_{nt}_threads"] = {"steps": len(tiny), "us_per_step": dt * 1e6 / len(tiny),
                                         "taxel_evals_per_s": n / dt}
    for key in ("scale", "differentiation"):
        s = scenes.get(key)
        if s is None:
            continue
        st = oracle.state64(s)
        t0 = time.perf_counter()
        oracle.force_field(s, st, nthreads=threads)
        dt = time.perf_counter() - t0
        res[key] = {"taxels": s.n_taxels, "s_per_step": dt, "taxel_evals_per_s": s.n_taxels / dt}
        if key == "differentiation":
            from paper_2408_06506_amd import workloads as wl
            wa, wb = wl.loss_weights(s.n_taxels, 5)
            t0 = time.perf_counter()
            oracle.grad(s, st, wa, wb, nthreads=threads)
            dt = time.perf_counter() - t0
            res["differentiation_dual_gradient"] = {"taxels": s.n_taxels, "s_per_gradient": dt,
                                                    "taxel_evals_per_s": s.n_taxels / dt}
    s = scenes.get("batched")
    if s is not None:
        sub = {}
        for step in (0, 1, 49, 99):
            if step >= s.obj_pose_steps.shape[0]:
                continue
            st = oracle.state64(s, step=step)
            t0 = time.perf_counter()
            oracle.force_field(s, st, nthreads=threads)
            sub[str(step)] = time.perf_counter() - t0
        res["batched_substeps"] = {"taxels_per_substep": s.n_taxels, "s_per_substep": sub,
                                   "taxel_evals_per_s": s.n_taxels * len(sub) / sum(sub.values())}
    return res


def run_cpu_baseline(sc, budget_threads, scenes=None):
    import oracle
    st = oracle.state64(sc)
    n_cpu, n_aff = host_cores()
    threads = max(1, min(budget_threads, n_aff))
    sel1 = np.arange(0, sc.n_inst, 8, dtype=np.int32)
    t0 = time.perf_counter()
    oracle.force_field(sc, st, sel=sel1, nthreads=1)
    t1 = time.perf_counter() - t0
    n1 = int(np.diff(sc.tmpl_offset)[sc.inst_tmpl[sel1]].sum())
    # the whole step on every thread, repeated for about 6 s (at most 8 times)
    reps = []
    t_start = time.perf_counter()
    while not reps or (time.perf_counter() - t_start < 6.0 and len(reps) < 8):
        t0 = time.perf_counter()
        oracle.force_field(sc, st, nthreads=threads)
        reps.append(time.perf_counter() - t0)
    tN = float(np.median(reps))
    res = {"value": sc.n_taxels / tN, "unit": "taxel-evals/s", "cores": threads, "kind": "oracle",
           "sample": f"FP64 C++ oracle (g++ -O2, OpenMP over pads): the full roofline-shape step "
                     f"({sc.n_taxels} taxels) on {threads} threads, median of {len(reps)} runs {tN:.2f} s; "
                     f"1 thread on every 8th pad ({n1} taxels) in {t1:.2f} s = {n1 / t1:.3e} taxel-evals/s",
           "single_thread_value": n1 / t1,
           "host": {"os_cpu_count": n_cpu, "affinity_cpus": n_aff, "threads_used": threads,
                    "thread_cap": budget_threads}}
    if scenes:
        res["per_workload"] = oracle_timings(scenes, threads)
    return res


def run_batched_vs_plain(args, torch, api, wl, autotune):
    t0 = time.time()
    sc = wl.make_c4()
    S = sc.obj_pose_steps.shape[0]
    log(f"c4 scene: {sc.n_env} envs, {sc.n_inst} pads, {sc.n_taxels} taxels/substep, {S} substeps "
        f"({time.time() - t0:.1f}s)")
    dt = float(sc.meta["dt"])

    def path_of(p, scene):
        """The substep pose path of a plan: poses at s dt from the step-0 pose and
        twist, written inside the graph before each substep's forward."""
        st0 = p.state(scene.state(0))
        return dict(pose0=st0["obj_pose"], twist=st0["obj_twist"], dt=dt,
                    poses=torch.empty(S, scene.n_env, 7, device=p.device))

    # batched: one plan, persistent schedules only, autotuned
    plan = api.Plan(sc, dict(tile_taxels=2048, schedule=2, order=2))
    states = [plan.state(sc.state(s)) for s in range(S)]
    tmp = plan.new_outputs()
    if not args.no_tune:
        res = autotune.autotune(plan, sc, states[0], tmp, reps=5, schedules=(1, 2), tag="c4-batched")
        log(f"batched autotune: {res['tuning']} {res['ms']:.4f} ms")
    out = plan.new_outputs()
    wrench = torch.empty(S, sc.n_inst, 6, device=plan.device)
    outs = [dict(out, wrench=wrench[s]) for s in range(S)]
    path_b = path_of(plan, sc)
    g_b = api.SubstepGraph(plan, states, outs, paths=path_b)
    # plain: one plan per (pad resolution, grid size) group, each autotuned
    # over every schedule (a superset of the batched plan's search), all
    # groups launched in every substep (one graph, substep-major)
    groups = wl.c4_groups(sc)
    subs = [wl.subset_scene(sc, g) for g in groups]
    plains, p_states, p_outs, pouts, p_paths, p_tun = [], [], [], [], [], []
    for gi, sub in enumerate(subs):
        p = api.Plan(sub)
        po = p.new_outputs()
        pst = [p.state(sub.state(s)) for s in range(S)]
        if not args.no_tune:
            r = autotune.autotune(p, sub, pst[0], po, reps=5, schedules=(0, 1, 2), tag=f"c4-plain-{gi}")
            ms_g = r["ms"]
        else:
            ms_g = None
        res_g = int(np.diff(sub.tmpl_offset)[sub.inst_tmpl[0]])
        p_tun.append({"taxels_per_pad": res_g, "grid": int(sub.sdf_dims[0][0]), "envs": sub.n_env,
                      "tuning": p.tuning, "tuned_ms": ms_g})
        pw = torch.empty(S, sub.n_inst, 6, device=p.device)
        plains.append(p)
        p_states.append(pst)
        p_outs.append([dict(po, wrench=pw[s]) for s in range(S)])
        p_paths.append(path_of(p, sub))
        pouts.append((po, pw))
    log(f"plain groups tuned: {[t['tuning'] for t in p_tun]}")
    graphs_p = [api.SubstepGraph(plains, p_states, p_outs, paths=p_paths)]
    torch.cuda.synchronize()

    def time_graphs(gs, reps):
        for g in gs:
            g.launch()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            for g in gs:
                g.launch()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = args.batched_reps
    ms_b = time_graphs([g_b], reps)
    ms_p = time_graphs(graphs_p, reps)
    log(f"batched {ms_b:.3f} ms / {S} substeps, plain {ms_p:.3f} ms")
    # parity: per-taxel outputs of the last substep and all substep wrenches
    off_all = plan.offsets()
    max_rel = 0.0
    bitwise = True
    for sub, (po, pw) in zip(subs, pouts):
        insts = sub.meta["insts"]
        rows = np.concatenate([np.arange(off_all[i], off_all[i + 1]) for i in insts])
        r = torch.as_tensor(rows, device=plan.device)
        for k in ("depth",):
            bitwise &= bool(torch.equal(out[k][r], po[k]))
        for k in ("normal", "fn", "ft"):
            bitwise &= bool(torch.equal(out[k][:, r], po[k]))
        wb = wrench[:, torch.as_tensor(insts, device=plan.device)]
        fmag = (torch.linalg.vector_norm(po["fn"] + po["ft"], dim=0))
        scale = max(float(fmag.sum().item()) / max(sub.n_inst, 1), 1e-9)
        max_rel = max(max_rel, float((wb - pw).abs().max().item()) / scale)
    # the poses the graphs stepped equal the closed form the workload records
    # (object translating at its velocity; FP64 then FP32 on both sides)
    host_poses = torch.as_tensor(sc.obj_pose_steps, device=plan.device)
    poses_equal = bool(torch.equal(path_b["poses"], host_poses))
    # roofline of one substep of the batched graph (pose step, prologue,
    # per-taxel pass, wrench reduction), same byte count as the main leg
    V = sdf_footprint_nodes("batched_uneven_4096_substep0", sc)
    B = algorithmic_bytes(sc, V)
    res = {"speedup": ms_p / ms_b, "batched_ms_per_substep": ms_b / S, "plain_ms_per_substep": ms_p / S,
           "substeps": S, "taxel_evals_per_substep": sc.n_taxels, "plain_launch_groups": len(subs),
           "batched_tuning": plan.tuning, "plain_group_tunings": p_tun, "per_taxel_bitwise_equal": bitwise,
           "wrench_max_rel_diff": max_rel, "tolerance": 1e-4,
           "recorded_poses_equal_closed_form": poses_equal,
           "batched_taxel_evals_per_s": sc.n_taxels * S / (ms_b * 1e-3),
           "algorithmic_bytes_per_substep": B, "sdf_footprint_nodes_substep0": V,
           "batched_frac_of_hbm_peak": B / (ms_b / S * 1e-3) / HBM_PEAK}
    for g in graphs_p:
        g.close()
    g_b.close()
    for p in plains:
        p.close()
    plan.close()
    return res


def run_backward(args, torch, api, wl):
    """Adjoint throughput on the differentiation workload (1024 envs x 2 pads
    x 40x50, 128^3): per step the forward prologue is recomputed, then the
    adjoint kernel (recomputation + reverse mode) and the per-env reduction.
    Algorithmic bytes: 24 B/taxel of upstream weights read once, 4 B per
    distinct scalar SDF node touched, the template, state and 64 B/env of
    gradients."""
    sc = wl.make_c5()
    plan = api.Plan(sc)
    st = plan.state(sc.state())
    st["obj_pose_delta"] = torch.zeros(sc.n_env, 6, device=plan.device)
    wa, wb = wl.loss_weights(sc.n_taxels, 5)
    wa_t = torch.as_tensor(wa, device=plan.device)
    wb_t = torch.as_tensor(wb, device=plan.device)
    g = plan.backward(st, wa_t, wb_t)
    torch.cuda.synchronize()
    # small launch-shape search for the adjoint (HIP events around each call)
    best, best_ms = None, float("inf")
    for tun in (dict(), dict(block=256, tile_taxels=0, schedule=0, order=3),
                dict(block=256, tile_taxels=0, schedule=0, order=5), dict(block=256, tile_taxels=512, schedule=0, order=5),
                dict(block=512, tile_taxels=0, schedule=0, order=5), dict(block=128, tile_taxels=0, schedule=0, order=5),
                dict(block=256, tile_taxels=0, schedule=2, grid=1024, order=5),
                dict(block=128, tile_taxels=256, schedule=0, order=5)):
        plan.set_tuning(tun)
        for _ in range(2):
            plan.backward(st, wa_t, wb_t, g)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            plan.backward(st, wa_t, wb_t, g)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 5
        if ms < best_ms:
            best, best_ms = tun, ms
    plan.set_tuning(best)
    for _ in range(3):
        plan.backward(st, wa_t, wb_t, g)
    steps = max(10, args.steps)
    plan.timer_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.backward(st, wa_t, wb_t, g)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = plan.timer_read(steps)
    plan_tuning = plan.tuning
    plan.close()
    V = sdf_footprint_nodes("differentiation_1024x2x40x50_128", sc)
    B = (24 * sc.n_taxels + 4 * V + 12 * int(sc.tmpl_offset[-1]) + (7 + 6) * 4 * sc.n_inst
         + (7 + 6 + 4 + 6) * 4 * sc.n_env + 64 * sc.n_env)
    k_avg = float(np.mean(kms))
    log(f"backward: {wall * 1e3 / steps:.4f} ms/step, kernel {k_avg:.4f} ms")
    return {"workload": "differentiation: 1024 envs x 2 pads x 40x50 taxels, 5 objects at 128^3",
            "taxels": sc.n_taxels, "ms_per_step": wall * 1e3 / steps,
            "taxel_evals_per_s": sc.n_taxels * steps / wall, "kernel": "k_force_bwd", "tuning": plan_tuning,
            "kernel_avg_ms": k_avg, "algorithmic_bytes_per_launch": B,
            "achieved_GBps": B / (k_avg * 1e-3) / 1e9, "frac_of_hbm_peak": B / (k_avg * 1e-3) / HBM_PEAK}


def run_observation(args, torch, api, wl, sc, tun):
    """Fused observation epilogue on the roofline batch (14 x 10 bins x 3
    channels per pad): observation only (no per-taxel stores) and observation
    with the per-taxel fields, the main leg's tuning with one tile per pad.  Algorithmic bytes
    of the observation-only pass: the stencil footprint, the template and bin
    map, state in, wrench and observation out."""
    # one tile per pad: the pooled partials are then one row per pad
    plan = api.Plan(sc, dict(tun, tile_taxels=0))
    bins = wl.scene_observation_bins(sc)
    plan.set_observation(bins, 140, scale=(1.0, 1.0, 1.0))
    st = plan.state(sc.state())
    obs = plan.new_observation()
    out_o = dict(wrench=torch.empty(sc.n_inst, 6, device=plan.device))
    res = {}
    for label, out in (("observation_only", out_o), ("observation_and_fields", plan.new_outputs())):
        for _ in range(args.warmup):
            plan.observe(st, obs=obs, out=out)
        steps = max(10, args.steps)
        plan.timer_start(steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.observe(st, obs=obs, out=out)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = float(np.mean(plan.timer_read(steps)))
        plan.timer_start(0)
        res[label] = {"ms_per_step": wall * 1e3 / steps, "kernel_avg_ms": kms,
                      "taxel_evals_per_s": sc.n_taxels * steps / wall}
        log(f"observation {label}: {wall * 1e3 / steps:.4f} ms/step, kernel {kms:.4f} ms")
        del out
    V = sdf_footprint_nodes("roofline_8192x2x80x100_256", sc)
    B = (4 * V + 16 * int(sc.tmpl_offset[-1]) + (7 + 6) * 4 * sc.n_inst + (7 + 6 + 4) * 4 * sc.n_env
         + (6 + 140 * 3) * 4 * sc.n_inst)
    k = res["observation_only"]["kernel_avg_ms"]
    res["observation_only"].update({"algorithmic_bytes_per_launch": B, "achieved_GBps": B / (k * 1e-3) / 1e9})
    res["workload"] = "roofline batch, 14 x 10 x 3 observation per pad (channels |f_n|, f_t,x, f_t,y)"
    plan.close()
    torch.cuda.empty_cache()
    return res


def run_nonlinear_law(args, torch, api, wl, sc, tun):
    """The roofline batch with the penetration to the power 1.5 in the normal
    law (same tuning as the main leg): cost of the nonlinear variant."""
    plan = api.Plan(sc, tun)
    plan.set_normal_law(1.5)
    st = plan.state(sc.state())
    out = plan.new_outputs()
    for _ in range(args.warmup):
        plan.forward(st, out)
    steps = max(10, args.steps // 2)
    plan.timer_start(steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forward(st, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = float(np.mean(plan.timer_read(steps)))
    plan.close()
    del out
    torch.cuda.empty_cache()
    log(f"normal law p=1.5: {wall * 1e3 / steps:.4f} ms/step, kernel {kms:.4f} ms")
    return {"exponent": 1.5, "ms_per_step": wall * 1e3 / steps, "kernel_avg_ms": kms,
            "taxel_evals_per_s": sc.n_taxels * steps / wall}


def run_depth(args, torch, api, wl, sc):
    """Tactile depth image of the roofline batch: every pad seen by an 80 x 60
    pinhole camera 20 mm behind a 4 mm gel (16384 images per frame)."""
    plan = api.Plan(sc)
    rows, cols = 80, 60
    plan.set_camera(rows, cols, -wl.PAD_W / 2, -wl.PAD_H / 2, wl.PAD_W / cols, wl.PAD_H / rows, 20e-3, 4e-3)
    st = plan.state(sc.state())
    status = torch.zeros(1, device=plan.device, dtype=torch.int32)
    img = plan.depth_image(st, status=status)
    for _ in range(args.warmup):
        plan.depth_image(st, image=img, status=status)
    reps = max(10, args.steps // 2)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        plan.depth_image(st, image=img, status=status)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    px = sc.n_inst * rows * cols
    hit = float((img < 20e-3 - 1e-9).float().mean().item())
    res = {"workload": "roofline batch, 80 x 60 pinhole camera per pad (20 mm behind a 4 mm gel)",
           "pads": sc.n_inst, "pixels_per_frame": px, "ms_per_frame": ms, "wall_ms_per_frame": wall * 1e3 / reps,
           "pixels_per_s": px / (ms * 1e-3), "env_frames_per_s": sc.n_env / (ms * 1e-3),
           "pixels_on_object": hit, "step_limit_hit": bool(int(status.item()) & 0x8)}
    log(f"depth image: {ms:.3f} ms/frame, {px / (ms * 1e-3):.3e} px/s, {hit:.3f} of pixels on the object")
    plan.close()
    torch.cuda.empty_cache()
    return res


def run_copy(torch, mib=1024, reps=10):
    """Bandwidth of a plain device-to-device copy of `mib` MiB (the runtime's
    copy kernel), warm buffers, each copy bracketed by its own events: the
    reference for what the HBM sustains with equal reads and writes."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda")
    dst = torch.ones_like(src)
    for _ in range(3):
        dst.copy_(src)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        dst.copy_(src)
        b.record()
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    del src, dst
    torch.cuda.empty_cache()
    moved = 2 * n * 4
    log(f"copy {mib} MiB: {ms:.4f} ms, {moved / (ms * 1e-3) / 1e12:.2f} TB/s read + write")
    return {"bytes_moved_per_copy": moved, "ms_per_copy": ms, "TBps": moved / (ms * 1e-3) / 1e12,
            "frac_of_hbm_peak": moved / (ms * 1e-3) / HBM_PEAK}


def run_impulse(args, torch, api, wl):
    """Batched implicit soft-contact impulse: per call 16 B read (eps, eps_dot,
    1/m, env) and 8 B written (lambda, dv) per contact, plus 8 B per
    environment of (kappa, c).  Each call is bracketed by its own event pair on
    the stream it is launched on."""
    res = {}
    for label, n_env, per_env in (("pads of the roofline batch x 64 contacts", 16384, 64),
                                  ("33.5 M contact stream", 262144, 128)):
        c = wl.make_contacts(n_env=n_env, per_env=per_env, seed=11)
        f = lambda a: torch.as_tensor(a, device="cuda")
        eps, ed, im, env, kc = f(c.eps), f(c.eps_dot), f(c.inv_mass), f(c.env), f(c.kc)
        lam = torch.empty_like(eps)
        dv = torch.empty_like(eps)
        for _ in range(5):
            api.contact_impulse(eps, ed, im, kc, c.dt, env=env, lam=lam, dv=dv)
        reps = max(20, args.steps)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in ev:
            a.record()
            api.contact_impulse(eps, ed, im, kc, c.dt, env=env, lam=lam, dv=dv)
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        B = 24 * c.n + 8 * n_env
        res["scene" if n_env == 16384 else "stream"] = {
            "workload": label, "contacts": c.n, "kernel": "k_contact_impulse_x4", "kernel_avg_ms": ms,
            "contacts_per_s": c.n / (ms * 1e-3), "wall_ms_per_call": wall * 1e3 / reps,
            "algorithmic_bytes_per_launch": B, "achieved_GBps": B / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": B / (ms * 1e-3) / HBM_PEAK}
        log(f"impulse {label}: {c.n} contacts, {ms * 1e3:.2f} us, {B / (ms * 1e-3) / 1e9:.0f} GB/s")
        del eps, ed, im, env, kc, lam, dv
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-impulse", action="store_true")
    ap.add_argument("--no-observation", action="store_true")
    ap.add_argument("--no-depth", action="store_true")
    ap.add_argument("--no-nonlinear", action="store_true")
    ap.add_argument("--no-tiny", action="store_true")
    ap.add_argument("--no-scale", action="store_true")
    ap.add_argument("--batched-reps", type=int, default=5)
    ap.add_argument("--threads", type=int, default=16)
    ap.add_argument("--tuning", type=str, default=None,
                    help='fixed tuning as JSON, e.g. {"block":256,"tile_taxels":512,"schedule":2,"grid":1024,"order":1}')
    ap.add_argument("--only-main", action="store_true", help="roofline workload only (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB copied by a plain device copy before the run (counter scale reference)")
    ap.add_argument("--only-copy", action="store_true", help="the plain device copy bandwidth only")
    args = ap.parse_args()
    if args.only_main:
        args.no_batched = True
        args.no_cpu_baseline = True
        args.no_backward = True
        args.no_impulse = True
        args.no_observation = True
        args.no_depth = True
        args.no_nonlinear = True
        args.no_tiny = True
        args.no_scale = True
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (environments shard "
              f"across GPUs without exchange; only the single-GPU shard is built here).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2408_06506_amd import api, autotune
    from paper_2408_06506_amd import workloads as wl
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {n * 4} bytes read, {n * 4} bytes written")
        del src, dst
    copy = run_copy(torch)
    if args.only_copy:
        print(json.dumps({"copy_bandwidth": copy}), flush=True)
        return
    m = run_main(args, torch, api, wl, autotune)
    sc = m["scene"]
    traffic = measured_traffic(m["tuning"])
    observation = None
    if not args.no_observation:
        observation = run_observation(args, torch, api, wl, sc, m["tuning"])
    nonlinear = None
    if not args.no_nonlinear:
        nonlinear = run_nonlinear_law(args, torch, api, wl, sc, m["tuning"])
    roof = {"bound": "hbm", "achieved": m["achieved"] / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": m["achieved"] / HBM_PEAK, "traffic": traffic, "kernel": "k_force_fwd",
            "kernel_avg_ms": m["kernel_ms"], "algorithmic_bytes_per_launch": m["bytes"],
            "bytes_per_taxel": m["bytes"] / sc.n_taxels, "sdf_footprint_nodes": m["footprint"],
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated; null if the kernel or "
                            "tuning changed since the counters were taken)",
            "traffic_GBps": None if traffic is None else traffic / (m["kernel_ms"] * 1e-3) / 1e9}
    m["plan"].close()
    del m["out"]
    torch.cuda.empty_cache()
    batched = None
    if not args.no_batched:
        batched = run_batched_vs_plain(args, torch, api, wl, autotune)
    backward = None
    if not args.no_backward:
        backward = run_backward(args, torch, api, wl)
    depth = None
    if not args.no_depth:
        depth = run_depth(args, torch, api, wl, sc)
    cpu_scenes = {}
    tiny = None
    if not args.no_tiny:
        tiny, cpu_scenes["tiny"] = run_tiny(args, torch, api, wl)
    scale = None
    if not args.no_scale:
        scale, cpu_scenes["scale"] = run_scale(args, torch, api, wl, autotune)
    impulse = None
    if not args.no_impulse:
        impulse = run_impulse(args, torch, api, wl)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        if not args.no_backward:
            cpu_scenes["differentiation"] = wl.make_c5()
        if not args.no_batched:
            cpu_scenes["batched"] = wl.make_c4()
        cpu = run_cpu_baseline(sc, args.threads, cpu_scenes)
        log(f"oracle {cpu['value']:.3e} taxel-evals/s on {cpu['cores']} threads")
    line = {
        "metric": METRIC, "value": m["value"], "unit": "taxel-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "roofline shape: 8192 envs x 2 pads x 80x100 taxels (1.31e8 taxel evals/step), "
                               "8 analytic objects voxelized at 256^3 FP32, ~70% of taxels in contact",
                   "n_env": sc.n_env, "n_pads": sc.n_inst, "taxels_per_step": sc.n_taxels,
                   "contact_fraction": m["contact"], "tuning": m["tuning"], "parallelism": "single GPU"},
        "roofline": roof, "cpu_baseline": cpu, "batched_vs_plain": batched, "differentiation": backward,
        "contact_impulse": impulse, "observation": observation, "depth_image": depth,
        "nonlinear_normal_law": nonlinear, "tiny": tiny, "scale": scale, "copy_bandwidth": copy,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
