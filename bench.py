#!/usr/bin/env python3
"""Throughput benchmark of the Allen-Cahn stepper on one MI355X.

One bench step is one full solve of the shrinking-circle workload: a 2048x2048
FP32 grid, h = 1/2048, dt = 0.1 h^2, eps = eps_4, phi0 = tanh((0.25 - r)/(sqrt2 eps)),
20000 explicit steps (8.39e10 grid-point updates).  The state lives in HBM
before the timed region starts; the timed region is K back-to-back solves.

Printed as one JSON line on stdout:
  value     grid-point updates per second, in GLUPS
  roofline  the dominant kernel (the tiled 2D stencil) against the 8 TB/s HBM
            peak, counting the algorithmic 2*sizeof(T) bytes per update; with
            temporal blocking one launch advances tb_depth steps per HBM pass,
            so the fraction can exceed 1 ("effective" roofline).  `traffic` is
            the measured HBM bytes per launch from rocprofv3 counters when a
            summary for the current kernel source is stored under profiles/.
  cpu_baseline  the FP64 CPU oracle timed on this host's cores on a bounded
            sample of the same workload.
  extra     the other workloads: the FP64 circle, the 3D 256^3 FP32 grid at
            every temporal-blocking depth, the 3D sphere radius check, the
            512-grid batch, the learned surrogate's time-to-T against the
            plain stepper, and the 64x64 FP64 phase-separation grid.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NSTEPS = 20000
REG3D_MAX_DEPTH = 8     # FP32
CSRC = os.path.join(ROOT, "paper_2105_09671_amd", "csrc")
# stored HBM-traffic counters: (summary file, the kernel sources they were taken on)
TRAFFIC_HEADLINE = {   # by the plan's kernel: 64-wide or 128-wide register tiles
    4: (os.path.join(ROOT, "profiles", "traffic_tile2d_reg_circle2048_fp32.json"),
        [os.path.join(CSRC, f) for f in ("stencil2d.hip", "reg2d.h", "update.h")]),
    6: (os.path.join(ROOT, "profiles", "traffic_tile2d_regw_circle2048_fp32.json"),
        [os.path.join(CSRC, f) for f in ("stencil2d.hip", "reg2d.h", "reg2w.h", "update.h")])}
TRAFFIC_BATCH = (os.path.join(ROOT, "profiles", "traffic_batched_phase_batch512_fp32.json"),
                 [os.path.join(CSRC, f) for f in ("batched.hip", "reg2d.h", "reg2w.h", "update.h")])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def timed(fn, reps: int):
    """Median seconds of reps calls of fn on the current stream (HIP events)."""
    import torch
    ts = []
    for _ in range(reps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        ts.append(s.elapsed_time(e) / 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def measured_traffic(which):
    """HBM bytes per launch from stored rocprofv3 counters, if they were taken on
    the current source of the kernel; else None."""
    if which is None:
        return None
    path, srcs = which
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("src_sha256") != src_hash(srcs):
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(phi0, g, budget_s: float) -> dict:
    """The FP64 oracle on this host: all available cores, then one core."""
    import oracle
    threads = oracle.cpus_available()
    cells = g.nx * g.ny
    # per-step cost from a probe long enough to hide thread start-up
    probe, el = 2, 0.0
    while True:
        t0 = time.perf_counter()
        oracle.step2d(phi0, g.h, g.dt, g.eps, probe, threads)
        el = time.perf_counter() - t0
        if el > 0.05 * budget_s or probe >= NSTEPS // 4:
            break
        probe *= 4
    per = el / probe
    steps = int(max(2, min(NSTEPS, budget_s / max(per, 1e-9))))
    t0 = time.perf_counter()
    oracle.step2d(phi0, g.h, g.dt, g.eps, steps, threads)
    el = time.perf_counter() - t0
    v_all = cells * steps / el / 1e9
    t0 = time.perf_counter()
    s1 = max(1, steps // max(1, threads) // 2)
    oracle.step2d(phi0, g.h, g.dt, g.eps, s1, 1)
    el1 = time.perf_counter() - t0
    return {"value": round(v_all, 4), "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": "2048x2048 circle, FP64 plain loops, first %d of the %d steps on %d threads "
                      "(%.1f s); one thread: %d steps, %.4f GLUPS"
                      % (steps, NSTEPS, threads, el, s1, cells * s1 / el1 / 1e9)}


def extras(api, torch, workloads, params, cpu_budget) -> dict:
    out = {}
    # FP64 circle, same workload
    g = workloads.circle2048()
    phi = torch.from_numpy(g.initial()).cuda()
    api.step2d(phi, g.h, g.dt, g.eps, 2000)
    t = timed(lambda: api.step2d(phi, g.h, g.dt, g.eps, NSTEPS), 1)
    glups = g.nx * g.ny * NSTEPS / t / 1e9
    out["circle2048_fp64"] = {"GLUPS": round(glups, 2), "f_eff": round(glups * 16 / HBM_PEAK_GBS, 3),
                              "ms": round(t * 1e3, 2), "plan": api.plan2d(g.nx, g.ny, NSTEPS, torch.float64)}
    log("extra circle2048_fp64", out["circle2048_fp64"])
    del phi
    # 3D 256^3 FP32, 2000 steps, every temporal-blocking depth: on the z-streamed
    # register kernel (the default for this grid) and on the LDS kernel
    g3 = workloads.sep256c()
    p3 = torch.from_numpy(g3.initial()).float().cuda()
    n3 = g3.nx * g3.ny * g3.nz
    by_kernel = {}
    for kname, kern, maxk in (("reg3d", 5, REG3D_MAX_DEPTH), ("stream3d_lds", 2, 8)):
        depth = {}
        for k in range(1, maxk + 1):
            tune = ({"kernel": 5, "tb_depth": k, "tile_x": 64, "tile_y": 32} if kern == 5 else
                    {"kernel": 2, "tb_depth": k, "tile_x": 32 if k <= 4 else 64, "tile_y": 32,
                     "tile_z": 32})
            try:
                api.step3d(p3, g3.h, g3.dt, g3.eps, 2000, tune=tune)   # warm-up, same call
                t = timed(lambda: api.step3d(p3, g3.h, g3.dt, g3.eps, 2000, tune=tune), 1)
            except Exception as ex:   # an infeasible tile for this depth
                depth[k] = {"error": str(ex)}
                continue
            gl = n3 * 2000 / t / 1e9
            depth[k] = {"GLUPS": round(gl, 2), "f_eff": round(gl * 8 / HBM_PEAK_GBS, 3),
                        "plan": api.plan3d(256, 256, 256, 2000, tune=tune)}
        by_kernel[kname] = depth
    api.step3d(p3, g3.h, g3.dt, g3.eps, 2000)
    t = timed(lambda: api.step3d(p3, g3.h, g3.dt, g3.eps, 2000), 3)
    gl = n3 * 2000 / t / 1e9
    out["sep256c_fp32"] = {"GLUPS": round(gl, 2), "f_eff": round(gl * 8 / HBM_PEAK_GBS, 3),
                           "ms": round(t * 1e3, 2), "plan": api.plan3d(256, 256, 256, 2000),
                           "by_depth": by_kernel}
    log("extra sep256c_fp32", {k: v for k, v in out["sep256c_fp32"].items() if k != "by_depth"})
    del p3
    # sphere: R^2 = R0^2 - 4t
    gs = workloads.sphere256()
    ps = torch.from_numpy(gs.initial()).float().cuda()
    api.step3d(ps, gs.h, gs.dt, gs.eps, 2000)
    V = float(torch.sum(0.5 * (1.0 + ps.double())).item()) * gs.h ** 3
    R = (V / (4.0 / 3.0 * math.pi)) ** (1.0 / 3.0)
    law = params.radius_law(0.3, 2000 * gs.dt, 3)
    out["sphere256_fp32"] = {"R_T": round(R, 6), "R_law": round(law, 6),
                             "err_over_h": round(abs(R - law) / gs.h, 3)}
    del ps
    out["batch512_fp32"] = batch512(api, torch, workloads, cpu_budget)
    # learned K=100-step surrogate vs the plain stepper: 256 held-out 256^2
    # grids to T = 2000 steps, judge + fallback included (stored weights)
    import numpy as np
    from paper_2105_09671_amd import sur_train, surrogate
    wpath = os.path.join(ROOT, "paper_2105_09671_amd", "weights", "sur256.npz")
    net = surrogate.Surrogate(256, 256)
    net.set_weights(np.load(wpath)["weights"])
    out["sur256"] = sur_train.evaluate(net, list(range(100000, 100256)))
    out["sur256"]["roofline"] = {"bound": "mfma", "peak": 2500.0, "unit": "TFLOP/s",
                                 "achieved": out["sur256"]["forward"]["TFLOPs"],
                                 "frac": round(out["sur256"]["forward"]["TFLOPs"] / 2500.0, 4)}
    net.close()
    log("extra sur256", {k: v for k, v in out["sur256"].items() if k != "by_kind"})
    # 64 independent 3D grids (sides 24..128), 1000 steps, one persistent launch
    insts3 = workloads.batch3d_instances(64)
    b3 = api.Batch3D([g3.initial().astype("float32") for g3 in insts3],
                     [(g3.h, g3.dt, g3.eps) for g3 in insts3])
    info3 = b3.step(1000)
    t = timed(lambda: b3.step(1000), 3)
    glups = b3.cells * 1000 / t / 1e9
    out["batch3d64_fp32"] = {"GLUPS": round(glups, 2), "f_eff": round(glups * 8 / HBM_PEAK_GBS, 3),
                             "ms": round(t * 1e3, 2), "cells": b3.cells, "launch": info3}
    log("extra batch3d64_fp32", out["batch3d64_fp32"])
    del b3
    # 64x64 FP64 phase separation, 500 steps, one launch (the whole grid as one register tile)
    g1 = workloads.phase64()
    p1 = torch.from_numpy(g1.initial()).cuda()
    t = timed(lambda: api.step2d(p1, g1.h, g1.dt, g1.eps, 500), 5)
    out["phase64_fp64"] = {"GLUPS": round(64 * 64 * 500 / t / 1e9, 3), "ms": round(t * 1e3, 3),
                           "plan": api.plan2d(64, 64, 500, torch.float64)}
    del p1
    out.update(hbm_resident(api, torch, workloads))
    # the paper's own workloads at its tables' step counts (its times: other
    # hardware, context only)
    from paper_2105_09671_amd import paper_suite
    out["paper_suite_fp32"] = paper_suite.timings(torch.float32)
    log("extra paper_suite_fp32", out["paper_suite_fp32"])
    out["table3_err_fp32_vs_fp64"] = paper_suite.err_table()
    log("extra table3_err_fp32_vs_fp64", out["table3_err_fp32_vs_fp64"])
    # the fused FP32 + FP64 trace kernel on 2048^2: 24 algorithmic bytes per
    # cell and step (read 4 + 8, write 4 + 8); depth-7 register tiles, so the
    # effective fraction of 8 TB/s can exceed 1
    g = workloads.circle2048()
    p32 = torch.from_numpy(g.initial()).float().cuda()
    p64 = p32.double()
    api.err_trace(p32, p64, g.h, g.dt, g.eps, 20)
    n = 200
    sec = timed(lambda: api.err_trace(p32, p64, g.h, g.dt, g.eps, n), 3)
    gbs = 24.0 * g.nx * g.ny * n / sec / 1e9
    out["err_trace_2048"] = {"steps": n, "ms": round(sec * 1e3, 3), "GBps_eff": round(gbs, 1),
                             "f_eff": round(gbs / HBM_PEAK_GBS, 3),
                             "G_pair_updates_s": round(g.nx * g.ny * n / sec / 1e9, 1)}
    log("extra err_trace_2048", out["err_trace_2048"])
    del p32, p64
    return out


def batch512(api, torch, workloads, cpu_budget: float) -> dict:
    """512 uneven 2D grids (sides 96..1024, m 3..8, mixed starts), FP32, 5000
    steps per call, replayed from the cached hipGraph: the default graph of one
    launch per temporal block (the line's figure), the single persistent launch
    with a phase barrier per block, and the plan the autotuner picks for this
    batch.  Its own roofline (the batched tile kernel: algorithmic 8 B per
    update, tb_depth updates per cell and launch, over the mean launch time of
    the graph), and the FP64 oracle on a bounded number of steps of all 512
    grids on every host core."""
    n = 5000
    insts = workloads.batch_instances(512)
    fields = [gi.initial().astype("float32") for gi in insts]
    prm = [(gi.h, gi.dt, gi.eps) for gi in insts]
    b = api.Batch(fields, prm)
    cells = b.cells
    modes = {}
    try:
        for name, persistent in (("graph", False), ("persistent", True)):
            api.batched_persistent(persistent)
            info = b.step(n)                      # builds and caches the plan + graph
            torch.cuda.synchronize()
            t = timed(lambda: b.step(n), 1)
            api.check()
            modes[name] = {"GLUPS": round(cells * n / t / 1e9, 2), "ms": round(t * 1e3, 2),
                           "launch": info}
            log("extra batch512_fp32 %s" % name, modes[name])
    finally:
        api.batched_persistent(False)
    api.tune_clear()
    best = b.autotune(probe_steps=200)
    info = b.step(n)
    torch.cuda.synchronize()
    t = timed(lambda: b.step(n), 1)
    modes["autotuned_graph"] = {"GLUPS": round(cells * n / t / 1e9, 2), "ms": round(t * 1e3, 2),
                                "tune": best, "launch": info}
    log("extra batch512_fp32 autotuned_graph", modes["autotuned_graph"])
    api.tune_clear()
    g = modes["graph"]
    launches = g["launch"]["blocks"]
    sec = g["ms"] / 1e3
    alg = 8.0 * cells * n / launches
    traffic = measured_traffic(TRAFFIC_BATCH)
    res = {"GLUPS": g["GLUPS"], "f_eff": round(g["GLUPS"] * 8 / HBM_PEAK_GBS, 3), "ms": g["ms"],
           "cells": cells, "mode": "graph of one launch per temporal block (built-in tile)",
           "modes": modes,
           "roofline": {"bound": "hbm", "kernel": "batched_phase_kernel<float>",
                        "achieved": round(alg / (sec / launches) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(alg / (sec / launches) / 1e9 / HBM_PEAK_GBS, 4),
                        "traffic": traffic,
                        "frac_meas": (round(traffic / (sec / launches) / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic is not None else None),
                        "algorithmic_bytes_per_launch": int(alg),
                        "avg_launch_us": round(sec / launches * 1e6, 3), "launches_timed": launches}}
    del b
    if cpu_budget > 0:
        res["cpu_baseline"] = cpu_baseline_batch(fields, prm, cells, n, cpu_budget)
        log("extra batch512_fp32 cpu_baseline", res["cpu_baseline"])
    return res


def cpu_baseline_batch(fields, prm, cells: int, nsteps: int, budget_s: float) -> dict:
    """The FP64 oracle on all 512 grids, every host core, as many steps as fit
    about budget_s."""
    import numpy as np
    import oracle
    threads = oracle.cpus_available()
    f64 = [f.astype(np.float64) for f in fields]
    hs, dts, es = ([p[i] for p in prm] for i in range(3))
    probe = 2
    while True:
        t0 = time.perf_counter()
        oracle.step_batched2d(f64, hs, dts, es, probe, threads)
        el = time.perf_counter() - t0
        if el > 0.05 * budget_s or probe >= nsteps // 4:
            break
        probe *= 4
    steps = int(max(2, min(nsteps, budget_s / max(el / probe, 1e-9))))
    t0 = time.perf_counter()
    oracle.step_batched2d(f64, hs, dts, es, steps, threads)
    el = time.perf_counter() - t0
    return {"value": round(cells * steps / el / 1e9, 4), "unit": "GLUPS", "cores": threads,
            "kind": "oracle",
            "sample": "all 512 grids (%d cells), FP64 plain loops, first %d of the %d steps on %d "
                      "threads (%.1f s)" % (cells, steps, nsteps, threads, el)}


def hbm_resident(api, torch, workloads) -> dict:
    """Grids far larger than the last-level cache: every launch streams its
    tile rows from HBM.  Also the device's achievable copy bandwidth."""
    from paper_2105_09671_amd import inputs
    out = {}
    n = workloads.HBM_STEPS
    g = workloads.hbm16k()
    t = inputs.random_field_torch((g.ny, g.nx), g.seed, g.stream, dtype=torch.float32, device="cuda")
    api.step2d(t, g.h, g.dt, g.eps, n)
    sec = timed(lambda: api.step2d(t, g.h, g.dt, g.eps, n), 3)
    glups = g.nx * g.ny * n / sec / 1e9
    out["hbm16k_fp32"] = {"GLUPS": round(glups, 2), "f_eff": round(glups * 8 / HBM_PEAK_GBS, 3),
                          "ms": round(sec * 1e3, 2), "steps": n,
                          "plan": api.plan2d(g.nx, g.ny, n, torch.float32)}
    log("extra hbm16k_fp32", out["hbm16k_fp32"])
    # achievable HBM bandwidth: a 1 GiB device-to-device copy (read + write)
    dst = torch.empty_like(t)
    dst.copy_(t)
    sec = timed(lambda: dst.copy_(t), 5)
    out["copy_1GiB"] = {"GBps": round(2 * t.numel() * 4 / sec / 1e9, 1), "ms": round(sec * 1e3, 3)}
    log("extra copy_1GiB", out["copy_1GiB"])
    del t, dst
    api.release_work()
    g3 = workloads.hbm1024c()
    t = inputs.random_field_torch((g3.nz, g3.ny, g3.nx), g3.seed, 0, dtype=torch.float32, device="cuda")
    api.step3d(t, g3.h, g3.dt, g3.eps, n)
    sec = timed(lambda: api.step3d(t, g3.h, g3.dt, g3.eps, n), 3)
    glups = g3.nx * g3.ny * g3.nz * n / sec / 1e9
    out["hbm1024c_fp32"] = {"GLUPS": round(glups, 2), "f_eff": round(glups * 8 / HBM_PEAK_GBS, 3),
                            "ms": round(sec * 1e3, 2), "steps": n,
                            "plan": api.plan3d(g3.nx, g3.ny, g3.nz, n, torch.float32)}
    log("extra hbm1024c_fp32", out["hbm1024c_fp32"])
    del t
    api.release_work()
    torch.cuda.empty_cache()
    return out


def only(name: str) -> dict:
    """One secondary workload alone (for profiling its kernels): one warm-up
    call, one timed call."""
    import torch
    from paper_2105_09671_amd import api, workloads
    if name == "batch512":
        insts = workloads.batch_instances(512)
        b = api.Batch([g.initial().astype("float32") for g in insts], [(g.h, g.dt, g.eps) for g in insts])
        b.step(5000)
        t = timed(lambda: b.step(5000), 1)
        return {"workload": name, "GLUPS": round(b.cells * 5000 / t / 1e9, 2), "ms": round(t * 1e3, 2)}
    if name == "sep256c":
        g3 = workloads.sep256c()
        p3 = torch.from_numpy(g3.initial()).float().cuda()
        api.step3d(p3, g3.h, g3.dt, g3.eps, 2000)
        t = timed(lambda: api.step3d(p3, g3.h, g3.dt, g3.eps, 2000), 3)
        return {"workload": name, "GLUPS": round(256 ** 3 * 2000 / t / 1e9, 2), "ms": round(t * 1e3, 2)}
    if name == "batch3d64":
        insts = workloads.batch3d_instances(64)
        b3 = api.Batch3D([g.initial().astype("float32") for g in insts], [(g.h, g.dt, g.eps) for g in insts])
        info = b3.step(1000)
        t = timed(lambda: b3.step(1000), 3)
        return {"workload": name, "GLUPS": round(b3.cells * 1000 / t / 1e9, 2), "ms": round(t * 1e3, 2),
                "launch": info}
    if name == "hbm16k":
        from paper_2105_09671_amd import inputs
        g = workloads.hbm16k()
        t = inputs.random_field_torch((g.ny, g.nx), g.seed, g.stream, dtype=torch.float32, device="cuda")
        n = workloads.HBM_STEPS
        api.step2d(t, g.h, g.dt, g.eps, n)
        sec = timed(lambda: api.step2d(t, g.h, g.dt, g.eps, n), 1)
        return {"workload": name, "GLUPS": round(g.nx * g.ny * n / sec / 1e9, 2),
                "ms": round(sec * 1e3, 2), "plan": api.plan2d(g.nx, g.ny, n, torch.float32)}
    if name == "sur_forward":
        import numpy as np
        from paper_2105_09671_amd import sur_train
        from paper_2105_09671_amd.surrogate import Surrogate
        net = Surrogate(256, 256)
        net.set_weights(np.load(os.path.join(ROOT, "paper_2105_09671_amd", "weights", "sur256.npz"))["weights"])
        res = sur_train.forward_rate(net, 256, reps=2)
        net.close()
        return {"workload": name, **res}
    if name == "sur256":
        import numpy as np
        from paper_2105_09671_amd import sur_train
        from paper_2105_09671_amd.surrogate import Surrogate
        net = Surrogate(256, 256)
        net.set_weights(np.load(os.path.join(ROOT, "paper_2105_09671_amd", "weights", "sur256.npz"))["weights"])
        res = sur_train.evaluate(net, list(range(100000, 100256)))
        net.close()
        return {"workload": name, "plain_ms": res["plain_ms"], "surrogate_ms": res["surrogate_ms"]}
    raise SystemExit("bench.py --only: unknown workload %r" % name)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed solves of the workload")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves before timing")
    ap.add_argument("--no-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of oracle work")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run a 256 MiB device copy (counter scale reference)")
    ap.add_argument("--only", default="", choices=["", "batch512", "batch3d64", "sep256c", "hbm16k", "sur256", "sur_forward"],
                    help="run one secondary workload alone (to profile its kernels)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this stepper runs on one GPU only; --gpus %d (WORLD_SIZE %d) is not "
              "supported" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2105_09671_amd import api, params, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_ref:
        # a device-to-device copy of 256 MiB: the scale reference of the counters
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.only:
        print(json.dumps(only(args.only)))
        return
    g = workloads.circle2048()
    phi0 = g.initial()
    phi_init = torch.from_numpy(phi0.astype("float32")).cuda()
    phi = phi_init.clone()
    api.work_like(phi)
    plan = api.plan2d(g.nx, g.ny, NSTEPS, torch.float32)
    log("plan", plan)


    for i in range(args.warmup):
        api.step2d(phi, g.h, g.dt, g.eps, NSTEPS)
        torch.cuda.synchronize()
        log("warmup %d done" % (i + 1))
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        api.step2d(phi, g.h, g.dt, g.eps, NSTEPS)
    end.record()
    torch.cuda.synchronize()
    sec = start.elapsed_time(end) / 1e3
    ms_per_step = sec * 1e3 / max(args.steps, 1)
    cells = g.nx * g.ny
    value = cells * NSTEPS * args.steps / sec / 1e9
    log("timed %d solves: %.2f ms each, %.1f GLUPS" % (args.steps, ms_per_step, value))

    # roofline of the dominant kernel: algorithmic bytes per launch / mean launch time
    launches = plan["launches"] * args.steps
    avg_launch = sec / launches
    alg_bytes = 2 * 4 * cells * NSTEPS / plan["launches"]
    achieved = alg_bytes / avg_launch / 1e9
    traffic = measured_traffic(TRAFFIC_HEADLINE.get(plan["kernel"]))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            # the true HBM fraction: counter bytes per launch / launch time
            "frac_meas": (round(traffic / avg_launch / 1e9 / HBM_PEAK_GBS, 4)
                          if traffic is not None else None),
            "kernel": {4: "tile2d_reg_kernel<float>", 6: "tile2d_regw_kernel<float>",
                       3: "tile2d_inplace_kernel<float>"}.get(
                plan["kernel"], "tile2d_kernel<float,%d>" % plan["tile_x"]),
            "algorithmic_bytes_per_launch": int(alg_bytes),
            "avg_launch_us": round(avg_launch * 1e6, 3), "launches_timed": launches}

    # the same launches against the instruction-issue bound of the register
    # kernels: 9 VALU instructions per computed cell in 64-wide tiles (two
    # cross-lane shifts, one folded into an add), 8 in 128-wide tiles (one
    # shift, folded), halo recomputation included; 256 CUs x 64 lanes x 2.4 GHz
    # with packed FP32 off.  Register tiles sit flush against the domain edges.
    roof_alu = None
    vpc = {4: 9, 6: 8}.get(plan["kernel"])
    if vpc:
        K, LX, LY = plan["tb_depth"], plan["tile_x"], plan["tile_y"]

        def flush_tiles(n, L):
            return 1 if n <= L else 1 + -(-(n - L) // (L - 2 * K))
        tiles = flush_tiles(g.nx, LX) * flush_tiles(g.ny, LY)
        computed = tiles * LX * LY * NSTEPS / plan["launches"]
        peak = 256 * 64 * 2.4e9 / vpc / 1e9
        ach = computed / avg_launch / 1e9
        roof_alu = {"bound": "alu", "achieved": round(ach, 1), "peak": round(peak, 1),
                    "unit": "G computed cell-updates/s", "frac": round(ach / peak, 4),
                    "valu_per_cell": vpc, "useful_fraction": round(cells / (tiles * LX * LY), 4)}

    # correctness check of the timed workload: one fresh solve, radius vs the law
    phi.copy_(phi_init)
    api.step2d(phi, g.h, g.dt, g.eps, NSTEPS)
    V = float(torch.sum(0.5 * (1.0 + phi.double())).item()) * g.h ** 2
    R = math.sqrt(V / math.pi)
    law = params.radius_law(0.25, NSTEPS * g.dt, 2)
    check = {"R_T": round(R, 6), "R_law": round(law, 6), "err_over_h": round(abs(R - law) / g.h, 3)}
    log("radius check", check)

    extra = {} if args.no_extra else extras(api, torch, workloads, params,
                                              0 if args.no_cpu else args.cpu_budget)
    cpu = None
    if not args.no_cpu:
        log("cpu baseline ...")
        cpu = cpu_baseline(phi0, g, args.cpu_budget)
        log("cpu baseline", cpu)

    line = {
        "metric": "grid-point updates/s (GLUPS), % HBM roofline", "value": round(value, 2),
        "unit": "GLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "circle2048: 2D 2048x2048, h=1/2048, dt=0.1h^2, eps_4, "
                               "circle R0=0.25, 20000 explicit steps per solve",
                   "nx": g.nx, "ny": g.ny, "nsteps": NSTEPS, "plan": plan},
        "roofline": roof, "roofline_alu": roof_alu, "cpu_baseline": cpu, "radius_check": check, "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
