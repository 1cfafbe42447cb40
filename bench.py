"""Benchmark: explicit APIC-MPM step on one MI355X.

Workload: the elastic cube of the benchmark spec's metric -- 3D, 128^3 cells on the
unit cube, quadratic B-spline, cube [0.25, 0.75]^3 at 8 particles per cell
(2,097,152 particles), neo-Hookean E = 1e4, nu = 0.3, rho = 1000, gravity
-9.8 along z, sticky floor, dt = 1e-4, binary32 cell + offset positions with
compensated grid accumulation.  Inputs are seeded and synthetic and resident
in HBM before the timed region.

One step = (re-sort every --sort-every steps) + P2G + grid update + G2P,
each through the C ABI on torch's current stream.  The timed region runs
without instrumentation; the same steps are then repeated with HIP events
bracketing every phase, and the dominant phase's average duration gives the
roofline figure.  The FP64 CPU oracle is timed on a bounded sample of
the same workload as the CPU baseline.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "APIC particle-updates/s (P2G+grid+G2P), 3D 2M ptcl; served p50/p99 latency"

# Algorithmic bytes (binary32, 3D) -- what the method itself must move:
#   particle read by P2G: cell 4 + off 12 + v 12 + B 36 + F 36 + m 4 = 104 B
#   particle read by G2P: cell 4 + off 12 + F 36 = 52 B; written: cell, off, v, B, F = 100 B
#   grid node: P2G writes m + mv (16 B; +16 B error terms when compensated),
#   the grid update reads them and writes vt (12 B), G2P reads vt (12 B).
P2G_PARTICLE_B = 104
G2P_PARTICLE_B = 52 + 100
NODE_MMV_B = 16
NODE_VT_B = 12
# whole step: state read once (104 B) and written once (100 B) per particle;
# per active node m and m v written and read (2 x 16 B), vt written and read (2 x 12 B)
STEP_PARTICLE_B = 204
STEP_NODE_B = 56


def _ensure_built():
    lib = os.path.join(ROOT, "paper_1603_06188_amd", "libapic.so")
    if not os.path.exists(lib):
        from paper_1603_06188_amd.build import build_library
        build_library()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cube128.txt")


def measured_traffic(phase: str):
    """HBM bytes per launch of the phase's kernel from the committed counter
    summary, or None when there is none or the kernel sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    from paper_1603_06188_amd import profile_traffic

    summ = profile_traffic.read_summary(TRAFFIC_FILE)
    if summ.get("source_sha256") != profile_traffic.source_hash():
        return None
    v = summ.get(f"k_{phase}_traffic_bytes")
    return float(v) if v is not None else None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads() -> int:
    """Cores this process may use: its affinity set, capped by OMP_NUM_THREADS
    when that is set (the share of the host the job was given)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(n, 1)


def cpu_baseline(scene, budget_s: float = 12.0, max_steps: int = 40):
    """Time the FP64 oracle on the full particle set of the workload: on all
    the host cores this job has (particles split into blocks, private grids
    summed in thread order) for as many steps as fit in about budget_s, and
    on one thread (the serial checker) for one step."""
    import oracle

    g = oracle.Grid(scene.dim, scene.degree, scene.cells, scene.dx)

    def run(threads, steps_max, budget):
        oracle.set_threads(threads)
        x, v, B, F = scene.x, scene.v, scene.B, scene.F
        steps = 0
        t0 = time.perf_counter()
        try:
            while steps < steps_max:
                r = oracle.step(g, x, v, B, F, scene.m, scene.V, scene.model, scene.mu, scene.lam, scene.dt,
                                scene.gravity, scene.band)
                x, v, B, F = r["x_new"], r["v_new"], r["B_new"], r["F_new"]
                steps += 1
                if time.perf_counter() - t0 >= budget:
                    break
        finally:
            oracle.set_threads(1)
        return steps, time.perf_counter() - t0

    cores = _host_threads()
    steps, el = run(cores, max_steps, budget_s)
    steps1, el1 = run(1, 1, 0.0)
    return {
        "value": scene.n * steps / el,
        "unit": "particle-updates/s",
        "cores": cores,
        "kind": "oracle",
        "cpu_model": _cpu_model(),
        "sample": f"full {scene.n}-particle cube, {steps} step(s) in {el:.1f} s on {cores} thread(s) "
                  f"(FP64 C oracle, OpenMP over particle blocks)",
        "single_thread": {"value": scene.n * steps1 / el1, "steps": steps1, "seconds": round(el1, 2)},
    }


def served(pool_size: int, duration: float, load: float, seed: int = 6):
    """Config 5: Poisson arrivals at `load` x the saturated batched capacity,
    replayed against the batch server and against sequential per-scene solves."""
    from paper_1603_06188_amd import serve

    pool = serve.Pool(serve.request_pool(pool_size, seed=5))
    mean_n = sum(pool.particles(k) for k in range(len(pool))) / len(pool)
    capacity = serve.saturated_rate(pool)                       # particle-updates/s
    rate = load * capacity / (mean_n * 275.0)                   # requests/s (mean 275 steps)
    trace = serve.poisson_trace(rate, duration, len(pool), seed=seed)
    out = {"requests": len(trace), "rate_per_s": rate, "load": load, "capacity_updates_per_s": capacity,
           "pool_bodies": len(pool), "mean_particles": mean_n, "trace_s": duration}
    batch_server = serve.BatchServer(pool)
    out["mem_budget_bytes"] = batch_server.mem_budget
    for name, server in (("batched", batch_server), ("sequential", serve.SequentialServer(pool))):
        st = server.run([dataclasses.replace(r) for r in trace])
        out[name] = {"p50_s": st.percentile(50), "p99_s": st.percentile(99), "mean_s": float(st.latencies.mean()),
                     "throughput": st.throughput, "wall_s": st.wall}
    return out


def batched(n_scenes: int, steps: int):
    """Config 4: n_scenes bodies stepped by apic_step_batch (launch plan
    tuned by the library over its first calls, then with the K-step sequence
    replayed from a captured HIP graph) vs the per-scene loop."""
    import torch

    from paper_1603_06188_amd import binding as b
    from paper_1603_06188_amd import scenes

    hosts = scenes.many_bodies(n_scenes)
    ds = [b.DeviceScene(h, compensated=True) for h in hosts]
    batch = b.SceneBatch(ds)
    b.apic_batch_set_plan(-1)
    count = b.apic_batch_plan_count()
    for _ in range(2 * count + 1):  # the tuner times every plan twice, then keeps the fastest
        batch.step(1)
    plan, ns = batch.tuning()
    batch.step_each(2)
    torch.cuda.synchronize()
    total = sum(h.n for h in hosts)
    per_block, per_cu = b.apic_batch_plan_info(plan) if plan >= 0 else (None, None)
    res = {"scenes": n_scenes, "particles": total, "steps": steps,
           "plan": {"chosen": plan, "particles_per_block": per_block, "blocks_per_cu": per_cu,
                    "ns_per_update": [None if v == float("inf") else v for v in ns]}}

    def graph_step(k):
        batch.step(k)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    el = timed(batch.step)
    res["batched"] = {"value": total * steps / el, "ms_per_step": el / steps * 1e3}
    for d in ds:
        d.s.grid.options |= b.APIC_OPT_BATCH_GRAPH
    batch.step(steps)  # captures the graph of this step count
    el = timed(graph_step)
    res["batched_graph"] = {"value": total * steps / el, "ms_per_step": el / steps * 1e3}
    for d in ds:
        d.s.grid.options &= ~b.APIC_OPT_BATCH_GRAPH
    el = timed(batch.step_each)
    res["per_scene_loop"] = {"value": total * steps / el, "ms_per_step": el / steps * 1e3}
    res["speedup"] = res["batched_graph"]["value"] / res["per_scene_loop"]["value"]
    return res


def spheres(steps: int):
    """Config 3: two spinning spheres, 256^3 cells, cubic B-spline, no gravity,
    in binary32 with positions as cell + offset (compensated and plain
    accumulation) and as plain binary32 coordinates, and in binary64.  Momenta are conserved to round-off while the
    spheres touch neither each other nor a wall; the drift per step is
    reported relative to S = sum_p m_p (|x_p| |v_p| + |B_p|_F)."""
    import numpy as np
    import torch

    from paper_1603_06188_amd import binding as b
    from paper_1603_06188_amd import scenes

    out = {}
    for mode, precision, comp, absolute in (("f32_compensated", "fp32", True, False),
                                            ("f32_uncompensated", "fp32", False, False),
                                            ("f32_absolute_positions", "fp32", True, True),
                                            ("f64", "fp64", False, False)):
        s = scenes.spheres3d(precision=precision)
        if absolute:
            s = s.with_state(x=s.x.astype(np.float32).astype(np.float64))
        S = float(np.sum(s.m * (np.linalg.norm(s.x, axis=1) * np.linalg.norm(s.v, axis=1)
                                + np.linalg.norm(s.B.reshape(s.n, -1), axis=1))))
        ds = b.DeviceScene(s, compensated=comp, with_id=False, absolute=absolute)
        ds.step(2)
        torch.cuda.synchronize()
        d0 = ds.diagnostics()
        t0 = time.perf_counter()
        ds.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d1 = ds.diagnostics()
        drift_p = float(np.abs(d1[0:3] - d0[0:3]).max()) / S / steps
        drift_l = float(np.abs(d1[3:6] - d0[3:6]).max()) / S / steps
        out[mode] = {"value": s.n * steps / el, "ms_per_step": el / steps * 1e3, "particles": s.n,
                     "drift_p_per_step": drift_p, "drift_l_per_step": drift_l, "flags": ds.flags()}
        del ds
        torch.cuda.empty_cache()
    return out


def midpoint(steps: int, cells: int = 128):
    """Implicit midpoint steps (apic_step_midpoint, binary64) on the elastic
    cube at two step sizes, with the explicit binary64 step beside it:
    particle-updates/s and simulated time per wall second.  The library
    brackets the particle pass of every CG iteration (and of every force
    evaluation) with HIP events on this stream during the timed steps."""
    import dataclasses

    import torch

    from paper_1603_06188_amd import binding as b
    from paper_1603_06188_amd import scenes

    base = scenes.cube3d(cells=cells, precision="fp64")
    out = {"particles": base.n, "tiles": midpoint_tiles(base)}
    ds = b.DeviceScene(base, with_id=False)
    ds.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ds.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["explicit_dt1e-4"] = {"value": base.n * steps / el, "ms_per_step": el / steps * 1e3,
                              "sim_time_per_s": base.dt * steps / el, "flags": ds.flags()}
    del ds
    torch.cuda.empty_cache()
    for dt in (1e-3, 5e-3):
        s = dataclasses.replace(base, dt=dt)
        ds = b.DeviceScene(s, with_id=False, midpoint=True)
        ds.step_midpoint(1)
        torch.cuda.synchronize()
        b.apic_timing_enable(True)
        b.apic_timing_read()
        t0 = time.perf_counter()
        st = ds.step_midpoint(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        tm = b.apic_timing_read()
        b.apic_timing_enable(False)
        out[f"midpoint_dt{dt:g}"] = {"value": s.n * steps / el, "ms_per_step": el / steps * 1e3,
                                     "sim_time_per_s": dt * steps / el, "newton_per_step": st["newton_iters"] / steps,
                                     "cg_per_step": st["cg_iters"] / steps, "halvings": st["halvings"],
                                     "converged": st["converged"], "flags": st["flags"],
                                     "apply_launches": tm["mid_apply"][0], "apply_us": tm["mid_apply"][1] * 1e3,
                                     "force_launches": tm["mid_force"][0], "force_us": tm["mid_force"][1] * 1e3}
        print(f"midpoint dt={dt:g}: {out[f'midpoint_dt{dt:g}']}", file=sys.stderr, flush=True)
        del ds
        torch.cuda.empty_cache()
    return out


def midpoint_tiles(scene):
    """Key tiles (4^3 base nodes holding particles) and the node tiles their
    regions touch, for the initial state of a 3D scene."""
    import numpy as np

    h = scene.x / scene.dx
    cell = np.floor(h).astype(np.int64)
    off = h - cell
    if scene.degree == 2:
        base = np.where(off < 0.5, cell - 1, cell)
    elif scene.degree == 3:
        base = cell - 1
    else:
        base = cell
    kt = np.unique(base // 4, axis=0)
    near = np.unique(np.concatenate([kt + np.array(d) for d in np.ndindex(2, 2, 2)]), axis=0)
    return {"key_tiles": int(len(kt)), "node_tiles": int(len(near))}


MIDPOINT_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_midpoint_cube128.txt")
MIDPOINT_APPLY_KERNEL = "k_mid_tile<3, 2, 2>"
MIDPOINT_PARTICLE_B = 188  # cell 4, offset 24, F 72, F_hat^{-T} 72, mu - lambda ln J 8, m 8


def midpoint_roofline(res):
    """Roofline of the midpoint step's dominant kernel, the particle pass of
    each CG iteration (operator application), timed live: algorithmic bytes
    per launch = particles x 188 B + the key tiles' region slabs written
    (216 nodes x 3 x 8 B) + the direction p read on the listed node tiles
    (64 nodes x 3 x 8 B), over the mean launch duration; traffic from the
    committed FETCH_SIZE / WRITE_SIZE summary when it matches the sources."""
    mode = res["midpoint_dt0.005"]
    if not mode.get("apply_launches"):
        return None
    tiles = res["tiles"]
    alg = res["particles"] * MIDPOINT_PARTICLE_B + tiles["key_tiles"] * 216 * 24 + tiles["node_tiles"] * 64 * 24
    achieved = alg / (mode["apply_us"] * 1e-6) / 1e9
    traffic = None
    if os.path.exists(MIDPOINT_TRAFFIC):
        from paper_1603_06188_amd import profile_traffic

        summ = profile_traffic.read_summary(MIDPOINT_TRAFFIC)
        if summ.get("source_sha256") == profile_traffic.source_hash():
            v = summ.get("k_mid_tile_3_2_2_traffic_bytes")
            traffic = float(v) if v is not None else None
    return {"bound": "hbm", "kernel": MIDPOINT_APPLY_KERNEL, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
            "frac": achieved / 8000.0, "traffic": traffic, "algorithmic_bytes": alg,
            "duration_us": mode["apply_us"], "launches": mode["apply_launches"]}


def midpoint_cpu_baseline(cells: int = 64, dt: float = 5e-3):
    """The oracle's midpoint step (single thread) on a bounded sample: the
    elastic cube on cells^3, one step."""
    import oracle

    from paper_1603_06188_amd import scenes

    s = scenes.cube3d(cells=cells, precision="fp64")
    g = oracle.Grid(s.dim, s.degree, s.cells, s.dx)
    t0 = time.perf_counter()
    r = oracle.midpoint_step(g, s.x, s.v, s.B, s.F, s.m, s.V, s.model, s.mu, s.lam, dt, s.gravity, s.band,
                             newton_tol=1e-10, cg_tol=1e-8, max_newton=20, max_cg=500)
    el = time.perf_counter() - t0
    return {"value": s.n / el, "unit": "particle-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"elastic cube {cells}^3 cells ({s.n} particles), one midpoint step at dt={dt:g} "
                      f"({r['stats']['newton']} Newton, {r['stats']['cg']} CG iterations), {el:.1f} s"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--sort-every", type=int, default=0)
    ap.add_argument("--cells", type=int, default=128)
    ap.add_argument("--plain", action="store_true", help="uncompensated binary32 accumulation")
    ap.add_argument("--fused", action="store_true",
                    help="APIC_OPT_FUSED_TRANSFER: G2P fused with the next step's P2G")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["cube", "batch", "spheres", "midpoint"], default="cube",
                    help="cube: the 128^3 elastic cube (headline); batch: 512 bodies, batched vs per-scene loop; "
                         "spheres: two spheres on 256^3 cells, cubic, three precision modes; midpoint: implicit "
                         "midpoint steps on the cube in binary64")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-latency replay")
    ap.add_argument("--headline-only", action="store_true",
                    help="cube: skip the adaptive-step and multilinear legs (profiling runs)")
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    ap.add_argument("--serve-pool", type=int, default=16)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--scenes", type=int, default=512)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device-to-device copy three times (known bytes, for "
                         "scaling hardware byte counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU (the explicit APIC step of one scene is not sharded across "
              "GPUs); run with --gpus 1", file=sys.stderr)
        return 2

    _ensure_built()
    import numpy as np
    import torch

    from paper_1603_06188_amd import binding as b
    from paper_1603_06188_amd import scenes

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # a plain 256 MiB device copy (known bytes) that scales the traffic counters
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "batch":
        res = batched(args.scenes, args.steps if args.steps != 100 else 20)
        print(json.dumps({
            "metric": "APIC particle-updates/s, many bodies, batched (tuned launch plan, graph replay) vs per-scene "
                      "loop",
            "value": res["batched_graph"]["value"], "unit": "particle-updates/s", "n_gpus": 1, "steps": res["steps"],
            "warmup": 2, "ms_per_step": res["batched_graph"]["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{res['scenes']} bodies (box/sphere, 8 ppc, N log-uniform 1e3..2e5, grids "
                                   f"32..128), quadratic, neo-Hookean, gravity, dt=1e-4, compensated f32",
                       "particles": res["particles"]},
            "batched_direct": res["batched"], "plan": res["plan"],
            "per_scene_loop": res["per_scene_loop"], "speedup": res["speedup"]}), flush=True)
        return 0
    if args.workload == "spheres":
        res = spheres(args.steps if args.steps != 100 else 20)
        main_mode = res["f32_compensated"]
        print(json.dumps({
            "metric": "APIC particle-updates/s, two spheres 256^3 cubic (~9M particles), angular-momentum drift",
            "value": main_mode["value"], "unit": "particle-updates/s", "n_gpus": 1,
            "steps": args.steps if args.steps != 100 else 20, "warmup": 2, "ms_per_step": main_mode["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "two spheres r=0.2 at 8 ppc, 256^3 cells, cubic B-spline, neo-Hookean, g=0, "
                                   "dt=1e-4", "particles": main_mode["particles"]},
            "modes": res}), flush=True)
        return 0
    if args.workload == "midpoint":
        nsteps = args.steps if args.steps != 100 else 3
        res = midpoint(nsteps, args.cells)
        main_mode = res["midpoint_dt0.005"]
        print(json.dumps({
            "metric": "implicit midpoint APIC particle-updates/s, elastic cube 128^3 (2,097,152 particles)",
            "value": main_mode["value"], "unit": "particle-updates/s", "n_gpus": 1, "steps": nsteps, "warmup": 1,
            "ms_per_step": main_mode["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "elastic cube 128^3, quadratic, neo-Hookean, gravity, sticky floor, implicit "
                                   "midpoint (Newton + mass-inner-product CG), dt=5e-3",
                       "particles": res["particles"]},
            "roofline": midpoint_roofline(res),
            "cpu_baseline": None if args.no_cpu_baseline else midpoint_cpu_baseline(),
            "modes": res}), flush=True)
        return 0
    scene = scenes.cube3d(cells=args.cells)
    compensated = not args.plain
    ds = b.DeviceScene(scene, compensated=compensated, with_id=False, fused=args.fused)
    st = torch.cuda.current_stream()

    # active grid nodes of the initial state (for the byte accounting)
    ds.p2g()
    active = int(np.count_nonzero(ds.export(b.APIC_GRID_MASS)))

    ds.step(args.warmup, args.sort_every)
    torch.cuda.synchronize()
    ds.upload(scene)  # timed steps start from the initial state of the workload
    ds.clear_flags()
    torch.cuda.synchronize()

    # timed region: K whole steps in one apic_step call, no instrumentation
    # (HIP events between phases add ~10 % to the wall time)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ds.step(args.steps, args.sort_every)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    flags = ds.flags()
    # the CFL rule of Sec. 4.3 on the state the timed steps produced (outside the timed region)
    t1 = time.perf_counter()
    cfl_dt = ds.cfl_dt()
    cfl_ms = (time.perf_counter() - t1) * 1e3
    # the same K steps again from the same state, the library bracketing every
    # phase with HIP events on this stream: per-kernel durations for the roofline
    ds.upload(scene)
    ds.clear_flags()
    torch.cuda.synchronize()
    b.apic_timing_enable(True)
    b.apic_timing_read()
    ds.step(args.steps, args.sort_every)
    torch.cuda.synchronize()
    timing = b.apic_timing_read()
    b.apic_timing_enable(False)
    phases = list(timing)
    dur = {p: timing[p][1] for p in phases}
    adaptive = multilinear = None
    if not args.headline_only:
        # the same K steps with adaptive steps (APIC_OPT_ADAPTIVE_DT, nu = 0.5):
        # the CFL rule allows ~0.06 here, so the 1e-4 cap is every step's dt and
        # the work is the fixed-step work plus choosing dt on the device
        ad = b.DeviceScene(dataclasses.replace(scene, cfl=0.5), compensated=compensated, with_id=False, adaptive=True)
        ad.step(args.warmup, args.sort_every)
        ad.upload(scene)
        ad.clear_flags()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ad.step(args.steps, args.sort_every)
        torch.cuda.synchronize()
        el_ad = time.perf_counter() - t2
        ad_dt, _ = ad.step_time()
        adaptive = {"ms_per_step": el_ad / args.steps * 1e3, "vs_fixed": el / el_ad, "cfl": 0.5, "dt_last": ad_dt,
                    "flags": ad.flags()}
        del ad
        # the multilinear kernel with the lagged affine matrix (APIC_MULTILINEAR,
        # Sec. 5.9) against the quadratic one on the same cube as transfer plus
        # gravity only (model 0): with the neo-Hookean force the lagged C_p grows
        # tenfold per step at the free surface (the oracle inverts elements by
        # step 5 at 128^3), so the elastic multilinear cube has no valid steps
        def transfer_run(degree):
            sc = dataclasses.replace(scenes.cube3d(cells=args.cells, degree=degree), model=0)
            dv = b.DeviceScene(sc, compensated=compensated, with_id=False)
            dv.step(args.warmup, args.sort_every)
            dv.upload(sc)
            dv.clear_flags()
            torch.cuda.synchronize()
            t = time.perf_counter()
            dv.step(args.steps, args.sort_every)
            torch.cuda.synchronize()
            el_t = time.perf_counter() - t
            fl = dv.flags()
            dv.upload(sc)
            torch.cuda.synchronize()
            b.apic_timing_enable(True)
            b.apic_timing_read()
            dv.step(args.steps, args.sort_every)
            torch.cuda.synchronize()
            tm = b.apic_timing_read()
            b.apic_timing_enable(False)
            del dv
            return {"value": sc.n * args.steps / el_t if fl == 0 else None, "unit": "particle-updates/s",
                    "ms_per_step": el_t / args.steps * 1e3, "phase_ms": {p: round(tm[p][1], 5) for p in tm},
                    "g2p_GBps": (sc.n * G2P_PARTICLE_B) / (tm["g2p"][1] * 1e-3) / 1e9, "flags": fl}
        multilinear = {"workload": "the cube as transfer + gravity (model 0)", "multilinear": transfer_run(1),
                       "quadratic": transfer_run(2)}

    n = scene.n
    comp_b = 16 if compensated else 0
    alg_bytes = {
        "p2g": n * P2G_PARTICLE_B + active * (NODE_MMV_B + comp_b),
        "grid_update": active * (NODE_MMV_B + comp_b + NODE_VT_B),
        "g2p": n * G2P_PARTICLE_B + active * NODE_VT_B,
    }
    dom = max(("p2g", "grid_update", "g2p"), key=lambda p: dur[p])
    achieved = alg_bytes[dom] / (dur[dom] * 1e-3) / 1e9
    value = n * args.steps / el
    # the whole step against the roofline: what the method itself moves per
    # step (particle state read once and written once, 204 B; m, m v written
    # and read and vt written and read, 56 B per active node) over the
    # measured time per step
    step_bytes = n * STEP_PARTICLE_B + active * STEP_NODE_B
    step_achieved = step_bytes / (el / args.steps) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"elastic cube, {args.cells}^3 grid, quadratic B-spline, {n} particles, neo-Hookean, "
                        f"gravity, dt=1e-4, {'compensated' if compensated else 'plain'} f32 cell+offset",
            "particles": n,
            "grid_cells": args.cells,
            "active_nodes": active,
            "sort_every": args.sort_every,
            **({"fused_transfer": True} if args.fused else {}),
        },
        "phase_ms": {p: round(dur[p], 5) for p in phases},
        "cfl": {"dt_max": cfl_dt, "call_ms": round(cfl_ms, 4)},
        **({"adaptive_dt": adaptive, "multilinear": multilinear} if not args.headline_only else {}),
        "flags": flags,
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if args.fused else measured_traffic(dom),  # counters cover the unfused kernels
            "step_bytes": step_bytes,
            "step_achieved": step_achieved,
            "step_frac": step_achieved / HBM_PEAK_GBS,
        },
    }
    del ds
    torch.cuda.empty_cache()
    if not args.headline_only:
        # config 4 (many bodies, batched vs the per-scene loop), config 3
        # (two spheres, cubic, four precision modes) and the implicit
        # midpoint step, a few steps each
        print("bench: batch leg", file=sys.stderr, flush=True)
        out["batch"] = batched(args.scenes, 10)
        torch.cuda.empty_cache()
        print("bench: spheres leg", file=sys.stderr, flush=True)
        out["spheres"] = spheres(10)
        torch.cuda.empty_cache()
        # the implicit midpoint step on the same cube in binary64 (Sec. 4.1, 4.2)
        print("bench: midpoint leg", file=sys.stderr, flush=True)
        mres = midpoint(3, args.cells)
        out["midpoint"] = {"dt5e-3": mres["midpoint_dt0.005"], "dt1e-3": mres["midpoint_dt0.001"],
                           "explicit_f64_dt1e-4": mres["explicit_dt1e-4"], "roofline": midpoint_roofline(mres)}
        torch.cuda.empty_cache()
    if not args.no_serve:
        print("bench: served leg", file=sys.stderr, flush=True)
        out["served"] = served(args.serve_pool, args.serve_seconds, args.serve_load)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(scene)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
