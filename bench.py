#!/usr/bin/env python3
"""Benchmark of the SPH fluid / rigid-body step on one MI355X.

Workload: 3D closed box filled with fluid, 100^3 interior sites (dx = 0.01),
3 wall layers, 64 rigid spheres (radii U(4, 8) dx, densities 1.2-3 x fluid),
1,191,016 particles; FP32 pair sweep, FP64 per-body reductions and rigid
integration.  Inputs are seeded and synthetic (no dataset).

A step is one full time step of the method (kick/drift, neighbour search,
density, extrapolation, forces, per-body reduction, second kick).  The
metric is pair interactions per second: ordered particle pairs within the
kernel support with at least one fluid member, once per step, over the
timed steps, with the scene resident in HBM.

Printed as one JSON line: value, the roofline of the dominant kernel (the
force/heat gather, measured live with HIP events), the FP64 path's
throughput and the FP32 error against the FP64 oracle, p50/p99 step latency,
and the oracle timed on the host cores (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SPH pair interactions/s, FP32 vs FP64 at stated error; p50/p99 step latency"
UNIT = "pair interactions/s"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0

# Algorithmic floating-point operations per pair (each add, subtract,
# multiply, divide and square root of the paper's formulas counted once):
#   force pair (eq. nummeth_fluid_momentum, 3D): distance 8, sqrt 1, dW/dr 15,
#   volumes 5, averaged pressure 5, averaged viscosity 4, coefficient 2,
#   three components x 6 = 18  -> 58
#   conduction adds 11 per thermal pair.
FLOPS_FORCE_PAIR = 58
FLOPS_DENSITY_PAIR = 28
FLOPS_EXTRAP_PAIR = 46
#   neighbour search (Sec. "Parallelization via spatial decomposition":
#   cells of edge r_c, every particle of the 27 surrounding cells is a
#   candidate): one distance test = 3 subtractions, 3 multiplications,
#   2 additions -> 8
FLOPS_CANDIDATE = 8


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=40)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-side", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--other-steps", type=int, default=100,
                    help="steps of the reduced thermal / moving-wall workloads; 0 skips them")
    ap.add_argument("--serve-scenes", type=int, default=24,
                    help="scenes of the serving run (continuous batching); 0 skips it")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (calibrates HBM byte counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic_3d_column_64_spheres.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2103_07925_amd", "csrc", "sph_kernels.hip")


def measured_traffic(kernel):
    """Memory traffic per launch of `kernel` ("build" or "forces") from the
    committed counter summary, or None when the kernel source has changed
    since the counters were taken."""
    import hashlib
    import re
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    b = re.search(r"traffic_bytes_per_launch_%s:\s*([0-9.eE+]+)" % kernel, txt)
    if not m or not b:
        return None
    if hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest() != m.group(1):
        return None
    return float(b.group(1))


def candidate_tests(cell_of_id, grid):
    """Distance tests of the cell-list search: every particle tests every
    other particle of the 27 (9 in 2D) cells around its own."""
    nx, ny, nz = (int(grid[0]), int(grid[1]), max(int(grid[2]), 1))
    cnt = np.bincount(np.asarray(cell_of_id, np.int64), minlength=nx * ny * nz).astype(np.int64)
    c3 = cnt.reshape(nz, ny, nx)
    pad = np.pad(c3, 1)
    box = np.zeros_like(c3)
    dzs = (-1, 0, 1) if nz > 1 else (0,)
    for dz in dzs:
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                box += pad[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
    return int(np.sum(c3 * box) - cnt.sum())


def serving_run(n_scenes, seed):
    """A short continuous-batching run: n_scenes requests of 1e4-1e5
    particles (2D box, 3D column, thermal grains), 50 steps each, arrivals
    at 0.8 of the capacity measured on the same requests, pool budget a
    third of their total footprint."""
    from paper_2103_07925_amd import serve as SV
    be = SV.GpuBackend()
    reqs = SV.make_requests(n_scenes, seed=seed, n_range=(1e4, 1e5), steps=50)
    total = sum(be.footprint(r) for r in reqs)
    budget = max(total // 3, max(be.footprint(r) for r in reqs))
    cal = SV.Server(be, budget, 128).run(reqs)
    rate = 0.8 * len(reqs) / cal["makespan_s"]
    rng = np.random.default_rng(seed + 1)
    t = 0.0
    for r in reqs:
        t += float(rng.exponential(1.0 / rate))
        r.arrival = t
    rep = SV.Server(be, budget, 128).run(reqs)
    rep.update({"budget_bytes": int(budget), "total_footprint_bytes": int(total), "arrival_rate_per_s": rate,
                "capacity_pair_interactions_per_s": cal["pair_interactions_per_s"],
                "requests": f"{n_scenes} scenes, 1e4-1e5 particles log-uniform, 50 steps each, FP32 sweep"})
    return rep


def timed_workload(B, sc, steps, label):
    """FP32 sweep timing of another workload with the per-stage split."""
    import torch
    g = B.SphScene(sc, precision=B.SPH_FP32_SWEEP)
    g.step(5)
    g.sync()
    p0 = g.stats().pairs_total
    g.sph_scene_enable_timers(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    g.sync()
    st = g.stats()
    tm = g.sph_scene_read_timers()
    nrec = max(tm["steps"], 1)
    stage = {k: tm[k] / nrec for k in B.SphScene.STAGES}
    out = {
        "workload": label, "n_particles": int(sc.n), "counts": sc.counts(), "steps": steps,
        "ms_per_step": 1e3 * el / steps, "pair_interactions_per_s": (st.pairs_total - p0) / el,
        "stage_ms_per_step": stage,
        # the split the moving-wall configuration asks for
        "split_ms_per_step": {
            "neighbour_search": stage["integrate"] + stage["neighbor_search"],
            "interaction_sweep": stage["density"] + stage["extrapolate"] + stage["forces"],
            "per_body_reduction": stage["body_reduce"] + stage["rigid_velocity"],
        },
        "bodies_end": int(st.n_bodies), "melted": int(st.n_melted), "solidified": int(st.n_solidified),
    }
    del g
    torch.cuda.empty_cache()
    return out


def calibrate_copy(mib):
    """A plain device-to-device copy of a known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the same profiler run."""
    import torch
    n = mib * (1 << 20)
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n, "launches": 5}), flush=True)


def field_errors(sc, g, o, O, S):
    """Max field-scaled errors of a GPU scene against the oracle."""
    gf = g.sph_scene_read_particles(["X", "U", "RHO", "P"])
    fl = sc.kind == S.FLUID
    c = math.sqrt(sc.materials[0].p0 / sc.materials[0].rho0)
    e = {
        "x_over_dx": float(np.max(np.abs(gf["X"] - o.get(O.F_X))) / sc.dx),
        "u_over_c10": float(np.max(np.abs(gf["U"] - o.get(O.F_U))) / (c / 10.0)),
        "rho_over_rho0": float(np.max(np.abs(gf["RHO"][fl] - o.get(O.F_RHO)[fl])) / sc.materials[0].rho0),
        "p_over_p0": float(np.max(np.abs(gf["P"][fl] - o.get(O.F_P)[fl])) / sc.materials[0].p0),
    }
    gb, ob = g.bodies(), o.bodies()
    e["body_r_over_dx"] = float(np.max(np.abs(gb[:, 1:4] - ob[:, 1:4])) / sc.dx)
    e["body_u_over_c10"] = float(np.max(np.abs(gb[:, 8:11] - ob[:, 8:11])) / (c / 10.0))
    return e


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              f"(multi-GPU sharding is a design note, not implemented).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2103_07925_amd import scenes as S
    from paper_2103_07925_amd import sphrb as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    sc = S.config_c2(seed=args.seed, n_side=args.n_side)
    counts = sc.counts()

    # ---- FP32 sweep: timed region ----------------------------------------
    g = B.SphScene(sc, precision=B.SPH_FP32_SWEEP)
    g.step(args.warmup)
    g.sync()
    p_before = g.stats().pairs_total
    g.sph_scene_enable_timers(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.sync()
    st = g.stats()
    pairs_timed = st.pairs_total - p_before
    elapsed = t1 - t0
    value = pairs_timed / elapsed
    tm = g.sph_scene_read_timers(with_steps=True)
    nrec = max(tm["steps"], 1)
    step_ms = tm["step_ms"]
    forces_ms = tm["forces"] / nrec
    build_ms = tm["density"] / nrec
    # pairs the force kernel evaluates per launch: all neighbours of fluid
    # particles plus the fluid neighbours of rigid particles
    force_pairs = st.pairs_fluid + st.pairs_rigid
    achieved_tflops = force_pairs * FLOPS_FORCE_PAIR / (forces_ms * 1e-3) / 1e12
    # the list build: the cell-list distance tests of every particle and the
    # density sum of every fluid particle (its own W(0) included)
    _, cell_of_id = g.cell_order()
    cand = candidate_tests(cell_of_id, st.grid)
    dens_terms = st.pairs_fluid + counts["fluid"]
    build_flops = cand * FLOPS_CANDIDATE + dens_terms * FLOPS_DENSITY_PAIR
    build_tflops = build_flops / (build_ms * 1e-3) / 1e12
    stage_avg = {k: tm[k] / nrec for k in B.SphScene.STAGES}
    g.sph_scene_enable_timers(False)
    del g

    # ---- FP64 path ---------------------------------------------------------
    g64 = B.SphScene(sc, precision=B.SPH_FP64)
    g64.step(3)
    g64.sync()
    p0 = g64.stats().pairs_total
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g64.step(args.fp64_steps)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    g64.sync()
    value64 = (g64.stats().pairs_total - p0) / t64
    del g64
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "3D fluid column in a closed box with 3-layer walls and 64 rigid spheres "
                        "(radii 4-8 dx, density 1.2-3x fluid), FP32 pair sweep, FP64 body sums",
            "n_particles": counts["n"], "n_fluid": counts["fluid"], "n_wall": counts["wall"],
            "n_rigid": counts["rigid"], "n_bodies": counts["bodies"], "dx": sc.dx,
            "pairs_per_step": int(st.pairs_last), "seed": args.seed,
        },
        "roofline": None,   # the kernel of the two below with the longer launches
        "rooflines": {
            "build": {
                "bound": "alu",
                "kernel": "list build + density + EOS (k_build_density)",
                "achieved": build_tflops,
                "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s",
                "frac": build_tflops / PEAK_FP32_TFLOPS,
                "traffic": measured_traffic("build"),
                "candidate_tests_per_launch": cand,
                "flops_per_candidate": FLOPS_CANDIDATE,
                "density_terms_per_launch": int(dens_terms),
                "flops_per_density_term": FLOPS_DENSITY_PAIR,
                "avg_launch_ms": build_ms,
            },
            "forces": {
                "bound": "alu",
                "kernel": "forces (momentum + coupling + contact gather, k_forces_list)",
                "achieved": achieved_tflops,
                "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s",
                "frac": achieved_tflops / PEAK_FP32_TFLOPS,
                "traffic": measured_traffic("forces"),
                "pairs_per_launch": int(force_pairs),
                "flops_per_pair": FLOPS_FORCE_PAIR,
                "avg_launch_ms": forces_ms,
            },
        },
        "stage_ms_per_step": stage_avg,
        "step_latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "fp64_path": {"value": value64, "unit": UNIT, "steps": args.fp64_steps,
                      "fp32_speedup": value / value64},
    }

    dom = "build" if build_ms >= forces_ms else "forces"
    out["roofline"] = dict(out["rooflines"][dom])

    if args.other_steps > 0:
        tv = S.config_c2(seed=args.seed)
        tv.p_b = tv.materials[0].p0
        out["other_workloads"] = [
            timed_workload(B, tv, args.other_steps,
                           "the same 3D column with the transport-velocity formulation on (background pressure "
                           "p_b = p0, as in the paper's examples)"),
        ]
        del tv
        gs = S.config_gastric(seed=args.seed)
        out["other_workloads"].append(
            timed_workload(B, gs, args.other_steps,
                           "2D gastric-shaped box 40 x 16 (dx 0.1): moving constriction, 60 boluses dissolving "
                           "into chyme by concentration, juice held at C = 1, p_b = 5 p0"))
        del gs
        c3 = S.config_c3(seed=args.seed)
        out["other_workloads"] += [
            timed_workload(B, c3, args.other_steps,
                           "two-phase thermal grains with conduction, moving heat source and phase switching, "
                           "200x200x100 fluid sites, 2000 grains requested (log-normal radii, median 4.3 dx)"),
        ]
        del c3
        torch.cuda.empty_cache()
        c4 = S.config_c4(seed=args.seed)
        out["other_workloads"].append(
            timed_workload(B, c4, args.other_steps,
                           "container with a moving perforated wall plate and 500 fragments of 2-6 spheres in "
                           "contact, 400x200x100 fluid sites"))
        del c4
        torch.cuda.empty_cache()
    if args.serve_scenes > 0:
        out["serving"] = serving_run(args.serve_scenes, args.seed)
        torch.cuda.empty_cache()

    # ---- CPU baseline: the oracle on a bounded sample ------------------------
    if not args.no_cpu_baseline:
        import oracle as O
        o = O.OracleScene(sc)
        t0 = time.perf_counter()
        pairs = 0
        for _ in range(args.cpu_steps):
            o.step(1)
            pairs += o.pair_count
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": pairs / tc, "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": f"{args.cpu_steps} time steps of the same {counts['n']}-particle scene after set-up "
                      f"({tc:.1f} s, single thread)",
        }
        # accuracy of both GPU paths against the oracle after the same steps
        g32 = B.SphScene(sc, precision=B.SPH_FP32_SWEEP)
        g32.step(args.cpu_steps)
        g32.sync()
        out["fp32_error_vs_oracle"] = field_errors(sc, g32, o, O, S)
        del g32
        g64 = B.SphScene(sc, precision=B.SPH_FP64)
        g64.step(args.cpu_steps)
        g64.sync()
        out["fp64_error_vs_oracle"] = field_errors(sc, g64, o, O, S)
        del g64
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
