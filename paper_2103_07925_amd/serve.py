"""Serving loop: continuous batching of independent resident scenes.

Requests (a scene description and a number of steps) arrive over time.  A
request is admitted as soon as its device arena (``sph_scene_arena_bytes``)
fits the pool budget and an active slot is free; it is created on an
admission stream, so set-up overlaps with the steps of the scenes already on
the device.  All admitted scenes are advanced together through one
``SphBatch`` (one launch per interaction sweep over all of them), one step
per launch group, with at most one group in flight while the host admits and
retires.  A scene leaves the batch once its steps are enqueued, its arena
returns to the pool when its last step has completed.

Per (scene, step) the latency is the completion time of that step minus that
of the scene's previous step (the first step counts from admission);
completion times are taken on the host when the step's event completes.
Throughput is the pairs of all completed steps over the makespan.

The scheduling logic is independent of the GPU: ``Server`` drives a backend
object (``GpuBackend`` here; the CPU tests use a stand-in).
"""
from __future__ import annotations

import dataclasses
import json
import math
import sys
import time
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    scene: object             # scenes.Scene
    steps: int
    arrival: float            # seconds after the start of the run
    precision: int = 1        # SPH_FP32_SWEEP


@dataclasses.dataclass
class Record:
    rid: int
    n: int
    steps: int
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    done: List[float] = dataclasses.field(default_factory=list)   # completion time of every step
    pairs: int = 0
    result: Optional[dict] = None


class GpuBackend:
    """Scenes, batches and step events on the GPU through the C ABI."""

    def __init__(self, keep_fields=None):
        import torch
        from . import sphrb
        self.torch = torch
        self.B = sphrb
        self.stream = torch.cuda.Stream()
        self.admit_stream = torch.cuda.Stream()
        self.keep_fields = keep_fields

    def footprint(self, req):
        return self.B.sph_scene_arena_bytes(self.B.Desc(req.scene, req.precision))

    def create(self, req):
        return self.B.SphScene(req.scene, precision=req.precision, stream=self.admit_stream)

    def batch(self, scenes):
        return self.B.SphBatch(scenes, stream=self.stream)

    def step(self, batch, k):
        batch.step(k)
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def wait(self, ev):
        ev.synchronize()

    def finish(self, scene):
        """Pairs of the scene's steps and (optionally) its final fields."""
        scene.sync()
        st = scene.stats()
        res = None
        if self.keep_fields:
            res = scene.sph_scene_read_particles(self.keep_fields)
            res["bodies"] = scene.bodies()
        return int(st.pairs_total), res

    def release(self, scene):
        scene.close()


class Server:
    def __init__(self, backend, budget_bytes: int, max_active: int = 64, steps_per_launch: int = 1,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep):
        self.be = backend
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.k = int(steps_per_launch)
        self.clock = clock
        self.sleep = sleep

    def run(self, requests: List[Request]) -> dict:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        foot = {r.rid: int(self.be.footprint(r)) for r in reqs}
        for r in reqs:
            if foot[r.rid] > self.budget:
                raise ValueError(f"request {r.rid} needs {foot[r.rid]} bytes, above the pool budget {self.budget}")
        recs = {r.rid: Record(r.rid, r.scene.n, r.steps, r.arrival) for r in reqs}
        pending = list(reqs)
        active = []            # [req, scene, steps enqueued]
        draining = []          # scenes whose steps are all enqueued: (req, scene)
        used = 0
        batch = None
        dirty = True
        inflight = None        # (event, [rids stepped], [(req, scene) that finish with it])
        t0 = self.clock()
        peak_active = 0
        launches = 0

        def now():
            return self.clock() - t0

        def complete(fl):
            nonlocal used
            ev, rids, fin = fl
            self.be.wait(ev)
            tc = now()
            for rid in rids:
                recs[rid].done.extend([tc] * self.k)
            for (rq, sc) in fin:
                pairs, res = self.be.finish(sc)
                rec = recs[rq.rid]
                rec.pairs = pairs
                rec.result = res
                rec.finished = tc
                self.be.release(sc)
                used -= foot[rq.rid]

        while pending or active or inflight is not None:
            # admission: arrived, fits the pool, a slot is free
            while pending and pending[0].arrival <= now() and len(active) < self.max_active \
                    and used + foot[pending[0].rid] <= self.budget:
                rq = pending.pop(0)
                sc = self.be.create(rq)
                used += foot[rq.rid]
                recs[rq.rid].admitted = now()
                active.append([rq, sc, 0])
                dirty = True
            peak_active = max(peak_active, len(active))
            if not active:
                if inflight is not None:
                    complete(inflight)
                    inflight = None
                    continue
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - now()))
                continue
            if dirty:
                batch = self.be.batch([a[1] for a in active])
                dirty = False
            ev = self.be.step(batch, self.k)
            launches += 1
            rids = [a[0].rid for a in active]
            fin = []
            for a in active:
                a[2] += self.k
            for a in [a for a in active if a[2] >= a[0].steps]:
                fin.append((a[0], a[1]))
                active.remove(a)
                dirty = True
            if inflight is not None:
                complete(inflight)
            inflight = (ev, rids, fin)
            if dirty:
                batch = None
        makespan = now()
        return self.report(recs, makespan, peak_active, launches)

    def report(self, recs, makespan, peak_active, launches):
        lat, wait, e2e = [], [], []
        pairs = 0
        for rec in recs.values():
            prev = rec.admitted
            for tc in rec.done:
                lat.append(tc - prev)
                prev = tc
            wait.append(rec.admitted - rec.arrival)
            e2e.append(rec.finished - rec.arrival)
            pairs += rec.pairs
        lat_ms = np.array(lat) * 1e3
        self.records = recs
        return {
            "scenes": len(recs),
            "makespan_s": makespan,
            "pair_interactions_per_s": pairs / makespan if makespan > 0 else 0.0,
            "scene_steps": int(sum(len(r.done) for r in recs.values())),
            "step_latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))}
            if len(lat_ms) else None,
            "queue_wait_s": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
            "end_to_end_s": {"p50": float(np.percentile(e2e, 50)), "p99": float(np.percentile(e2e, 99))},
            "peak_active": peak_active,
            "batch_launches": launches,
        }


# ---------------------------------------------------------------------------
# synthetic request stream
# ---------------------------------------------------------------------------

def scene_of_size(kind: str, n_target: int, bodies: int, seed: int):
    """A scene shaped like one of the configurations with about n_target
    particles: "2d" (the falling-disc box), "3d" (fluid column with spheres
    on a grid), "thermal" (two-phase grains with conduction and switching)."""
    from . import scenes as S
    if kind == "2d":
        side = max(8, int(round(math.sqrt(n_target))))
        return S.config_c1(seed=seed, n_side=side, dx=0.8 / side, with_disc=bodies > 0)
    if kind == "3d":
        side = max(10, int(round(n_target ** (1.0 / 3.0))))
        per = max(0, min(5, int(round(bodies ** (1.0 / 3.0)))))
        spacing = max(6, side // max(per, 1))
        rmax = max(1.5, min(0.3 * spacing, 0.55 * (0.3 * spacing ** 3) ** (1.0 / 3.0)))
        sc = S.config_c2(seed=seed, n_side=side, dx=1.0 / side, n_per_axis=per, spacing_sites=spacing,
                         r_range=(0.6 * rmax, rmax))
        return sc
    if kind == "thermal":
        side = max(12, int(round(n_target ** (1.0 / 3.0))))
        g = max(1, bodies)
        med = max(1.5, min(4.3, 0.45 * (0.25 * side ** 3 / g) ** (1.0 / 3.0)))
        return S.config_c3(seed=seed, nsites=(side, side, side), n_grains=g, median_r=med)
    raise ValueError(kind)


def make_requests(n: int, seed: int = 0, n_range=(1e4, 5e5), steps: int = 100, rate: float = 0.0,
                  kinds=("2d", "3d", "thermal"), max_bodies: int = 200, precision: int = 1) -> List[Request]:
    """n requests: kind uniform over `kinds`, particle count log-uniform in
    n_range, bodies uniform in 0..max_bodies, Poisson arrivals at `rate`
    per second (0: all at once)."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    for i in range(n):
        kind = kinds[int(rng.integers(len(kinds)))]
        nt = int(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1]))))
        nb = int(rng.integers(0, max_bodies + 1))
        sc = scene_of_size(kind, nt, nb, seed=int(rng.integers(1 << 30)))
        if rate > 0:
            t += float(rng.exponential(1.0 / rate))
        out.append(Request(rid=i, scene=sc, steps=steps, arrival=t if rate > 0 else 0.0, precision=precision))
    return out


def main():
    import argparse
    ap = argparse.ArgumentParser(description="continuous-batching serving run on one GPU")
    ap.add_argument("--scenes", type=int, default=64)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--n-min", type=float, default=1e4)
    ap.add_argument("--n-max", type=float, default=5e5)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate as a fraction of the measured capacity")
    ap.add_argument("--budget-gb", type=float, default=0.0, help="pool budget; 0: a third of the total footprint")
    ap.add_argument("--max-active", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    be = GpuBackend()
    reqs = make_requests(args.scenes, seed=args.seed, n_range=(args.n_min, args.n_max), steps=args.steps)
    print(f"{len(reqs)} requests, {sum(r.scene.n for r in reqs)} particles", file=sys.stderr, flush=True)
    total = sum(be.footprint(r) for r in reqs)
    budget = int(args.budget_gb * 1e9) if args.budget_gb > 0 else max(total // 3, max(be.footprint(r) for r in reqs))
    # capacity: the same requests all at once (closed loop)
    cal = Server(be, budget, args.max_active).run(reqs)
    cap = len(reqs) / cal["makespan_s"]
    print(f"closed loop: {cal['makespan_s']:.2f} s, {cal['pair_interactions_per_s']:.3g} pairs/s", file=sys.stderr,
          flush=True)
    rate = args.load * cap
    rng = np.random.default_rng(args.seed + 1)
    t = 0.0
    for r in reqs:
        t += float(rng.exponential(1.0 / rate))
        r.arrival = t
    rep = Server(be, budget, args.max_active).run(reqs)
    rep.update({"budget_bytes": budget, "total_footprint_bytes": total, "capacity_scenes_per_s": cap,
                "arrival_rate_per_s": rate, "calibration": cal,
                "n_range": [args.n_min, args.n_max], "steps_per_scene": args.steps})
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
