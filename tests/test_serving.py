"""Serving: admission by footprint and continuous batching (host logic on the
CPU with a stand-in backend), and on the GPU the bitwise equality of every
scene's result alone and in a changing mix."""
import numpy as np
import pytest

from paper_2103_07925_amd import scenes as S
from paper_2103_07925_amd.serve import Request, Server


class FakeScene:
    def __init__(self, req):
        self.req = req
        self.steps = 0


class FakeBackend:
    """Records what the server asks for; every step completes at once."""

    def __init__(self, clock):
        self.clock = clock
        self.batches = []
        self.live = set()
        self.peak_bytes = 0
        self.used = 0

    def footprint(self, req):
        return 100 * req.scene.n

    def create(self, req):
        assert req.arrival <= self.clock.t + 1e-12
        sc = FakeScene(req)
        self.live.add(sc)
        self.used += self.footprint(req)
        self.peak_bytes = max(self.peak_bytes, self.used)
        return sc

    def batch(self, scenes):
        assert all(s in self.live for s in scenes)
        self.batches.append([s.req.rid for s in scenes])
        return list(scenes)

    def step(self, batch, k):
        for s in batch:
            assert s in self.live
            s.steps += k
            assert s.steps <= s.req.steps
        self.clock.t += 0.01
        return object()

    def wait(self, ev):
        pass

    def finish(self, scene):
        assert scene.steps == scene.req.steps
        return scene.steps * scene.req.scene.n, None

    def release(self, scene):
        self.live.remove(scene)
        self.used -= self.footprint(scene.req)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class _Sc:
    def __init__(self, n):
        self.n = n


def test_server_admission_and_batching_on_cpu():
    clock = Clock()
    be = FakeBackend(clock)
    rng = np.random.default_rng(0)
    reqs = [Request(rid=i, scene=_Sc(int(rng.integers(10, 100))), steps=int(rng.integers(1, 6)),
                    arrival=float(0.015 * i)) for i in range(40)]
    budget = 100 * 250
    srv = Server(be, budget, max_active=4, clock=clock, sleep=clock.sleep)
    rep = srv.run(reqs)
    assert be.peak_bytes <= budget
    assert not be.live                                     # every arena returned
    assert max(len(b) for b in be.batches) <= 4
    assert len(be.batches) > 5                             # the mix changed as scenes came and went
    for r in reqs:
        rec = srv.records[r.rid]
        assert len(rec.done) == r.steps
        assert rec.admitted >= r.arrival
        assert rec.pairs == r.steps * r.scene.n
        assert np.all(np.diff([rec.admitted] + rec.done) >= 0)
    assert rep["scene_steps"] == sum(r.steps for r in reqs)
    assert rep["step_latency_ms"]["p99"] >= rep["step_latency_ms"]["p50"] > 0


def test_server_refuses_a_request_above_the_budget():
    clock = Clock()
    be = FakeBackend(clock)
    with pytest.raises(ValueError):
        Server(be, 1000, clock=clock, sleep=clock.sleep).run([Request(0, _Sc(50), 1, 0.0)])


def _mix_requests(B):
    from test_gpu_parity import _scripted_switch_scene, small_3d
    th = S.config_c3(seed=4, nsites=(16, 12, 10), n_grains=3, median_r=2.0, dim=3)
    rg = th.kind == S.RIGID
    th.T[rg & (th.body == np.unique(th.body[rg])[0])] = 70.0
    return [
        Request(0, S.config_c1(seed=3), 12, 0.0, B.SPH_FP64),
        Request(1, small_3d(seed=6), 9, 0.0, B.SPH_FP32_SWEEP),
        Request(2, th, 10, 0.0, B.SPH_FP32_SWEEP),
        Request(3, _scripted_switch_scene(), 10, 0.005, B.SPH_FP64),
        Request(4, small_3d(seed=7), 7, 0.01, B.SPH_FP64),
        Request(5, _tvf(small_3d(seed=8)), 8, 0.0, B.SPH_FP32_SWEEP),
    ]


def _tvf(sc):
    sc.p_b = sc.materials[0].p0
    return sc


FIELDS = ["X", "U", "A", "RHO", "P", "T", "PW", "UW", "FR", "AB", "UD"]


@pytest.mark.gpu
def test_results_alone_and_in_the_mix_are_bitwise_equal():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07925_amd import sphrb as B
    from paper_2103_07925_amd.serve import GpuBackend
    reqs = _mix_requests(B)
    alone = {}
    for r in reqs:
        g = B.SphScene(r.scene, precision=r.precision)
        g.step(r.steps)
        g.sync()
        f = g.sph_scene_read_particles(FIELDS)
        f["bodies"] = g.bodies()
        alone[r.rid] = f
        g.close()
    be = GpuBackend(keep_fields=FIELDS)
    foot = sorted(be.footprint(r) for r in reqs)
    srv = Server(be, budget_bytes=foot[-1] + foot[-2] + foot[-3], max_active=2)
    rep = srv.run(reqs)
    assert rep["scene_steps"] == sum(r.steps for r in reqs)
    waited = [srv.records[r.rid].admitted - r.arrival for r in reqs]
    assert max(waited) > 0                       # admission did bind
    for r in reqs:
        mix = srv.records[r.rid].result
        for key in FIELDS + ["bodies"]:
            assert np.array_equal(alone[r.rid][key], mix[key]), (r.rid, key)


@pytest.mark.gpu
def test_batch_graph_replays_match_lone_steps():
    """A batch steps through captured graphs after its first steps; replays
    interleaved with eager reads give, bit for bit, the lone results."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07925_amd import sphrb as B
    reqs = _mix_requests(B)
    n = 9
    alone = []
    for r in reqs:
        g = B.SphScene(r.scene, precision=r.precision)
        g.step(n)
        g.sync()
        alone.append(g.sph_scene_read_particles(FIELDS))
        g.close()
    scenes = [B.SphScene(r.scene, precision=r.precision) for r in reqs]
    bt = B.SphBatch(scenes, stream=torch.cuda.Stream())    # graphs need a stream of its own
    bt.step(3)
    mid = scenes[0].sph_scene_read_particles(["X"])      # eager work between replays
    assert np.all(np.isfinite(mid["X"]))
    bt.step(2)
    scenes[1].sync()
    bt.step(n - 5)
    for sc, ref in zip(scenes, alone):
        sc.sync()
        got = sc.sph_scene_read_particles(FIELDS)
        for key in FIELDS:
            assert np.array_equal(ref[key], got[key]), key
        assert sc.stats().step == n
