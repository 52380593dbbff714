"""Periodic boundaries on the GPU against the oracle: channels periodic along
y (and z) between walls normal to x, with a rigid body straddling the
periodic boundary; FP64 neighbour lists, cell order and fields bit for bit /
within 1e-10; FP32 within the gates; the FP32 sweep reproduces the plane
Poiseuille profile."""
import numpy as np
import pytest

import oracle as O
from paper_2103_07925_amd import scenes as S

from parity_util import body_errors, field_errors, gpu_fields, oracle_fields, run_pair
from test_gpu_parity import FP64_TOL, B, assert_bitwise_structure

pytestmark = pytest.mark.gpu


def channel(dim, tvf=False):
    if dim == 2:
        sc = S.periodic_channel(dim=2, n_sites=(16, 12, 1), dx=0.1, g=1.0, nu=0.05, c=10.0, seed=2,
                                body_radius=0.25, body_centre=(0.8, 0.05))
        sc.bodies[0].u = (0.0, -1.0, 0.0)
        sc.bodies[0].w = (0.0, 0.0, 2.0)
    else:
        sc = S.periodic_channel(dim=3, n_sites=(12, 9, 9), dx=0.1, g=1.0, nu=0.05, c=10.0, seed=2,
                                body_radius=0.22, body_centre=(0.6, 0.05, 0.85))
        sc.bodies[0].u = (0.0, -1.0, 0.5)
        sc.bodies[0].w = (0.5, -1.0, 2.0)
    if tvf:
        sc.p_b = sc.materials[0].p0
    return sc


@pytest.mark.parametrize("dim,steps", [(2, 150), (3, 30)])
def test_periodic_fp64_parity(B, dim, steps):
    sc = channel(dim)
    o, g = run_pair(sc, B.SPH_FP64, steps)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert max(e.values()) <= FP64_TOL, e
    eb = body_errors(sc, g.bodies(), o.bodies())
    assert max(eb.values()) <= FP64_TOL, eb
    # particles did cross the periodic boundary
    P = sc.hi[1] - sc.lo[1]
    moved = np.abs(o.get(O.F_X)[:, 1] - sc.x[:, 1])
    assert np.any(moved > 0.5 * P)


def test_periodic_tvf_fp64_parity(B):
    sc = channel(2, tvf=True)
    o, g = run_pair(sc, B.SPH_FP64, 60)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert max(e.values()) <= FP64_TOL, e


@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_fp32_gates(B, dim):
    sc = channel(dim)
    o, g = run_pair(sc, B.SPH_FP32_SWEEP, 1)
    e1 = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    for k in ("x", "u", "rho", "p", "pw", "uw"):
        assert e1[k] <= 1e-5, (k, e1)
    n = 100
    o.step(n - 1)
    g.step(n - 1)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert e["x"] <= 1e-3 and e["u"] <= 1e-3 and e["rho"] <= 1e-4, e


def test_poiseuille_fp32(B):
    g0, nu, H = 1.0, 0.5, 1.0
    sc = S.periodic_channel(dim=2, n_sites=(20, 9, 1), dx=H / 20, g=g0, nu=nu, c=2.5, jitter_amp=0.0)
    g = B.SphScene(sc, precision=B.SPH_FP32_SWEEP)
    dt = O.OracleScene(sc).dt
    g.step(int(round(1.5 / dt)))
    g.sync()
    f = g.sph_scene_read_particles(["X", "U"])
    fl = sc.kind == S.FLUID
    x, u = f["X"][fl, 0], f["U"][fl, 1]
    ref = g0 * x * (H - x) / (2.0 * nu)
    umax = g0 * H * H / (8.0 * nu)
    assert np.max(np.abs(u - ref)) < 0.02 * umax
