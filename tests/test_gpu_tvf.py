"""Transport-velocity formulation on the GPU against the oracle (Sec.
"Momentum equation" with the background pressure p_b = p0 of the paper's
examples): FP64 structure bit for bit and fields (a_b and u~ - u included)
within 1e-10 after the run, with bodies, walls, conduction and phase
switching; FP32 within the one-step and run gates of the other parity
tests."""
import numpy as np
import pytest

import oracle as O
from paper_2103_07925_amd import scenes as S

from parity_util import body_errors, field_errors, gpu_fields, oracle_fields, run_pair
from test_gpu_parity import (FP64_TOL, B, _assert_switch_parity, _run_switch_pair, _scripted_switch_scene,
                             assert_bitwise_structure, small_3d)

pytestmark = pytest.mark.gpu


def tvf(sc, factor=1.0):
    fl = sorted(set(sc.phase[sc.kind == S.FLUID].tolist()))
    sc.p_b = factor * max(sc.materials[p].p0 for p in fl)
    return sc


@pytest.mark.parametrize("make,steps", [("c1", 200), ("3d", 20)])
def test_tvf_fp64_parity(B, make, steps):
    sc = tvf(S.config_c1(seed=2) if make == "c1" else small_3d(seed=3))
    o, g = run_pair(sc, B.SPH_FP64, steps)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert "ab" in e and "ud" in e
    assert max(e.values()) <= FP64_TOL, e
    eb = body_errors(sc, g.bodies(), o.bodies())
    assert max(eb.values()) <= FP64_TOL, eb
    # the formulation is active
    assert np.max(np.abs(o.get(O.F_UD))) > 0.0


def test_tvf_background_five_times_p0_fp64(B):
    """The gastric example's p_b = 5 p0."""
    sc = tvf(S.config_c1(seed=4), factor=5.0)
    o, g = run_pair(sc, B.SPH_FP64, 60)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert max(e.values()) <= FP64_TOL, e


@pytest.mark.parametrize("dim", [2, 3])
def test_tvf_thermal_fp64_parity(B, dim):
    sc = tvf(S.config_c3(seed=2, nsites=(20, 14, 12), n_grains=4 if dim == 3 else 3, median_r=2.5, dim=dim))
    sc.phase_switch = 0
    o, g = run_pair(sc, B.SPH_FP64, 20)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert max(e.values()) <= FP64_TOL, e


def test_tvf_phase_switch_fp64_parity(B):
    """Melting and solidification with the formulation on: a melted particle
    starts without a background acceleration."""
    sc = tvf(_scripted_switch_scene())
    o, g, prev = _run_switch_pair(B, sc, 3)
    _assert_switch_parity(sc, o, g, prev)
    kind = o.get_int(O.I_KIND)
    fl = kind == S.FLUID
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), kind)
    assert e["ab"] <= FP64_TOL and e["ud"] <= FP64_TOL, e
    assert np.any(fl & (sc.kind == S.RIGID))       # some particles melted


@pytest.mark.parametrize("make", ["c1", "3d"])
def test_tvf_fp32_gates(B, make):
    sc = tvf(S.config_c1(seed=5) if make == "c1" else small_3d(seed=5))
    o, g = run_pair(sc, B.SPH_FP32_SWEEP, 1)
    e1 = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    for k in ("x", "u", "rho", "p", "pw", "uw", "ab", "ud"):
        assert e1[k] <= 1e-5, (k, e1)
    n = 200
    o.step(n - 1)
    g.step(n - 1)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), o.get_int(O.I_KIND))
    assert e["x"] <= 1e-3 and e["u"] <= 1e-3, e
    assert e["rho"] <= 1e-4, e
    eb = body_errors(sc, g.bodies(), o.bodies())
    assert eb["r"] <= 1e-3 and eb["m"] <= 1e-12, eb


def test_tvf_off_matches_the_plain_method(B):
    """p_b = 0 is the printed momentum equation: the same results as a scene
    without the field, bit for bit."""
    a = small_3d(seed=9)
    b = small_3d(seed=9)
    b.p_b = 0.0
    ga = B.SphScene(a, precision=B.SPH_FP32_SWEEP)
    gb = B.SphScene(b, precision=B.SPH_FP32_SWEEP)
    ga.step(5)
    gb.step(5)
    ga.sync()
    gb.sync()
    fa, fb = gpu_fields(ga), gpu_fields(gb)
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    assert not np.any(fa["AB"]) and not np.any(fa["UD"])
