"""GPU (HIP library through the C ABI) against the FP64 oracle.

FP64 mode: neighbour lists, cell order and particle flags bit for bit; every
field within 1e-10 (field-scaled) after the run.  FP32 mode: the gates fixed
before measuring -- after one step every field within 1e-5; after the run
positions and velocities within 1e-3 and densities within 1e-4.
"""
import numpy as np
import pytest

import oracle as O
from paper_2103_07925_amd import scenes as S

from parity_util import body_errors, field_errors, gpu_fields, oracle_fields, run_pair

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_07925_amd import sphrb
    sphrb.lib()
    return sphrb


def small_3d(seed=0):
    return S.config_c2(seed=seed, n_side=24, n_per_axis=2, spacing_sites=12, r_range=(2.5, 4.0))


def assert_bitwise_structure(o, g, sc):
    off_o, ids_o = o.neighbors()
    off_g, ids_g = g.neighbors()
    assert np.array_equal(off_o, off_g)
    assert np.array_equal(ids_o, ids_g)
    so, co = o.cell_order()
    sg, cg = g.cell_order()
    assert np.array_equal(co, cg)
    assert np.array_equal(so, sg)
    k, ph, b = g.flags()
    assert np.array_equal(k, o.get_int(O.I_KIND))
    assert np.array_equal(ph, o.get_int(O.I_PHASE))
    assert np.array_equal(b, o.get_int(O.I_BODY))


@pytest.mark.parametrize("steps", [0, 1, 25])
def test_c1_fp64_parity(B, steps):
    sc = S.config_c1(seed=1)
    o, g = run_pair(sc, B.SPH_FP64, steps)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert max(e.values()) <= FP64_TOL, e
    eb = body_errors(sc, g.bodies(), o.bodies())
    assert max(eb.values()) <= FP64_TOL, eb
    assert g.stats().pairs_last == o.pair_count


def test_c1_fp64_full_run(B):
    sc = S.config_c1(seed=0)
    o, g = run_pair(sc, B.SPH_FP64, 1000)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), o.get_int(O.I_KIND))
    assert max(e.values()) <= FP64_TOL, e
    eb = body_errors(sc, g.bodies(), o.bodies())
    assert max(eb.values()) <= FP64_TOL, eb


@pytest.mark.parametrize("steps", [0, 20])
def test_3d_bodies_fp64_parity(B, steps):
    sc = small_3d()
    o, g = run_pair(sc, B.SPH_FP64, steps)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert max(e.values()) <= FP64_TOL, e
    eb = body_errors(sc, g.bodies(), o.bodies())
    assert max(eb.values()) <= FP64_TOL, eb


def test_contact_fp64_parity(B):
    sc = S.two_particle_bodies(dim=3, dx=0.1, gap=0.05, speed=0.2, k_c=1e4, d_c=0.5)
    o, g = run_pair(sc, B.SPH_FP64, 8000, dt=2e-5)
    eb = body_errors(sc, g.bodies(), o.bodies())
    assert max(eb.values()) <= FP64_TOL, eb
    assert abs(o.bodies()[0, 8] - 0.2) > 0.1      # the bodies did collide


@pytest.mark.parametrize("dim", [2, 3])
def test_thermal_fp64_parity(B, dim):
    sc = S.config_c3(seed=2, nsites=(20, 14, 12), n_grains=4 if dim == 3 else 3, median_r=2.5, dim=dim)
    sc.phase_switch = 0
    o, g = run_pair(sc, B.SPH_FP64, 20)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert max(e.values()) <= FP64_TOL, e


def test_moving_walls_fp64_parity(B):
    sc = S.config_c4(seed=3, nsites=(30, 16, 12), n_frag=3, r_range=(1.5, 2.5))
    o, g = run_pair(sc, B.SPH_FP64, 20)
    assert_bitwise_structure(o, g, sc)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    assert max(e.values()) <= FP64_TOL, e


def test_fp64_run_twice_is_bitwise_identical(B):
    sc = small_3d(seed=4)
    g1 = B.SphScene(sc, precision=B.SPH_FP64)
    g2 = B.SphScene(sc, precision=B.SPH_FP64)
    g1.step(10)
    g2.step(10)
    f1, f2 = gpu_fields(g1), gpu_fields(g2)
    for k in f1:
        assert np.array_equal(f1[k], f2[k]), k
    assert np.array_equal(g1.bodies(), g2.bodies())


@pytest.mark.parametrize("make", ["c1", "3d"])
def test_fp32_gates(B, make):
    sc = S.config_c1(seed=5) if make == "c1" else small_3d(seed=5)
    o, g = run_pair(sc, B.SPH_FP32_SWEEP, 1)
    e1 = field_errors(sc, gpu_fields(g), oracle_fields(o), sc.kind)
    for k in ("x", "u", "rho", "p", "pw", "uw"):
        assert e1[k] <= 1e-5, (k, e1)
    n = 200
    o.step(n - 1)
    g.step(n - 1)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), o.get_int(O.I_KIND))
    assert e["x"] <= 1e-3 and e["u"] <= 1e-3, e
    assert e["rho"] <= 1e-4, e
    eb = body_errors(sc, g.bodies(), o.bodies())
    assert eb["r"] <= 1e-3 and eb["m"] <= 1e-12, eb


@pytest.mark.parametrize("p_b", [0.0, 1.0])
def test_fp32_full_run_gates(B, p_b):
    """The C1 run's full 1000 steps in the FP32 sweep (with and without the
    transport-velocity formulation): positions and velocities within 1e-3,
    densities and every body error within 1e-4 (gates fixed before
    measuring)."""
    sc = S.config_c1(seed=0)
    sc.p_b = p_b * sc.materials[0].p0
    o, g = run_pair(sc, B.SPH_FP32_SWEEP, 1000)
    e = field_errors(sc, gpu_fields(g), oracle_fields(o), o.get_int(O.I_KIND))
    assert e["x"] <= 1e-3 and e["u"] <= 1e-3, e
    assert e["rho"] <= 1e-4 and e["p"] <= 1e-4, e
    eb = body_errors(sc, g.bodies(), o.bodies())
    assert max(eb.values()) <= 1e-4, eb


# ---- reversible phase transition -------------------------------------------

def _scripted_switch_scene():
    """The oracle's scripted switch scene: two rigid particles melt, one fluid
    particle next to the disc joins it, two far fluid clusters form new
    bodies; T exactly at T_t does not switch."""
    from test_oracle_bodies import _switch_scene
    sc = _switch_scene()
    rigid = np.nonzero(sc.kind == S.RIGID)[0]
    fl = np.nonzero(sc.kind == S.FLUID)[0]
    sc.T[rigid[0]] = 70.0
    sc.T[rigid[5]] = 50.0
    sc.T[rigid[-1]] = 50.0 + 1e-9
    dist = np.linalg.norm(sc.x[fl, :2] - np.array([0.4, 0.6]), axis=1)
    sc.T[fl[np.argsort(dist)[0]]] = 40.0
    for c in ((0.15, 0.15), (0.62, 0.15)):
        sc.T[fl[np.linalg.norm(sc.x[fl, :2] - np.array(c), axis=1) < 0.06]] = 10.0
    return sc


def _run_switch_pair(B, sc, steps):
    """Run both sides; also return the kinds before the last step."""
    o, g = run_pair(sc, B.SPH_FP64, steps - 1)
    prev = o.get_int(O.I_KIND)
    o.step(1)
    g.step(1)
    g.sync()
    return o, g, prev


def _assert_switch_parity(sc, o, g, prev_kind):
    """Structure bit for bit, fields and bodies within 1e-10.  The
    per-evaluation wall/rigid diagnostics (p_w, u~_w, particle force) of a
    particle that switched after the last evaluation are not defined on
    either side and are left out."""
    assert_bitwise_structure(o, g, sc)
    kind = o.get_int(O.I_KIND)
    gf, of = gpu_fields(g), oracle_fields(o)
    sw = prev_kind != kind
    for key in ("PW", "UW", "FR"):
        gf[key][sw] = of[key][sw]
    e = field_errors(sc, gf, of, kind)
    assert max(e.values()) <= FP64_TOL, e
    ob, gb = o.bodies(), g.bodies()
    assert gb.shape == ob.shape
    assert np.array_equal(gb[:, 32], ob[:, 32])          # active flags
    act = ob[:, 32] > 0
    eb = body_errors(sc, gb[act], ob[act])
    assert max(eb.values()) <= FP64_TOL, eb
    st = g.stats()
    assert st.n_rigid == int(np.sum(kind == S.RIGID))
    assert st.n_fluid == int(np.sum(kind == S.FLUID))
    assert st.n_bodies == ob.shape[0]


@pytest.mark.parametrize("steps", [1, 30])
def test_phase_switch_scripted_fp64_parity(B, steps):
    sc = _scripted_switch_scene()
    o, g, prev = _run_switch_pair(B, sc, steps)
    _assert_switch_parity(sc, o, g, prev)
    assert o.bodies().shape[0] == 3


def test_phase_switch_bulk_solidification_fp64_parity(B):
    """Every fluid particle below T_t at once: the particles within r_c of
    the disc join it, all others form new bodies in one switch (a large
    joiner sort and component search)."""
    from test_oracle_bodies import _switch_scene
    sc = _switch_scene()
    sc.T[sc.kind == S.FLUID] = 10.0
    sc.max_bodies = 64
    o, g, prev = _run_switch_pair(B, sc, 1)
    _assert_switch_parity(sc, o, g, prev)
    assert np.all(o.get_int(O.I_KIND)[sc.kind == S.FLUID] == S.RIGID)
    o.step(4)
    g.step(4)
    prev = o.get_int(O.I_KIND)
    o.step(1)
    g.step(1)
    g.sync()
    _assert_switch_parity(sc, o, g, prev)


@pytest.mark.parametrize("dim", [2, 3])
def test_phase_switch_thermal_fp64_parity(B, dim):
    """Two-phase thermal scene with conduction and the moving heat source:
    one grain heated above T_t melts entirely (its body goes inactive), part
    of another melts; 40 steps with switching on every step."""
    sc = S.config_c3(seed=2, nsites=(20, 14, 12), n_grains=4 if dim == 3 else 3, median_r=2.5, dim=dim)
    rg = sc.kind == S.RIGID
    bodies = np.unique(sc.body[rg])
    assert bodies.size >= 2
    sc.T[rg & (sc.body == bodies[0])] = 70.0
    b1 = rg & (sc.body == bodies[1])
    cut = np.median(sc.x[b1, 0])
    sc.T[b1 & (sc.x[:, 0] < cut)] = 52.0
    o, g, prev = _run_switch_pair(B, sc, 40)
    _assert_switch_parity(sc, o, g, prev)
    kind = o.get_int(O.I_KIND)
    assert np.any(kind[rg] == S.FLUID)          # something melted


def test_phase_switch_body_capacity_error(B):
    """More new bodies than max_bodies: a sticky device error, reported by sync."""
    sc = _scripted_switch_scene()
    sc.max_bodies = 2
    g = B.SphScene(sc, precision=B.SPH_FP64)
    g.step(1)
    with pytest.raises(RuntimeError):
        g.sync()
    assert g.stats().device_error & 16


# ---- checkpoint / resume ----------------------------------------------------

@pytest.mark.parametrize("case", ["c1_fp64", "switch_fp64", "3d_fp32", "3d_tvf_fp32"])
def test_checkpoint_resume_is_bitwise(B, case):
    """k steps, state image, re-create, N-k steps == N steps, bit for bit."""
    if case == "c1_fp64":
        sc, prec = S.config_c1(seed=2), B.SPH_FP64
    elif case == "switch_fp64":
        sc, prec = _scripted_switch_scene(), B.SPH_FP64
    elif case == "3d_tvf_fp32":
        sc, prec = small_3d(seed=4), B.SPH_FP32_SWEEP
        sc.p_b = sc.materials[0].p0
    else:
        sc, prec = small_3d(seed=3), B.SPH_FP32_SWEEP
    k, n = 7, 19
    ref = B.SphScene(sc, precision=prec)
    ref.step(n)
    ref.sync()
    a = B.SphScene(sc, precision=prec)
    a.step(k)
    blob = a.read_state()
    del a
    r = B.SphScene.from_state(blob, sc)
    r.step(n - k)
    r.sync()
    f1, f2 = gpu_fields(ref), gpu_fields(r)
    for key in f1:
        assert np.array_equal(f1[key], f2[key]), key
    assert np.array_equal(ref.bodies(), r.bodies())
    assert np.array_equal(np.concatenate(ref.flags()), np.concatenate(r.flags()))
    s1, s2 = ref.stats(), r.stats()
    assert (s1.step, s1.pairs_total, s1.n_bodies) == (s2.step, s2.pairs_total, s2.n_bodies)


# ---- global FP64 checks ------------------------------------------------------

def _oracle_globals(sc, o):
    kind = o.get_int(O.I_KIND)
    ph = o.get_int(O.I_PHASE)
    fl = kind == S.FLUID
    m = o.get(O.F_M)[fl]
    u = o.get(O.F_U)[fl]
    x = o.get(O.F_X)[fl]
    b = np.array([sc.materials[p].b for p in ph[fl]], np.float64)
    bo = o.bodies()
    act = bo[:, 32] > 0
    bo = bo[act]
    mass = m.sum() + bo[:, 0].sum()
    mom = (m[:, None] * u).sum(0) + (bo[:, 0:1] * bo[:, 8:11]).sum(0)
    ke = 0.5 * (m * (u * u).sum(1)).sum() + 0.5 * (bo[:, 0] * (bo[:, 8:11] ** 2).sum(1)).sum()
    for rec in bo:
        w = rec[11:14]
        if sc.dim == 3:
            I = np.array([[rec[26], rec[29], rec[30]], [rec[29], rec[27], rec[31]], [rec[30], rec[31], rec[28]]])
            ke += 0.5 * w @ I @ w
        else:
            ke += 0.5 * rec[28] * w[2] ** 2
    pe = -(m * (b * x).sum(1)).sum()
    # body force of a body: that of its particles' phase
    body = o.get_int(O.I_BODY)
    for k, rec in zip(np.nonzero(act)[0], bo):
        p = ph[(kind == S.RIGID) & (body == k)][0]
        pe -= rec[0] * np.dot(sc.materials[p].b[:sc.dim], rec[1:1 + sc.dim])
    return mass, mom, ke, pe


@pytest.mark.parametrize("case", ["c1", "3d", "switch"])
def test_global_checks_match_the_oracle_fields(B, case):
    if case == "c1":
        sc = S.config_c1(seed=1)
    elif case == "3d":
        sc = small_3d(seed=2)
        sc.bodies[0].w = (0.3, -0.2, 0.5)
    else:
        sc = _scripted_switch_scene()
    o, g = run_pair(sc, B.SPH_FP64, 6)
    mass, mom, ke, pe = _oracle_globals(sc, o)
    st = g.stats()
    assert abs(st.mass - mass) <= 1e-12 * mass
    scale = max(np.abs(mom).max(), 1e-30)
    assert np.max(np.abs(np.array(st.momentum) - mom)) <= 1e-10 * scale + 1e-15 * mass
    assert abs(st.kinetic - ke) <= 1e-10 * max(ke, 1e-30)
    assert abs(st.potential - pe) <= 1e-10 * max(abs(pe), 1e-30)
    if case == "switch":
        o0 = O.OracleScene(sc)
        k0 = o0.get_int(O.I_KIND)
        g1 = B.SphScene(sc, precision=B.SPH_FP64)
        g1.step(1)
        o0.step(1)
        k1 = o0.get_int(O.I_KIND)
        s1 = g1.stats()
        assert s1.n_melted == int(np.sum((k0 == S.RIGID) & (k1 == S.FLUID)))
        assert s1.n_solidified == int(np.sum((k0 == S.FLUID) & (k1 == S.RIGID)))
        assert s1.n_melted > 0 and s1.n_solidified > 0
