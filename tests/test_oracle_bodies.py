"""Pins of the oracle's rigid-body part, time step and phase switch (CPU).

  * disc mass and inertia against the analytic values and plotted ranges of
    Sec. "Spatial discretization of a rigid circular disk" (golden fixture);
  * processor-wise quantities combined by Huygens-Steiner equal the single
    partition result (eqs. global_centerofmass, global_inertia; Remark on the
    serial case);
  * time step sizes printed for the examples (golden fixture);
  * free fall: velocity Verlet is exact for a constant acceleration;
  * torque-free spin: orientation is q(n dt omega) o q0, particle positions
    rotate as scipy's independent rotation says;
  * head-on contact of two particles: duration pi sqrt(mu/k_c), restitution
    of the linear spring-dashpot;
  * phase switch with scripted temperatures: strict comparisons, mass
    conservation, unchanged velocities of surviving rigid particles, body
    quantities equal to a fresh recomputation, new bodies per component.
"""
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2103_07925_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            out[k] = [float(t) for t in v] if len(v) > 1 else float(v[0])
    return out


def test_disc_mass_and_inertia(oracle_lib):
    g = read_golden("disc_mass_inertia.txt")
    D, rho = g["diameter"], g["density"]
    errs_m, errs_I = [], []
    for dx in g["dx_values"]:
        x = S.disc_sites(2, D, dx, "vertex")
        m = np.full(x.shape[0], rho * dx * dx)
        M, r, I = oracle_lib.mass_props(2, dx, x, m)
        assert g["mass_axis_min"] <= M <= g["mass_axis_max"]
        assert g["inertia_axis_min"] <= I[2, 2] <= g["inertia_axis_max"]
        errs_m.append(abs(M / g["mass_analytic"] - 1.0))
        errs_I.append(abs(I[2, 2] / g["inertia_analytic"] - 1.0))
        assert np.allclose(r[:2], 0.0, atol=1e-15)
    # converges to the analytic values
    assert errs_m[-1] < 0.01 and errs_I[-1] < 0.01
    assert errs_m[-1] < errs_m[0] and errs_I[-1] < errs_I[0]


def test_particle_inertia_reading(oracle_lib):
    # A single particle: I = 0.5 m r_eff^2 with r_eff = dx / sqrt(pi) in 2D and
    # 0.4 m r_eff^2 with r_eff = (0.75/pi)^(1/3) dx in 3D: the inertia of a disc
    # or ball of area / volume dx^d.
    dx, m = 0.3, 2.0
    _, _, I2 = oracle_lib.mass_props(2, dx, np.zeros((1, 3)), np.array([m]))
    assert abs(I2[2, 2] - m * dx * dx / (2.0 * math.pi)) < 1e-15
    _, _, I3 = oracle_lib.mass_props(3, dx, np.zeros((1, 3)), np.array([m]))
    R = (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0) * dx
    assert abs(I3[0, 0] - 0.4 * m * R * R) < 1e-14 and abs(I3[0, 1]) == 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_steiner_partition_invariance(oracle_lib, dim):
    rng = np.random.default_rng(11)
    n = 700
    x = rng.normal(0.0, 1.0, size=(n, 3)) + np.array([5.0, -3.0, 2.0])
    if dim == 2:
        x[:, 2] = 0.0
    m = rng.uniform(0.5, 2.0, n)
    M1, r1, I1 = oracle_lib.mass_props(dim, 0.1, x, m)
    for nparts in (2, 7, 40):
        part = rng.integers(0, nparts, n).astype(np.int32)
        M2, r2, I2 = oracle_lib.mass_props_partitioned(dim, 0.1, x, m, part, nparts)
        assert abs(M2 - M1) <= 1e-14 * M1
        assert np.max(np.abs(r2 - r1)) <= 1e-14 * np.max(np.abs(r1))
        assert np.max(np.abs(I2 - I1)) <= 1e-13 * np.max(np.abs(I1))
    # brute force: the definitions with math.fsum
    assert abs(M1 - math.fsum(m)) <= 1e-15 * M1
    for a in range(dim):
        assert abs(r1[a] - math.fsum(m * x[:, a]) / math.fsum(m)) <= 1e-14 * abs(r1[a])


def test_timestep_examples(oracle_lib):
    with open(os.path.join(GOLDEN, "timestep_examples.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for name, dx, rho0, p0, nu, dt_printed in rows:
        dx, rho0, p0, nu, dt_printed = map(float, (dx, rho0, p0, nu, dt_printed))
        sc = S.fluid_box(3, 4, dx=dx, rho0=rho0, c=math.sqrt(p0 / rho0), nu=nu, jitter_amp=0.0, g=1.0)
        dt = oracle_lib.timestep(sc)
        assert abs(dt / dt_printed - 1.0) < 1e-12, name


def test_timestep_multiphase_uses_fastest_sound(oracle_lib):
    # With a gas phase present (rho 0.1, same p0) the CFL bound strictly
    # taken is 0.25 h / sqrt(p0 / 0.1); the printed PBFAM step used the liquid's c.
    sc = S.fluid_box(2, 6, dx=0.1, rho0=1.0, c=4000.0, nu=100.0, jitter_amp=0.0, g=1e4)
    sc.materials.append(S.Material(rho0=0.1, p0=16.0e6, nu=100.0, b=(0.0, -1e4, 0.0)))
    sc.phase[0] = len(sc.materials) - 1
    assert abs(oracle_lib.timestep(sc) - 0.25 * 0.1 / math.sqrt(16.0e6 / 0.1)) < 1e-18


@pytest.mark.parametrize("dim", [2, 3])
def test_free_fall_exact(oracle_lib, dim):
    g = 9.81
    u0 = (0.3, -0.1, 0.2)
    sc = S.single_body(dim, g=g, u0=u0)
    o = oracle_lib.OracleScene(sc, dt=1e-3)
    b0 = o.bodies()[0].copy()
    n = 250
    o.step(n)
    b = o.bodies()[0]
    t = n * 1e-3
    gv = np.zeros(3)
    gv[dim - 1] = -g
    for a in range(dim):
        ref = b0[1 + a] + u0[a] * t + 0.5 * gv[a] * t * t
        assert abs(b[1 + a] - ref) < 1e-12 * (1 + abs(ref))
        assert abs(b[8 + a] - (u0[a] + gv[a] * t)) < 1e-12 * (1 + abs(g * t))


@pytest.mark.parametrize("dim", [2, 3])
def test_torque_free_spin(oracle_lib, dim):
    w = np.array([0.0, 0.0, 3.0]) if dim == 2 else np.array([1.0, -2.0, 0.5])
    q0 = (1.0, 0.0, 0.0, 0.0) if dim == 2 else tuple(Rotation.from_rotvec([0.3, 0.2, -0.4]).as_quat(scalar_first=True))
    sc = S.single_body(dim, g=0.0, w0=tuple(w), q0=q0)
    dt = 1e-3
    o = oracle_lib.OracleScene(sc, dt=dt)
    x0 = o.get(oracle_lib.F_X)
    r0 = o.bodies()[0, 1:4].copy()
    n = 400
    o.step(n)
    b = o.bodies()[0]
    Rn = Rotation.from_rotvec(n * dt * w)
    qref = (Rn * Rotation.from_quat(q0, scalar_first=True)).as_quat(scalar_first=True)
    q = b[4:8]
    if np.dot(q, qref) < 0:
        qref = -qref
    assert np.max(np.abs(q - qref)) < 1e-13
    assert np.max(np.abs(b[11:14] - w)) < 1e-13
    x = o.get(oracle_lib.F_X)
    xref = Rn.apply(x0 - r0) + r0
    assert np.max(np.abs(x[:, :dim] - xref[:, :dim])) < 1e-13


def _collide(oracle_lib, d_c):
    k_c = 1.0e4
    sc = S.two_particle_bodies(dim=2, dx=0.1, gap=0.05, speed=0.2, k_c=k_c, d_c=d_c)
    dt = 2e-5
    o = oracle_lib.OracleScene(sc, dt=dt)
    m = o.bodies()[0, 0]
    t_on = t_off = None
    for n in range(20000):
        o.step(1)
        f = np.abs(o.bodies()[0, 20])
        if f > 0 and t_on is None:
            t_on = o.time
        if t_on is not None and f == 0 and t_off is None:
            t_off = o.time
            break
    v = o.bodies()[:, 8]
    return m, k_c, dt, t_on, t_off, v


def test_contact_elastic(oracle_lib):
    m, k_c, dt, t_on, t_off, v = _collide(oracle_lib, 0.0)
    mu = 0.5 * m
    assert abs((t_off - t_on) - math.pi * math.sqrt(mu / k_c)) < 3 * dt
    assert abs(v[0] + 0.2) < 1e-3 and abs(v[1] - 0.2) < 1e-3


def test_contact_damped_restitution(oracle_lib):
    m0, k_c = None, 1.0e4
    d_c = 0.5
    m, k_c, dt, t_on, t_off, v = _collide(oracle_lib, d_c)
    mu = 0.5 * m
    zeta = d_c / (2.0 * math.sqrt(k_c * mu))
    e_ref = math.exp(-zeta * math.pi / math.sqrt(1.0 - zeta * zeta))
    e = abs(v[1] - v[0]) / 0.4
    # the tension cut-off ends contact a little before the dashpot would
    assert abs(e - e_ref) < 0.05 * e_ref
    assert e < 1.0


def _switch_scene(dim=2):
    """Fluid box with one rigid disc; liquid phase 0 (switch to 2), solid
    phase 2 (switch to 0), T_t = 50, no conduction (kappa = 0)."""
    sc = S.config_c1(seed=1, n_side=16, dx=0.05)
    sc.materials[0].switch_to = 2
    sc.materials[0].T_t = 50.0
    sc.materials[2].switch_to = 0
    sc.materials[2].T_t = 50.0
    sc.thermal = 1
    sc.phase_switch = 1
    sc.max_bodies = 8
    sc.T[:] = 60.0
    sc.T[sc.kind == S.RIGID] = 40.0
    sc.bodies[0].w = (0.0, 0.0, 1.5)
    sc.bodies[0].u = (0.1, 0.05, 0.0)
    return sc


def test_phase_switch_scripted(oracle_lib):
    sc = _switch_scene()
    rigid = np.nonzero(sc.kind == S.RIGID)[0]
    fl = np.nonzero(sc.kind == S.FLUID)[0]
    # two rigid particles melt; T exactly at T_t does not switch
    sc.T[rigid[0]] = 70.0
    sc.T[rigid[5]] = 50.0
    sc.T[rigid[-1]] = 50.0 + 1e-9
    # one fluid cluster far from the disc solidifies into a new body; one fluid
    # particle next to the disc joins it
    dist = np.linalg.norm(sc.x[fl, :2] - np.array([0.4, 0.6]), axis=1)
    near = fl[np.argsort(dist)[0]]
    sc.T[near] = 40.0
    far = fl[np.linalg.norm(sc.x[fl, :2] - np.array([0.15, 0.15]), axis=1) < 0.06]
    sc.T[far] = 10.0
    far2 = fl[np.linalg.norm(sc.x[fl, :2] - np.array([0.62, 0.15]), axis=1) < 0.06]
    sc.T[far2] = 10.0
    sw = oracle_lib.OracleScene(sc)
    sc_off = _switch_scene()
    sc_off.T[:] = sc.T
    sc_off.phase_switch = 0
    ref = oracle_lib.OracleScene(sc_off)
    m_before = sw.get(oracle_lib.F_M).sum()
    sw.step(1)
    ref.step(1)
    kind = sw.get_int(oracle_lib.I_KIND)
    body = sw.get_int(oracle_lib.I_BODY)
    assert kind[rigid[0]] == S.FLUID and kind[rigid[-1]] == S.FLUID
    assert kind[rigid[5]] == S.RIGID
    assert kind[near] == S.RIGID and body[near] == 0
    assert np.all(kind[far] == S.RIGID) and np.all(kind[far2] == S.RIGID)
    nb = sw.bodies().shape[0]
    assert nb == 3
    assert np.all(body[far] == (1 if far.min() < far2.min() else 2))
    assert np.all(body[far2] == (2 if far.min() < far2.min() else 1))
    # mass conserved
    assert sw.get(oracle_lib.F_M).sum() == m_before
    # surviving rigid particles keep their velocity across the switch
    surv = rigid[(kind[rigid] == S.RIGID)]
    u_sw = sw.get(oracle_lib.F_U)[surv]
    u_ref = ref.get(oracle_lib.F_U)[surv]
    assert np.max(np.abs(u_sw - u_ref)) <= 1e-14 * np.max(np.abs(u_ref))
    # body quantities equal a fresh recomputation
    b = sw.bodies()
    x = sw.get(oracle_lib.F_X)
    m = sw.get(oracle_lib.F_M)
    for k in range(nb):
        sel = body == k
        M, r, I = oracle_lib.mass_props(2, sc.dx, x[sel], m[sel])
        assert abs(b[k, 0] - M) <= 1e-15 * M
        assert np.max(np.abs(b[k, 1:3] - r[:2])) <= 1e-14
        assert abs(b[k, 28] - I[2, 2]) <= 1e-13 * I[2, 2]


def test_phase_switch_gas_never_solidifies(oracle_lib):
    sc = _switch_scene()
    sc.materials[0].switch_to = -1
    sc.T[:] = 0.0
    o = oracle_lib.OracleScene(sc)
    o.step(1)
    kind = o.get_int(oracle_lib.I_KIND)
    assert np.array_equal(kind[sc.kind == S.FLUID], np.zeros(int(np.sum(sc.kind == S.FLUID)), np.int32))
