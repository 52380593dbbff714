"""Pins of the oracle's transport-velocity formulation (CPU only).

Sec. "Momentum equation" applies a constant background pressure p_b to all
particles and refers to Adami, Hu, Adams (2013) for the modified advection
velocity and the extra momentum term.  What fixes the oracle here, other
than its own formulas:
  * the paper's statement that the background-pressure contribution
    vanishes where the kernel sums form a partition of unity (a regular
    lattice with full support);
  * a particle displaced by delta inside a lattice, all volumes equal: the
    kernel sum of the remaining sites is flat to ~1e-4, so the background
    term is the missing self-site's gradient,
    a_b = (2 p_b V / rho) W'(|delta|) delta/|delta| (restoring), up to that
    flatness;
  * the divergence of A = rho u (u~ - u) with uniform u = U and
    u~ - u = G x on a lattice is exactly U tr(G) V G_d / dx^d, with the
    lattice constant G_d = -dx^d sum x_b^2 W'/r (the same constant as the
    conduction pin: G_2 = 1.000795443058, G_3 = 1.001001280684);
  * exact conservation of linear momentum of an isolated fluid + body system
    with the extra term on (it is pairwise antisymmetric);
  * the drift moves a particle with u~ = u + (dt/2) a_b.
"""
import math

import numpy as np
import pytest

from paper_2103_07925_amd import scenes as S

G_D = {2: 1.000795443058, 3: 1.001001280684}


def interior_mask(x, dim, lo, hi, margin):
    m = np.ones(x.shape[0], bool)
    for a in range(dim):
        m &= (x[:, a] > lo + margin) & (x[:, a] < hi - margin)
    return m


def lattice(O, dim, n_side, p_b, rho0=1.0, **kw):
    sc = S.frozen_lattice(dim, n_side, rho0=rho0, **kw)
    sc.p_b = p_b
    return sc


@pytest.mark.parametrize("dim,n_side", [(2, 20), (3, 15)])
def test_background_term_vanishes_with_full_support(oracle_lib, dim, n_side):
    O = oracle_lib
    p_b = 7.0
    sc = lattice(O, dim, n_side, p_b)
    o = O.OracleScene(sc)
    ab = o.get(O.F_AB)
    rho = o.get(O.F_RHO)
    # full support of every neighbour too (uniform volumes): 6 dx from the surface
    inner = interior_mask(sc.x, dim, 0.0, n_side * sc.dx, 6.0 * sc.dx)
    scale = p_b / (rho[inner].min() * sc.dx)
    assert np.max(np.abs(ab[inner])) < 1e-11 * scale
    # near the free surface the background pressure pushes outwards
    edge = ~interior_mask(sc.x, dim, 0.0, n_side * sc.dx, sc.dx)
    centre = np.full(3, 0.5 * n_side * sc.dx)
    centre[dim:] = 0.0
    out = np.sum(ab[edge] * (sc.x[edge] - centre), axis=1)
    assert np.all(out > 0.0)


@pytest.mark.parametrize("dim,n_side", [(2, 20), (3, 12)])
@pytest.mark.parametrize("axis", [0, 1])
def test_background_term_restores_a_displaced_particle(oracle_lib, dim, n_side, axis):
    O = oracle_lib
    p_b = 3.0
    sc = lattice(O, dim, n_side, p_b)
    mid = np.full(3, (n_side // 2 + 0.5) * sc.dx)
    mid[dim:] = 0.0
    k = int(np.argmin(np.sum((sc.x - mid) ** 2, axis=1)))
    delta = 0.2 * sc.dx
    sc.x[k, axis] += delta
    o = O.OracleScene(sc)
    # uniform volumes (the bulk density everywhere), so that the sum is the
    # kernel-gradient sum alone
    rho = float(np.median(o.get(O.F_RHO)))
    o.set(O.F_RHO, np.full(sc.n, rho))
    o.stage(O.S_FORCES)
    ab = o.get(O.F_AB)[k]
    m = o.get(O.F_M)[k]
    V = m / rho
    expect = 2.0 * p_b * V / rho * O.kernel_dW(dim, sc.dx, delta)
    assert expect < 0.0
    assert abs(ab[axis] / expect - 1.0) < 0.01
    for b in range(dim):
        if b != axis:
            assert abs(ab[b]) < 1e-9 * abs(expect)


@pytest.mark.parametrize("dim,n_side", [(2, 22), (3, 15)])
def test_divergence_of_the_extra_stress(oracle_lib, dim, n_side):
    O = oracle_lib
    sc = lattice(O, dim, n_side, p_b=1.0, rho0=1.5)
    o = O.OracleScene(sc)
    o.stage(O.S_NEIGHBORS)
    o.stage(O.S_DENSITY)
    rho = o.get(O.F_RHO)
    m = o.get(O.F_M)
    U = np.array([0.4, -0.3, 0.2])
    U[dim:] = 0.0
    G = np.array([[0.7, 0.2, -0.1], [0.3, -0.4, 0.5], [0.1, 0.6, 0.25]])
    G[dim:, :] = 0.0
    G[:, dim:] = 0.0
    o.set(O.F_U, np.tile(U, (sc.n, 1)))
    o.set(O.F_UD, sc.x @ G.T)
    o.set(O.F_P, np.zeros(sc.n))
    o.stage(O.S_FORCES)
    a = o.get(O.F_A)
    inner = interior_mask(sc.x, dim, 0.0, n_side * sc.dx, 6.0 * sc.dx)
    V = m[inner] / rho[inner]
    expect = (V * np.trace(G) * G_D[dim] / sc.dx ** dim)[:, None] * U[None, :]
    scale = np.max(np.abs(expect))
    assert np.max(np.abs(a[inner] - expect)) < 1e-9 * scale
    # u~ - u uniform: no contribution
    o.set(O.F_UD, np.tile(np.array([0.3, 0.1, -0.2]), (sc.n, 1)))
    o.stage(O.S_FORCES)
    a = o.get(O.F_A)
    assert np.max(np.abs(a[inner])) < 1e-9 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_isolated_momentum_conservation_with_tvf(oracle_lib, dim):
    O = oracle_lib
    sc = S.isolated_blob_with_body(dim=dim, n_side=14 if dim == 2 else 8)
    sc.p_b = sc.materials[0].p0
    o = O.OracleScene(sc)
    fl = sc.kind == S.FLUID

    def momentum():
        u = o.get(O.F_U)
        m = o.get(O.F_M)
        b = o.bodies()
        P = np.array([math.fsum(m[fl] * u[fl, a]) + math.fsum(b[:, 0] * b[:, 8 + a]) for a in range(3)])
        scale = math.fsum(m[fl] * np.linalg.norm(u[fl], axis=1)) + \
            math.fsum(b[:, 0] * np.linalg.norm(b[:, 8:11], axis=1))
        return P, scale

    P0, scale = momentum()
    o.step(40)
    P1, _ = momentum()
    assert np.max(np.abs(P1 - P0)) < 1e-12 * scale
    # the formulation is active: u~ - u is non-zero on fluid particles
    assert np.max(np.abs(o.get(O.F_UD)[fl])) > 0.0


def test_drift_uses_the_transport_velocity(oracle_lib):
    O = oracle_lib
    sc = S.fluid_box(dim=3, n_side=6, g=9.81, walls=False)
    keep = np.array([40])
    for f in ("x", "u", "T", "kind", "phase", "body", "moving"):
        setattr(sc, f, np.ascontiguousarray(getattr(sc, f)[keep]))
    sc.u[0] = (0.3, -0.1, 0.2)
    sc.p_b = 2.0
    o = O.OracleScene(sc)
    ab = np.array([[1.5, -2.0, 0.5]])
    o.set(O.F_AB, ab)
    x0, u0, a0 = o.get(O.F_X), o.get(O.F_U), o.get(O.F_A)
    dt = o.dt
    hdt = 0.5 * dt
    o.step(1)
    uhalf = u0 + hdt * a0
    x1 = x0 + dt * (uhalf + hdt * ab)
    assert np.max(np.abs(o.get(O.F_X) - x1)) <= 1e-15 * np.max(np.abs(x1))
    assert np.array_equal(o.get(O.F_UD), hdt * ab)
    # an isolated particle has no background-pressure acceleration
    assert np.all(o.get(O.F_AB) == 0.0)
