"""Pins of the oracle's interaction physics (CPU only).

Each check is fixed by the mathematics or by the paper, not by the oracle's
own formulas:
  * partition of unity on a regular lattice (uniform density, within 1e-4 of
    the reference density);
  * the pressure-gradient and viscous terms of eq. nummeth_fluid_momentum on
    a frozen lattice against the continuum values -grad p / rho and
    nu lap u (lattice sums put them within 0.2 %);
  * the conduction operator of eq. nummeth_thermo_heat_equation: zero for a
    linear field, kappa lap T / (rho c_p) for a quadratic one, and the erf
    solution of 1D conduction between two blocks;
  * the wall extrapolation returns the exact linear extension of a
    hydrostatic field;
  * exact conservation of linear momentum for an isolated fluid + free body
    system (eqs. nummeth_fluid_conservlinmom, nummeth_fluid_couplingforce);
  * hydrostatic pressure slope -rho0 g in a closed box at rest.
"""
import math

import numpy as np
import pytest
from scipy import special

from paper_2103_07925_amd import scenes as S


def interior_mask(x, dim, lo, hi, margin):
    m = np.ones(x.shape[0], bool)
    for a in range(dim):
        m &= (x[:, a] > lo + margin) & (x[:, a] < hi - margin)
    return m


def frozen(oracle, dim, n_side, **kw):
    sc = S.frozen_lattice(dim, n_side, **kw)
    o = oracle.OracleScene(sc)
    o.stage(oracle.S_NEIGHBORS)
    o.stage(oracle.S_DENSITY)
    return sc, o


@pytest.mark.parametrize("dim,n_side", [(2, 20), (3, 12)])
def test_partition_of_unity_on_lattice(oracle_lib, dim, n_side):
    sc, o = frozen(oracle_lib, dim, n_side, rho0=1000.0)
    rho = o.get(oracle_lib.F_RHO)
    inner = interior_mask(sc.x, dim, 0.0, n_side * sc.dx, 3.0 * sc.dx)
    r = rho[inner]
    assert r.max() - r.min() <= 1e-12 * r.max()
    assert abs(r.mean() / 1000.0 - 1.0) < 1e-4


def test_c1_unjittered_full_support(oracle_lib):
    # 3 wall layers continue the lattice and the disc sites are lattice sites,
    # so every fluid particle of the unjittered C1 box has full support.
    sc = S.config_c1(jitter_amp=0.0)
    o = oracle_lib.OracleScene(sc)
    rho = o.get(oracle_lib.F_RHO)[sc.kind == S.FLUID]
    assert rho.max() - rho.min() <= 1e-12 * 1000.0
    assert abs(rho.mean() / 1000.0 - 1.000063224595) < 1e-11
    p = o.get(oracle_lib.F_P)[sc.kind == S.FLUID]
    mat = sc.materials[0]
    assert np.allclose(p, mat.p0 * (rho / mat.rho0 - 1.0), rtol=0, atol=1e-9 * mat.p0)


@pytest.mark.parametrize("dim,n_side", [(2, 22), (3, 15)])
def test_pressure_gradient_term(oracle_lib, dim, n_side):
    sc, o = frozen(oracle_lib, dim, n_side, rho0=2.0)
    B = 3.0
    rho = o.get(oracle_lib.F_RHO)
    o.set(oracle_lib.F_P, B * sc.x[:, 0])
    o.set(oracle_lib.F_U, np.zeros((sc.n, 3)))
    o.stage(oracle_lib.S_EXTRAP)
    o.stage(oracle_lib.S_FORCES)
    a = o.get(oracle_lib.F_A)
    inner = interior_mask(sc.x, dim, 0.0, n_side * sc.dx, 6.0 * sc.dx)
    ax = a[inner, 0] * rho[inner] / (-B)
    assert np.all(np.abs(ax - 1.0) < 2e-3)
    for k in range(1, dim):
        assert np.all(np.abs(a[inner, k]) < 1e-9 * B / rho[inner])


@pytest.mark.parametrize("dim,n_side", [(2, 22), (3, 15)])
def test_viscous_term(oracle_lib, dim, n_side):
    nu = 0.7
    sc, o = frozen(oracle_lib, dim, n_side, rho0=1.5, nu=nu)
    A = 2.0
    rho = o.get(oracle_lib.F_RHO)
    u = np.zeros((sc.n, 3))
    u[:, 0] = A * sc.x[:, 1] ** 2
    o.set(oracle_lib.F_P, np.zeros(sc.n))
    o.set(oracle_lib.F_U, u)
    o.stage(oracle_lib.S_FORCES)
    a = o.get(oracle_lib.F_A)
    inner = interior_mask(sc.x, dim, 0.0, n_side * sc.dx, 6.0 * sc.dx)
    expect = 2.0 * nu * A * 1.5 / rho[inner]      # eta lap u / rho with eta = rho0 nu
    assert np.all(np.abs(a[inner, 0] / expect - 1.0) < 2e-3)
    # a linear field has zero Laplacian
    u[:, 0] = A * sc.x[:, 1]
    o.set(oracle_lib.F_U, u)
    o.stage(oracle_lib.S_FORCES)
    a = o.get(oracle_lib.F_A)
    assert np.all(np.abs(a[inner, 0]) < 1e-9 * np.abs(expect))


@pytest.mark.parametrize("dim,n_side", [(2, 22), (3, 15)])
def test_heat_operator(oracle_lib, dim, n_side):
    kappa, cp, rho0 = 2.0, 3.0, 1.5
    sc, o = frozen(oracle_lib, dim, n_side, rho0=rho0, cp=cp, kappa=kappa)
    rho = o.get(oracle_lib.F_RHO)
    inner = interior_mask(sc.x, dim, 0.0, n_side * sc.dx, 6.0 * sc.dx)
    o.set(oracle_lib.F_T, 5.0 + 7.0 * sc.x[:, 0] - 2.0 * sc.x[:, dim - 1])
    o.stage(oracle_lib.S_HEAT)
    r = o.get(oracle_lib.F_DTDT)
    assert np.all(np.abs(r[inner]) < 1e-9)
    A = 4.0
    o.set(oracle_lib.F_T, A * sc.x[:, 0] ** 2)
    o.stage(oracle_lib.S_HEAT)
    r = o.get(oracle_lib.F_DTDT)
    expect = 2.0 * kappa * A / (rho[inner] * cp)
    assert np.all(np.abs(r[inner] / expect - 1.0) < 2e-3)


def test_one_dimensional_conduction_erf(oracle_lib):
    """Two blocks at T1, T2 in contact (a fixed rigid strip, so no particle
    moves); compare with T1/2 + T2/2 + (T2 - T1)/2 erf(x / (2 sqrt(alpha t)))."""
    dx = 0.1
    nx, ny = 80, 21
    sites = S.lattice_sites(2, [-nx // 2, 0], [nx // 2, ny], dx)
    kappa, rho, cp = 1.0, 1.0, 1.0
    mats = [S.Material(rho0=rho, p0=1.0), S.Material(rho0=rho), S.Material(rho0=rho, cp=cp, kappa=kappa)]
    T1, T2 = 10.0, 30.0
    T0 = np.where(sites[:, 0] < 0.0, T1, T2)
    lo = np.array([-10.0, -5.0, 0.0])
    hi = np.array([10.0, 5.0, 0.0])
    sc = S._assemble("strip", 2, dx, lo, hi, [(sites, S.RIGID, 2, 0, 0, T0)], mats,
                     [S.BodyInit(fixed=1)], max_bodies=1, thermal=1, contact=0)
    o = oracle_lib.OracleScene(sc)
    alpha = kappa / (rho * cp)
    dt = o.dt
    nsteps = int(round(25.0 * dx * dx / alpha / dt))
    o.step(nsteps)
    t = o.time
    T = o.get(oracle_lib.F_T)
    mid = np.abs(sc.x[:, 1] - (ny // 2 + 0.5) * dx) < 1e-9
    xs = sc.x[mid, 0]
    ref = 0.5 * (T1 + T2) + 0.5 * (T2 - T1) * special.erf(xs / (2.0 * math.sqrt(alpha * t)))
    err = np.max(np.abs(T[mid] - ref)) / (T2 - T1)
    assert err < 0.01


def test_extrapolation_hydrostatic_is_exact(oracle_lib):
    """With p_f = P - rho0 g y_f and rho_f = rho0, the extrapolated wall
    pressure is the linear extension P - rho0 g y_w (local force balance of
    Sec. "Boundary and coupling conditions"); a uniform velocity U of fluid
    and wall gives u~_w = U."""
    g, rho0, P = 9.81, 1000.0, 5000.0
    sc = S.fluid_box(2, 16, dx=0.05, jitter_amp=0.0, g=g, rho0=rho0)
    o = oracle_lib.OracleScene(sc)
    fl = sc.kind == S.FLUID
    rho = np.full(sc.n, rho0)
    p = np.where(fl, P - rho0 * g * sc.x[:, 1], 0.0)
    U = np.array([0.3, -0.2, 0.0])
    u = np.tile(U, (sc.n, 1))
    o.set(oracle_lib.F_RHO, rho)
    o.set(oracle_lib.F_P, p)
    o.set(oracle_lib.F_U, u)
    o.stage(oracle_lib.S_EXTRAP)
    pw = o.get(oracle_lib.F_PW)
    uw = o.get(oracle_lib.F_UW)
    w = ~fl
    has_fluid = np.array([np.any(np.sum((sc.x[fl, :2] - sc.x[i, :2]) ** 2, axis=1) < (3 * sc.dx) ** 2)
                          for i in np.nonzero(w)[0]])
    idx = np.nonzero(w)[0][has_fluid]
    ref = P - rho0 * g * sc.x[idx, 1]
    assert np.max(np.abs(pw[idx] - ref)) < 1e-10 * P
    assert np.max(np.abs(uw[idx, :2] - U[:2])) < 1e-13
    idx0 = np.nonzero(w)[0][~has_fluid]
    assert np.all(pw[idx0] == 0.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_isolated_momentum_conservation(oracle_lib, dim):
    sc = S.isolated_blob_with_body(dim=dim, n_side=14 if dim == 2 else 8)
    o = oracle_lib.OracleScene(sc)
    fl = sc.kind == S.FLUID

    def momentum():
        u = o.get(oracle_lib.F_U)
        m = o.get(oracle_lib.F_M)
        b = o.bodies()
        P = np.array([math.fsum(m[fl] * u[fl, a]) + math.fsum(b[:, 0] * b[:, 8 + a]) for a in range(3)])
        scale = math.fsum(m[fl] * np.linalg.norm(u[fl], axis=1)) + math.fsum(b[:, 0] * np.linalg.norm(b[:, 8:11], axis=1))
        return P, scale

    P0, scale = momentum()
    o.step(40)
    P1, _ = momentum()
    assert np.max(np.abs(P1 - P0)) < 1e-12 * scale
    # the body has actually been pushed by the fluid
    b = o.bodies()
    assert np.linalg.norm(b[0, 20:23]) > 0.0


def test_hydrostatic_box_at_rest(oracle_lib):
    g = 9.81
    sc = S.fluid_box(2, 20, dx=0.05, jitter_amp=0.0, g=g, nu=2.0, c=20.0, rho0=1000.0)
    o = oracle_lib.OracleScene(sc)
    o.step(1500)
    x = o.get(oracle_lib.F_X)
    p = o.get(oracle_lib.F_P)
    fl = sc.kind == S.FLUID
    inner = fl & interior_mask(x, 2, 0.0, 20 * 0.05, 3 * 0.05)
    slope = np.polyfit(x[inner, 1], p[inner], 1)[0]
    assert abs(slope / (-1000.0 * g) - 1.0) < 0.02
    u = o.get(oracle_lib.F_U)
    assert np.max(np.linalg.norm(u[fl], axis=1)) < 0.05 * math.sqrt(2 * g * 1.0)
