"""Pins of the oracle's concentration transport and concentration-driven
dissolution (CPU only).

The remark on concentration-driven transitions (Sec. "Reversible phase
transition") solves dC/dt = (1/rho) div(D grad C) with the discretisation of
the heat equation, and the gastric example holds the gastric juice at a
fixed concentration while food boluses dissolve into chyme above C_t.  What
fixes the oracle here, other than its own formulas:
  * 1D diffusion into a block from a reservoir held at C_1 (a phase with a
    prescribed value): C = C_1 + (C_0 - C_1) erf((x - x_b) / (2 sqrt(D t)))
    while sqrt(D t) is small against the block, within 1 % at two times; the
    held rows are Dirichlet nodes, so the boundary x_b is the first held row
    (x_b = -dx/2; a boundary at the interface x = 0 misses by an O(dx)
    offset that shrinks like 1/sqrt(t));
  * the prescribed phase keeps its value exactly, and the discrete operator
    keeps every concentration inside the initial range;
  * the strict transition rule at C_t: after every step no bolus particle
    is above C_t and every dissolved particle is chyme with C > C_t at the
    step it switched; mass is conserved exactly.
"""
import math

import numpy as np
from scipy import special

from paper_2103_07925_amd import scenes as S


def test_diffusion_from_a_prescribed_reservoir(oracle_lib):
    O = oracle_lib
    dx = 0.1
    nx, ny = 80, 21
    sites = S.lattice_sites(2, [-nx // 2, 0], [nx // 2, ny], dx)
    D, rho = 0.5, 1.0
    mats = [S.Material(rho0=rho, p0=1.0), S.Material(rho0=rho),
            S.Material(rho0=rho, cp=1.0, kappa=D),                 # the block
            S.Material(rho0=rho, cp=1.0, kappa=D, dirichlet=1)]    # the reservoir
    C0, C1 = 0.0, 1.0
    res = sites[:, 0] < 0.0
    groups = [(sites[~res], S.RIGID, 2, 0, 0, C0), (sites[res], S.RIGID, 3, 1, 0, C1)]
    lo = np.array([-10.0, -5.0, 0.0])
    hi = np.array([10.0, 5.0, 0.0])
    sc = S._assemble("strip", 2, dx, lo, hi, groups, mats, [S.BodyInit(fixed=1), S.BodyInit(fixed=1)],
                     max_bodies=2, thermal=1, contact=0)
    o = O.OracleScene(sc)
    kind_res = sc.phase == 3
    mid = (np.abs(sc.x[:, 1] - (ny // 2 + 0.5) * dx) < 1e-9) & ~kind_res
    xs = sc.x[mid, 0]
    done = 0
    for mult in (25.0, 100.0):
        nsteps = int(round(mult * dx * dx / D / o.dt))
        o.step(nsteps - done)
        done = nsteps
        t = o.time
        C = o.get(O.F_T)
        assert np.array_equal(C[kind_res], np.full(int(kind_res.sum()), C1))
        ref = C1 + (C0 - C1) * special.erf((xs + 0.5 * dx) / (2.0 * math.sqrt(D * t)))
        assert np.max(np.abs(C[mid] - ref)) < 0.01 * (C1 - C0)
        assert C.min() >= C0 and C.max() <= C1


def test_boluses_dissolve_by_the_strict_rule(oracle_lib):
    O = oracle_lib
    sc = S.config_gastric(size=(6.0, 3.0), n_bolus=3, d_range=(0.8, 1.2), amplitude=1.2, seed=1)
    bol = sc.kind == S.RIGID
    sc.T[bol] = 0.8 - 2e-4           # close to C_t, so dissolution starts within the run
    o = O.OracleScene(sc)
    m0 = math.fsum(o.get(O.F_M))
    juice = sc.phase == 1
    switched = np.zeros(sc.n, bool)
    for _ in range(40):
        prev_kind = o.get_int(O.I_KIND)
        o.step(1)
        kind = o.get_int(O.I_KIND)
        ph = o.get_int(O.I_PHASE)
        C = o.get(O.F_T)
        new = (prev_kind == S.RIGID) & (kind == S.FLUID)
        assert np.all(ph[new] == 2) and np.all(C[new] > 0.8)
        assert np.all(C[(kind == S.RIGID)] <= 0.8)
        assert np.all(C[juice] == 1.0)
        assert math.fsum(o.get(O.F_M)) == m0
        switched |= new
    assert switched.any()
    # dissolution proceeds from the surface in: dissolved sites touch juice or chyme
    assert C.min() >= 0.0 and C.max() <= 1.0
