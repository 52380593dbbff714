"""Helpers shared by the GPU parity tests: run a scene on the HIP library and
on the oracle, and compare field by field with field-scaled errors."""
import math

import numpy as np

import oracle as O
from paper_2103_07925_amd import scenes as S


def scales(sc):
    """Per-field scales: dx for positions, a reference speed for velocities
    (one tenth of the largest speed of sound of a fluid phase), rho0 for
    densities, p0 for pressures."""
    fl_ph = sorted(set(sc.phase[sc.kind == S.FLUID].tolist()))
    c = max([math.sqrt(sc.materials[p].p0 / sc.materials[p].rho0) for p in fl_ph] or [1.0])
    rho0 = max([sc.materials[p].rho0 for p in fl_ph] or [1.0])
    p0 = max([sc.materials[p].p0 for p in fl_ph] or [1.0])
    Tr = float(np.ptp(sc.T)) if sc.thermal and np.ptp(sc.T) > 0 else 1.0
    return {"x": sc.dx, "u": c / 10.0, "rho": rho0, "p": p0, "T": Tr}


def oracle_fields(o):
    return {
        "X": o.get(O.F_X), "U": o.get(O.F_U), "A": o.get(O.F_A), "RHO": o.get(O.F_RHO), "P": o.get(O.F_P),
        "T": o.get(O.F_T), "PW": o.get(O.F_PW), "UW": o.get(O.F_UW), "FR": o.get(O.F_FR),
        "AB": o.get(O.F_AB), "UD": o.get(O.F_UD),
    }


def gpu_fields(g):
    return g.sph_scene_read_particles(["X", "U", "A", "RHO", "P", "T", "PW", "UW", "FR", "AB", "UD"])


def field_errors(sc, gf, of, kind):
    """Max field-scaled errors of the GPU fields against the oracle's."""
    s = scales(sc)
    fl = kind == S.FLUID
    nf = kind != S.FLUID
    rg = kind == S.RIGID
    out = {}
    out["x"] = np.max(np.abs(gf["X"] - of["X"])) / s["x"]
    out["u"] = np.max(np.abs(gf["U"] - of["U"])) / s["u"]
    a_scale = max(np.max(np.abs(of["A"][fl])), 1e-300) if fl.any() else 1.0
    out["a"] = np.max(np.abs(gf["A"][fl] - of["A"][fl])) / a_scale if fl.any() else 0.0
    out["rho"] = np.max(np.abs(gf["RHO"][fl] - of["RHO"][fl])) / s["rho"] if fl.any() else 0.0
    out["p"] = np.max(np.abs(gf["P"][fl] - of["P"][fl])) / s["p"] if fl.any() else 0.0
    out["pw"] = np.max(np.abs(gf["PW"][nf] - of["PW"][nf])) / s["p"] if nf.any() else 0.0
    out["uw"] = np.max(np.abs(gf["UW"][nf] - of["UW"][nf])) / s["u"] if nf.any() else 0.0
    if rg.any():
        f_scale = max(np.max(np.abs(of["FR"][rg])), 1e-300)
        out["fr"] = np.max(np.abs(gf["FR"][rg] - of["FR"][rg])) / f_scale
    if sc.thermal:
        out["T"] = np.max(np.abs(gf["T"] - of["T"])) / s["T"]
    if getattr(sc, "p_b", 0.0) > 0.0 and fl.any():
        # transport-velocity formulation: a_b against the size of one pair
        # term, p_b / (rho0 dx); u~ - u against the velocity scale
        out["ab"] = np.max(np.abs(gf["AB"][fl] - of["AB"][fl])) / (sc.p_b / (s["rho"] * sc.dx))
        out["ud"] = np.max(np.abs(gf["UD"][fl] - of["UD"][fl])) / s["u"]
    return out


def body_errors(sc, gb, ob):
    s = scales(sc)
    if len(ob) == 0:
        return {}
    e = {}
    e["m"] = np.max(np.abs(gb[:, 0] - ob[:, 0]) / ob[:, 0])
    e["r"] = np.max(np.abs(gb[:, 1:4] - ob[:, 1:4])) / s["x"]
    dq = np.minimum(np.max(np.abs(gb[:, 4:8] - ob[:, 4:8]), axis=1), np.max(np.abs(gb[:, 4:8] + ob[:, 4:8]), axis=1))
    e["q"] = np.max(dq)
    e["u"] = np.max(np.abs(gb[:, 8:11] - ob[:, 8:11])) / s["u"]
    R = max(sc.dx, 1e-300) * 4
    e["w"] = np.max(np.abs(gb[:, 11:14] - ob[:, 11:14])) * R / s["u"]
    return e


def run_pair(sc, precision, steps, dt=None):
    from paper_2103_07925_amd import sphrb as B
    o = O.OracleScene(sc, dt=dt)
    g = B.SphScene(sc, precision=precision, dt=dt)
    if steps:
        o.step(steps)
        g.step(steps)
    g.sync()
    return o, g
