"""Scene generators against the counts the paper prints (CPU only)."""
import os

import numpy as np

from paper_2103_07925_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()[:2]
                out[k] = float(v)
    return out


def test_strong_scaling_scene_counts(oracle_lib):
    g = read_golden("strong_scaling_scene.txt")
    sc = S.config_e7(dx=g["dx"])
    c = sc.counts()
    assert c["n"] == int(g["total_particles"])
    assert c["fluid"] == int(g["fluid_particles"])
    assert c["rigid"] == int(g["rigid_particles"])
    assert c["wall"] == int(g["boundary_particles"])
    assert c["bodies"] == int(g["spheres"])
    assert np.all(np.bincount(sc.body[sc.kind == S.RIGID]) == 1021)
    assert sc.cell_edge == g["cell_edge"]
    # the oracle's cell grid for this domain: 48 cells of 0.65 per axis
    keep = np.nonzero(sc.kind == S.FLUID)[0][:20]
    small = S.Scene(name="e7grid", dim=3, dx=sc.dx, lo=sc.lo, hi=sc.hi, cell_edge=sc.cell_edge,
                    x=sc.x[keep], u=sc.u[keep], T=sc.T[keep], kind=sc.kind[keep], phase=sc.phase[keep],
                    body=sc.body[keep], moving=sc.moving[keep], materials=sc.materials, bodies=[])
    o = oracle_lib.OracleScene(small)
    assert list(o.grid()) == [int(g["cells_per_axis"])] * 3
    # p0 = rho0 c^2 and dt from the stability bounds
    assert sc.materials[0].p0 == g["p0"]
    assert abs(oracle_lib.timestep(small) - g["dt"]) < 1e-15


def test_c1_counts():
    c = S.config_c1().counts()
    assert (c["n"], c["fluid"], c["wall"], c["rigid"], c["bodies"]) == (1444, 972, 420, 52, 1)


def test_seeded_and_jittered():
    a = S.config_c1(seed=4)
    b = S.config_c1(seed=4)
    c = S.config_c1(seed=5)
    assert np.array_equal(a.x, b.x)
    assert not np.array_equal(a.x, c.x)
    fl = a.kind == S.FLUID
    lat = S.config_c1(jitter_amp=0.0)
    d = np.abs(a.x[fl] - lat.x[fl])
    assert d.max() <= 0.01 * a.dx and d.max() > 0.005 * a.dx
    assert np.array_equal(a.x[~fl], lat.x[~fl])


def test_c2_small_shape():
    sc = S.config_c2(n_side=30, n_per_axis=2, spacing_sites=15)
    c = sc.counts()
    assert c["n"] == 36 ** 3 and c["bodies"] == 8 and c["wall"] == 36 ** 3 - 30 ** 3
