"""Neighbour search and cell order of the oracle against an O(N^2) brute
force written with numpy (CPU only).

The pair set {(a, b): a != b, |x_a - x_b|^2 < r_c^2} has a plain definition;
the cell-list search must reach it exactly.  The order by (cell, id) is
unique, so it is compared element by element.
"""
import numpy as np
import pytest

from paper_2103_07925_amd import scenes as S


def brute_pairs(x, dim, rc):
    d = x[:, None, :dim] - x[None, :, :dim]
    r2 = np.sum(d * d, axis=2)
    m = r2 < rc * rc
    np.fill_diagonal(m, False)
    return m


def check_scene(oracle, sc):
    o = oracle.OracleScene(sc)
    off, ids = o.neighbors()
    m = brute_pairs(sc.x, sc.dim, 3.0 * sc.dx)
    for i in range(sc.n):
        mine = ids[off[i]:off[i + 1]]
        ref = np.nonzero(m[i])[0]
        assert np.array_equal(mine, ref), f"row {i}"
    order, cell = o.cell_order()
    L = sc.cell_edge
    nc = o.grid()
    c3 = np.floor((sc.x[:, :3] - sc.lo[None, :]) / L).astype(np.int64)
    if sc.dim == 2:
        c3[:, 2] = 0
    lin = c3[:, 0] + nc[0] * (c3[:, 1] + nc[1] * c3[:, 2])
    assert np.array_equal(cell, lin)
    ref_order = np.lexsort((np.arange(sc.n), lin))
    assert np.array_equal(order, ref_order)
    return o


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("clustered", [False, True])
@pytest.mark.parametrize("seed", [0, 1])
def test_random_clouds(oracle_lib, dim, clustered, seed):
    n = 900 if dim == 2 else 1500
    sc = S.random_cloud(dim, n, extent=1.0, dx=0.02 if dim == 2 else 0.04, seed=seed, clustered=clustered)
    check_scene(oracle_lib, sc)


def test_c1_scene(oracle_lib):
    check_scene(oracle_lib, S.config_c1(seed=3))


def test_small_3d_box_with_bodies(oracle_lib):
    sc = S.config_c2(n_side=14, n_per_axis=1, spacing_sites=14, r_range=(3.0, 4.0))
    check_scene(oracle_lib, sc)


def test_larger_cell_edge(oracle_lib):
    sc = S.random_cloud(3, 1200, extent=1.0, dx=0.03, seed=5)
    sc.cell_edge = 0.13          # any edge >= r_c = 0.09 gives the same pairs
    check_scene(oracle_lib, sc)


def test_escape_is_an_error(oracle_lib):
    sc = S.fluid_box(2, 6, walls=False)
    sc.x[0, 0] = sc.hi[0] + 1.0
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.OracleScene(sc)
