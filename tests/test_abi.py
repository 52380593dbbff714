"""The C-ABI library loads and exports every entry point its header declares;
host-side descriptor validation and arena sizing (no GPU call)."""
import ctypes as C

import numpy as np
import pytest

from paper_2103_07925_amd import scenes as S
from paper_2103_07925_amd import sphrb as B


@pytest.fixture(scope="module")
def L():
    return B.lib()


def test_exports_every_header_symbol(L):
    syms = B.header_symbols()
    assert len(syms) >= 17
    for s in syms:
        assert hasattr(L, s), s


def test_version_and_status(L):
    assert B.sph_abi_version() == 3
    assert B.sph_status_string(B.SPH_E_INVALID) == "invalid argument"


def test_arena_bytes_scale_with_precision_and_size():
    sc = S.config_c1()
    b64 = B.sph_scene_arena_bytes(B.Desc(sc, B.SPH_FP64))
    b32 = B.sph_scene_arena_bytes(B.Desc(sc, B.SPH_FP32_SWEEP))
    assert 0 < b32 < b64
    big = S.fluid_box(3, 20)
    assert B.sph_scene_arena_bytes(B.Desc(big, B.SPH_FP32_SWEEP)) > b32
    # FP32 footprint per particle: state, sort buffers and the fixed-capacity
    # neighbour lists (320 16-bit entries per particle in 3D)
    assert B.sph_scene_arena_bytes(B.Desc(big, B.SPH_FP32_SWEEP)) / big.n < 1500


@pytest.mark.parametrize("mutate,what", [
    (lambda sc: setattr(sc, "cell_edge", sc.dx), "cell edge"),
    (lambda sc: sc.phase.__setitem__(0, 99), "bad phase"),
    (lambda sc: sc.kind.__setitem__(3, 7), "bad kind"),
    (lambda sc: sc.x.__setitem__((5, 0), np.nan), "non-finite"),
    (lambda sc: sc.body.__setitem__(int(np.nonzero(sc.kind == S.RIGID)[0][0]), 5), "bad body"),
])
def test_invalid_descriptors_rejected(mutate, what):
    sc = S.config_c1()
    mutate(sc)
    with pytest.raises(B.SphError) as e:
        B.sph_scene_arena_bytes(B.Desc(sc, B.SPH_FP64))
    assert e.value.status == B.SPH_E_INVALID
    assert what in B.sph_last_error()


def _many_phases(sc, n, fluid_phase=None, thermal=0):
    """sc with n materials; optionally its fluid particles moved to fluid_phase."""
    extra = [S.Material(rho0=sc.materials[0].rho0, p0=sc.materials[0].p0, nu=sc.materials[0].nu)
             for _ in range(n - len(sc.materials))]
    sc.materials = list(sc.materials) + extra
    if fluid_phase is not None:
        sc.phase[sc.kind == S.FLUID] = fluid_phase
    sc.thermal = thermal
    return sc


@pytest.mark.parametrize("mutate,status,what", [
    (lambda sc: _many_phases(sc, 20, fluid_phase=17), "UNSUPPORTED", "fluid phases"),
    (lambda sc: _many_phases(sc, 20, thermal=1), "UNSUPPORTED", "thermal scene"),
    (lambda sc: setattr(sc, "phase_switch", 1), "INVALID", "scalar (thermal) solver"),
    (lambda sc: setattr(sc, "p_b", -1.0), "INVALID", "background pressure"),
])
def test_scene_limits_rejected(mutate, status, what):
    """The sweeps' LDS phase table, phase switching and the transport-velocity
    option have set-up conditions; a descriptor that breaks one is refused
    before any device call."""
    sc = S.config_c1()
    mutate(sc)
    with pytest.raises(B.SphError) as e:
        B.sph_scene_arena_bytes(B.Desc(sc, B.SPH_FP32_SWEEP))
    assert e.value.status == getattr(B, "SPH_E_" + status)
    assert what in B.sph_last_error()


def _periodic(sc, axes, ny=None):
    sc.periodic = axes
    if ny is not None:
        sc.hi[1] = sc.lo[1] + ny * 3.0 * sc.dx
    return sc


@pytest.mark.parametrize("mutate,status,what", [
    (lambda sc: _periodic(sc, (1, 0, 0)), "UNSUPPORTED", "x axis"),
    (lambda sc: _periodic(sc, (0, 1, 0), ny=2), "INVALID", "at least 3 cells"),
    (lambda sc: setattr(sc, "hi", sc.hi + np.array([0.0, 0.01, 0.0])) or _periodic(sc, (0, 1, 0)), "INVALID",
     "whole number of cells"),
])
def test_periodic_limits_rejected(mutate, status, what):
    sc = S.periodic_channel(dim=2, n_sites=(12, 9, 1), dx=0.1)
    sc.periodic = (0, 0, 0)
    mutate(sc)
    with pytest.raises(B.SphError) as e:
        B.sph_scene_arena_bytes(B.Desc(sc, B.SPH_FP32_SWEEP))
    assert e.value.status == getattr(B, "SPH_E_" + status)
    assert what in B.sph_last_error()


def test_many_rigid_phases_accepted():
    """Rigid phases beyond the first 16 materials are fine (the 3D column
    gives every sphere its own density)."""
    sc = S.config_c2(seed=0, n_side=24, n_per_axis=3, spacing_sites=8, r_range=(2.0, 3.0))
    assert len(sc.materials) > 16
    assert B.sph_scene_arena_bytes(B.Desc(sc, B.SPH_FP32_SWEEP)) > 0


@pytest.mark.parametrize("blob", [b"", b"not a state image at all" * 4, b"SPHRBST1" + b"\0" * 64])
def test_state_images_rejected(blob):
    """A buffer that is not a whole state image is refused before any device call."""
    with pytest.raises(B.SphError) as e:
        B.sph_state_arena_bytes(np.frombuffer(blob, np.uint8) if blob else np.zeros(0, np.uint8))
    assert e.value.status == B.SPH_E_INVALID
