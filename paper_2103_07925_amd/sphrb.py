"""ctypes binding of libsphrb.so (include/sphrb.h), same names as the C ABI.

Argument marshalling only: device memory (the scene arena) comes from a
torch uint8 tensor and the HIP stream from torch's current stream; every
step of the method runs in the library's HIP kernels.  If the built library
is missing, loading fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SPHRB_LIB selects another build of the same library (same ABI)
LIB_PATH = os.environ.get("SPHRB_LIB") or os.path.join(HERE, "libsphrb.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sphrb.h")

SPH_OK, SPH_E_INVALID, SPH_E_NOMEM, SPH_E_DEVICE, SPH_E_STATE, SPH_E_UNSUPPORTED = range(6)
SPH_FP64, SPH_FP32_SWEEP = 0, 1
SPH_FLUID, SPH_WALL, SPH_RIGID = 0, 1, 2
SPH_ERR_ESCAPE, SPH_ERR_CELL, SPH_ERR_NONFINITE, SPH_ERR_COINCIDENT, SPH_ERR_BODYCAP = 1, 2, 4, 8, 16
SPH_BODY_REC = 36
ABI_VERSION = 3
FIELDS = ["X", "U", "A", "RHO", "P", "T", "PW", "UW", "FR", "M", "DTDT", "AB", "UD"]
FIELD_BIT = {f: 1 << k for k, f in enumerate(FIELDS)}
VEC_FIELDS = {"X", "U", "A", "UW", "FR", "AB", "UD"}


class sph_material(C.Structure):
    _fields_ = [("rho0", C.c_double), ("p0", C.c_double), ("nu", C.c_double), ("cp", C.c_double),
                ("kappa", C.c_double), ("b", C.c_double * 3), ("T_t", C.c_double),
                ("switch_to", C.c_int32), ("dirichlet", C.c_int32)]


class sph_body_init(C.Structure):
    _fields_ = [("u", C.c_double * 3), ("w", C.c_double * 3), ("q", C.c_double * 4),
                ("fixed", C.c_int32), ("pad", C.c_int32)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class sph_scene_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("dx", C.c_double),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("cell_edge", C.c_double),
                ("dt", C.c_double), ("n", C.c_int64),
                ("x", _dp), ("u", _dp), ("T", _dp),
                ("kind", _ip), ("phase", _ip), ("body", _ip), ("moving", _ip),
                ("n_mat", C.c_int32), ("n_body", C.c_int32),
                ("mat", C.POINTER(sph_material)), ("bodies", C.POINTER(sph_body_init)),
                ("max_bodies", C.c_int32), ("thermal", C.c_int32), ("contact", C.c_int32),
                ("phase_switch", C.c_int32), ("k_c", C.c_double), ("d_c", C.c_double),
                ("wall_A", C.c_double), ("wall_Omega", C.c_double), ("wall_dir", C.c_double * 3),
                ("heat_src", C.c_int32), ("pad1", C.c_int32),
                ("src_Q", C.c_double), ("src_sigma", C.c_double), ("src_s0", C.c_double * 2),
                ("src_v", C.c_double * 2), ("src_ztop", C.c_double), ("src_depth", C.c_double),
                ("p_b", C.c_double), ("periodic", C.c_int32 * 3), ("pad2", C.c_int32)]


class sph_stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("dt", C.c_double), ("k_c", C.c_double),
                ("d_c", C.c_double), ("n", C.c_int64), ("n_fluid", C.c_int64), ("n_wall", C.c_int64),
                ("n_rigid", C.c_int64), ("n_bodies", C.c_int32), ("grid", C.c_int32 * 3),
                ("pairs_last", C.c_int64), ("pairs_total", C.c_int64), ("pairs_fluid", C.c_int64),
                ("pairs_rigid", C.c_int64), ("pairs_wall", C.c_int64), ("device_error", C.c_uint32),
                ("pad", C.c_uint32), ("mass", C.c_double), ("momentum", C.c_double * 3),
                ("kinetic", C.c_double), ("potential", C.c_double), ("n_melted", C.c_int64),
                ("n_solidified", C.c_int64)]


_lib = None


class SphError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib():
    """Load libsphrb.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    L.sph_abi_version.restype = C.c_int
    if L.sph_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {L.sph_abi_version()}, this binding needs {ABI_VERSION}: "
                           "rebuild it with __graft_entry__.build()")
    L.sph_status_string.argtypes = [C.c_int]
    L.sph_status_string.restype = C.c_char_p
    L.sph_last_error.restype = C.c_char_p
    L.sph_scene_arena_bytes.argtypes = [C.POINTER(sph_scene_desc), C.POINTER(C.c_int)]
    L.sph_scene_arena_bytes.restype = C.c_size_t
    L.sph_scene_create.argtypes = [C.POINTER(sph_scene_desc), C.c_void_p, C.c_size_t, C.c_void_p,
                                   C.POINTER(C.c_void_p)]
    L.sph_scene_step.argtypes = [C.c_void_p, C.c_int64]
    L.sph_batch_bytes.argtypes = [C.c_int32]
    L.sph_batch_bytes.restype = C.c_size_t
    L.sph_batch_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                   C.POINTER(C.c_void_p)]
    L.sph_batch_step.argtypes = [C.c_void_p, C.c_int64]
    L.sph_batch_destroy.argtypes = [C.c_void_p]
    L.sph_batch_destroy.restype = None
    L.sph_scene_sync.argtypes = [C.c_void_p]
    L.sph_scene_read_particles.argtypes = [C.c_void_p, C.c_uint32, _dp]
    L.sph_scene_read_bodies.argtypes = [C.c_void_p, _dp, C.c_int32, C.POINTER(C.c_int32)]
    L.sph_scene_read_neighbors.argtypes = [C.c_void_p, C.POINTER(C.c_int64), _ip, C.c_int64]
    L.sph_scene_read_neighbors.restype = C.c_int64
    L.sph_scene_read_cell_order.argtypes = [C.c_void_p, _ip, _ip]
    L.sph_scene_read_flags.argtypes = [C.c_void_p, _ip, _ip, _ip]
    L.sph_scene_read_stats.argtypes = [C.c_void_p, C.POINTER(sph_stats)]
    L.sph_scene_enable_timers.argtypes = [C.c_void_p, C.c_int32]
    L.sph_scene_read_timers.argtypes = [C.c_void_p, _dp, C.POINTER(C.c_int64), _dp, C.c_int64]
    L.sph_scene_state_bytes.argtypes = [C.c_void_p]
    L.sph_scene_state_bytes.restype = C.c_size_t
    L.sph_scene_read_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    L.sph_state_arena_bytes.argtypes = [C.c_void_p, C.c_size_t, C.POINTER(C.c_int)]
    L.sph_state_arena_bytes.restype = C.c_size_t
    L.sph_scene_create_from_state.argtypes = [C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_void_p,
                                              C.POINTER(C.c_void_p)]
    L.sph_scene_destroy.argtypes = [C.c_void_p]
    L.sph_scene_destroy.restype = None
    _lib = L
    return L


def header_symbols():
    """Entry points declared in include/sphrb.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", txt)))


def _check(status, what):
    if status != SPH_OK:
        msg = lib().sph_last_error().decode(errors="replace")
        raise SphError(status, f"{what}: {msg}")


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


class Desc:
    """sph_scene_desc built from a scenes.Scene; keeps the arrays alive."""

    def __init__(self, sc, precision=SPH_FP64, dt=None):
        self.x = np.ascontiguousarray(sc.x, np.float64)
        self.u = np.ascontiguousarray(sc.u, np.float64)
        self.T = np.ascontiguousarray(sc.T, np.float64)
        self.kind = np.ascontiguousarray(sc.kind, np.int32)
        self.phase = np.ascontiguousarray(sc.phase, np.int32)
        self.body = np.ascontiguousarray(sc.body, np.int32)
        self.moving = np.ascontiguousarray(sc.moving, np.int32)
        nm = len(sc.materials)
        self.mats = (sph_material * max(nm, 1))()
        for k, m in enumerate(sc.materials):
            M = self.mats[k]
            M.rho0, M.p0, M.nu, M.cp, M.kappa = m.rho0, m.p0, m.nu, m.cp, m.kappa
            for a in range(3):
                M.b[a] = m.b[a]
            M.T_t, M.switch_to, M.dirichlet = m.T_t, m.switch_to, m.dirichlet
        nb = len(sc.bodies)
        self.bodies = (sph_body_init * max(nb, 1))()
        for k, b in enumerate(sc.bodies):
            B = self.bodies[k]
            for a in range(3):
                B.u[a] = b.u[a]
                B.w[a] = b.w[a]
            for a in range(4):
                B.q[a] = b.q[a]
            B.fixed = b.fixed
        d = sph_scene_desc()
        d.dim = sc.dim
        d.precision = precision
        d.dx = sc.dx
        for a in range(3):
            d.lo[a] = sc.lo[a]
            d.hi[a] = sc.hi[a]
            d.wall_dir[a] = sc.wall_dir[a]
        d.cell_edge = sc.cell_edge
        d.dt = sc.dt if dt is None else dt
        d.n = sc.n
        d.x, d.u, d.T = _d(self.x), _d(self.u), _d(self.T)
        d.kind, d.phase, d.body, d.moving = _i(self.kind), _i(self.phase), _i(self.body), _i(self.moving)
        d.n_mat, d.n_body = nm, nb
        d.mat = self.mats
        d.bodies = self.bodies
        d.max_bodies = max(sc.max_bodies, nb)
        d.thermal, d.contact, d.phase_switch = sc.thermal, sc.contact, sc.phase_switch
        d.k_c, d.d_c = sc.k_c, sc.d_c
        d.wall_A, d.wall_Omega = sc.wall_A, sc.wall_Omega
        d.heat_src = sc.heat_src
        d.src_Q, d.src_sigma = sc.src_Q, sc.src_sigma
        for a in range(2):
            d.src_s0[a] = sc.src_s0[a]
            d.src_v[a] = sc.src_v[a]
        d.src_ztop, d.src_depth = sc.src_ztop, sc.src_depth
        d.p_b = getattr(sc, "p_b", 0.0)
        for a in range(3):
            d.periodic[a] = int(getattr(sc, "periodic", (0, 0, 0))[a])
        self.desc = d


def sph_abi_version():
    return lib().sph_abi_version()


def sph_status_string(status):
    return lib().sph_status_string(status).decode()


def sph_last_error():
    return lib().sph_last_error().decode(errors="replace")


def sph_scene_arena_bytes(desc: Desc) -> int:
    st = C.c_int(0)
    nbytes = lib().sph_scene_arena_bytes(C.byref(desc.desc), C.byref(st))
    _check(st.value, "sph_scene_arena_bytes")
    return int(nbytes)


def sph_state_arena_bytes(blob) -> int:
    """Device arena bytes a scene re-created from a state image needs."""
    blob = np.ascontiguousarray(blob, np.uint8)
    st = C.c_int(0)
    nbytes = lib().sph_state_arena_bytes(C.c_void_p(blob.ctypes.data), C.c_size_t(blob.nbytes), C.byref(st))
    _check(st.value, "sph_state_arena_bytes")
    return int(nbytes)


class SphScene:
    """One resident scene: a torch-owned device arena plus the library handle."""

    @classmethod
    def sph_scene_create_from_state(cls, blob, like, device="cuda", stream=None, arena=None):
        """Re-create a scene from a state image; `like` is the scene
        description it was made from (particle count and dimension)."""
        import torch
        blob = np.ascontiguousarray(blob, np.uint8)
        self = cls.__new__(cls)
        self.sc = like
        self.n = like.n
        self.dim = like.dim
        self.precision = None
        self._desc = None
        self.arena_bytes = sph_state_arena_bytes(blob)
        if arena is None:
            arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device=device)
        assert arena.numel() >= self.arena_bytes and arena.data_ptr() % 256 == 0
        self.arena = arena
        self.stream = stream if stream is not None else torch.cuda.current_stream(arena.device)
        h = C.c_void_p()
        st = lib().sph_scene_create_from_state(C.c_void_p(blob.ctypes.data), C.c_size_t(blob.nbytes),
                                               C.c_void_p(arena.data_ptr()), C.c_size_t(arena.numel()),
                                               C.c_void_p(self.stream.cuda_stream), C.byref(h))
        _check(st, "sph_scene_create_from_state")
        self.handle = h
        return self

    from_state = sph_scene_create_from_state

    def __init__(self, sc, precision=SPH_FP64, dt=None, device="cuda", stream=None, arena=None):
        import torch
        self.sc = sc
        self.n = sc.n
        self.dim = sc.dim
        self.precision = precision
        self._desc = Desc(sc, precision, dt)
        self.arena_bytes = sph_scene_arena_bytes(self._desc)
        if arena is None:
            arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device=device)
        assert arena.numel() >= self.arena_bytes and arena.data_ptr() % 256 == 0
        self.arena = arena
        self.stream = stream if stream is not None else torch.cuda.current_stream(arena.device)
        h = C.c_void_p()
        st = lib().sph_scene_create(C.byref(self._desc.desc), C.c_void_p(arena.data_ptr()),
                                    C.c_size_t(arena.numel()), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        _check(st, "sph_scene_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().sph_scene_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- ABI calls ----------------------------------------------------------
    def sph_scene_step(self, nsteps=1):
        _check(lib().sph_scene_step(self.handle, int(nsteps)), "sph_scene_step")

    step = sph_scene_step

    def sph_scene_sync(self):
        _check(lib().sph_scene_sync(self.handle), "sph_scene_sync")

    sync = sph_scene_sync

    def sph_scene_read_particles(self, fields):
        mask = 0
        for f in fields:
            mask |= FIELD_BIT[f]
        total = sum(3 * self.n if f in VEC_FIELDS else self.n for f in FIELDS if mask & FIELD_BIT[f])
        buf = np.zeros(max(total, 1), np.float64)
        _check(lib().sph_scene_read_particles(self.handle, mask, _d(buf)), "sph_scene_read_particles")
        out, off = {}, 0
        for f in FIELDS:
            if mask & FIELD_BIT[f]:
                w = 3 if f in VEC_FIELDS else 1
                a = buf[off:off + w * self.n]
                out[f] = a.reshape(self.n, 3) if w == 3 else a
                off += w * self.n
        return out

    def get(self, field):
        return self.sph_scene_read_particles([field])[field]

    def sph_scene_read_bodies(self):
        nb = C.c_int32(0)
        _check(lib().sph_scene_read_bodies(self.handle, None, 0, C.byref(nb)), "sph_scene_read_bodies")
        out = np.zeros((max(nb.value, 1), SPH_BODY_REC), np.float64)
        _check(lib().sph_scene_read_bodies(self.handle, _d(out), nb.value, C.byref(nb)), "sph_scene_read_bodies")
        return out[:nb.value]

    bodies = sph_scene_read_bodies

    def sph_scene_read_neighbors(self):
        off = np.zeros(self.n + 1, np.int64)
        tot = lib().sph_scene_read_neighbors(self.handle, off.ctypes.data_as(C.POINTER(C.c_int64)), None, 0)
        if tot < 0:
            raise SphError(SPH_E_DEVICE, sph_last_error())
        ids = np.zeros(max(tot, 1), np.int32)
        tot2 = lib().sph_scene_read_neighbors(self.handle, off.ctypes.data_as(C.POINTER(C.c_int64)), _i(ids), tot)
        if tot2 != tot:
            raise SphError(SPH_E_DEVICE, sph_last_error())
        return off, ids[:tot]

    neighbors = sph_scene_read_neighbors

    def sph_scene_read_cell_order(self):
        s = np.zeros(self.n, np.int32)
        c = np.zeros(self.n, np.int32)
        _check(lib().sph_scene_read_cell_order(self.handle, _i(s), _i(c)), "sph_scene_read_cell_order")
        return s, c

    cell_order = sph_scene_read_cell_order

    def sph_scene_read_flags(self):
        k = np.zeros(self.n, np.int32)
        p = np.zeros(self.n, np.int32)
        b = np.zeros(self.n, np.int32)
        _check(lib().sph_scene_read_flags(self.handle, _i(k), _i(p), _i(b)), "sph_scene_read_flags")
        return k, p, b

    flags = sph_scene_read_flags

    def sph_scene_read_stats(self):
        st = sph_stats()
        _check(lib().sph_scene_read_stats(self.handle, C.byref(st)), "sph_scene_read_stats")
        return st

    stats = sph_scene_read_stats

    def sph_scene_read_state(self):
        """State image (header + device arena) as a numpy uint8 array."""
        nbytes = lib().sph_scene_state_bytes(self.handle)
        blob = np.empty(nbytes, np.uint8)
        _check(lib().sph_scene_read_state(self.handle, C.c_void_p(blob.ctypes.data), C.c_size_t(nbytes)),
               "sph_scene_read_state")
        return blob

    read_state = sph_scene_read_state

    def sph_scene_enable_timers(self, enable=True):
        _check(lib().sph_scene_enable_timers(self.handle, int(enable)), "sph_scene_enable_timers")

    STAGES = ["integrate", "neighbor_search", "density", "extrapolate", "forces", "body_reduce", "rigid_velocity"]

    def sph_scene_read_timers(self, with_steps=False):
        """Per-stage milliseconds summed over the recorded steps, the number
        of recorded steps and (optionally) each step's duration."""
        ms = np.zeros(7, np.float64)
        nrec = C.c_int64(0)
        steps = np.zeros(4096, np.float64)
        _check(lib().sph_scene_read_timers(self.handle, _d(ms), C.byref(nrec), _d(steps), 4096),
               "sph_scene_read_timers")
        out = {k: float(v) for k, v in zip(self.STAGES, ms)}
        out["steps"] = int(nrec.value)
        if with_steps:
            out["step_ms"] = steps[:nrec.value].copy()
        return out


class SphBatch:
    """Scenes advanced together (one launch per interaction sweep over all of
    them); the device workspace is a torch tensor owned by this object."""

    def __init__(self, scenes, stream=None, device="cuda"):
        import torch
        self.scenes = list(scenes)
        n = len(self.scenes)
        nbytes = int(lib().sph_batch_bytes(n))
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        arr = (C.c_void_p * max(n, 1))(*[s.handle.value for s in self.scenes])
        h = C.c_void_p()
        _check(lib().sph_batch_create(arr, n, C.c_void_p(self.ws.data_ptr()), C.c_size_t(self.ws.numel()),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)), "sph_batch_create")
        self.handle = h

    def sph_batch_step(self, nsteps=1):
        _check(lib().sph_batch_step(self.handle, int(nsteps)), "sph_batch_step")

    step = sph_batch_step

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            lib().sph_batch_destroy(self.handle)
            self.handle = C.c_void_p()

    sph_batch_destroy = close

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sph_batch_bytes(n):
    return int(lib().sph_batch_bytes(int(n)))
