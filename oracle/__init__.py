"""Python binding of the plain FP64 CPU oracle (oracle/sph_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark are the only callers.  The product path never
imports this package.

`build()` compiles sph_oracle.c with gcc (-O2 -ffp-contract=off, no
fast-math) into oracle/liboracle.so.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FLUID, WALL, RIGID = 0, 1, 2
BODY_REC = 36
F_X, F_U, F_A, F_RHO, F_P, F_T, F_PW, F_UW, F_FR, F_M, F_DTDT, F_AB, F_UD = range(13)
I_KIND, I_PHASE, I_BODY, I_CELL = range(4)
S_NEIGHBORS, S_DENSITY, S_EXTRAP, S_HEAT, S_FORCES, S_BODYSUMS, S_BODYACC = range(4, 11)
_VEC_FIELDS = {F_X, F_U, F_A, F_UW, F_FR, F_AB, F_UD}


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
               "-o", _LIB_PATH, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
    return _LIB_PATH


class Material(C.Structure):
    _fields_ = [("rho0", C.c_double), ("p0", C.c_double), ("nu", C.c_double), ("cp", C.c_double),
                ("kappa", C.c_double), ("b", C.c_double * 3), ("T_t", C.c_double),
                ("switch_to", C.c_int32), ("dirichlet", C.c_int32)]


class BodyInit(C.Structure):
    _fields_ = [("u", C.c_double * 3), ("w", C.c_double * 3), ("q", C.c_double * 4),
                ("fixed", C.c_int32), ("pad", C.c_int32)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class Desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("pad0", C.c_int32), ("dx", C.c_double),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("cell_edge", C.c_double),
                ("dt", C.c_double), ("n", C.c_int64),
                ("x", _dp), ("u", _dp), ("T", _dp),
                ("kind", _ip), ("phase", _ip), ("body", _ip), ("moving", _ip),
                ("n_mat", C.c_int32), ("n_body", C.c_int32),
                ("mat", C.POINTER(Material)), ("bodies", C.POINTER(BodyInit)),
                ("max_bodies", C.c_int32), ("thermal", C.c_int32), ("contact", C.c_int32),
                ("phase_switch", C.c_int32), ("k_c", C.c_double), ("d_c", C.c_double),
                ("wall_A", C.c_double), ("wall_Omega", C.c_double), ("wall_dir", C.c_double * 3),
                ("heat_src", C.c_int32), ("pad1", C.c_int32),
                ("src_Q", C.c_double), ("src_sigma", C.c_double), ("src_s0", C.c_double * 2),
                ("src_v", C.c_double * 2), ("src_ztop", C.c_double), ("src_depth", C.c_double),
                ("p_b", C.c_double), ("periodic", C.c_int32 * 3), ("pad2", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.orc_create.argtypes = [C.POINTER(Desc), C.POINTER(C.c_void_p)]
        L.orc_create.restype = C.c_int
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_step.restype = C.c_int
        for nm in ("orc_get_dt", "orc_get_time", "orc_get_kc", "orc_get_dc"):
            getattr(L, nm).argtypes = [C.c_void_p]
            getattr(L, nm).restype = C.c_double
        L.orc_n_bodies.argtypes = [C.c_void_p]
        L.orc_n_bodies.restype = C.c_int32
        L.orc_pair_count.argtypes = [C.c_void_p]
        L.orc_pair_count.restype = C.c_int64
        L.orc_get.argtypes = [C.c_void_p, C.c_int32, _dp]
        L.orc_set.argtypes = [C.c_void_p, C.c_int32, _dp]
        L.orc_get_int.argtypes = [C.c_void_p, C.c_int32, _ip]
        L.orc_get_bodies.argtypes = [C.c_void_p, _dp]
        L.orc_stage.argtypes = [C.c_void_p, C.c_int32]
        L.orc_stage.restype = C.c_int
        L.orc_neighbors.argtypes = [C.c_void_p, C.POINTER(C.c_int64), _ip, C.c_int64]
        L.orc_neighbors.restype = C.c_int64
        L.orc_cell_order.argtypes = [C.c_void_p, _ip, _ip]
        L.orc_grid.argtypes = [C.c_void_p, _ip]
        L.orc_kernel_W.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.orc_kernel_W.restype = C.c_double
        L.orc_kernel_dW.argtypes = [C.c_int32, C.c_double, C.c_double]
        L.orc_kernel_dW.restype = C.c_double
        L.orc_fsum.argtypes = [_dp, C.c_int64]
        L.orc_fsum.restype = C.c_double
        L.orc_timestep.argtypes = [C.POINTER(Desc)]
        L.orc_timestep.restype = C.c_double
        L.orc_mass_props.argtypes = [C.c_int32, C.c_double, C.c_int64, _dp, _dp, _dp, _dp, _dp]
        L.orc_mass_props_partitioned.argtypes = [C.c_int32, C.c_double, C.c_int64, _dp, _dp, _ip,
                                                 C.c_int32, _dp, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


class _DescHolder:
    """Keeps the numpy arrays alive while the C side reads them."""

    def __init__(self, sc, dt=None):
        self.x = np.ascontiguousarray(sc.x, np.float64)
        self.u = np.ascontiguousarray(sc.u, np.float64)
        self.T = np.ascontiguousarray(sc.T, np.float64)
        self.kind = np.ascontiguousarray(sc.kind, np.int32)
        self.phase = np.ascontiguousarray(sc.phase, np.int32)
        self.body = np.ascontiguousarray(sc.body, np.int32)
        self.moving = np.ascontiguousarray(sc.moving, np.int32)
        nm = len(sc.materials)
        self.mats = (Material * max(nm, 1))()
        for k, m in enumerate(sc.materials):
            M = self.mats[k]
            M.rho0, M.p0, M.nu, M.cp, M.kappa = m.rho0, m.p0, m.nu, m.cp, m.kappa
            for a in range(3):
                M.b[a] = m.b[a]
            M.T_t, M.switch_to, M.dirichlet = m.T_t, m.switch_to, m.dirichlet
        nb = len(sc.bodies)
        self.bodies = (BodyInit * max(nb, 1))()
        for k, b in enumerate(sc.bodies):
            B = self.bodies[k]
            for a in range(3):
                B.u[a] = b.u[a]
                B.w[a] = b.w[a]
            for a in range(4):
                B.q[a] = b.q[a]
            B.fixed = b.fixed
        d = Desc()
        d.dim = sc.dim
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


class OracleError(RuntimeError):
    pass


class OracleScene:
    """One scene advanced by the oracle (FP64, original-id order)."""

    def __init__(self, sc, dt=None):
        self.sc = sc
        self.n = sc.n
        self.dim = sc.dim
        self._h = _DescHolder(sc, dt)
        ptr = C.c_void_p()
        st = lib().orc_create(C.byref(self._h.desc), C.byref(ptr))
        if st != 0:
            raise OracleError(f"orc_create failed with status {st}")
        self._p = ptr

    def close(self):
        if self._p:
            lib().orc_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        st = lib().orc_step(self._p, int(n))
        if st != 0:
            raise OracleError(f"orc_step failed with status {st}")

    @property
    def dt(self):
        return lib().orc_get_dt(self._p)

    @property
    def time(self):
        return lib().orc_get_time(self._p)

    @property
    def k_c(self):
        return lib().orc_get_kc(self._p)

    @property
    def d_c(self):
        return lib().orc_get_dc(self._p)

    @property
    def pair_count(self):
        return int(lib().orc_pair_count(self._p))

    def get(self, field):
        w = 3 if field in _VEC_FIELDS else 1
        out = np.zeros((self.n, w) if w == 3 else self.n, np.float64)
        st = lib().orc_get(self._p, field, _d(out))
        if st != 0:
            raise OracleError("bad field")
        return out

    def set(self, field, values):
        w = 3 if field in _VEC_FIELDS else 1
        v = np.ascontiguousarray(values, np.float64).reshape((self.n, w) if w == 3 else self.n)
        lib().orc_set(self._p, field, _d(v))

    def get_int(self, field):
        out = np.zeros(self.n, np.int32)
        lib().orc_get_int(self._p, field, _i(out))
        return out

    def bodies(self):
        nb = lib().orc_n_bodies(self._p)
        out = np.zeros((max(nb, 0), BODY_REC), np.float64)
        if nb:
            lib().orc_get_bodies(self._p, _d(out))
        return out

    def stage(self, st):
        r = lib().orc_stage(self._p, st)
        if r != 0:
            raise OracleError(f"stage {st} failed with status {r}")

    def neighbors(self):
        L = lib()
        off = np.zeros(self.n + 1, np.int64)
        tot = L.orc_neighbors(self._p, off.ctypes.data_as(C.POINTER(C.c_int64)), None, 0)
        ids = np.zeros(max(tot, 1), np.int32)
        L.orc_neighbors(self._p, off.ctypes.data_as(C.POINTER(C.c_int64)), _i(ids), tot)
        return off, ids[:tot]

    def cell_order(self):
        s = np.zeros(self.n, np.int32)
        c = np.zeros(self.n, np.int32)
        st = lib().orc_cell_order(self._p, _i(s), _i(c))
        if st != 0:
            raise OracleError("cell order failed")
        return s, c

    def grid(self):
        g = np.zeros(3, np.int32)
        lib().orc_grid(self._p, _i(g))
        return g


def kernel_W(dim, h, r):
    return lib().orc_kernel_W(dim, h, r)


def kernel_dW(dim, h, r):
    return lib().orc_kernel_dW(dim, h, r)


def fsum(v):
    v = np.ascontiguousarray(v, np.float64)
    return lib().orc_fsum(_d(v), v.size)


def timestep(sc, dt_override=None):
    h = _DescHolder(sc, dt_override)
    return lib().orc_timestep(C.byref(h.desc))


def mass_props(dim, dx, x, m):
    x = np.ascontiguousarray(x, np.float64)
    m = np.ascontiguousarray(m, np.float64)
    om = np.zeros(1)
    orr = np.zeros(3)
    oI = np.zeros(9)
    lib().orc_mass_props(dim, dx, m.size, _d(x), _d(m), _d(om), _d(orr), _d(oI))
    return om[0], orr, oI.reshape(3, 3)


def mass_props_partitioned(dim, dx, x, m, part, nparts):
    x = np.ascontiguousarray(x, np.float64)
    m = np.ascontiguousarray(m, np.float64)
    part = np.ascontiguousarray(part, np.int32)
    om = np.zeros(1)
    orr = np.zeros(3)
    oI = np.zeros(9)
    lib().orc_mass_props_partitioned(dim, dx, m.size, _d(x), _d(m), _i(part), nparts, _d(om), _d(orr), _d(oI))
    return om[0], orr, oI.reshape(3, 3)
