"""Python view of the CPU oracle (liboracle.so, built from lbm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports it.

Arrays are numpy float64 in the canonical order [component][z][y][x]
(rho: (nz, ny, nx), u: (3, nz, ny, nx), populations: (Q, nz, ny, nx)).
``tau`` is the lattice relaxation time: omega = 1/tau, nu = (tau - 1/2)/3.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

D2Q9, D3Q19, D3Q27 = 0, 1, 2
PERIODIC, SOLID_ENDS, WALLS_OUTSIDE, WALLS_NODAL = 0, 1, 2, 3
_QOF = {D2Q9: 9, D3Q19: 19, D3Q27: 27}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.orc_create.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, _dp, _ip, ctypes.POINTER(vp)]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_destroy.restype = None
    lib.orc_init_equilibrium.argtypes = [vp, _dp, _dp, _dp]
    lib.orc_set_populations.argtypes = [vp, _dp]
    lib.orc_get_populations.argtypes = [vp, _dp]
    lib.orc_step.argtypes = [vp, ctypes.c_int]
    lib.orc_moments.argtypes = [vp, _dp, _dp]
    lib.orc_geometry.argtypes = [vp, ctypes.POINTER(ctypes.c_ubyte)]
    lib.orc_reduce.argtypes = [vp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_long)]
    lib.orc_lattice_tables.argtypes = [ctypes.c_int, _ip, _ip, _ip, _dp]
    lib.orc_equilibrium_node.argtypes = [ctypes.c_int, ctypes.c_double, _dp, ctypes.c_int, _dp]
    lib.orc_collide_node.argtypes = [ctypes.c_int, ctypes.c_double, _dp, ctypes.c_int, _dp, _dp]
    lib.orc_set_compressible.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.orc_collide_node_cs.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
    _up = ctypes.POINTER(ctypes.c_ubyte)
    lib.orc_cs_objective.argtypes = (
        [ctypes.c_int] * 4 + [ctypes.c_double, ctypes.c_double, _dp, _dp, _ip, _up, ctypes.c_int,
                              _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp])
    lib.orc_adjoint.argtypes = (
        [ctypes.c_int] * 4 + [ctypes.c_double, _dp, _ip, _up, ctypes.c_int, _dp, _dp, _dp,
                              ctypes.c_int, _dp, _dp, _dp, _dp])
    lib.orc_set_solid.argtypes = [vp, ctypes.POINTER(ctypes.c_ubyte)]
    lib.orc_wall_force.argtypes = [vp, _dp]
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def set_num_threads(n):
    """Thread count of the oracle's parallel loops."""
    _check(_load().orc_set_num_threads(int(n)), "set_num_threads")


def num_threads():
    """OpenMP threads the oracle's loops run on."""
    return _load().orc_num_threads()


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _vec3(v):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (3,)))


def _bc3(bc):
    return (ctypes.c_int * 3)(*[int(b) for b in bc])


def _check(st, what):
    if st != 0:
        raise ValueError(f"oracle {what} failed with status {st}")


def lattice_tables(lattice):
    """(e [Q,3] int, t [Q] float64) of the oracle's lattice."""
    lib = _load()
    Q, D = ctypes.c_int(), ctypes.c_int()
    e = np.zeros((27, 3), dtype=np.int32)
    t = np.zeros(27)
    _check(lib.orc_lattice_tables(lattice, ctypes.byref(Q), ctypes.byref(D),
                                  e.ctypes.data_as(_ip), _d(t)), "lattice_tables")
    return e[: Q.value].astype(np.int64), t[: Q.value].copy()


def equilibrium_node(lattice, rho, u, compressible=False):
    lib = _load()
    Q = _QOF[lattice]
    out = np.zeros(Q)
    _check(lib.orc_equilibrium_node(lattice, float(rho), _d(_vec3(u)), int(compressible), _d(out)),
           "equilibrium")
    return out


def collide_node(lattice, tau, F, f, compressible=False):
    lib = _load()
    f = _f64(f)
    out = np.zeros_like(f)
    _check(lib.orc_collide_node(lattice, float(tau), _d(_vec3(F)), int(compressible), _d(f),
                                _d(out)), "collide")
    return out


def collide_node_complex(lattice, tau, F, f):
    """Collision in complex arithmetic (tau, F, f may be complex)."""
    lib = _load()
    tau = np.array([complex(tau).real, complex(tau).imag])
    Fc = np.broadcast_to(np.asarray(F, dtype=np.complex128), (3,))
    F2 = np.ascontiguousarray(np.stack([Fc.real, Fc.imag], -1).reshape(-1))
    fc = np.asarray(f, dtype=np.complex128)
    f2 = np.ascontiguousarray(np.stack([fc.real, fc.imag], -1).reshape(-1))
    out = np.zeros_like(f2)
    _check(lib.orc_collide_node_cs(lattice, _d(tau), _d(F2), _d(f2), _d(out)), "collide_cs")
    return out[0::2] + 1j * out[1::2]


class Sim:
    """The oracle's simulation state: paper-order FP64 time stepping."""

    def __init__(self, lattice, nx, ny, nz, tau, force=(0.0, 0.0, 0.0), bc=(0, 0, 0),
                 compressible=False):
        self._lib = _load()
        self.lattice = lattice
        self.Q = _QOF[lattice]
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.tau = float(tau)
        self.force = _vec3(force)
        self.bc = tuple(int(b) for b in bc)
        h = ctypes.c_void_p()
        _check(self._lib.orc_create(lattice, nx, ny, nz, float(tau), _d(self.force),
                                    _bc3(self.bc), ctypes.byref(h)), "create")
        self._h = h
        if compressible:
            _check(self._lib.orc_set_compressible(self._h, 1), "set_compressible")

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_equilibrium(self, rho, u, noise=None):
        rho = _f64(rho, self.shape)
        u = _f64(u, (3,) + self.shape)
        noise = _f64(noise, (self.Q,) + self.shape)
        _check(self._lib.orc_init_equilibrium(self._h, _d(rho), _d(u), _d(noise)), "init")

    def set_populations(self, f):
        f = _f64(f, (self.Q,) + self.shape)
        _check(self._lib.orc_set_populations(self._h, _d(f)), "set_populations")

    def get_populations(self):
        f = np.zeros((self.Q,) + self.shape)
        _check(self._lib.orc_get_populations(self._h, _d(f)), "get_populations")
        return f

    def step(self, n=1):
        _check(self._lib.orc_step(self._h, int(n)), "step")

    def moments(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        _check(self._lib.orc_moments(self._h, _d(rho), _d(u)), "moments")
        return rho, u

    def geometry(self):
        g = np.zeros(self.shape, dtype=np.uint8)
        _check(self._lib.orc_geometry(self._h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))),
               "geometry")
        return g.astype(bool)

    def set_solid(self, solid):
        """Solid mask [z][y][x] (nonzero = solid), before initialisation."""
        m = np.ascontiguousarray(np.asarray(solid).reshape(self.shape), dtype=np.uint8)
        _check(self._lib.orc_set_solid(self._h, m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))),
               "set_solid")

    def wall_force(self):
        """Momentum-exchange force on all walls during the last propagation."""
        F = np.zeros(3)
        _check(self._lib.orc_wall_force(self._h, _d(F)), "wall_force")
        return F

    def reduce(self):
        m, k, um = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        bad = ctypes.c_long()
        _check(self._lib.orc_reduce(self._h, ctypes.byref(m), ctypes.byref(k), ctypes.byref(um),
                                    ctypes.byref(bad)), "reduce")
        return {"mass": m.value, "ke": k.value, "umax": um.value, "nonfinite": bad.value}


def _mask(solid, shape):
    if solid is None:
        return None, None
    m = np.ascontiguousarray(np.asarray(solid).reshape(shape), dtype=np.uint8)
    return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))


def cs_objective(lattice, dims, tau, force, bc, rho0, u0, u_tgt, nsteps, *, dtau=0.0,
                 dforce=(0.0, 0.0, 0.0), du0=None, noise=None, h=1e-30, solid=None,
                 compressible=False):
    """(J, dJ) with J = 1/2 sum |u^N - u_tgt|^2 and dJ its complex-step
    derivative along (du0, dtau, dforce)."""
    lib = _load()
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    Q = _QOF[lattice]
    rho0 = _f64(rho0, shape)
    u0 = _f64(u0, (3,) + shape)
    u_tgt = _f64(u_tgt, (3,) + shape)
    du0 = np.zeros_like(u0) if du0 is None else _f64(du0, (3,) + shape)
    noise = _f64(noise, (Q,) + shape)
    J, dJ = ctypes.c_double(), ctypes.c_double()
    keep, mp = _mask(solid, shape)
    _check(lib.orc_cs_objective(lattice, nx, ny, nz, float(tau), float(dtau), _d(_vec3(force)),
                                _d(_vec3(dforce)), _bc3(bc), mp, int(compressible), _d(rho0),
                                _d(u0), _d(du0), _d(noise),
                                int(nsteps), float(h), _d(u_tgt), ctypes.byref(J),
                                ctypes.byref(dJ)), "cs_objective")
    return J.value, dJ.value


def adjoint(lattice, dims, tau, force, bc, rho0, u0, ubar, nsteps, noise=None, *, solid=None,
            compressible=False):
    """Gradients (u0bar [3,nz,ny,nx], taubar, Fbar [3]) of a functional whose
    derivative with respect to the final velocity u^N is ``ubar``."""
    lib = _load()
    nx, ny, nz = dims
    shape = (nz, ny, nx)
    Q = _QOF[lattice]
    rho0 = _f64(rho0, shape)
    u0 = _f64(u0, (3,) + shape)
    ubar = _f64(ubar, (3,) + shape)
    noise = _f64(noise, (Q,) + shape)
    u0bar = np.zeros((3,) + shape)
    taubar = ctypes.c_double()
    Fbar = np.zeros(3)
    keep, mp = _mask(solid, shape)
    _check(lib.orc_adjoint(lattice, nx, ny, nz, float(tau), _d(_vec3(force)), _bc3(bc), mp,
                           int(compressible), _d(rho0), _d(u0), _d(noise), int(nsteps), _d(ubar),
                           _d(u0bar),
                           ctypes.byref(taubar), _d(Fbar)), "adjoint")
    return u0bar, taubar.value, Fbar
