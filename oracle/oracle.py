"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Array conventions (all float64, C order):
  chart        [3, nz, ny, nx]   node positions, wall layers included
  populations  [19, nz, H, nx]   H = ny - 2 fluid layers
  history      [10, nz, H, nx]   A, B^x, B^y, B^z, C^xx, C^xy, C^xz, C^yy, C^yz, C^zz
  displacement [nz, nx]          y-displacement of a wall
  wall vel.    [nz, nx, 3]       Cartesian
  plate disp.  [nz, nx]          y-displacement of the plate's cross-section row
  plate vel.   [nz, nx, 3]       Cartesian, per column (columns off the plate
                                 take the nearest plate column's)
  geometry     [28, nz, H, nx]   sqrt g, g^ij (6), Gamma^i_jk (18), F^i (3)
  jacobian     [9, nz, H, nx]    J[a][i] = d h^a / d xi^i, row major
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_D = ctypes.POINTER(ctypes.c_double)


def lib_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def _lib():
    global _LIB
    if _LIB is None:
        p = lib_path()
        if not os.path.exists(p):
            from . import build as _b

            _b.build()
        L = ctypes.CDLL(p)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_threads.restype = ctypes.c_int
        L.orc_threads.argtypes = []
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_fluid_nodes.restype = ctypes.c_long
        L.orc_fluid_nodes.argtypes = [ctypes.c_void_p]
        for name, extra in [
            ("orc_set_body_force", [_D]),
            ("orc_set_metric", [_D, ctypes.c_int]),
            ("orc_set_wall_displacement", [ctypes.c_int, _D, ctypes.c_int]),
            ("orc_set_wall_velocity", [ctypes.c_int, _D]),
            ("orc_init_equilibrium", [_D, _D]),
            ("orc_set_populations", [_D]),
            ("orc_get_populations", [_D]),
            ("orc_get_history", [_D]),
            ("orc_step", [ctypes.c_int]),
            ("orc_moments", [_D, _D, ctypes.c_int]),
            ("orc_wall_force", [ctypes.c_int, _D, _D]),
            ("orc_set_plate_displacement", [_D, ctypes.c_int]),
            ("orc_set_plate_velocity", [_D]),
            ("orc_plate_force", [_D, _D]),
            ("orc_geometry", [_D]),
            ("orc_chart", [_D]),
            ("orc_jacobian", [_D]),
        ]:
            fn = getattr(L, name)
            fn.argtypes = [ctypes.c_void_p] + extra
            fn.restype = None
        L.orc_set_plate.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_set_plate.restype = ctypes.c_int
        L.orc_wall_force_mem.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D]
        L.orc_wall_force_mem.restype = ctypes.c_int
        L.orc_set_ablation.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_set_ablation.restype = None
        L.orc_set_open_x.argtypes = [ctypes.c_void_p, _D]
        L.orc_set_open_x.restype = ctypes.c_int
        L.orc_run_forces.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, _D, _D, _D, ctypes.c_int, ctypes.c_int, _D, _D]
        L.orc_run_forces.restype = None
        L.orc_dual_forces.argtypes = (
            [ctypes.c_int] * 3 + [ctypes.c_double, _D, _D, _D, _D, _D, ctypes.c_int, ctypes.c_int, _D, _D, _D]
        )
        L.orc_dual_forces.restype = None
        _LIB = L
    return _LIB


def threads() -> int:
    """OpenMP threads the oracle's node loops use."""
    return int(_lib().orc_threads())


def set_threads(n: int) -> int:
    """Set the OpenMP threads of the oracle's node loops; returns the count."""
    return int(_lib().orc_set_threads(int(n)))


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_D)


def _c(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """One FP64 oracle simulation (owns its CPU state)."""

    def __init__(self, nx: int, ny: int, nz: int, tau: float):
        self.nx, self.ny, self.nz, self.tau = nx, ny, nz, tau
        self.H = ny - 2
        self._h = _lib().orc_create(nx, ny, nz, float(tau))
        if not self._h:
            raise ValueError("invalid oracle grid or tau")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib().orc_destroy(h)
            self._h = None

    @property
    def fluid_shape(self):
        return (self.nz, self.H, self.nx)

    def set_body_force(self, F):
        F = _c(F, (3,))
        _lib().orc_set_body_force(self._h, _p(F))

    def set_metric(self, chart, reproject=False):
        chart = _c(chart, (3, self.nz, self.ny, self.nx))
        _lib().orc_set_metric(self._h, _p(chart), int(bool(reproject)))

    def set_wall_displacement(self, wall, d, reproject=False):
        d = _c(d, (self.nz, self.nx))
        _lib().orc_set_wall_displacement(self._h, int(wall), _p(d), int(bool(reproject)))

    def set_wall_velocity(self, wall, v):
        v = _c(v, (self.nz, self.nx, 3))
        _lib().orc_set_wall_velocity(self._h, int(wall), _p(v))

    def set_plate(self, jp, i0, i1):
        """Interior plate between fluid rows jp-1 and jp over columns i0..i1
        (jp = 0 removes it)."""
        if _lib().orc_set_plate(self._h, int(jp), int(i0), int(i1)) != 0:
            raise ValueError("invalid plate")

    def set_open_x(self, uin):
        """Open ends in x with the Cartesian inlet velocity [nz, H, 3] at
        column 0 (None: periodic x again)."""
        uin = _c(uin, (self.nz, self.H, 3))
        if _lib().orc_set_open_x(self._h, _p(uin)) != 0:
            raise ValueError("open ends need nx >= 3 and a plate at least 2 columns from each end")

    def set_ablation(self, drop_C=False):
        """Diagnostic only (not the method): drop the velocity-gradient
        coefficient C^ij of Eq. (forcing-C) from every forcing term."""
        _lib().orc_set_ablation(self._h, 1 if drop_C else 0)

    def set_plate_displacement(self, d, reproject=False):
        d = _c(d, (self.nz, self.nx))
        _lib().orc_set_plate_displacement(self._h, _p(d), int(bool(reproject)))

    def set_plate_velocity(self, v):
        v = _c(v, (self.nz, self.nx, 3))
        _lib().orc_set_plate_velocity(self._h, _p(v))

    def plate_force(self, per_column=False):
        tot = np.empty(3)
        pc = np.empty((self.nz, self.nx, 3)) if per_column else None
        _lib().orc_plate_force(self._h, _p(tot), _p(pc))
        return (tot, pc) if per_column else tot

    def init_equilibrium(self, rho=None, ucart=None):
        rho = _c(rho, self.fluid_shape)
        ucart = _c(ucart, (3,) + self.fluid_shape)
        _lib().orc_init_equilibrium(self._h, _p(rho), _p(ucart))

    def set_populations(self, f):
        f = _c(f, (19,) + self.fluid_shape)
        _lib().orc_set_populations(self._h, _p(f))

    def populations(self):
        out = np.empty((19,) + self.fluid_shape)
        _lib().orc_get_populations(self._h, _p(out))
        return out

    def history(self):
        out = np.empty((10,) + self.fluid_shape)
        _lib().orc_get_history(self._h, _p(out))
        return out

    def step(self, n=1):
        _lib().orc_step(self._h, int(n))

    def moments(self, cartesian=False):
        rho = np.empty(self.fluid_shape)
        u = np.empty((3,) + self.fluid_shape)
        _lib().orc_moments(self._h, _p(rho), _p(u), int(bool(cartesian)))
        return rho, u

    def wall_force(self, wall, per_node=False):
        tot = np.empty(3)
        pn = np.empty((self.nz, self.nx, 3)) if per_node else None
        _lib().orc_wall_force(self._h, int(wall), _p(tot), _p(pn))
        return (tot, pn) if per_node else tot

    def wall_force_mem(self, wall, per_node=False):
        """Momentum-exchange force on a wall at rest (diagnostic)."""
        tot = np.empty(3)
        pn = np.empty((self.nz, self.nx, 3)) if per_node else None
        if _lib().orc_wall_force_mem(self._h, int(wall), _p(tot), _p(pn)) != 0:
            raise ValueError("the momentum-exchange force needs the wall at rest")
        return (tot, pn) if per_node else tot

    def geometry(self):
        out = np.empty((28,) + self.fluid_shape)
        _lib().orc_geometry(self._h, _p(out))
        return out

    def chart(self):
        """The chart in use, [3, nz, ny, nx]."""
        out = np.empty((3, self.nz, self.ny, self.nx))
        _lib().orc_chart(self._h, _p(out))
        return out

    def jacobian(self):
        out = np.empty((9,) + self.fluid_shape)
        _lib().orc_jacobian(self._h, _p(out))
        return out


def run_forces(nx, ny, nz, tau, F, d_top, f0, K, wall=1, vwall=None):
    """Wall forces [K, 3] at states 1..K from f0 under top displacement d_top;
    vwall [2, nz, nx, 3]: Cartesian wall velocities (None: at rest)."""
    F = _c(F, (3,))
    d_top = _c(d_top, (nz, nx))
    f0 = _c(f0, (19, nz, ny - 2, nx))
    vw = None if vwall is None else _c(vwall, (2, nz, nx, 3))
    out = np.empty((K, 3))
    _lib().orc_run_forces(nx, ny, nz, float(tau), _p(F), _p(d_top), _p(f0), int(K), int(wall), _p(out),
                          None if vw is None else _p(vw))
    return out


def dual_forces(nx, ny, nz, tau, F, d_top, dd_top, f0, df0, K, wall=1, vwall=None):
    """Forces [K,3] and their exact derivative along (dd_top, df0) (forward
    mode); vwall [2, nz, nx, 3]: Cartesian wall velocities (None: at rest)."""
    F = _c(F, (3,))
    d_top = _c(d_top, (nz, nx))
    dd_top = _c(dd_top, (nz, nx))
    f0 = _c(f0, (19, nz, ny - 2, nx))
    df0 = _c(df0, (19, nz, ny - 2, nx))
    out = np.empty((K, 3))
    dout = np.empty((K, 3))
    vw = None if vwall is None else _c(vwall, (2, nz, nx, 3))
    _lib().orc_dual_forces(
        nx, ny, nz, float(tau), _p(F), _p(d_top), _p(dd_top), _p(f0), _p(df0), int(K), int(wall), _p(out), _p(dout),
        None if vw is None else _p(vw)
    )
    return out, dout
