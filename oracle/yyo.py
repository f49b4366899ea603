"""ctypes wrapper of the C oracle (oracle/yyo.c).

TEST INFRASTRUCTURE ONLY: the product package never imports this module.
Arrays cross the boundary as contiguous float64 numpy arrays.
"""
import ctypes
import os

import numpy as np

from . import build as _build

T, U1R, U1T, U1P, P1, U2R, U2T, U2P, P2 = range(9)
NF = 9
LEV_N, LEV_NM1, LEV_K = 0, 1, 2
MAC, PADDED = 0, 1
OP_DRR, OP_DTT, OP_DTT_HAT, OP_DPP, OP_DPP_HAT, OP_LR, OP_LT, OP_LP = range(8)
FIELD_NAMES = ["T", "u1r", "u1t", "u1p", "p1", "u2r", "u2t", "u2p", "p2"]
NORM_NAMES = FIELD_NAMES + ["div_u2"]

_lib = None


def load_library(path):
    """A configured ctypes handle of an oracle library at `path` (the tests
    also load deliberately altered builds this way)."""
    L = ctypes.CDLL(path)
    vp, d, i, dp = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    L.yyo_create.restype = vp
    L.yyo_create.argtypes = [i, i, i, d, d, d]
    L.yyo_destroy.argtypes = [vp]
    L.yyo_set_params.argtypes = [vp, d, d, d, d, d, d]
    L.yyo_set_mode.argtypes = [vp, i]
    L.yyo_set_verbose.argtypes = [vp, i]
    L.yyo_set_mass_fix.argtypes = [vp, i]
    L.yyo_set_mass_fix_params.argtypes = [vp, d, d]
    L.yyo_set_pressure_exchange.argtypes = [vp, i]
    L.yyo_set_t_bc.argtypes = [vp, i, d, d]
    L.yyo_set_u_bc.argtypes = [vp, i, d, d]
    L.yyo_field_count.restype = ctypes.c_int64
    L.yyo_field_count.argtypes = [vp, i, i]
    L.yyo_set_field.argtypes = [vp, i, i, i, dp]
    L.yyo_get_field.argtypes = [vp, i, i, i, dp]
    L.yyo_set_forcing.argtypes = [vp, i, dp]
    L.yyo_set_wall.argtypes = [vp, i, i, i, dp]
    L.yyo_step.argtypes = [vp, i]
    L.yyo_step_tol.argtypes = [vp, i, d]
    L.yyo_get_norms.argtypes = [vp, dp, i]
    L.yyo_fill.argtypes = [vp, i]
    L.yyo_sweep.argtypes = [vp, i, i, dp, dp]
    L.yyo_apply_op.argtypes = [vp, i, i, dp, dp]
    L.yyo_sweep_op.argtypes = [vp, i, dp, dp]
    L.yyo_residual.argtypes = [vp, i, dp]
    L.yyo_extrapolate.argtypes = [vp]
    L.yyo_thomas.argtypes = [i, dp, dp, dp, dp, dp]
    L.yyo_involution.argtypes = [d, d, dp, dp]
    L.yyo_rotation.argtypes = [d, d, dp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = load_library(_build.LIB)
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def thomas(lo, di, up, rhs):
    n = len(di)
    x = np.zeros(n)
    lo, di, up, rhs = map(_f64, (lo, di, up, rhs))
    lib().yyo_thomas(n, _ptr(lo), _ptr(di), _ptr(up), _ptr(rhs), _ptr(x))
    return x


def involution(th, ph):
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().yyo_involution(th, ph, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def rotation(th, ph):
    m = np.zeros(4)
    lib().yyo_rotation(th, ph, _ptr(m))
    return m.reshape(2, 2)


def omp_threads():
    return lib().yyo_omp_threads()


def set_threads(n):
    """threads of the following oracle calls (n <= 0: one per host core)"""
    lib().yyo_set_threads(int(n))


class Shell:
    """One Yin-Yang shell held by the oracle."""

    def __init__(self, nr, nt, np_, r1=0.5, r2=1.0, delta=0.0, _lib=None):
        self.nr, self.nt, self.np = nr, nt, np_
        self._L = _lib if _lib is not None else lib()
        self.h = self._L.yyo_create(nr, nt, np_, r1, r2, delta)
        if not self.h:
            raise ValueError("oracle rejected the grid (arguments or donor-window fit)")

    def close(self):
        if self.h:
            self._L.yyo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, pr=1.0, ra=0.0, tau=1e-3, chi=1.0, t_inner=0.0, t_outer=0.0):
        if self._L.yyo_set_params(self.h, pr, ra, tau, chi, t_inner, t_outer) != 0:
            raise ValueError("bad parameters")

    def set_verbose(self, on):
        self._L.yyo_set_verbose(self.h, 1 if on else 0)

    def set_mode(self, mode):
        if self._L.yyo_set_mode(self.h, mode) != 0:
            raise ValueError("bad mode")

    def padded_shape(self):
        return (2, self.nr + 2, self.nt + 2, self.np + 2)

    def mac_shape(self, field):
        n = [self.nr, self.nt, self.np]
        loc = {U1R: 0, U2R: 0, U1T: 1, U2T: 1, U1P: 2, U2P: 2}.get(field)
        if loc is not None:
            n[loc] += 1
        return (2, *n)

    def set_field(self, field, level, a, layout=MAC):
        a = _f64(a)
        if a.size != self._L.yyo_field_count(self.h, field, layout):
            raise ValueError("size mismatch")
        self._L.yyo_set_field(self.h, field, level, layout, _ptr(a))

    def get_field(self, field, level=LEV_N, layout=MAC):
        shape = self.padded_shape() if layout == PADDED else self.mac_shape(field)
        a = np.zeros(shape)
        self._L.yyo_get_field(self.h, field, level, layout, _ptr(a))
        return a

    def set_forcing(self, field, a):
        if a is None:
            self._L.yyo_set_forcing(self.h, field, None)
            return
        a = _f64(a)
        assert a.shape == self.mac_shape(field)
        self._L.yyo_set_forcing(self.h, field, _ptr(a))

    def set_t_bc(self, wall, a, b):
        """Robin condition a T + b dT/dn = g on a wall (0: R1, 1: R2)"""
        if self._L.yyo_set_t_bc(self.h, wall, a, b) != 0:
            raise RuntimeError("set_t_bc failed")

    def set_u_bc(self, wall, a, b):
        """Robin condition a u + b R dn(u/r) = g of the tangential velocity
        on a wall (0: R1, 1: R2); (0, 1) is stress-free"""
        if self._L.yyo_set_u_bc(self.h, wall, a, b) != 0:
            raise RuntimeError("set_u_bc failed")

    def set_mass_fix(self, on):
        if self._L.yyo_set_mass_fix(self.h, 1 if on else 0) != 0:
            raise RuntimeError("set_mass_fix failed")

    def set_mass_fix_params(self, eps, tol):
        """epsilon of step 4's functional (0: the limit) and its flux trigger"""
        if self._L.yyo_set_mass_fix_params(self.h, float(eps), float(tol)) != 0:
            raise ValueError("yyo_set_mass_fix_params: eps and tol must be >= 0")

    def set_pressure_exchange(self, nring):
        """Algorithm step 7: the outermost nring cells take the other
        patch's pressure (0: off)"""
        if self._L.yyo_set_pressure_exchange(self.h, int(nring)) != 0:
            raise ValueError("set_pressure_exchange failed")

    def set_wall(self, field, level, wall, a):
        """Dirichlet wall data (2, nt+2, np+2) of T, u_r, u_theta or u_phi
        for a level and a wall (0: R1, 1: R2); None clears"""
        if a is None:
            if self._L.yyo_set_wall(self.h, field, level, wall, None) != 0:
                raise RuntimeError("set_wall failed")
            return
        a = _f64(a)
        assert a.shape == (2, self.nt + 2, self.np + 2)
        if self._L.yyo_set_wall(self.h, field, level, wall, _ptr(a)) != 0:
            raise RuntimeError("set_wall failed")

    def step(self, K):
        if self._L.yyo_step(self.h, K) != 0:
            raise RuntimeError("step failed")

    def step_tol(self, kmax, tol):
        """one step, Schwarz iterations until every increment norm < tol
        (at most kmax); returns the iteration count"""
        k = self._L.yyo_step_tol(self.h, kmax, tol)
        if k < 1:
            raise RuntimeError("step_tol failed")
        return k

    def norms(self, K):
        out = np.zeros(K * 2 * 10)
        self._L.yyo_get_norms(self.h, _ptr(out), out.size)
        return out.reshape(K, 2, 10)

    def fill(self, level):
        self._L.yyo_fill(self.h, level)

    def extrapolate(self):
        self._L.yyo_extrapolate(self.h)

    def sweep(self, field, d, x):
        x = _f64(x)
        y = np.zeros(self.padded_shape())
        if self._L.yyo_sweep(self.h, field, d, _ptr(x), _ptr(y)) != 0:
            raise ValueError("bad sweep")
        return y

    def sweep_op(self, op, x):
        """(I - tau/2 Pr D_op) y = x along D_op's direction (centre unknowns)"""
        x = _f64(x)
        y = np.zeros(self.padded_shape())
        if self._L.yyo_sweep_op(self.h, op, _ptr(x), _ptr(y)) != 0:
            raise ValueError("bad sweep_op")
        return y

    def apply_op(self, field, op, x):
        x = _f64(x)
        y = np.zeros(self.padded_shape())
        self._L.yyo_apply_op(self.h, field, op, _ptr(x), _ptr(y))
        return y

    def residual(self, field):
        y = np.zeros(self.padded_shape())
        self._L.yyo_residual(self.h, field, _ptr(y))
        return y
