"""Thin ctypes binding of libyy.so (C-ABI in include/yy.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libyy.so.  PyTorch provides device memory (the workspace and the
I/O buffers) and streams.  Importing works without a GPU; creating a shell
needs the built library and a HIP device and raises otherwise.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libyy.so")

YY_OK, YY_ERR_ARG, YY_ERR_GEOMETRY, YY_ERR_WORKSPACE, YY_ERR_HIP, YY_ERR_NONFINITE, YY_ERR_STATE = (
    0, -1, -2, -3, -4, -5, -6)
YY_FP64, YY_FP32_MIXED = 0, 1
YY_MAC, YY_PADDED = 0, 1
YY_LEVEL_N, YY_LEVEL_NM1, YY_LEVEL_K = 0, 1, 2
T, U1R, U1T, U1P, P1, U2R, U2T, U2P, P2 = range(9)
NNORMS = 10
EXPORTS = ["yy_workspace_bytes", "yy_create", "yy_set_params", "yy_set_field", "yy_get_field",
           "yy_set_forcing", "yy_step", "yy_get_norms", "yy_destroy", "yy_strerror",
           "yy_internal_dims", "yy_fill", "yy_extrapolate", "yy_sweep", "yy_sweep_diffusion",
           "yy_residual", "yy_profile", "yy_profile_read", "yy_profile_name",
           "yy_ensemble_workspace_bytes", "yy_ensemble_create", "yy_ensemble_shell",
           "yy_ensemble_step", "yy_ensemble_destroy", "yy_autotune", "yy_set_tuning", "yy_step_tol",
           "yy_set_wall", "yy_set_mass_fix", "yy_set_t_bc",
           "yy_set_pressure_exchange", "yy_step_static", "yy_set_u_bc", "yy_ensemble_autotune",
           "yy_ensemble_info", "yy_get_tuning", "yy_stream_copy", "yy_set_mass_fix_params"]
NPROF = 17


class YYError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {strerror(status)} ({status})")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nt", ctypes.c_int32), ("np", ctypes.c_int32),
                ("r1", ctypes.c_double), ("r2", ctypes.c_double), ("delta", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("pr", ctypes.c_double), ("ra", ctypes.c_double), ("dt", ctypes.c_double),
                ("chi", ctypes.c_double), ("t_inner", ctypes.c_double), ("t_outer", ctypes.c_double),
                ("mode", ctypes.c_int32)]


_lib = None


def load():
    """Load libyy.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libyy.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER
    L.yy_workspace_bytes.argtypes = [P(Grid), i32, P(u64)]
    L.yy_create.argtypes = [P(Grid), i32, vp, u64, P(vp)]
    L.yy_set_params.argtypes = [vp, P(Params)]
    L.yy_set_field.argtypes = [vp, i32, i32, i32, vp, vp]
    L.yy_get_field.argtypes = [vp, i32, i32, i32, vp, vp]
    L.yy_set_forcing.argtypes = [vp, i32, vp, vp]
    L.yy_set_wall.argtypes = [vp, i32, i32, i32, vp, vp]
    L.yy_set_mass_fix.argtypes = [vp, i32]
    L.yy_set_mass_fix_params.argtypes = [vp, ctypes.c_double, ctypes.c_double]
    L.yy_set_pressure_exchange.argtypes = [vp, i32]
    L.yy_set_t_bc.argtypes = [vp, i32, ctypes.c_double, ctypes.c_double]
    L.yy_set_u_bc.argtypes = [vp, i32, ctypes.c_double, ctypes.c_double]
    L.yy_step.argtypes = [vp, i32, vp]
    L.yy_step_static.argtypes = [vp, i32, vp]
    L.yy_step_tol.argtypes = [vp, i32, ctypes.c_double, P(i32), vp]
    L.yy_get_norms.argtypes = [vp, P(ctypes.c_double), i32, vp]
    L.yy_destroy.argtypes = [vp]
    L.yy_strerror.argtypes = [ctypes.c_int]
    L.yy_strerror.restype = ctypes.c_char_p
    L.yy_internal_dims.argtypes = [vp, P(i64), P(i32), P(i32)]
    L.yy_fill.argtypes = [vp, i32, vp]
    L.yy_extrapolate.argtypes = [vp, vp]
    L.yy_sweep.argtypes = [vp, i32, i32, vp, vp, vp]
    L.yy_sweep_diffusion.argtypes = [vp, i32, i32, vp, vp, vp]
    L.yy_residual.argtypes = [vp, i32, vp, vp]
    L.yy_profile.argtypes = [vp, i32]
    L.yy_profile_read.argtypes = [vp, P(ctypes.c_double), P(i64), vp]
    L.yy_profile_name.argtypes = [i32]
    L.yy_profile_name.restype = ctypes.c_char_p
    L.yy_ensemble_workspace_bytes.argtypes = [i32, P(Grid), i32, P(u64)]
    L.yy_ensemble_create.argtypes = [i32, P(Grid), i32, vp, u64, P(vp)]
    L.yy_ensemble_shell.argtypes = [vp, i32]
    L.yy_ensemble_shell.restype = vp
    L.yy_ensemble_step.argtypes = [vp, i32, i32, vp]
    L.yy_ensemble_destroy.argtypes = [vp]
    L.yy_ensemble_autotune.argtypes = [vp, ctypes.c_char_p, i32, vp]
    L.yy_ensemble_info.argtypes = [vp, P(i32), P(i64), P(i64)]
    L.yy_autotune.argtypes = [vp, ctypes.c_char_p, i32, vp]
    L.yy_set_tuning.argtypes = [vp, ctypes.c_char_p]
    L.yy_get_tuning.argtypes = [vp, ctypes.c_char_p, i32]
    L.yy_stream_copy.argtypes = [vp, vp, u64, vp]
    _lib = L
    return L


def strerror(status):
    try:
        return load().yy_strerror(status).decode()
    except Exception:
        return "status %d" % status


def _check(st, what):
    if st < 0:
        raise YYError(st, what)
    return st


def workspace_bytes(nr, nt, np_, r1=0.5, r2=1.0, delta=0.0, prec=YY_FP64):
    g = Grid(nr, nt, np_, r1, r2, delta)
    out = ctypes.c_uint64()
    _check(load().yy_workspace_bytes(ctypes.byref(g), prec, ctypes.byref(out)), "yy_workspace_bytes")
    return out.value


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def stream_copy(dst, src, stream=None):
    """plain streaming copy of device tensor src into dst (same byte size)"""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("dst and src differ in size")
    _check(load().yy_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nb,
                                 _stream_ptr(stream)), "yy_stream_copy")


class Shell:
    """One Yin-Yang shell on the current HIP device."""

    def __init__(self, nr, nt, np_, r1=0.5, r2=1.0, delta=0.0, prec=YY_FP64, device="cuda",
                 _handle=None, _ws=None):
        import torch
        L = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: libyy.so runs on MI355X only")
        self.nr, self.nt, self.np, self.prec = nr, nt, np_, prec
        self._keep_w = {}
        self.grid = Grid(nr, nt, np_, r1, r2, delta)
        self._owned = _handle is None
        if _handle is None:
            nbytes = workspace_bytes(nr, nt, np_, r1, r2, delta, prec)
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.ws.data_ptr()
            self._off = (-base) % 256
            h = ctypes.c_void_p()
            _check(L.yy_create(ctypes.byref(self.grid), prec, ctypes.c_void_p(base + self._off),
                               nbytes, ctypes.byref(h)), "yy_create")
            self.h = h
        else:
            self.ws = _ws
            self.h = ctypes.c_void_p(_handle)
        dims = (ctypes.c_int64 * 4)()
        eb, kf = ctypes.c_int32(), ctypes.c_int32()
        _check(L.yy_internal_dims(self.h, dims, ctypes.byref(eb), ctypes.byref(kf)), "yy_internal_dims")
        self.internal_dims = tuple(dims)
        self.elem_bytes = eb.value
        self.k_first = kf.value       # row element of the ghost k = -1
        self.K = 0

    def close(self):
        if getattr(self, "h", None) and self._owned:
            load().yy_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- shapes ----
    def mac_shape(self, field):
        n = [self.nr, self.nt, self.np]
        loc = {U1R: 0, U2R: 0, U1T: 1, U2T: 1, U1P: 2, U2P: 2}.get(field)
        if loc is not None:
            n[loc] += 1
        return (2, *n)

    def padded_shape(self):
        return (2, self.nr + 2, self.nt + 2, self.np + 2)

    def internal_tensor(self):
        """zero array in the internal layout and compute precision"""
        import torch
        dt = torch.float64 if self.elem_bytes == 8 else torch.float32
        return torch.zeros(self.internal_dims, dtype=dt, device=self.ws.device)

    # ---- calls ----
    def set_params(self, pr=1.0, ra=0.0, dt=1e-3, chi=1.0, t_inner=0.0, t_outer=0.0, mode=0):
        self.params = Params(pr, ra, dt, chi, t_inner, t_outer, mode)
        _check(load().yy_set_params(self.h, ctypes.byref(self.params)), "yy_set_params")

    def set_field(self, field, level, a, layout=YY_MAC, stream=None):
        import torch
        t = torch.as_tensor(a, dtype=torch.float64).to(self.ws.device).contiguous()
        want = self.padded_shape() if layout == YY_PADDED else self.mac_shape(field)
        if tuple(t.shape) != want:
            raise ValueError(f"shape {tuple(t.shape)} != {want}")
        _check(load().yy_set_field(self.h, field, level, layout, ctypes.c_void_p(t.data_ptr()),
                                   _stream_ptr(stream)), "yy_set_field")
        self._keep = t

    def get_field(self, field, level=YY_LEVEL_N, layout=YY_MAC, stream=None):
        import torch
        shape = self.padded_shape() if layout == YY_PADDED else self.mac_shape(field)
        t = torch.empty(shape, dtype=torch.float64, device=self.ws.device)
        _check(load().yy_get_field(self.h, field, level, layout, ctypes.c_void_p(t.data_ptr()),
                                   _stream_ptr(stream)), "yy_get_field")
        return t

    def set_forcing(self, field, a, stream=None):
        import torch
        if a is None:
            _check(load().yy_set_forcing(self.h, field, None, _stream_ptr(stream)), "yy_set_forcing")
            return
        t = torch.as_tensor(a, dtype=torch.float64).to(self.ws.device).contiguous()
        if tuple(t.shape) != self.mac_shape(field):
            raise ValueError("forcing shape")
        _check(load().yy_set_forcing(self.h, field, ctypes.c_void_p(t.data_ptr()),
                                     _stream_ptr(stream)), "yy_set_forcing")
        self._keep_f = t

    def set_t_bc(self, wall, a, b):
        """Robin wall condition a T + b dT/dn = g of T (wall 0: R1, 1: R2)"""
        _check(load().yy_set_t_bc(self.h, wall, ctypes.c_double(a), ctypes.c_double(b)), "yy_set_t_bc")

    def set_u_bc(self, wall, a, b):
        """Robin wall condition a u + b R dn(u/r) = g of the tangential
        velocity (wall 0: R1, 1: R2); (0, 1) is stress-free"""
        _check(load().yy_set_u_bc(self.h, wall, ctypes.c_double(a), ctypes.c_double(b)), "yy_set_u_bc")

    def set_mass_fix(self, on):
        """Algorithm step 4 (boundary mass-flux correction) on every velocity fill"""
        _check(load().yy_set_mass_fix(self.h, 1 if on else 0), "yy_set_mass_fix")

    def set_mass_fix_params(self, eps, tol):
        """epsilon of step 4's functional (0: the limit) and its flux trigger"""
        _check(load().yy_set_mass_fix_params(self.h, float(eps), float(tol)), "yy_set_mass_fix_params")

    def set_pressure_exchange(self, nring):
        """Algorithm step 7: the outermost nring cells take the other
        patch's pressure after every pressure update (0: off)"""
        _check(load().yy_set_pressure_exchange(self.h, int(nring)), "yy_set_pressure_exchange")

    def set_wall(self, field, level, wall, a, stream=None):
        """Dirichlet wall data (2, nt+2, np+2) of T, u_r, u_theta or u_phi
        (field T, U1R, U1T, U1P) for a level (0: n, 1: n-1, 2: the step's
        target) and wall (0: R1, 1: R2); None clears the slot"""
        import torch
        if a is None:
            _check(load().yy_set_wall(self.h, field, level, wall, None, _stream_ptr(stream)), "yy_set_wall")
            return
        t = torch.as_tensor(a, dtype=torch.float64).to(self.ws.device).contiguous()
        if tuple(t.shape) != (2, self.nt + 2, self.np + 2):
            raise ValueError("wall data shape")
        _check(load().yy_set_wall(self.h, field, level, wall, ctypes.c_void_p(t.data_ptr()),
                                  _stream_ptr(stream)), "yy_set_wall")
        self._keep_w[(field, level, wall)] = t    # alive until the stream has copied it

    def step(self, K, stream=None):
        _check(load().yy_step(self.h, K, _stream_ptr(stream)), "yy_step")
        self.K = K

    def step_static(self, K, stream=None):
        """yy_step with its scratch in the library's static device array"""
        _check(load().yy_step_static(self.h, K, _stream_ptr(stream)), "yy_step_static")
        self.K = K

    def step_tol(self, kmax, tol, stream=None):
        """one step, Schwarz iterations until every increment norm < tol
        (at most kmax); returns the iteration count"""
        k = ctypes.c_int32(0)
        _check(load().yy_step_tol(self.h, kmax, ctypes.c_double(tol), ctypes.byref(k),
                                  _stream_ptr(stream)), "yy_step_tol")
        self.K = k.value
        return k.value

    def norms(self, stream=None):
        n = max(self.K, 1) * 2 * NNORMS
        out = (ctypes.c_double * n)()
        _check(load().yy_get_norms(self.h, out, n, _stream_ptr(stream)), "yy_get_norms")
        return np.array(out[:self.K * 2 * NNORMS]).reshape(self.K, 2, NNORMS)

    def fill(self, level, stream=None):
        _check(load().yy_fill(self.h, level, _stream_ptr(stream)), "yy_fill")

    def extrapolate(self, stream=None):
        _check(load().yy_extrapolate(self.h, _stream_ptr(stream)), "yy_extrapolate")

    def sweep(self, field, d, x, y, stream=None):
        _check(load().yy_sweep(self.h, field, d, ctypes.c_void_p(x.data_ptr()),
                               ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)), "yy_sweep")

    def sweep_diffusion(self, d, x, y, stream=None, metric=0):
        """(I - tau/2 Pr D) y = x along d; metric 0: D_rr, Dhat_thth,
        Dhat_phph (the split operators), 1: the true D_thth, D_phph"""
        _check(load().yy_sweep_diffusion(self.h, d, metric, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)),
               "yy_sweep_diffusion")

    def residual(self, field, out, stream=None):
        _check(load().yy_residual(self.h, field, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
               "yy_residual")

    def autotune(self, stream=None):
        """time the line-solver tile variants; returns the choices (JSON)"""
        buf = ctypes.create_string_buffer(4096)
        _check(load().yy_autotune(self.h, buf, 4096, _stream_ptr(stream)), "yy_autotune")
        return buf.value.decode()

    def tuning_json(self):
        """the current tile choices (JSON)"""
        buf = ctypes.create_string_buffer(4096)
        _check(load().yy_get_tuning(self.h, buf, len(buf)), "yy_get_tuning")
        return buf.value.decode()

    def set_tuning(self, js):
        _check(load().yy_set_tuning(self.h, js.encode()), "yy_set_tuning")

    def profile(self, enable=True):
        _check(load().yy_profile(self.h, 1 if enable else 0), "yy_profile")

    def profile_read(self, stream=None):
        """{kernel class: (total ms, timed launch groups)} since profile(True)"""
        L = load()
        ms = (ctypes.c_double * NPROF)()
        cnt = (ctypes.c_int64 * NPROF)()
        _check(L.yy_profile_read(self.h, ms, cnt, _stream_ptr(stream)), "yy_profile_read")
        return {L.yy_profile_name(c).decode(): (ms[c], cnt[c]) for c in range(NPROF)}

    # ---- layout helpers (host side) ----
    def to_internal(self, padded):
        """(2, nr+2, nt+2, np+2) array -> internal-layout tensor"""
        import torch
        t = self.internal_tensor()
        o = self.k_first
        t[..., o:o + self.np + 2] = torch.as_tensor(padded, dtype=t.dtype, device=t.device)
        return t

    def from_internal(self, t):
        o = self.k_first
        return t[..., o:o + self.np + 2]


class Ensemble:
    """Independent shells in one workspace, stepped by one captured graph."""

    def __init__(self, grids, prec=YY_FP32_MIXED, device="cuda"):
        """grids: list of (nr, nt, np) or (nr, nt, np, r1, r2, delta)"""
        import torch
        L = load()
        n = len(grids)
        arr = (Grid * n)()
        for q, g in enumerate(grids):
            g = tuple(g) + (0.5, 1.0, 0.0)[len(g) - 3:] if len(g) < 6 else tuple(g)
            arr[q] = Grid(*g)
        nbytes = ctypes.c_uint64()
        _check(L.yy_ensemble_workspace_bytes(n, arr, prec, ctypes.byref(nbytes)),
               "yy_ensemble_workspace_bytes")
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _check(L.yy_ensemble_create(n, arr, prec, ctypes.c_void_p(base + off), nbytes.value,
                                    ctypes.byref(h)), "yy_ensemble_create")
        self.h = h
        self.shells = []
        for q in range(n):
            sh = L.yy_ensemble_shell(self.h, q)
            self.shells.append(Shell(arr[q].nr, arr[q].nt, arr[q].np, arr[q].r1, arr[q].r2,
                                     arr[q].delta, prec, device, _handle=sh, _ws=self.ws))

    def step(self, K, graph=True, stream=None):
        """graph: True / 1 batched launches in a graph, 2 one stream per
        shell in a graph, False / 0 the shells one after another"""
        g = 1 if graph is True else (0 if graph is False else int(graph))
        _check(load().yy_ensemble_step(self.h, K, g, _stream_ptr(stream)), "yy_ensemble_step")
        for sh in self.shells:
            sh.K = K

    def autotune(self, stream=None):
        """per-bucket tiles (unknown, direction, line-length bucket); returns the JSON"""
        buf = ctypes.create_string_buffer(65536)
        _check(load().yy_ensemble_autotune(self.h, buf, len(buf), _stream_ptr(stream)), "yy_ensemble_autotune")
        return buf.value.decode()

    def info(self):
        """(batched, batched launches per step, the shells' own launches per
        step they replace) of the captured graphs"""
        b, n, m = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().yy_ensemble_info(self.h, ctypes.byref(b), ctypes.byref(n), ctypes.byref(m)),
               "yy_ensemble_info")
        return bool(b.value), n.value, m.value

    def close(self):
        if getattr(self, "h", None):
            for sh in self.shells:
                sh.h = None
            load().yy_ensemble_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
