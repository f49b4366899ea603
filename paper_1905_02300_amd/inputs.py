"""Seeded, synthetic inputs of the Yin-Yang shell workloads.

This module describes problems, not the method: MAC point positions, the
manufactured solution and its forcing, seeded initial states and seeded
right-hand sides.  It holds none of the scheme's arithmetic (no operator,
no interpolation, no solver) and serves both the HIP path's tests and
benchmark and the oracle's.

Layout of every array: (2 patches, n_r, n_theta, n_phi) in the field's MAC
extent -- centres (Nr, Nt, Np); u_r on r-faces (Nr+1, Nt, Np); u_theta on
theta-faces (Nr, Nt+1, Np); u_phi on phi-faces (Nr, Nt, Np+1).  Patch 0 is
Yin, patch 1 is Yang.
"""
import math

import numpy as np

# field ids (same order as the library's)
T, U1R, U1T, U1P, P1, U2R, U2T, U2P, P2 = range(9)
FIELD_NAMES = ["T", "u1r", "u1t", "u1p", "p1", "u2r", "u2t", "u2p", "p2"]
LOC = {T: "c", P1: "c", P2: "c", U1R: "r", U2R: "r", U1T: "t", U2T: "t", U1P: "p", U2P: "p"}


class Grid:
    """Cell sizes and extents of one patch (both patches are identical in
    their own coordinates).  delta <= 0 selects the one-cell overlap
    delta = pi / (2 (Nt - 2))."""

    def __init__(self, nr, nt, np_, r1=0.5, r2=1.0, delta=0.0):
        self.nr, self.nt, self.np = nr, nt, np_
        self.r1, self.r2 = r1, r2
        self.delta = delta if delta > 0 else math.pi / (2.0 * (nt - 2))
        self.dr = (r2 - r1) / nr
        self.th0 = math.pi / 4 - self.delta
        self.ph0 = -3 * math.pi / 4 - self.delta
        self.dth = (math.pi / 2 + 2 * self.delta) / nt
        self.dph = (1.5 * math.pi + 2 * self.delta) / np_

    @property
    def cells(self):
        return 2 * self.nr * self.nt * self.np

    def mac_shape(self, field):
        n = [self.nr, self.nt, self.np]
        loc = LOC[field]
        if loc == "r":
            n[0] += 1
        elif loc == "t":
            n[1] += 1
        elif loc == "p":
            n[2] += 1
        return (2, *n)

    def axes(self, field, padded=False):
        """1-D coordinates (r, theta, phi) of the field's MAC points, or of
        every slot of the padded layout (logical index -1..N per direction,
        face f stored at logical index f)."""
        loc = LOC[field]
        out = []
        for d, (x0, h, n, key) in enumerate([(self.r1, self.dr, self.nr, "r"),
                                             (self.th0, self.dth, self.nt, "t"),
                                             (self.ph0, self.dph, self.np, "p")]):
            face = loc == key
            idx = np.arange(-1, n + 1) if padded else np.arange(n + face)
            out.append(x0 + (idx + (0.0 if face else 0.5)) * h)
        return tuple(out)


def _patch_frame(patch, v):
    """Map a vector (or point) given in a patch's own Cartesian frame to
    the global (Yin) frame.  Yang's frame is (x,y,z) -> (-x, z, y)."""
    if patch == 0:
        return v
    return np.stack([-v[0], v[2], v[1]])


def points(grid, field, patch, padded=False):
    """Global Cartesian coordinates and the local unit vectors (global
    frame) of a field's MAC (or padded-layout) points on one patch."""
    r, t, p = grid.axes(field, padded)
    return _frame_points(r, t, p, patch)


def _frame_points(r, t, p, patch):
    R, TH, PH = np.meshgrid(r, t, p, indexing="ij")
    st, ct, sp, cp = np.sin(TH), np.cos(TH), np.sin(PH), np.cos(PH)
    X = _patch_frame(patch, np.stack([R * st * cp, R * st * sp, R * ct]))
    er = _patch_frame(patch, np.stack([st * cp, st * sp, ct]))
    et = _patch_frame(patch, np.stack([ct * cp, ct * sp, -st]))
    ep = _patch_frame(patch, np.stack([-sp, cp, np.zeros_like(sp)]))
    return X, (er, et, ep)


# ---------------------------------------------------------------------------
# second-order jets in (x, y, z): exact first and second derivatives
# ---------------------------------------------------------------------------
class Jet:
    """value v, gradient g[3], Hessian H[3][3] of a function of (x,y,z)."""

    def __init__(self, v, g, H):
        self.v, self.g, self.H = v, g, H

    @staticmethod
    def var(X, d):
        z = np.zeros_like(X[0])
        o = np.ones_like(X[0])
        g = [o if e == d else z for e in range(3)]
        H = [[z for _ in range(3)] for _ in range(3)]
        return Jet(X[d], g, H)

    @staticmethod
    def const(c, like):
        z = np.zeros_like(like)
        return Jet(np.full_like(like, c), [z, z, z], [[z] * 3 for _ in range(3)])

    def _lift(self, o):
        return o if isinstance(o, Jet) else Jet.const(o, self.v)

    def __add__(self, o):
        o = self._lift(o)
        return Jet(self.v + o.v, [a + b for a, b in zip(self.g, o.g)],
                   [[self.H[i][j] + o.H[i][j] for j in range(3)] for i in range(3)])

    __radd__ = __add__

    def __neg__(self):
        return Jet(-self.v, [-a for a in self.g], [[-self.H[i][j] for j in range(3)] for i in range(3)])

    def __sub__(self, o):
        return self + (-self._lift(o))

    def __rsub__(self, o):
        return self._lift(o) - self

    def __mul__(self, o):
        o = self._lift(o)
        v = self.v * o.v
        g = [self.g[i] * o.v + self.v * o.g[i] for i in range(3)]
        H = [[self.H[i][j] * o.v + self.g[i] * o.g[j] + self.g[j] * o.g[i] + self.v * o.H[i][j]
              for j in range(3)] for i in range(3)]
        return Jet(v, g, H)

    __rmul__ = __mul__

    def compose(self, f0, f1, f2):
        """phi(self) with phi, phi', phi'' given at self.v"""
        g = [f1 * a for a in self.g]
        H = [[f2 * self.g[i] * self.g[j] + f1 * self.H[i][j] for j in range(3)] for i in range(3)]
        return Jet(f0, g, H)

    def __truediv__(self, o):
        o = self._lift(o)
        inv = o.compose(1.0 / o.v, -1.0 / o.v ** 2, 2.0 / o.v ** 3)
        return self * inv

    def sqrt(self):
        s = np.sqrt(self.v)
        return self.compose(s, 0.5 / s, -0.25 / s ** 3)

    def lap(self):
        return self.H[0][0] + self.H[1][1] + self.H[2][2]


def _mms_jets(X, r1, r2):
    """Spatial parts U (3 jets), P, Theta of the manufactured solution
    u = curl(g(r) sin t (xy, yz, zx)), g = (r-R1)^2 (R2-r)^2,
    p = sin t xyz/r, T = sin t (r-R1)(R2-r) z/r."""
    x, y, z = (Jet.var(X, d) for d in range(3))
    r = (x * x + y * y + z * z).sqrt()
    a, b = r - r1, (-r) + r2
    g = a * a * b * b
    gp = 2.0 * a * b * b - 2.0 * a * a * b          # g'(r)
    q = gp / r
    xyz = x * y * z
    U = [q * (xyz - y * z * z) - g * y,
         q * (xyz - x * x * z) - g * z,
         q * (xyz - x * y * y) - g * x]
    P = xyz / r
    TH = a * b * z / r
    return U, P, TH, r


def _mms_values(X, r1, r2):
    """Values only of U, P, Theta (the same formulas as _mms_jets)."""
    x, y, z = X
    r = np.sqrt(x * x + y * y + z * z)
    a, b = r - r1, r2 - r
    g = a * a * b * b
    q = (2.0 * a * b * b - 2.0 * a * a * b) / r
    xyz = x * y * z
    U = [q * (xyz - y * z * z) - g * y, q * (xyz - x * x * z) - g * z, q * (xyz - x * y * y) - g * x]
    return U, xyz / r, a * b * z / r


def _paper_jets(X):
    """Spatial parts of the manufactured solution of the numerical-tests
    section (eq. Exact): u = cos t (2x^2yz, -xy^2z, -xyz^2), p = cos t xyz,
    T = 2 cos t x^2yz.  It is divergence-free and non-zero on the walls."""
    x, y, z = (Jet.var(X, d) for d in range(3))
    r = (x * x + y * y + z * z).sqrt()
    U = [x * x * y * z * 2.0, -(x * y * y * z), -(x * y * z * z)]
    return U, x * y * z, x * x * y * z * 2.0, r


def _paper_values(X):
    x, y, z = X
    return [2.0 * x * x * y * z, -x * y * y * z, -x * y * z * z], x * y * z, 2.0 * x * x * y * z


# time factor a(t) and a'(t) of each manufactured solution: "shell" (ours,
# zero on the walls) and "paper" (eq. Exact)
_TIME = {"shell": (math.sin, math.cos), "paper": (math.cos, lambda t: -math.sin(t))}


def _values(kind, X, r1, r2):
    return _mms_values(X, r1, r2) if kind == "shell" else _paper_values(X)


def _jets(kind, X, r1, r2):
    return _mms_jets(X, r1, r2) if kind == "shell" else _paper_jets(X)


def _field_value(field, U, P, TH, e):
    loc = LOC[field]
    if loc == "c":
        return TH if field == T else P
    ev = {"r": e[0], "t": e[1], "p": e[2]}[loc]
    return U[0] * ev[0] + U[1] * ev[1] + U[2] * ev[2]


def mms_fields(grid, t, field, padded=False, kind="shell"):
    """Exact value of a field of a manufactured solution ("shell": ours,
    "paper": eq. Exact) at time t on its MAC points (both patches), or on
    every slot of the padded layout.  Velocity fields are the same for
    systems 1 and 2, pressure fields for p1 and p2."""
    shape = (2, grid.nr + 2, grid.nt + 2, grid.np + 2) if padded else grid.mac_shape(field)
    out = np.zeros(shape)
    s = _TIME[kind][0](t)
    for patch in range(2):
        X, (er, et, ep) = points(grid, field, patch, padded)
        U, P, TH = _values(kind, X, grid.r1, grid.r2)
        loc = LOC[field]
        if loc == "c":
            out[patch] = s * (TH if field == T else P)
        else:
            e = {"r": er, "t": et, "p": ep}[loc]
            out[patch] = s * (U[0] * e[0] + U[1] * e[1] + U[2] * e[2])
    return out


def time_factor(kind, t):
    """(a(t), a'(t)): every field of a manufactured solution is a(t) times
    its spatial part"""
    return _TIME[kind][0](t), _TIME[kind][1](t)


def forcing_parts(grid, field, pr, ra, padded=False, kind="shell"):
    """Spatial parts (A, B, C) of the forcing that makes the manufactured
    solution exact, f(t) = a(t) A + a'(t) B + a(t)^2 C, from
    f_u = du/dt + (u.grad)u + grad p - Pr lap u - Pr Ra T e_r and
    f_T = dT/dt + u.grad T - lap T  (field T, U1R, U1T or U1P)."""
    shape = (2, grid.nr + 2, grid.nt + 2, grid.np + 2) if padded else grid.mac_shape(field)
    A, B, C = np.zeros(shape), np.zeros(shape), np.zeros(shape)
    for patch in range(2):
        X, (er, et, ep) = points(grid, field, patch, padded)
        U, P, TH, r = _jets(kind, X, grid.r1, grid.r2)
        if field == T:
            A[patch] = -TH.lap()
            B[patch] = TH.v
            C[patch] = sum(U[d].v * TH.g[d] for d in range(3))
            continue
        rhat = [X[d] / r.v for d in range(3)]
        e = {U1R: er, U1T: et, U1P: ep}[field]
        for comp in range(3):
            A[patch] += e[comp] * (P.g[comp] - pr * U[comp].lap() - pr * ra * TH.v * rhat[comp])
            B[patch] += e[comp] * U[comp].v
            C[patch] += e[comp] * sum(U[d].v * U[comp].g[d] for d in range(3))
    return A, B, C


def mms_forcing(grid, t, field, pr, ra, padded=False, kind="shell"):
    """Forcing at time t that makes the manufactured solution exact (see
    forcing_parts)."""
    a, da = time_factor(kind, t)
    A, B, C = forcing_parts(grid, field, pr, ra, padded, kind)
    return a * A + da * B + (a * a) * C


def mms_state(grid, t, padded=False, kind="shell"):
    """All nine fields of the manufactured solution at time t."""
    st = {f: mms_fields(grid, t, f, padded, kind) for f in (T, U1R, U1T, U1P, P1)}
    for f, base in ((U2R, U1R), (U2T, U1T), (U2P, U1P), (P2, P1)):
        st[f] = st[base].copy()
    return st


def wall_values(grid, t, field, kind="paper"):
    """Exact Dirichlet data of T, u_r, u_theta or u_phi (field T, U1R, U1T
    or U1P) at time t on the walls r = R1 (index 0) and r = R2 (index 1), at
    the field's own (theta, phi) positions of the padded layout: shape
    (2 walls, 2 patches, nt+2, np+2)."""
    return _TIME[kind][0](t) * wall_parts(grid, field, kind)


def wall_parts(grid, field, kind="paper"):
    """Spatial part of wall_values (the values at a(t) = 1)."""
    _, th, ph = grid.axes(field, padded=True)
    out = np.zeros((2, 2, grid.nt + 2, grid.np + 2))
    for w, r in enumerate((grid.r1, grid.r2)):
        for patch in range(2):
            X, e = _frame_points(np.array([r]), th, ph, patch)
            U, P, TH = _values(kind, X, grid.r1, grid.r2)
            out[w, patch] = _field_value(field, U, P, TH, e)[0]
    return out


# ---------------------------------------------------------------------------
# seeded workloads
# ---------------------------------------------------------------------------
def conductive_T(grid, t_inner=1.0, t_outer=0.0):
    """Conductive profile T(r) with T(R1) = t_inner, T(R2) = t_outer at
    cell centres (solution of r^-2 (r^2 T')' = 0)."""
    r, _, _ = grid.axes(T)
    r1, r2 = grid.r1, grid.r2
    prof = t_outer + (t_inner - t_outer) * r1 * (r2 - r) / ((r2 - r1) * r)
    return np.broadcast_to(prof[None, :, None, None], grid.mac_shape(T)).copy()


def convection_state(grid, pr, ra, seed, noise=1e-3):
    """u = 0, T = conductive profile + seeded Gaussian noise, p1 = p2 =
    hydrostatic balance of the noise-free T integrated cell by cell along r
    with p = 0 in the innermost cell."""
    Tc = conductive_T(grid)
    rng = np.random.default_rng(seed)
    Tn = Tc + noise * rng.standard_normal(grid.mac_shape(T))
    p = np.zeros_like(Tc)
    for i in range(1, grid.nr):
        p[:, i] = p[:, i - 1] + grid.dr * pr * ra * 0.5 * (Tc[:, i - 1] + Tc[:, i])
    st = {f: np.zeros(grid.mac_shape(f)) for f in range(9)}
    st[T] = Tn
    st[P1] = p.copy()
    st[P2] = p.copy()
    return st


def line_rhs(grid, seed=2):
    """Right-hand side of the line-solve workload: uniform[-1,1] on the
    padded grid (2, Nr+2, Nt+2, Np+2)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (2, grid.nr + 2, grid.nt + 2, grid.np + 2))


def ensemble_shapes(n=32, seed=5):
    """Shell sizes and Rayleigh numbers of the batched ensemble."""
    rng = np.random.default_rng(seed)
    nr = rng.integers(16, 64, n, endpoint=True)
    nt = rng.integers(48, 192, n, endpoint=True)
    ra = 10 ** rng.uniform(3, 6, n)
    return [(int(a), int(b), int(3 * b), float(c)) for a, b, c in zip(nr, nt, ra)]
