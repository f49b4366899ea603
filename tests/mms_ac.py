"""A non-solenoidal manufactured field for pinning the grad-div and
div-dependent viscous terms of the momentum residual.

For a divergence-free field the grad-div blocks D_ij (Sec. 3.3) vanish, so
the plain manufactured solution cannot see a wrong sign or factor in them.
This field adds W = w0 sin t (xy, yz, zx) (div W != 0) to the manufactured
velocity and builds the forcing of the equation the converged AC step
actually discretises:
  du/dt + (u.grad)u + grad p - Pr V(u) - (1/(2 chi)) grad div u
      - Pr Ra T e_r = f,
where V(u) is the viscous operator written with div u = 0 used in the r
and theta components (Sec. 3.3.1-3.3.2):
  V(u) = vector Laplacian + (2/r) div(u) e_r + (2 cot(theta)/r) div(u) e_theta,
theta being the patch's own polar angle.
"""
import math

import numpy as np

from paper_1905_02300_amd import inputs as I

W0 = 0.3


def _jets(X, g):
    U, P, TH, r = I._mms_jets(X, g.r1, g.r2)
    x, y, z = (I.Jet.var(X, d) for d in range(3))
    U = [U[0] + W0 * x * y, U[1] + W0 * y * z, U[2] + W0 * z * x]
    return U, P, TH, r


def _local_theta(g, field, patch, padded):
    r, t, p = g.axes(field, padded)
    return np.broadcast_to(t[None, :, None], (r.size, t.size, p.size))


def fields(g, t, field, padded=False):
    shape = (2, g.nr + 2, g.nt + 2, g.np + 2) if padded else g.mac_shape(field)
    out = np.zeros(shape)
    s = math.sin(t)
    for patch in range(2):
        X, (er, et, ep) = I.points(g, field, patch, padded)
        U, P, TH = I._mms_values(X, g.r1, g.r2)
        x, y, z = X
        U = [U[0] + W0 * x * y, U[1] + W0 * y * z, U[2] + W0 * z * x]
        loc = I.LOC[field]
        if loc == "c":
            out[patch] = s * (TH if field == I.T else P)
        else:
            e = {"r": er, "t": et, "p": ep}[loc]
            out[patch] = s * sum(U[d] * e[d] for d in range(3))
    return out


def state(g, t, padded=True):
    st = {f: fields(g, t, f, padded) for f in (I.T, I.U1R, I.U1T, I.U1P, I.P1)}
    for f, base in ((I.U2R, I.U1R), (I.U2T, I.U1T), (I.U2P, I.U1P), (I.P2, I.P1)):
        st[f] = st[base].copy()
    return st


def forcing(g, t, field, pr, ra, chi):
    out = np.zeros(g.mac_shape(field))
    s, c = math.sin(t), math.cos(t)
    for patch in range(2):
        X, (er, et, ep) = I.points(g, field, patch)
        U, P, TH, r = _jets(X, g)
        if field == I.T:
            adv = sum(U[d].v * TH.g[d] for d in range(3))
            out[patch] = c * TH.v + s * s * adv - s * TH.lap()
            continue
        div = sum(U[d].g[d] for d in range(3))
        graddiv = [sum(U[d].H[comp][d] for d in range(3)) for comp in range(3)]
        rhat = [X[d] / r.v for d in range(3)]
        cot = 1.0 / np.tan(_local_theta(g, field, patch, False))
        F = []
        for comp in range(3):
            adv = sum(U[d].v * U[comp].g[d] for d in range(3))
            visc = U[comp].lap() + (2.0 / r.v) * div * er[comp] + (2.0 * cot / r.v) * div * et[comp]
            F.append(c * U[comp].v + s * s * adv
                     + s * (P.g[comp] - pr * visc - graddiv[comp] / (2.0 * chi)
                            - pr * ra * TH.v * rhat[comp]))
        e = {I.U1R: er, I.U1T: et, I.U1P: ep}[field]
        out[patch] = F[0] * e[0] + F[1] * e[1] + F[2] * e[2]
    return out
