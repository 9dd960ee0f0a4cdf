"""Whole-grid second implementation of the step, no subdomains (test
infrastructure only).

Written directly from the scheme (Sec. 2.2.1 eq. VF_scheme, the
Lax-Friedrichs flux of Sec. 2.2.1, the Euler system of Sec. 5, the spray
system of Sec. 6.1) with numpy array shifts instead of the subdomain tasks.
It evaluates the same operations in the same order as the C oracle, so for
advection and Euler the two must agree bit for bit at any partition; this is
what pins the task decomposition (overlap copies, interior/border split) to
the unpartitioned scheme. A torch version of the same formula gives the exact
discrete adjoint through torch.autograd for small grids.
"""
from __future__ import annotations

import math

import numpy as np

ADV, EULER, SPRAY = 0, 1, 2
PERIODIC, TRANSMISSIVE, DIRICHLET = 0, 1, 2
TINY = 1e-300


def _neighbours(W, axis, bc, ghost=None):
    """(left, right) neighbour arrays along a spatial axis (2 = x, 1 = y).
    Dirichlet: ghost is (nVar, 4) states west, east, south, north; the
    neighbour beyond each side is that side's state."""
    if bc == PERIODIC:
        return np.roll(W, 1, axis=axis), np.roll(W, -1, axis=axis)
    if bc == DIRICHLET:
        g = np.asarray(ghost, dtype=np.float64)
        lo, hi = (0, 1) if axis == 2 else (2, 3)
        shape = list(W.shape)
        shape[axis] = 1
        gl = np.broadcast_to(g[:, lo].reshape(-1, 1, 1), shape)
        gr = np.broadcast_to(g[:, hi].reshape(-1, 1, 1), shape)
        n = W.shape[axis]
        left = np.concatenate([gl, np.take(W, np.arange(n - 1), axis=axis)], axis=axis)
        right = np.concatenate([np.take(W, np.arange(1, n), axis=axis), gr], axis=axis)
        return left, right
    n = W.shape[axis]
    idx_l = np.clip(np.arange(n) - 1, 0, n - 1)
    idx_r = np.clip(np.arange(n) + 1, 0, n - 1)
    return np.take(W, idx_l, axis=axis), np.take(W, idx_r, axis=axis)


def phys_flux(model, W, d, gamma=1.4, a=(0.0, 0.0)):
    if model == ADV:
        return a[d] * W, np.full(W.shape[1:], abs(a[d]))
    if model == EULER:
        r, ru, rv, e = W
        u = ru / r
        v = rv / r
        ke = 0.5 * (ru * u + rv * v)
        p = (gamma - 1.0) * (e - ke)
        c = np.sqrt(gamma * p / r)
        un = u if d == 0 else v
        f1 = ru * un
        f2 = rv * un
        if d == 0:
            f1 = f1 + p
        else:
            f2 = f2 + p
        F = np.stack([r * un, f1, f2, (e + p) * un])
        return F, np.abs(un) + c
    m2 = W[2]
    un = np.where(m2 > TINY, W[4 + d] / np.where(m2 > TINY, m2, 1.0), 0.0)
    return W * un, np.abs(un)


def num_flux(model, WL, WR, d, gamma=1.4, a=(0.0, 0.0)):
    if model == ADV:
        ap = a[d] if a[d] > 0.0 else 0.0
        am = a[d] if a[d] < 0.0 else 0.0
        return ap * WL + am * WR
    if model == EULER:
        FL, sl = phys_flux(model, WL, d, gamma)
        FR, sr = phys_flux(model, WR, d, gamma)
        sigma = np.where(sl >= sr, sl, sr)
        return 0.5 * (FL + FR) - 0.5 * sigma * (WR - WL)
    m2l, m2r = WL[2], WR[2]
    ul = np.where(m2l > TINY, WL[4 + d] / np.where(m2l > TINY, m2l, 1.0), 0.0)
    ur = np.where(m2r > TINY, WR[4 + d] / np.where(m2r > TINY, m2r, 1.0), 0.0)
    up = np.where(ul > 0.0, ul, 0.0)
    um = np.where(ur < 0.0, ur, 0.0)
    return WL * up + WR * um


def spray_source(W, ug, K, theta, s_eps):
    m0, m1, m2 = W[0], W[1], W[2]
    ok = (m0 > TINY) & (m1 > TINY) & (m2 > TINY)
    safe = lambda x: np.where(ok, x, 1.0)
    m0s, m1s, m2s = safe(m0), safe(m1), safe(m2)
    ux = W[4] / m2s
    uy = W[5] / m2s
    L1 = np.log(m1s / m0s)
    L2 = np.log(m2s / m0s)
    s2 = 4.0 * (L2 - 2.0 * L1)
    s2 = np.where(s2 < 1e-8, 1e-8, s2)
    mu = 2.0 * L1 - s2 / 4.0
    mmh = m0s * np.exp(-mu / 2.0 + s2 / 8.0)
    z = math.log(s_eps) - mu
    n0 = m0s / (s_eps * np.sqrt(2.0 * math.pi * s2)) * np.exp(-(z * z) / (2.0 * s2))
    S = np.stack([-K * n0, -(K / 2.0) * mmh, -K * m0s, -(1.5 * K) * m1s,
                  -K * m0s * ux + m0s * (ug[0] - ux) / theta,
                  -K * m0s * uy + m0s * (ug[1] - uy) / theta])
    return np.where(ok[None], S, 0.0)


def step(model, W, dt, *, bc=PERIODIC, lx=1.0, ly=1.0, gamma=1.4,
         a=(0.0, 0.0), ug=None, K=1.0, theta=0.1, s_eps=0.01, ghost=None):
    """One step W^n -> W^{n+1} with the given dt on the whole grid
    (ghost: Dirichlet states, 4 x nVar, west, east, south, north)."""
    W = np.asarray(W, dtype=np.float64)
    nx, ny = W.shape[2], W.shape[1]
    mux = dt / (lx / nx)
    muy = dt / (ly / ny)
    gT = None if ghost is None else np.asarray(ghost, dtype=np.float64).T
    Wl, Wr = _neighbours(W, 2, bc, gT)
    Ws, Wn = _neighbours(W, 1, bc, gT)
    FE = num_flux(model, W, Wr, 0, gamma, a)
    FW = num_flux(model, Wl, W, 0, gamma, a)
    GN = num_flux(model, W, Wn, 1, gamma, a)
    GS = num_flux(model, Ws, W, 1, gamma, a)
    t = mux * (FE - FW) + muy * (GN - GS)
    Wstar = W + (-t)
    if model == SPRAY:
        Wstar = Wstar + dt * spray_source(Wstar, ug, K, theta, s_eps)
    return Wstar


def speeds(model, W, gamma=1.4, a=(0.0, 0.0)):
    _, sx = phys_flux(model, W, 0, gamma, a)
    _, sy = phys_flux(model, W, 1, gamma, a)
    return float(np.max(sx)), float(np.max(sy))


def cfl_dt(model, W, cfl, *, lx=1.0, ly=1.0, gamma=1.4, a=(0.0, 0.0)):
    nx, ny = W.shape[2], W.shape[1]
    sx, sy = speeds(model, W, gamma, a)
    return cfl / (sx / (lx / nx) + sy / (ly / ny))


# --------------------------------------------------------------------------
# torch version (fp64, CPU) for the exact discrete adjoint via autograd
# --------------------------------------------------------------------------

def torch_step(model, W, dt, *, bc=PERIODIC, lx=1.0, ly=1.0, gamma=1.4,
               a=(0.0, 0.0), ug=None, K=1.0, theta=0.1, s_eps=0.01):
    """Differentiable whole-grid step: the transport (advection, Euler or the
    spray's kinetic upwind flux) and, for the spray, the lognormal-closure
    source at W* (ug: the gas velocity, 2 planes)."""
    import torch

    def nb(X, axis):
        if bc == PERIODIC:
            return torch.roll(X, 1, dims=axis), torch.roll(X, -1, dims=axis)
        n = X.shape[axis]
        il = torch.clamp(torch.arange(n) - 1, 0, n - 1)
        ir = torch.clamp(torch.arange(n) + 1, 0, n - 1)
        return torch.index_select(X, axis, il), torch.index_select(X, axis, ir)

    def pflux(X, d):
        if model == ADV:
            return a[d] * X, None
        r, ru, rv, e = X[0], X[1], X[2], X[3]
        u = ru / r
        v = rv / r
        p = (gamma - 1.0) * (e - 0.5 * (ru * u + rv * v))
        c = torch.sqrt(gamma * p / r)
        un = u if d == 0 else v
        f1 = ru * un + (p if d == 0 else 0.0)
        f2 = rv * un + (p if d == 1 else 0.0)
        return torch.stack([r * un, f1, f2, (e + p) * un]), torch.abs(un) + c

    def vel(X, d):
        ok = X[2] > TINY
        return torch.where(ok, X[4 + d] / torch.where(ok, X[2], torch.ones_like(X[2])),
                           torch.zeros_like(X[2]))

    def nflux(XL, XR, d):
        if model == ADV:
            ap = a[d] if a[d] > 0.0 else 0.0
            am = a[d] if a[d] < 0.0 else 0.0
            return ap * XL + am * XR
        if model == SPRAY:
            ul, ur = vel(XL, d), vel(XR, d)
            up = torch.where(ul > 0.0, ul, torch.zeros_like(ul))
            um = torch.where(ur < 0.0, ur, torch.zeros_like(ur))
            return XL * up + XR * um
        FL, sl = pflux(XL, d)
        FR, sr = pflux(XR, d)
        sigma = torch.where(sl >= sr, sl, sr)
        return 0.5 * (FL + FR) - 0.5 * sigma * (XR - XL)

    nx, ny = W.shape[2], W.shape[1]
    mux = dt / (lx / nx)
    muy = dt / (ly / ny)
    Wl, Wr = nb(W, 2)
    Ws, Wn = nb(W, 1)
    t = mux * (nflux(W, Wr, 0) - nflux(Wl, W, 0)) + muy * (nflux(W, Wn, 1) - nflux(Ws, W, 1))
    Wstar = W - t
    if model != SPRAY:
        return Wstar
    ug = torch.as_tensor(ug, dtype=W.dtype)
    m0, m1, m2 = Wstar[0], Wstar[1], Wstar[2]
    ok = (m0 > TINY) & (m1 > TINY) & (m2 > TINY)
    one = torch.ones_like(m0)
    m0s, m1s, m2s = torch.where(ok, m0, one), torch.where(ok, m1, one), torch.where(ok, m2, one)
    ux, uy = Wstar[4] / m2s, Wstar[5] / m2s
    L1 = torch.log(m1s / m0s)
    L2 = torch.log(m2s / m0s)
    s2 = 4.0 * (L2 - 2.0 * L1)
    s2 = torch.where(s2 < 1e-8, torch.full_like(s2, 1e-8), s2)
    mu = 2.0 * L1 - s2 / 4.0
    mmh = m0s * torch.exp(-mu / 2.0 + s2 / 8.0)
    z = math.log(s_eps) - mu
    n0 = m0s / (s_eps * torch.sqrt(2.0 * math.pi * s2)) * torch.exp(-(z * z) / (2.0 * s2))
    it = 0.0 if math.isinf(theta) else 1.0 / theta
    S = torch.stack([-K * n0, -(K / 2.0) * mmh, -K * m0s, -(1.5 * K) * m1s,
                     -K * m0s * ux + m0s * (ug[0] - ux) * it,
                     -K * m0s * uy + m0s * (ug[1] - uy) * it])
    return Wstar + dt * torch.where(ok[None], S, torch.zeros_like(S))
