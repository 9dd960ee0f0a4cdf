"""Seeded synthetic inputs and the named workload presets.

This module is the only code shared by the HIP path and the CPU oracle: it
draws initial states and read-only fields with numpy's PCG64 generator and
holds the preset parameters of the five workloads. It contains none of the
time-step arithmetic (no flux, no update, no source, no CFL logic); the only
formulas here build the inputs themselves (cell centres, primitive-to-
conservative conversion of initial data, lognormal moments of the initial
size distributions, the gas velocity field).

Arrays are float64 structure-of-arrays ``W[v, j, i]`` (x fastest), cell
centres ``x_i = (i + 1/2) dx`` on the unit square unless stated (point values
at the centres, not cell averages).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ADV, EULER, SPRAY = 0, 1, 2
PERIODIC, TRANSMISSIVE = 0, 1
NVAR = {ADV: 1, EULER: 4, SPRAY: 6}
GAMMA = 1.4


@dataclasses.dataclass(frozen=True)
class Preset:
    """Parameters of one workload (names follow the paper: Nx, Ny, NPartX,
    NPartY, nVar)."""
    name: str
    model: int
    bc: int
    nx: int
    ny: int
    npart_x: int
    npart_y: int
    nsteps: int
    cfl: float
    gamma: float = GAMMA
    ax: float = 0.0
    ay: float = 0.0
    K: float = 1.0
    theta: float = 0.1
    s_eps: float = 0.01
    lx: float = 1.0
    ly: float = 1.0
    dt_max: float = 0.0

    @property
    def nvar(self) -> int:
        return NVAR[self.model]

    def replace(self, **kw) -> "Preset":
        return dataclasses.replace(self, **kw)


# 2-D linear advection, a = (1, 0.5), upwind, 64x64 periodic, CFL 0.9,
# 100 steps, 2x2 subdomains.
ADVECTION_64 = Preset("advection_64x64", ADV, PERIODIC, 64, 64, 2, 2, 100, 0.9,
                      ax=1.0, ay=0.5)
# 2-D Euler, Rusanov flux, 4096x4096, transmissive, CFL 0.45, 200 steps,
# 8x8 subdomains.
EULER_4096 = Preset("euler_4096x4096", EULER, TRANSMISSIVE, 4096, 4096, 8, 8,
                    200, 0.45)
# Spray moments (nVar = 6), kinetic upwind transport + evaporation/drag
# source, 2048x2048 periodic, 200 steps, 8x8 subdomains.
SPRAY_2048 = Preset("spray_2048x2048", SPRAY, PERIODIC, 2048, 2048, 8, 8, 200,
                    0.9, K=1.0, theta=0.1, s_eps=0.01)
# Batched Euler: 256 grids with n ~ floor(64 * 16**U), 100 steps.
BATCH_256 = Preset("euler_batch_256", EULER, TRANSMISSIVE, 0, 0, 1, 1, 100,
                   0.45)
BATCH_COUNT = 256
# Adjoint Euler: 1024x1024, 100 steps, checkpoint every 10 steps.
ADJOINT_1024 = Preset("euler_adjoint_1024x1024", EULER, TRANSMISSIVE, 1024,
                      1024, 1, 1, 100, 0.45)
ADJOINT_CKPT_EVERY = 10


def centres(n: int, length: float = 1.0) -> np.ndarray:
    """Cell-centre coordinates (i + 1/2) * length / n."""
    return (np.arange(n, dtype=np.float64) + 0.5) * (length / n)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_bumps(nx: int, ny: int, seed: int, nbumps: int = 3) -> np.ndarray:
    """Sum of ``nbumps`` periodic Gaussian bumps on the unit square, shape
    (ny, nx). Per bump the draws are, in order: centre x, centre y ~ U[0,1),
    amplitude ~ U[0.5,1], width (standard deviation) ~ U[0.05,0.15].
    Offsets to the centre use the minimum periodic image."""
    rng = _rng(seed)
    x = centres(nx)[None, :]
    y = centres(ny)[:, None]
    out = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(nbumps):
        cx, cy = rng.uniform(0.0, 1.0), rng.uniform(0.0, 1.0)
        amp = rng.uniform(0.5, 1.0)
        wid = rng.uniform(0.05, 0.15)
        ddx = x - cx
        ddx = ddx - np.round(ddx)
        ddy = y - cy
        ddy = ddy - np.round(ddy)
        out = out + amp * np.exp(-(ddx * ddx + ddy * ddy) / (2.0 * wid * wid))
    return out


def advection_state(nx: int, ny: int, seed: int) -> np.ndarray:
    """Initial scalar of the advection workload, shape (1, ny, nx)."""
    return gaussian_bumps(nx, ny, seed)[None]


def conservative_from_primitive(rho, u, v, p, gamma: float = GAMMA) -> np.ndarray:
    """(rho, u, v, p) -> (rho, rho u, rho v, rho E), rho E = p/(gamma-1) +
    rho (u^2+v^2)/2 (initial data only)."""
    rho, u, v, p = (np.asarray(a, dtype=np.float64) for a in (rho, u, v, p))
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, e]).astype(np.float64)


def riemann_primitives(nx: int, ny: int, seed: int):
    """Four-quadrant piecewise-constant Riemann data split at x = 1/2 and
    y = 1/2 (a centre exactly at 1/2 counts as west/south). Quadrants are
    drawn in the order NE, NW, SW, SE; per quadrant rho, u, v, p with
    rho, p ~ U[0.1,1] and u, v ~ U[-0.5,0.5]."""
    rng = _rng(seed)
    q = {}
    for name in ("NE", "NW", "SW", "SE"):
        rho = rng.uniform(0.1, 1.0)
        u = rng.uniform(-0.5, 0.5)
        v = rng.uniform(-0.5, 0.5)
        p = rng.uniform(0.1, 1.0)
        q[name] = (rho, u, v, p)
    east = (centres(nx) > 0.5)[None, :]
    north = (centres(ny) > 0.5)[:, None]
    prim = []
    for k in range(4):
        f = np.where(north,
                     np.where(east, q["NE"][k], q["NW"][k]),
                     np.where(east, q["SE"][k], q["SW"][k]))
        prim.append(np.broadcast_to(f, (ny, nx)).astype(np.float64))
    return prim


def riemann_state(nx: int, ny: int, seed: int, gamma: float = GAMMA) -> np.ndarray:
    """Conservative Euler state of the four-quadrant Riemann data, shape
    (4, ny, nx)."""
    return conservative_from_primitive(*riemann_primitives(nx, ny, seed), gamma)


def adjoint_target_density(nx: int, ny: int, seed: int) -> np.ndarray:
    """Target density of the adjoint workload: the density of the Riemann
    state perturbed by 1e-2 times a sum of three seeded Gaussian bumps
    normalised to a maximum of one (seed + 1 for the bumps)."""
    prim = riemann_primitives(nx, ny, seed)
    b = gaussian_bumps(nx, ny, seed + 1)
    b = b / np.max(np.abs(b))
    return prim[0] + 1e-2 * b


def perturbed_riemann_state(nx: int, ny: int, seed: int, amp: float = 1e-2,
                            gamma: float = GAMMA) -> np.ndarray:
    """Riemann state whose primitives (rho, u, v, p) are each shifted by
    ``amp`` times the normalised bump field of ``adjoint_target_density``."""
    prim = riemann_primitives(nx, ny, seed)
    b = gaussian_bumps(nx, ny, seed + 1)
    b = b / np.max(np.abs(b))
    return conservative_from_primitive(*(f + amp * b for f in prim), gamma)


def _smooth_periodic(nx: int, ny: int, rng: np.random.Generator) -> np.ndarray:
    """Sum of three periodic sinusoids with integer wavenumbers in [1,4] and
    random phases, normalised to max |g| = 1."""
    x = centres(nx)[None, :]
    y = centres(ny)[:, None]
    g = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(3):
        kx = int(rng.integers(1, 5))
        ky = int(rng.integers(1, 5))
        phx = rng.uniform(0.0, 2.0 * math.pi)
        phy = rng.uniform(0.0, 2.0 * math.pi)
        g = g + np.sin(2 * math.pi * kx * x + phx) * np.cos(2 * math.pi * ky * y + phy)
    return g / np.max(np.abs(g))


def gas_velocity(nx: int, ny: int, seed: int) -> np.ndarray:
    """Taylor-Green gas velocity u_g = A (sin(2 pi k x + px) cos(2 pi k y + py),
    -cos(2 pi k x + px) sin(2 pi k y + py)), A ~ U[0.5,1], k in {1,2},
    phases ~ U[0, 2 pi). Shape (2, ny, nx)."""
    rng = _rng(seed)
    amp = rng.uniform(0.5, 1.0)
    k = int(rng.integers(1, 3))
    phx = rng.uniform(0.0, 2.0 * math.pi)
    phy = rng.uniform(0.0, 2.0 * math.pi)
    x = centres(nx)[None, :]
    y = centres(ny)[:, None]
    ax = 2 * math.pi * k * x + phx
    ay = 2 * math.pi * k * y + phy
    ugx = amp * np.sin(ax) * np.cos(ay)
    ugy = -amp * np.cos(ax) * np.sin(ay)
    return np.stack([ugx, ugy]).astype(np.float64)


def lognormal_moments(n0, mu, s, kmax: int = 3) -> list:
    """Fractional moments m_{k/2} = N0 exp(k mu/2 + k^2 s^2/8), k = 0..kmax,
    of the (untruncated) lognormal N0 * LogNormal(mu, s^2) in S."""
    return [n0 * np.exp(k * mu / 2.0 + k * k * s * s / 8.0) for k in range(kmax + 1)]


def spray_state(nx: int, ny: int, seed: int):
    """Initial spray state (m_{0/2}, m_{1/2}, m_{2/2}, m_{3/2}, q_x, q_y) with
    q = m_{2/2} u and u = u_g, plus the gas velocity field. The size
    distribution is lognormal with smooth seeded parameters
    N0 = 1 + 0.5 g1, mu = ln 0.2 + 0.3 g2, s = 0.3 + 0.1 g3 (median sizes
    0.15-0.27, so the K = 1 evaporation of the workload keeps every moment
    positive over its 200 steps).
    Returns (W of shape (6, ny, nx), u_g of shape (2, ny, nx))."""
    ug = gas_velocity(nx, ny, seed)
    rng = _rng(seed + 7919)
    g1 = _smooth_periodic(nx, ny, rng)
    g2 = _smooth_periodic(nx, ny, rng)
    g3 = _smooth_periodic(nx, ny, rng)
    n0 = 1.0 + 0.5 * g1
    mu = math.log(0.2) + 0.3 * g2
    s = 0.3 + 0.1 * g3
    m = lognormal_moments(n0, mu, s)
    w = np.stack([m[0], m[1], m[2], m[3], m[2] * ug[0], m[2] * ug[1]])
    return w.astype(np.float64), ug


def batch_sizes(count: int, seed: int, nmin: int = 64, ratio: float = 16.0):
    """Side lengths n_g = floor(nmin * ratio**U), U ~ U[0,1) per grid (sizes
    log-uniform between 64 and 1024 for the defaults)."""
    rng = _rng(seed)
    u = rng.uniform(0.0, 1.0, size=count)
    return [int(math.floor(nmin * ratio ** float(t))) for t in u]


def localized_cosine_primitives(nx: int, ny: int, t: float = 0.0,
                                ubar: float = 1.0, vbar: float = 1.0,
                                gamma: float = GAMMA):
    """Localized cosine density bump advected by (ubar, vbar) on the periodic
    unit square, with p = 1/gamma; the bump is read as
    rho = 1 + (r < 1/4) (1 + cos(4 pi r)) / 2 so that it stays positive and
    continuous. Returns primitive fields at time t (exact translation)."""
    x = centres(nx)[None, :]
    y = centres(ny)[:, None]
    xs = x - ubar * t
    ys = y - vbar * t
    xs = xs - np.floor(xs)
    ys = ys - np.floor(ys)
    r = np.sqrt((xs - 0.5) ** 2 + (ys - 0.5) ** 2)
    rho = 1.0 + (r < 0.25) * 0.5 * (1.0 + np.cos(4.0 * math.pi * r))
    shape = (ny, nx)
    return [np.broadcast_to(rho, shape).astype(np.float64),
            np.full(shape, ubar), np.full(shape, vbar), np.full(shape, 1.0 / gamma)]


def isentropic_vortex_primitives(nx: int, ny: int, t: float = 0.0,
                                 omega: float = 1.0, R: float = 0.1,
                                 ubar: float = 1.0, vbar: float = 1.0,
                                 gamma: float = GAMMA):
    """Isentropic rotating Gaussian vortex translated by (ubar, vbar) on the
    periodic unit square: omega(r) = omega exp(-r^2/(2 R^2)), velocity
    perturbation (-y' omega/R, x' omega/R) with (x', y') the offset from the
    vortex centre, rho = (1 - (gamma-1)/2 omega^2)^(1/(gamma-1)),
    p = rho^gamma / gamma. Primitive fields at time t (quasi-exact)."""
    x = centres(nx)[None, :]
    y = centres(ny)[:, None]
    xs = x - ubar * t
    ys = y - vbar * t
    xs = xs - np.floor(xs) - 0.5
    ys = ys - np.floor(ys) - 0.5
    r2 = xs * xs + ys * ys
    om = omega * np.exp(-r2 / (2.0 * R * R))
    rho = (1.0 - 0.5 * (gamma - 1.0) * om * om) ** (1.0 / (gamma - 1.0))
    u = ubar - ys * om / R
    v = vbar + xs * om / R
    p = rho ** gamma / gamma
    shape = (ny, nx)
    return [np.broadcast_to(a, shape).astype(np.float64) for a in (rho, u, v, p)]
