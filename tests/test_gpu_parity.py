"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerance (per variable v): relative L-infinity
    max |W_gpu - W_orc| / max |W_orc[v]|  <=  1e-12
after one step from the same state, and along whole trajectories where each
side takes its own adaptive dt. The dt itself comes from maxima that are
order-independent, so the two sides may differ only through the per-cell
speed arithmetic: |dt_gpu - dt_orc| <= 4 ulp. Results that must not depend on
the work decomposition (subdomain counts, tile shapes, batched vs single
launches) are compared bit for bit.
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import fv as orc
from paper_1701_05431_amd import inputs
from paper_1701_05431_amd import _lib
from paper_1701_05431_amd.solver import Batch, Solver, aligned_pitch, params_from, fvrun

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

TOL = 1e-12
DT_ULP = 4


def rel_linf(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = 0.0
    for v in range(a.shape[0]):
        den = max(float(np.max(np.abs(b[v]))), 1e-300)
        out = max(out, float(np.max(np.abs(a[v] - b[v]))) / den)
    return out


def ulps(a, b):
    return abs(a - b) / math.ulp(abs(b))


def oparams(p: _lib.Params, ghost=None):
    return orc.params(p.model, p.nx, p.ny, bc=p.bc, npx=p.npart_x, npy=p.npart_y, lx=p.lx,
                      ly=p.ly, gamma=p.gamma, ax=p.ax, ay=p.ay, K=p.K, theta=p.theta,
                      s_eps=p.s_eps, cfl=p.cfl, dt_max=p.dt_max, ghost=ghost)


def gpu_state(s: Solver) -> np.ndarray:
    torch.cuda.synchronize()
    return s.state().cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    _lib.lib()
    torch.cuda.set_device(0)
    yield


# ---------------------------------------------------------------------------
# one step from an identical state
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape", [(200, 150, 203), (62, 1, 64), (1, 7, 1), (125, 64, 125)])
def test_euler_one_step(bc, shape):
    nx, ny, ld = shape
    print(f"euler one step bc={bc} shape={shape}", flush=True)
    W = inputs.riemann_state(nx, ny, 3)
    W = W + 0.01 * np.stack([inputs.gaussian_bumps(nx, ny, 10 + v) for v in range(4)])
    p = params_from(model=1, bc=bc, nx=nx, ny=ny, ld=ld, cfl=0.45)
    s = Solver(p)
    s.set_state(W)
    dts = s.run(1, record_dt=True).cpu().numpy()
    got = gpu_state(s)
    P = oparams(p)
    ref, odts = orc.run(P, W, 1)
    assert ulps(dts[0], odts[0]) <= DT_ULP
    ref1 = orc.run_dts(P, W, dts)
    assert rel_linf(got, ref1) <= TOL, rel_linf(got, ref1)


@pytest.mark.parametrize("bc", [0, 1])
def test_advection_workload_trajectory(bc):
    """64x64 advection, a = (1, 0.5), C = 0.9, 100 steps, 2x2 subdomains."""
    pre = inputs.ADVECTION_64.replace(bc=bc)
    for seed in (0, 1, 2):
        print(f"advection seed={seed} bc={bc}", flush=True)
        u0 = inputs.advection_state(64, 64, seed)
        p = params_from(pre)
        s = Solver(p)
        s.set_state(u0)
        dts = s.run(pre.nsteps, record_dt=True).cpu().numpy()
        got = gpu_state(s)
        ref, odts = orc.run(oparams(p), u0, pre.nsteps)
        assert np.all(dts == odts)
        assert rel_linf(got, ref) <= TOL


def test_euler_trajectory_each_step():
    nx, ny = 96, 80
    W = inputs.riemann_state(nx, ny, 5)
    p = params_from(model=1, bc=1, nx=nx, ny=ny, npart_x=4, npart_y=2, cfl=0.45)
    s = Solver(p)
    s.set_state(W)
    P = oparams(p)
    ref = W.copy()
    for k in range(40):
        dts = s.run(1, record_dt=True).cpu().numpy()
        ref, odt = orc.run(P, ref, 1)
        assert ulps(dts[0], odt[0]) <= DT_ULP, k
        assert rel_linf(gpu_state(s), ref) <= TOL, k


def test_spray_trajectory():
    n = 128
    W, ug = inputs.spray_state(n, n, 1)
    pre = inputs.SPRAY_2048.replace(nx=n, ny=n, npart_x=4, npart_y=4)
    p = params_from(pre)
    s = Solver(p, ug=ug)
    s.set_state(W)
    P = oparams(p)
    ref = W.copy()
    for k in range(10):
        dts = s.run(2, record_dt=True).cpu().numpy()
        ref = orc.run_dts(P, ref, dts, ug=ug)
        err = rel_linf(gpu_state(s), ref)
        assert err <= TOL, (k, err)
    _, _, odt = orc.cfl(P, ref)
    dt, _, _ = s.cfl_dt()
    assert ulps(dt, odt) <= DT_ULP


@pytest.mark.parametrize("bc,layout,cpl", [(0, 0, 2), (1, 1, 2), (0, 1, 1)])
def test_spray_maxent_trajectory(bc, layout, cpl):
    """The entropy-maximising closure (transport step, then the per-cell
    Newton source pass) against the oracle's, step after step; the oracle
    integrates the moments with a different, much finer rule."""
    nx, ny = 64, 48
    print(f"spray maxent trajectory bc={bc} layout={layout} cpl={cpl}", flush=True)
    W, ug = inputs.spray_state(nx, ny, 2)
    pre = inputs.SPRAY_2048.replace(nx=nx, ny=ny, npart_x=4, npart_y=4, bc=bc)
    p = params_from(pre, layout=layout, closure=_lib.FVM_CLOSURE_MAXENT)
    s = Solver(p, ug=ug)
    s.set_cells_per_lane(cpl)
    s.set_state(W)
    P = oparams(p)
    P.closure = 1
    ref = W.copy()
    for k in range(6):
        dts = s.run(1, record_dt=True).cpu().numpy()
        ref = orc.run_dts(P, ref, dts, ug=ug)
        got = gpu_state(s)
        assert np.all(np.isfinite(got)), k
        err = rel_linf(got, ref)
        assert err <= TOL, (k, err)
    _, _, odt = orc.cfl(P, ref)
    dt, _, _ = s.cfl_dt()
    assert ulps(dt, odt) <= DT_ULP
    assert s.sync() == 0


@pytest.mark.parametrize("chunk", [1, 6])
def test_spray_maxent_warm_start_matches_oracle(chunk):
    """Newton restarting from each cell's kept multipliers (one step per
    call, or six steps in one graph) reaches the oracle's cold-start result
    within the parity tolerance; setting a new state forgets them."""
    nx, ny = 64, 48
    print(f"spray maxent warm start chunk={chunk}", flush=True)
    W, ug = inputs.spray_state(nx, ny, 7)
    pre = inputs.SPRAY_2048.replace(nx=nx, ny=ny, npart_x=4, npart_y=4)
    p = params_from(pre, closure=_lib.FVM_CLOSURE_MAXENT)
    s = Solver(p, ug=ug)
    s.keep_closure_multipliers()
    P = oparams(p)
    P.closure = 1
    for rep in range(2):  # the second pass starts over from a new state
        s.set_state(W)
        dts = np.concatenate([s.run(chunk, record_dt=True).cpu().numpy()
                              for _ in range(6 // chunk)])
        ref = orc.run_dts(P, W, dts, ug=ug)
        err = rel_linf(gpu_state(s), ref)
        assert err <= TOL, (rep, err)
    assert s.sync() == 0


def test_spray_maxent_fixed_dt_and_cfl_check():
    """The entropy-closure spray under the paper's fixed-dt policy: explicit
    steps and a checked fixed-dt run match the oracle's fixed-dt steps; a dt
    that fails the check leaves the state unchanged (neither the transport
    nor the source pass moves it) and reports FVM_ECFL."""
    nx, ny = 48, 40
    print("spray maxent fixed dt", flush=True)
    W, ug = inputs.spray_state(nx, ny, 5)
    pre = inputs.SPRAY_2048.replace(nx=nx, ny=ny, npart_x=2, npart_y=2, bc=1)
    p = params_from(pre, closure=_lib.FVM_CLOSURE_MAXENT)
    s = Solver(p, ug=ug)
    s.set_state(W)
    P = oparams(p)
    P.closure = 1
    dt, sx, sy = s.cfl_dt()
    lim = min(1.0 / nx, 1.0 / ny) / max(sx, sy)
    s.step(0.5 * lim)
    s.run_fixed(3, 0.5 * lim)
    assert s.sync() == 0
    ref = W.copy()
    for _ in range(4):
        rc, ref = orc.step_fixed(P, ref, 0.5 * lim, ug=ug)
        assert rc == 0
    assert rel_linf(gpu_state(s), ref) <= TOL
    before = gpu_state(s)
    s.run_fixed(2, 8.0 * lim)
    assert s.sync() == _lib.FVM_ECFL
    assert np.array_equal(gpu_state(s), before)


def test_spray_maxent_differs_from_lognormal_only_in_evaporation():
    """With K = 0 the closure is never used: both closures give the same
    state bit for bit."""
    n = 64
    W, ug = inputs.spray_state(n, n, 4)
    out = []
    for closure in (_lib.FVM_CLOSURE_LOGNORMAL, _lib.FVM_CLOSURE_MAXENT):
        pre = inputs.SPRAY_2048.replace(nx=n, ny=n, npart_x=1, npart_y=1, K=0.0)
        s = Solver(params_from(pre, closure=closure), ug=ug)
        s.set_state(W)
        s.run(3)
        out.append(gpu_state(s))
    assert np.array_equal(out[0], out[1])


# ---------------------------------------------------------------------------
# invariance: bit-for-bit across subdomains, tiles and launch forms
# ---------------------------------------------------------------------------

def test_decomposition_invariance_bitwise():
    nx, ny = 250, 120
    W = inputs.riemann_state(nx, ny, 9)
    outs = []
    for (npx, npy, rows, wpb, cpl) in [(1, 1, 64, 4, 1), (5, 4, 1, 1, 1), (10, 8, 7, 2, 1),
                                       (2, 2, 120, 8, 1), (25, 3, 33, 4, 1), (1, 1, 64, 4, 2),
                                       (5, 4, 1, 1, 2), (10, 8, 7, 2, 2), (2, 2, 3, 8, 2)]:
        p = params_from(model=1, bc=1, nx=nx, ny=ny, npart_x=npx, npart_y=npy)
        s = Solver(p)
        s.set_tiling(rows, wpb)
        assert s.set_cells_per_lane(cpl) == cpl
        s.set_state(W)
        s.run(7)
        outs.append(gpu_state(s))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("model", [0, 1, 2])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("nx", [1, 2, 127, 128, 129, 300, 389])
def test_lane_layouts_agree_bitwise(model, bc, nx):
    """One and two cells per lane, odd and even widths, strips that end
    inside or at the end of the grid: bit-for-bit the same steps."""
    ny = 37
    ld = nx + (nx % 2)
    ug = None
    if model == 0:
        W = inputs.advection_state(nx, ny, nx)
        kw = dict(ax=0.6, ay=-0.8)
    elif model == 1:
        W = inputs.riemann_state(nx, ny, nx)
        kw = {}
    else:
        W, ug = inputs.spray_state(nx, ny, nx)
        kw = dict(cfl=0.9)
    res = []
    for layout in (_lib.FVM_LAYOUT_PLANES, _lib.FVM_LAYOUT_ROWS):
        for cpl in (1, 2):
            p = params_from(model=model, bc=bc, nx=nx, ny=ny, ld=ld, layout=layout, **kw)
            s = Solver(p, ug=ug)
            assert s.set_cells_per_lane(cpl) == cpl
            s.set_state(W)
            d = s.run(5, record_dt=True).cpu().numpy()
            res.append((gpu_state(s), d))
    for r in res[1:]:
        assert np.array_equal(res[0][0], r[0]) and np.array_equal(res[0][1], r[1])
    ref, odts = orc.run(oparams(params_from(model=model, bc=bc, nx=nx, ny=ny, **kw)), W, 5, ug=ug)
    assert rel_linf(res[1][0], ref) <= TOL


def _dirichlet_case(model, nx, ny, seed):
    """State, gas velocity, extra parameters and ghost states (west, east,
    south, north) of a Dirichlet test case."""
    ug = None
    if model == 0:
        W = inputs.advection_state(nx, ny, seed)
        kw = dict(ax=0.6, ay=-0.8)
        ghost = np.array([[0.9], [-0.4], [0.2], [1.3]])
    elif model == 1:
        W = inputs.riemann_state(nx, ny, seed)
        kw = {}
        ghost = np.stack([inputs.conservative_from_primitive(*q) for q in
                          [(0.6, 0.2, -0.1, 0.5), (1.1, -0.3, 0.05, 0.9),
                           (0.8, 0.1, 0.25, 0.4), (0.4, -0.05, -0.2, 0.7)]])
    else:
        W, ug = inputs.spray_state(nx, ny, seed)
        kw = dict(cfl=0.9)
        # states of the same family, taken from a larger field
        Wg, _ = inputs.spray_state(8, 8, seed + 1)
        ghost = np.stack([Wg[:, 1, 2], Wg[:, 5, 6], Wg[:, 3, 0], Wg[:, 7, 4]])
    return W, ug, kw, ghost


@pytest.mark.parametrize("model", [0, 1, 2])
@pytest.mark.parametrize("nx", [1, 64, 127, 128, 129, 300])
def test_dirichlet_matches_oracle_in_every_layout(model, nx):
    """Dirichlet boundaries: both storage layouts and both lane layouts give
    bitwise the same 5 adaptive steps, which are the oracle's."""
    ny = 37
    ld = nx + (nx % 2)
    W, ug, kw, ghost = _dirichlet_case(model, nx, ny, nx + 3)
    res = []
    for layout in (_lib.FVM_LAYOUT_PLANES, _lib.FVM_LAYOUT_ROWS):
        for cpl in (1, 2):
            p = params_from(model=model, bc=_lib.FVM_DIRICHLET, nx=nx, ny=ny, ld=ld,
                            layout=layout, **kw)
            s = Solver(p, ug=ug)
            s.set_boundary_states(ghost)
            assert s.set_cells_per_lane(cpl) == cpl
            s.set_state(W)
            d = s.run(5, record_dt=True).cpu().numpy()
            assert s.sync() == 0
            res.append((gpu_state(s), d))
    for r in res[1:]:
        assert np.array_equal(res[0][0], r[0]) and np.array_equal(res[0][1], r[1])
    P = oparams(params_from(model=model, bc=_lib.FVM_DIRICHLET, nx=nx, ny=ny, **kw), ghost)
    ref = orc.run_dts(P, W, res[0][1], ug=ug)
    assert rel_linf(res[0][0], ref) <= TOL
    _, odts = orc.run(P, W, 1, ug=ug)
    assert ulps(res[0][1][0], odts[0]) <= DT_ULP


def test_dirichlet_ghost_states_change_between_runs():
    """New ghost states apply to the next run (cached launch graphs are
    rebuilt) and to the adjoint step."""
    n = 96
    W, _, _, ghost = _dirichlet_case(1, n, n, 5)
    p = params_from(model=1, bc=_lib.FVM_DIRICHLET, nx=n, ny=n, npart_x=2, npart_y=3)
    s = Solver(p)
    s.set_boundary_states(ghost)
    s.set_state(W)
    d1 = s.run(4, record_dt=True).cpu().numpy()
    mid = gpu_state(s)
    ghost2 = ghost[::-1].copy()
    s.set_boundary_states(ghost2)
    d2 = s.run(4, record_dt=True).cpu().numpy()
    got = gpu_state(s)
    ref = orc.run_dts(oparams(p, ghost), W, d1)
    assert rel_linf(mid, ref) <= TOL
    ref = orc.run_dts(oparams(p, ghost2), ref, d2)
    assert rel_linf(got, ref) <= TOL
    lam = np.random.default_rng(3).standard_normal(W.shape)
    adj = s.adjoint_step(W, 1e-4, lam)
    torch.cuda.synchronize()
    oref = orc.adjoint_step(oparams(p, ghost2), W, 1e-4, lam)
    assert rel_linf(adj[:, :, :n].cpu().numpy(), oref) <= TOL


@pytest.mark.parametrize("model", [1, 2])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("layout,cpl", [(0, 2), (1, 2), (1, 1)])
def test_slabs_with_halo_rows_equal_the_whole_grid(model, bc, layout, cpl):
    """The one-GPU share of the slab decomposition: a grid cut into 4 slabs
    of whole rows, each stepped on its own with the neighbours' boundary
    rows copied into its halo buffers before every step (periodic: the
    first and last slabs exchange too; transmissive: those sides keep the
    boundary rule), gives bit for bit the whole-grid steps with the same
    dts."""
    nx, ny, k = 260, 96, 4
    ld = nx + (nx % 2)
    h = ny // k
    if model == 1:
        W = inputs.riemann_state(nx, ny, 21)
        ug, kw = None, {}
    else:
        W, ug = inputs.spray_state(nx, ny, 21)
        kw = dict(cfl=0.9)
    full = Solver(params_from(model=model, bc=bc, nx=nx, ny=ny, ld=ld, layout=layout, **kw),
                  ug=ug)
    assert full.set_cells_per_lane(cpl) == cpl
    full.set_state(W)
    dts = full.run(4, record_dt=True).cpu().numpy()
    ref = gpu_state(full)
    slabs, halos = [], []
    for q in range(k):
        # the slab's own gas velocity and physical extent (dy unchanged)
        p = params_from(model=model, bc=bc, nx=nx, ny=h, ld=ld, layout=layout, ly=h / ny, **kw)
        sl = Solver(p, ug=None if ug is None else ug[:, q * h:(q + 1) * h])
        assert sl.set_cells_per_lane(cpl) == cpl
        sl.set_state(W[:, q * h:(q + 1) * h])
        south = torch.zeros((sl.nv, ld), dtype=torch.float64, device="cuda")
        north = torch.zeros_like(south)
        has_s = q > 0 or bc == 0
        has_n = q < k - 1 or bc == 0
        sl.set_halo_rows(south if has_s else None, north if has_n else None)
        slabs.append(sl)
        halos.append((south, north, has_s, has_n))
    for dt in dts:
        cur = [sl.current() for sl in slabs]
        for q, (south, north, has_s, has_n) in enumerate(halos):
            if has_s:
                south.copy_(cur[(q - 1) % k][:, -1, :])
            if has_n:
                north.copy_(cur[(q + 1) % k][:, 0, :])
        for sl in slabs:
            sl.run_dts([dt])
    got = np.concatenate([gpu_state(sl) for sl in slabs], axis=1)
    assert np.array_equal(got, ref)


def _random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    model = int(rng.integers(0, 3))
    bc = int(rng.integers(0, 3))
    nx = int(rng.choice([1, 2, 3, 63, 64, 65, 127, 128, 129, 191, 255, 256, 257, 300, 513]))
    ny = int(rng.choice([1, 2, 5, 17, 33, 64, 100]))
    ld = nx + int(rng.integers(0, 9))
    layout = int(rng.integers(0, 2))
    cpl = int(rng.choice([1, 2]))
    rows = int(rng.choice([1, 2, 3, 8, 16, 64, 128]))
    wpb = int(rng.choice([1, 2, 4, 8]))
    npx = int(rng.choice([d for d in (1, 2, 3, 4) if nx % d == 0]))
    npy = int(rng.choice([d for d in (1, 2, 3, 4) if ny % d == 0]))
    return model, bc, nx, ny, ld, layout, cpl, rows, wpb, npx, npy


@pytest.mark.parametrize("seed", range(12))
def test_random_maxent_configurations_match_oracle(seed):
    """The entropy-closure spray over seeded random sizes, pitches, storage
    and lane layouts, tile shapes, subdomain counts, boundaries, evaporation
    rates and Newton starts (cold, or kept multipliers): 3 adaptive steps
    against the oracle, or the same status where the draw is degenerate."""
    rng = np.random.default_rng(5000 + seed)
    bc = int(rng.integers(0, 2))
    nx = int(rng.choice([1, 2, 3, 17, 64, 65, 128, 129]))
    ny = int(rng.choice([1, 2, 5, 17, 33]))
    ld = nx + int(rng.integers(0, 5))
    layout = int(rng.integers(0, 2))
    cpl = int(rng.choice([1, 2]))
    rows = int(rng.choice([1, 3, 8, 32]))
    wpb = int(rng.choice([1, 2, 4]))
    npx = int(rng.choice([d for d in (1, 2, 4) if nx % d == 0]))
    npy = int(rng.choice([d for d in (1, 2, 4) if ny % d == 0]))
    K = float(rng.choice([0.0, 0.2, 1.0]))
    warm = bool(rng.integers(0, 2))
    print(f"random maxent case {seed}: bc={bc} {nx}x{ny} ld={ld} layout={layout} cpl={cpl} "
          f"tile={rows}x{wpb} parts={npx}x{npy} K={K} warm={warm}", flush=True)
    W, ug = inputs.spray_state(nx, ny, 300 + seed)
    pre = inputs.SPRAY_2048.replace(nx=nx, ny=ny, npart_x=npx, npart_y=npy, bc=bc, K=K)
    p = params_from(pre, ld=ld, layout=layout, closure=_lib.FVM_CLOSURE_MAXENT)
    s = Solver(p, ug=ug)
    s.set_cells_per_lane(cpl)
    s.set_tiling(rows, wpb)
    if warm:
        s.keep_closure_multipliers()
    s.set_state(W)
    dts = s.run(3, record_dt=True).cpu().numpy()
    P = oparams(p)
    P.closure = 1
    orc_rc, _, _ = orc.run(P, W, 3, ug=ug, return_status=True)
    if orc_rc != 0:
        assert s.sync() == orc_rc
        return
    assert s.sync() == 0
    ref = orc.run_dts(P, W, dts, ug=ug)
    assert rel_linf(gpu_state(s), ref) <= TOL


@pytest.mark.parametrize("seed", range(40))
def test_random_configurations_match_oracle(seed):
    """Seeded random model, boundary, size, pitch, storage and lane layout,
    tile shape and subdomain counts: 3 adaptive steps against the oracle."""
    model, bc, nx, ny, ld, layout, cpl, rows, wpb, npx, npy = _random_case(seed)
    print(f"random case {seed}: model={model} bc={bc} {nx}x{ny} ld={ld} layout={layout} "
          f"cpl={cpl} tile={rows}x{wpb} parts={npx}x{npy}", flush=True)
    W, ug, kw, ghost = _dirichlet_case(model, nx, ny, seed)
    p = params_from(model=model, bc=bc, nx=nx, ny=ny, ld=ld, layout=layout, npart_x=npx,
                    npart_y=npy, **kw)
    s = Solver(p, ug=ug)
    if bc == _lib.FVM_DIRICHLET:
        s.set_boundary_states(ghost)
    got_cpl = s.set_cells_per_lane(cpl)
    assert got_cpl == (cpl if ld % 2 == 0 else 1)
    s.set_tiling(rows, wpb)
    s.set_state(W)
    dts = s.run(3, record_dt=True).cpu().numpy()
    P = oparams(p, ghost if bc == _lib.FVM_DIRICHLET else None)
    orc_rc, _, _ = orc.run(P, W, 3, ug=ug, return_status=True)
    if orc_rc != 0:
        # degenerate draws (e.g. a 2x1 spray grid whose CFL step lets the
        # source drive a moment negative): the same status on both sides
        assert s.sync() == orc_rc
        return
    assert s.sync() == 0
    got = gpu_state(s)
    ref = orc.run_dts(P, W, dts, ug=ug)
    assert rel_linf(got, ref) <= TOL
    _, odts = orc.run(P, W, 1, ug=ug)
    assert ulps(dts[0], odts[0]) <= DT_ULP


def test_pitch_padding_is_untouched():
    nx, ny, ld = 70, 33, 96
    W = inputs.riemann_state(nx, ny, 2)
    p = params_from(model=1, bc=0, nx=nx, ny=ny, ld=ld)
    s = Solver(p)
    s.wa.fill_(12345.0)
    s.wb.fill_(-777.0)
    s.set_state(W)
    s.run(3)
    torch.cuda.synchronize()
    cur = s.current().cpu().numpy()
    assert np.all(cur[:, :, nx:] == -777.0)
    ref, _ = orc.run(oparams(p), W, 3)
    assert rel_linf(cur[:, :, :nx], ref) <= TOL


def test_row_layout_addresses():
    """Row-interleaved storage: each variable's row j sits at (j * nVar + v)
    * ld, the padding columns stay untouched, and the result is the
    oracle's."""
    nx, ny, ld = 70, 33, 96
    W = inputs.riemann_state(nx, ny, 2)
    p = params_from(model=1, bc=0, nx=nx, ny=ny, ld=ld, layout=_lib.FVM_LAYOUT_ROWS)
    s = Solver(p)
    assert tuple(s.wa.shape) == (ny, 4, ld)
    s.wa.fill_(12345.0)
    s.wb.fill_(-777.0)
    s.set_state(W)
    s.run(3)
    torch.cuda.synchronize()
    raw = s.current_storage().cpu().numpy()
    assert np.all(raw[:, :, nx:] == -777.0)
    ref, _ = orc.run(oparams(p), W, 3)
    assert rel_linf(np.transpose(raw[:, :, :nx], (1, 0, 2)), ref) <= TOL


# ---------------------------------------------------------------------------
# fixed-dt steps, status and errors
# ---------------------------------------------------------------------------

def test_fixed_dt_step_and_cfl_check():
    n = 64
    W = inputs.riemann_state(n, n, 1)
    p = params_from(model=1, bc=1, nx=n, ny=n)
    s = Solver(p)
    s.set_state(W)
    dt, sx, sy = s.cfl_dt()
    P = oparams(p)
    osx, osy, odt = orc.cfl(P, W)
    assert ulps(sx, osx) <= DT_ULP and ulps(sy, osy) <= DT_ULP and ulps(dt, odt) <= DT_ULP
    lim = (1.0 / n) / max(sx, sy)
    s.step(0.999 * lim)
    rc, ref = orc.step_fixed(P, W, 0.999 * lim)
    assert rc == 0 and s.sync() == 0
    assert rel_linf(gpu_state(s), ref) <= TOL
    before = gpu_state(s)
    s.step(10.0 * lim)
    assert s.status(clear=True) == _lib.FVM_ECFL
    assert np.array_equal(gpu_state(s), before)
    assert s.status() == 0


def test_fixed_dt_run_checks_every_step():
    """fvm_run_fixed: every step checked against the CFL condition, each
    step the oracle's fixed-dt step; a run whose dt fails the check leaves
    the state unchanged and reports FVM_ECFL."""
    nx, ny = 96, 80
    W = inputs.riemann_state(nx, ny, 4)
    p = params_from(model=1, bc=1, nx=nx, ny=ny, npart_x=4, npart_y=2)
    P = oparams(p)
    s = Solver(p)
    s.set_state(W)
    dt, sx, sy = s.cfl_dt()
    lim = min(1.0 / nx, 1.0 / ny) / max(sx, sy)
    s.run_fixed(12, 0.5 * lim)
    assert s.sync() == 0
    ref = W.copy()
    for _ in range(12):
        rc, ref = orc.step_fixed(P, ref, 0.5 * lim)
        assert rc == 0
    assert rel_linf(gpu_state(s), ref) <= TOL
    before = gpu_state(s)
    s.run_fixed(3, 4.0 * lim)
    assert s.sync() == _lib.FVM_ECFL
    assert np.array_equal(gpu_state(s), before)
    rc, _ = orc.step_fixed(P, ref, 4.0 * lim)
    assert rc == orc.ECFL


@pytest.mark.parametrize("case", ["cosine", "vortex"])
def test_paper_test_cases_converge_on_gpu(case):
    """The paper's two analytic Euler cases (Sec. 5.1) run on the GPU with the
    paper's fixed-dt policy to T = 0.2: the state at 128^2 is the oracle's,
    and the L1 and L2 errors against the exact solution fall with the order
    the paper prints (about 0.95, Sec. 5.1.3)."""
    import json
    paper = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_numbers.json")))
    slope_paper = paper["convergence_slope"]["value"]
    fn = {"cosine": inputs.localized_cosine_primitives,
          "vortex": inputs.isentropic_vortex_primitives}[case]
    T = 0.2
    errs = []
    for n in (64, 128, 256, 512):
        W0 = inputs.conservative_from_primitive(*fn(n, n, 0.0))
        p = params_from(model=1, bc=0, nx=n, ny=n, npart_x=2, npart_y=2, cfl=0.4)
        s = Solver(p)
        s.set_state(W0)
        dt, _, _ = s.cfl_dt()
        steps = int(math.ceil(T / dt))
        s.run_fixed(steps, T / steps)
        assert s.sync() == 0
        W = gpu_state(s)
        if n == 128:
            ref = orc.run_dts(oparams(p), W0, [T / steps] * steps)
            print(f"{case} 128^2, {steps} fixed steps: rel Linf vs oracle "
                  f"{rel_linf(W, ref):.2e}", flush=True)
            assert rel_linf(W, ref) <= TOL, rel_linf(W, ref)  # measured 7e-16
        e = W[0] - fn(n, n, T)[0]
        errs.append((np.mean(np.abs(e)), math.sqrt(np.mean(e * e))))
    print(f"{case} errors {errs}", flush=True)
    for k in range(2):
        for a, b in ((1, 2), (2, 3)):
            slope = math.log2(errs[a][k] / errs[b][k])
            assert abs(slope - slope_paper) < 0.15, (case, k, a, slope, errs)


@pytest.mark.parametrize("what", ["nan", "rho", "p"])
def test_nonfinite_state_is_reported(what):
    n = 32
    W = inputs.riemann_state(n, n, 1)
    if what == "nan":
        W[2, 3, 4] = np.nan
    elif what == "rho":
        W[0, 3, 4] = -0.1
    else:
        W[3, 3, 4] = 0.0
    s = Solver(params_from(model=1, bc=1, nx=n, ny=n))
    s.set_state(W)
    with pytest.raises(_lib.FvmError) as e:
        s.cfl_dt()
    assert e.value.code == _lib.FVM_ENONFINITE


def test_invalid_arguments_are_rejected():
    L = _lib.lib()
    bad = params_from(model=1, nx=10, ny=10, npart_x=3)
    assert L.fvm_validate(bad) == _lib.FVM_EINVAL
    s = Solver(params_from(model=1, nx=16, ny=16))
    assert L.fvm_step(s.h, -1.0) == _lib.FVM_EINVAL
    assert L.fvm_step(s.h, float("nan")) == _lib.FVM_EINVAL
    assert L.fvm_run(s.h, -3, None) == _lib.FVM_EINVAL
    assert L.fvm_set_tiling(s.h, 0, 3) == _lib.FVM_EINVAL


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

def _batch_case(sizes, seed=100):
    plist = [params_from(model=1, bc=1, nx=n, ny=n, cfl=0.45) for n in sizes]
    states = [inputs.riemann_state(n, n, seed + k) for k, n in enumerate(sizes)]
    return plist, states


# (model, bc, nx, ny); Euler 48 x 48 fills the LDS exactly (2 x 4 x 2304 =
# 18432 doubles), 49 x 48 just does not (step launches either way)
@pytest.mark.parametrize("case", [(0, 0, 64, 64), (1, 0, 40, 33), (1, 1, 40, 33), (1, 2, 47, 48),
                                  (1, 1, 48, 48), (1, 1, 49, 48), (2, 0, 30, 20), (2, 1, 31, 17),
                                  (2, 2, 25, 25), (1, 1, 1, 1)])
def test_resident_runs_equal_step_launches(case):
    """fvm_run on a grid that fits in one workgroup's LDS runs in one launch:
    the states (both ping-pong buffers), the logged dts and the next dt are
    bitwise those of one launch per step, and match the oracle."""
    model, bc, nx, ny = case
    ug = None
    if model == 0:
        p = params_from(inputs.ADVECTION_64, nx=nx, ny=ny, npart_x=1, npart_y=1)
        W = inputs.advection_state(nx, ny, 4)
    elif model == 1:
        p = params_from(model=1, bc=bc, nx=nx, ny=ny, cfl=0.45)
        W = inputs.riemann_state(nx, ny, 4)
    else:
        p = params_from(inputs.SPRAY_2048, nx=nx, ny=ny, npart_x=1, npart_y=1, bc=bc, cfl=0.05)
        W, ug = inputs.spray_state(nx, ny, 4)
    ghost = None
    if bc == 2:
        ghost = np.stack([W[:, 0, 0], W[:, -1, -1], W[:, 0, -1], W[:, -1, 0]])
    out = []
    for resident in (True, False):
        s = Solver(p, ug=ug)
        if ghost is not None:
            s.set_boundary_states(ghost)
        s.set_resident_runs(resident)
        s.set_state(W)
        d1 = s.run(9, record_dt=True).cpu().numpy()
        d2 = s.run(4, record_dt=True).cpu().numpy()
        torch.cuda.synchronize()
        cur = s.current_storage().clone()
        other = (s.wb if s.current_storage() is s.wa else s.wa).clone()
        out.append((np.concatenate([d1, d2]), cur.cpu().numpy(), other.cpu().numpy(),
                    s.cfl_dt()[0], s.sync()))
    (da, ca, oa, na, sa), (db, cb, ob, nb, sb) = out
    assert sa == sb
    assert np.array_equal(da, db, equal_nan=True)
    assert np.array_equal(ca, cb, equal_nan=True) and np.array_equal(oa, ob, equal_nan=True)
    assert na == nb or (math.isnan(na) and math.isnan(nb))
    if sa == 0:
        P = oparams(p, ghost)
        ref = orc.run_dts(P, W, da, ug=ug)
        s = Solver(p, ug=ug)
        if ghost is not None:
            s.set_boundary_states(ghost)
        s.set_state(W)
        s.run(13)
        assert rel_linf(gpu_state(s), ref) <= TOL


def test_batch_equals_single_grid_runs():
    sizes = [64, 65, 97, 130, 200, 71, 64, 257]
    plist, states = _batch_case(sizes)
    b = Batch(plist)
    b.set_states(states)
    dts = b.run(9, record_dt=True).cpu().numpy()
    got = [x.cpu().numpy() for x in b.states()]
    b2 = Batch(plist)
    b2.set_states(states)
    dts2 = b2.run(9, record_dt=True, per_grid=True).cpu().numpy()
    got2 = [x.cpu().numpy() for x in b2.states()]
    b3 = Batch(plist)  # one workgroup per item instead of persistent workgroups
    b3.set_schedule(False)
    b3.set_tiling(16, 4)
    b3.set_states(states)
    dts3 = b3.run(9, record_dt=True).cpu().numpy()
    got3 = [x.cpu().numpy() for x in b3.states()]
    b4 = Batch(plist)  # row blocks fitted to whole workgroups
    b4.set_schedule(True, fit_blocks=True)
    b4.set_tiling(32, 8)
    b4.set_states(states)
    dts4 = b4.run(9, record_dt=True).cpu().numpy()
    got4 = [x.cpu().numpy() for x in b4.states()]
    narrow = []  # one cell per lane on every grid, persistent and grouped
    for persistent, tiling in ((True, (48, 4)), (False, (8, 2))):
        b5 = Batch(plist)
        b5.set_layout(1)
        b5.set_schedule(persistent)
        b5.set_tiling(*tiling)
        b5.set_states(states)
        narrow.append((b5.run(9, record_dt=True).cpu().numpy(),
                       [x.cpu().numpy() for x in b5.states()]))
    assert np.array_equal(dts3, dts) and np.array_equal(dts4, dts)
    for k in range(len(sizes)):
        assert np.array_equal(got3[k], got[k]), k
        assert np.array_equal(got4[k], got[k]), k
    for d5, got5 in narrow:
        assert np.array_equal(d5, dts)
        for k in range(len(sizes)):
            assert np.array_equal(got5[k], got[k]), k
    for k, n in enumerate(sizes):
        s = Solver(plist[k])
        s.set_state(states[k])
        d1 = s.run(9, record_dt=True).cpu().numpy()
        one = gpu_state(s)
        assert np.array_equal(got[k], one), k
        assert np.array_equal(got2[k], one), k
        assert np.array_equal(dts[:, k], d1) and np.array_equal(dts2[:, k], d1)
    ref, odts = orc.run(oparams(plist[3]), states[3], 9)
    assert rel_linf(got[3], ref) <= TOL


def test_batch_row_layout_equals_planar():
    sizes = [64, 97, 130, 71, 257]
    plist, states = _batch_case(sizes, 3)
    rows = [params_from(model=p.model, bc=p.bc, nx=p.nx, ny=p.ny, ld=p.ld, cfl=p.cfl,
                        layout=_lib.FVM_LAYOUT_ROWS if k % 2 == 0 else _lib.FVM_LAYOUT_PLANES)
            for k, p in enumerate(plist)]
    out = []
    for pl in (plist, rows):
        b = Batch(pl)
        b.set_states(states)
        d = b.run(7, record_dt=True).cpu().numpy()
        out.append(([x.cpu().numpy() for x in b.states()], d))
    assert np.array_equal(out[0][1], out[1][1])
    for k in range(len(sizes)):
        assert np.array_equal(out[0][0][k], out[1][0][k]), k


def test_batch_workload_sample_parity():
    """Sizes drawn as in the 256-grid workload; a few grids checked against
    the oracle after 5 steps."""
    sizes = inputs.batch_sizes(24, 4)
    plist, states = _batch_case(sizes, 4)
    b = Batch(plist)
    b.set_states(states)
    b.run(5)
    got = b.states()
    for k in (0, 5, 11, 23):
        ref, _ = orc.run(oparams(plist[k]), states[k], 5)
        assert rel_linf(got[k].cpu().numpy(), ref) <= TOL, k


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("model", [0, 1])
def test_adjoint_step(model, bc):
    nx, ny = 133, 70
    W, _, kw, ghost = _dirichlet_case(model, nx, ny, 6)
    if model == 1:
        W = W + 0.01 * np.stack([inputs.gaussian_bumps(nx, ny, 40 + v) for v in range(4)])
    p = params_from(model=model, bc=bc, nx=nx, ny=ny, **kw)
    gh = ghost if bc == _lib.FVM_DIRICHLET else None
    lam = np.random.default_rng(7).standard_normal(W.shape)
    s = Solver(p)
    if gh is not None:
        s.set_boundary_states(gh)
    P = oparams(p, gh)
    _, _, dt = orc.cfl(P, W)
    got = s.adjoint_step(W, dt, lam)
    torch.cuda.synchronize()
    ref = orc.adjoint_step(P, W, dt, lam)
    assert rel_linf(got[:, :, :nx].cpu().numpy(), ref) <= TOL
    p.layout = _lib.FVM_LAYOUT_ROWS
    p.ld = nx + 3
    for cpl in (1, 2):
        sr = Solver(p)
        if gh is not None:
            sr.set_boundary_states(gh)
        sr.set_adjoint_tiling(0, 0, cpl)
        got_rows = sr.adjoint_step(W, dt, lam)
        torch.cuda.synchronize()
        assert np.array_equal(got_rows[:, :, :nx].cpu().numpy(),
                              got[:, :, :nx].cpu().numpy()), cpl


@pytest.mark.parametrize("cpl", [1, 2])
@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("nx", [1, 2, 62, 63, 64, 124, 127, 128, 129, 130, 257, 500, 1024])
def test_adjoint_step_covers_every_column(nx, bc, cpl):
    """The adjoint strips (62 columns with one cell per lane, 128 with two)
    tile the whole width at every default workgroup size, ragged last strips
    and periodic wrap included."""
    ny = 9
    print(f"adjoint widths nx={nx} bc={bc} cpl={cpl}", flush=True)
    W = inputs.riemann_state(nx, ny, 8) + 0.01 * np.stack(
        [inputs.gaussian_bumps(nx, ny, 50 + v) for v in range(4)])
    p = params_from(model=1, bc=bc, nx=nx, ny=ny, ld=nx + nx % 2)
    lam = np.random.default_rng(nx).standard_normal(W.shape)
    gh = _dirichlet_case(1, 1, 1, 0)[3] if bc == _lib.FVM_DIRICHLET else None
    P = oparams(p, gh)
    _, _, dt = orc.cfl(P, W)
    s = Solver(p)
    if gh is not None:
        s.set_boundary_states(gh)
    s.set_adjoint_tiling(0, 0, cpl)
    got = s.adjoint_step(W, dt, lam)
    torch.cuda.synchronize()
    ref = orc.adjoint_step(P, W, dt, lam)
    assert rel_linf(got[:, :, :nx].cpu().numpy(), ref) <= TOL


def test_adjoint_tiling_invariance_bitwise():
    """Tile shapes and both lane layouts give the same multipliers bit for
    bit (every face is evaluated once with the same arguments and each cell
    sums its shares in the same order)."""
    nx, ny = 300, 77
    W = inputs.riemann_state(nx, ny, 13)
    lam = np.random.default_rng(5).standard_normal(W.shape)
    outs = []
    for bc in (0, 1):
        p = params_from(model=1, bc=bc, nx=nx, ny=ny)
        s = Solver(p)
        _, _, dt = orc.cfl(oparams(p), W)
        res = []
        for rows, wpb, cpl in ((64, 4, 1), (1, 1, 1), (7, 2, 1), (33, 8, 1), (256, 4, 1),
                               (64, 4, 2), (1, 1, 2), (7, 2, 2), (33, 8, 2), (16, 4, 2)):
            s.set_adjoint_tiling(rows, wpb, cpl)
            res.append(s.adjoint_step(W, dt, lam).cpu().numpy())
        for r in res[1:]:
            assert np.array_equal(r, res[0]), bc
        outs.append(res[0])
    assert not np.array_equal(outs[0], outs[1])


def test_adjoint_tuner_on_caller_buffers():
    """fvm_autotune_adjoint times dt = 0 steps on the given buffers: the
    output buffer ends up holding the input multipliers bit for bit, the
    state is untouched, and the chosen tiling still gives the oracle's
    adjoint step."""
    nx, ny = 200, 72
    W = inputs.riemann_state(nx, ny, 21)
    p = params_from(model=1, bc=1, nx=nx, ny=ny, ld=nx, layout=_lib.FVM_LAYOUT_ROWS)
    s = Solver(p)
    Ws = s._as_state(W)
    lam = np.random.default_rng(21).standard_normal(W.shape)
    la = s._as_state(lam)
    lb = torch.full_like(la, 7.0)
    w_before = Ws.clone()
    s.autotune_adjoint(Ws, la, lb)
    torch.cuda.synchronize()
    assert torch.equal(lb, la) and torch.equal(Ws, w_before)
    P = oparams(p)
    _, _, dt = orc.cfl(P, W)
    got = s.adjoint_step(W, dt, lam)
    torch.cuda.synchronize()
    assert rel_linf(got[:, :, :nx].cpu().numpy(), orc.adjoint_step(P, W, dt, lam)) <= TOL


@pytest.mark.parametrize("model", [1, 2])
def test_forward_tuner_keeps_the_state_and_caches_its_choice(model, tmp_path):
    """fvm_autotune (dry runs, then the fastest candidates re-timed) leaves
    the state bit for bit, writes its choice to the cache, reads the same
    choice back, and the chosen tiling still steps like the oracle."""
    nx, ny = 200, 72
    if model == 1:
        W, ug = inputs.riemann_state(nx, ny, 5), None
        p = params_from(model=1, bc=1, nx=nx, ny=ny, ld=nx, layout=_lib.FVM_LAYOUT_ROWS)
    else:
        W, ug = inputs.spray_state(nx, ny, 5)
        p = params_from(inputs.SPRAY_2048, nx=nx, ny=ny, npart_x=1, npart_y=1, cfl=0.45,
                        layout=_lib.FVM_LAYOUT_ROWS)
    s = Solver(p, ug=ug)
    s.set_state(W)
    cache = str(tmp_path / "tune.txt")
    chosen = s.autotune(cache)
    assert np.array_equal(gpu_state(s), W)
    lines = open(cache).read().splitlines()
    assert lines and all(" | rows=" in x for x in lines)
    s2 = Solver(p, ug=ug)
    s2.set_state(W)
    assert s2.autotune(cache) == chosen
    assert open(cache).read().splitlines() == lines  # read, not re-tuned
    dts = s.run(3, record_dt=True).cpu().numpy()
    ref = orc.run_dts(oparams(p), W, dts, ug=ug)
    assert rel_linf(gpu_state(s), ref) <= TOL
    print(f"model {model}: tuned tiling {chosen}", flush=True)


def test_fvrun_gradient_matches_oracle_and_fd():
    n = 32
    W0 = inputs.riemann_state(n, n, 0)
    tgt = torch.tensor(inputs.adjoint_target_density(n, n, 0), device="cuda")
    p = params_from(model=1, bc=1, nx=n, ny=n)
    s = Solver(p)
    X = torch.tensor(W0, device="cuda", requires_grad=True)
    Y = fvrun(X, s, 30, 5)
    loss = 0.5 * ((Y[0] - tgt) ** 2).sum()
    loss.backward()
    g = X.grad.cpu().numpy()
    # the same gradient from row-interleaved storage
    pr = params_from(model=1, bc=1, nx=n, ny=n, ld=n + 2, layout=_lib.FVM_LAYOUT_ROWS)
    Xr = torch.tensor(W0, device="cuda", requires_grad=True)
    Yr = fvrun(Xr, Solver(pr), 30, 5)
    (0.5 * ((Yr[0] - tgt) ** 2).sum()).backward()
    assert torch.equal(Yr, Y) and np.array_equal(Xr.grad.cpu().numpy(), g)
    P = oparams(p)
    WN, odts = orc.run(P, W0, 30)
    lamN = np.zeros_like(W0)
    lamN[0] = WN[0] - inputs.adjoint_target_density(n, n, 0)
    gref = orc.adjoint_run(P, W0, odts, lamN)
    print(f"euler gradient 32^2 x 30 steps: rel Linf vs oracle {rel_linf(g, gref):.2e}",
          flush=True)
    assert rel_linf(g, gref) <= TOL  # measured 5e-16
    # central differences with the forward dts frozen
    def L(W):
        out = orc.run_dts(P, W, odts)
        return 0.5 * np.sum((out[0] - inputs.adjoint_target_density(n, n, 0)) ** 2)
    rng = np.random.default_rng(11)
    for _ in range(6):
        v = rng.standard_normal(W0.shape)
        eps = 1e-6
        fd = (L(W0 + eps * v) - L(W0 - eps * v)) / (2 * eps)
        assert abs(float(np.sum(g * v)) - fd) <= 1e-6 * max(1.0, abs(fd))


def test_fvrun_gradient_with_dirichlet_boundaries():
    """The differentiable run with prescribed ghost states: the gradient the
    checkpointed GPU adjoint returns equals the oracle's adjoint run."""
    n = 40
    W0, _, _, ghost = _dirichlet_case(1, n, n, 9)
    tgt = torch.tensor(inputs.adjoint_target_density(n, n, 9), device="cuda")
    p = params_from(model=1, bc=_lib.FVM_DIRICHLET, nx=n, ny=n)
    s = Solver(p)
    s.set_boundary_states(ghost)
    X = torch.tensor(W0, device="cuda", requires_grad=True)
    Y = fvrun(X, s, 20, 4)
    (0.5 * ((Y[0] - tgt) ** 2).sum()).backward()
    g = X.grad.cpu().numpy()
    P = oparams(p, ghost)
    WN, odts = orc.run(P, W0, 20)
    lamN = np.zeros_like(W0)
    lamN[0] = WN[0] - inputs.adjoint_target_density(n, n, 9)
    e = rel_linf(g, orc.adjoint_run(P, W0, odts, lamN))
    print(f"dirichlet gradient 40^2 x 20 steps: rel Linf vs oracle {e:.2e}", flush=True)
    assert e <= TOL  # measured 5.5e-16


def _spray_adjoint_case(nx, ny, seed):
    """A spray state whose velocity differs from the gas velocity (the drag
    acts) and whose moments are not exactly lognormal."""
    W, ug = inputs.spray_state(nx, ny, seed)
    rng = np.random.default_rng(seed + 50)
    W = W.copy()
    W[:4] *= 1.0 + 0.02 * rng.standard_normal((4, ny, nx))
    W[4:] += 0.1 * W[2] * rng.standard_normal((2, ny, nx))
    return W, ug


def _spray_ghosts():
    g = []
    for k, (u, v) in enumerate([(0.3, -0.2), (-0.4, 0.1), (0.2, 0.35), (-0.1, -0.3)]):
        m = inputs.lognormal_moments(1.0 + 0.1 * k, math.log(0.2), 0.3)
        g.append([m[0], m[1], m[2], m[3], m[2] * u, m[2] * v])
    return np.array(g)


@pytest.mark.parametrize("theta", [0.1, math.inf])
@pytest.mark.parametrize("bc", [0, 1, 2])
def test_spray_adjoint_step(bc, theta):
    """One spray adjoint step (transport and lognormal-closure source) against
    the oracle; the row-interleaved layout with a padded pitch gives the same
    multipliers bit for bit."""
    nx, ny = 133, 70
    print(f"spray adjoint bc={bc} theta={theta}", flush=True)
    W, ug = _spray_adjoint_case(nx, ny, 3)
    gh = _spray_ghosts() if bc == _lib.FVM_DIRICHLET else None
    p = params_from(model=2, bc=bc, nx=nx, ny=ny, K=0.7, theta=theta, cfl=0.9)
    lam = np.random.default_rng(9).standard_normal(W.shape)
    P = oparams(p, gh)
    _, _, dt = orc.cfl(P, W)
    s = Solver(p, ug=ug)
    if gh is not None:
        s.set_boundary_states(gh)
    got = s.adjoint_step(W, dt, lam)
    torch.cuda.synchronize()
    ref = orc.adjoint_step(P, W, dt, lam, ug)
    assert rel_linf(got[:, :, :nx].cpu().numpy(), ref) <= TOL
    p.layout = _lib.FVM_LAYOUT_ROWS
    p.ld = nx + 3
    sr = Solver(p, ug=ug)
    if gh is not None:
        sr.set_boundary_states(gh)
    got_rows = sr.adjoint_step(W, dt, lam)
    torch.cuda.synchronize()
    assert np.array_equal(got_rows[:, :, :nx].cpu().numpy(), got[:, :, :nx].cpu().numpy())


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 6), (2, 5), (63, 3), (64, 4), (65, 9),
                                   (129, 7), (300, 2)])
def test_spray_adjoint_covers_every_cell(nx, ny, bc):
    """The spray adjoint's cell tiles cover every cell of ragged grids,
    periodic wrap onto the cell itself (nx = 1) included."""
    print(f"spray adjoint cells nx={nx} ny={ny} bc={bc}", flush=True)
    W, ug = _spray_adjoint_case(nx, ny, nx + ny)
    gh = _spray_ghosts() if bc == _lib.FVM_DIRICHLET else None
    p = params_from(model=2, bc=bc, nx=nx, ny=ny, ld=nx + 1, K=0.7, cfl=0.9)
    lam = np.random.default_rng(nx).standard_normal(W.shape)
    P = oparams(p, gh)
    dt = 0.3 / max(nx, ny)
    s = Solver(p, ug=ug)
    if gh is not None:
        s.set_boundary_states(gh)
    got = s.adjoint_step(W, dt, lam)
    torch.cuda.synchronize()
    ref = orc.adjoint_step(P, W, dt, lam, ug)
    assert rel_linf(got[:, :, :nx].cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_fvrun_spray_gradient(bc):
    """The differentiable spray run: the checkpointed GPU adjoint (forward
    recomputation with the fused source, then the spray adjoint steps)
    equals the oracle's adjoint run, and central differences of the oracle's
    forward steps agree with it."""
    n = 40
    print(f"spray fvrun gradient bc={bc}", flush=True)
    W0, ug = _spray_adjoint_case(n, n, 12)
    gh = _spray_ghosts() if bc == _lib.FVM_DIRICHLET else None
    p = params_from(model=2, bc=bc, nx=n, ny=n, K=0.5, cfl=0.5)
    s = Solver(p, ug=ug)
    if gh is not None:
        s.set_boundary_states(gh)
    tgt_np = 0.9 * W0[0]
    tgt = torch.tensor(tgt_np, device="cuda")
    X = torch.tensor(W0, device="cuda", requires_grad=True)
    Y = fvrun(X, s, 12, 4)
    (0.5 * ((Y[0] - tgt) ** 2).sum()).backward()
    g = X.grad.cpu().numpy()
    # the same gradient, bit for bit, from row-interleaved storage with a padded pitch
    pr = params_from(model=2, bc=bc, nx=n, ny=n, K=0.5, cfl=0.5, ld=n + 2,
                     layout=_lib.FVM_LAYOUT_ROWS)
    sr = Solver(pr, ug=ug)
    if gh is not None:
        sr.set_boundary_states(gh)
    Xr = torch.tensor(W0, device="cuda", requires_grad=True)
    Yr = fvrun(Xr, sr, 12, 4)
    (0.5 * ((Yr[0] - tgt) ** 2).sum()).backward()
    assert torch.equal(Yr, Y) and np.array_equal(Xr.grad.cpu().numpy(), g)
    P = oparams(p, gh)
    WN, odts = orc.run(P, W0, 12, ug)
    ey = rel_linf(Y.detach().cpu().numpy(), WN)
    lamN = np.zeros_like(W0)
    lamN[0] = WN[0] - tgt_np
    eg = rel_linf(g, orc.adjoint_run(P, W0, odts, lamN, ug))
    print(f"spray bc={bc} 40^2 x 12 steps: rel Linf state {ey:.2e}, gradient {eg:.2e}",
          flush=True)
    assert ey <= TOL  # measured 4e-16 - 6e-16
    assert eg <= TOL  # measured 8e-15 - 2e-14
    def L(W):
        out = orc.run_dts(P, W, odts, ug)
        return 0.5 * np.sum((out[0] - tgt_np) ** 2)
    rng = np.random.default_rng(13)
    for _ in range(4):
        v = rng.standard_normal(W0.shape) * np.abs(W0)
        eps = 1e-6
        fd = (L(W0 + eps * v) - L(W0 - eps * v)) / (2 * eps)
        assert abs(float(np.sum(g * v)) - fd) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_spray_adjoint_degenerate_cases(bc):
    """dt = 0 leaves the multipliers bit for bit unchanged; vacuum cells (all
    moments zero: no velocity, no source) next to droplets, with and without
    evaporation, match the oracle."""
    nx, ny = 70, 21
    W, ug = _spray_adjoint_case(nx, ny, 17)
    W[:, 5:12, 20:41] = 0.0   # a vacuum block
    W[:, :, 60] = 0.0         # and a vacuum column
    gh = _spray_ghosts() if bc == _lib.FVM_DIRICHLET else None
    lam = np.random.default_rng(19).standard_normal(W.shape)
    for K in (0.7, 0.0):
        print(f"spray adjoint degenerate bc={bc} K={K}", flush=True)
        p = params_from(model=2, bc=bc, nx=nx, ny=ny, K=K, cfl=0.9)
        s = Solver(p, ug=ug)
        if gh is not None:
            s.set_boundary_states(gh)
        same = s.adjoint_step(W, 0.0, lam)
        torch.cuda.synchronize()
        assert np.array_equal(same[:, :, :nx].cpu().numpy(), lam)
        dt = 0.3 / nx
        got = s.adjoint_step(W, dt, lam)
        torch.cuda.synchronize()
        ref = orc.adjoint_step(oparams(p, gh), W, dt, lam, ug)
        assert rel_linf(got[:, :, :nx].cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_spray_clipped_lognormal_width(bc):
    """Cells whose moments leave no room for a lognormal width
    (m_{1/2}^2 >= m_0 m_{2/2}: a monodisperse block, and a column beyond it)
    take the clipped width s^2 = 1e-8 in the closure, where m_{-1/2} and the
    closure Jacobian follow their clipped forms: one forward step with a
    fixed dt and one adjoint step against the oracle, on a state that mixes
    such cells with fitted ones."""
    nx, ny = 70, 21
    print(f"spray clipped width bc={bc}", flush=True)
    W, ug = _spray_adjoint_case(nx, ny, 23)
    n, S = W[0, 3:9, 10:30].copy(), 0.2
    for k in range(4):  # m_{k/2} = n S^{k/2}: zero width
        W[k, 3:9, 10:30] = n * S ** (0.5 * k)
    W[1, :, 50] = 1.05 * np.sqrt(W[0, :, 50] * W[2, :, 50])
    gh = _spray_ghosts() if bc == _lib.FVM_DIRICHLET else None
    p = params_from(model=2, bc=bc, nx=nx, ny=ny, K=0.7, cfl=0.9)
    P = oparams(p, gh)
    _, _, dt = orc.cfl(P, W)
    s = Solver(p, ug=ug)
    if gh is not None:
        s.set_boundary_states(gh)
    s.set_state(W)
    s.step(dt)
    assert s.sync() == 0
    rc, ref = orc.step_fixed(P, W, dt, ug=ug)
    assert rc == 0
    assert rel_linf(gpu_state(s), ref) <= TOL
    lam = np.random.default_rng(29).standard_normal(W.shape)
    got = s.adjoint_step(W, dt, lam)
    torch.cuda.synchronize()
    ref = orc.adjoint_step(P, W, dt, lam, ug)
    assert rel_linf(got[:, :, :nx].cpu().numpy(), ref) <= TOL


def test_spray_adjoint_2048_full_size_step():
    """One spray adjoint step on the 2048^2 spray workload's state (lognormal
    closure, K = 1, theta = 0.1) in the benchmark's storage layout against
    the oracle, whole grid."""
    pre = inputs.SPRAY_2048
    W, ug = inputs.spray_state(pre.nx, pre.ny, 0)
    p = params_from(pre, layout=_lib.FVM_LAYOUT_ROWS)
    lam = np.random.default_rng(5).standard_normal(W.shape)
    P = oparams(p)
    orc.set_threads(16)
    _, _, dt = orc.cfl(P, W)
    print("spray adjoint 2048^2", flush=True)
    got = Solver(p, ug=ug).adjoint_step(W, dt, lam)
    torch.cuda.synchronize()
    ref = orc.adjoint_step(P, W, dt, lam, ug)
    assert rel_linf(got[:, :, :pre.nx].cpu().numpy(), ref) <= TOL


# ---------------------------------------------------------------------------
# the full-size Euler workload in the benchmark's launch configuration
# ---------------------------------------------------------------------------

TUNING = os.path.join(ROOT, "paper_1701_05431_amd", "tuning_mi355x.txt")


@pytest.mark.parametrize("bench_config", [False, True])
def test_euler_4096_full_size_one_step_parity(bench_config):
    """One step of the 4096^2 workload after 20 steps, against the oracle:
    planar storage with the default tiling, and the benchmark's launch
    configuration (row-interleaved storage, the tuned tile shape)."""
    pre = inputs.EULER_4096
    p = params_from(pre, layout=_lib.FVM_LAYOUT_ROWS if bench_config else _lib.FVM_LAYOUT_PLANES)
    W = inputs.riemann_state(pre.nx, pre.ny, 0)
    s = Solver(p)
    s.set_state(W)
    if bench_config:
        print(f"euler 4096 bench tiling {s.autotune(TUNING)}", flush=True)
    s.run(20)
    Wk = gpu_state(s)
    dts = s.run(1, record_dt=True).cpu().numpy()
    got = gpu_state(s)
    P = oparams(p)
    orc.set_threads(16)
    _, _, odt = orc.cfl(P, Wk)
    assert ulps(dts[0], odt) <= DT_ULP
    ref = orc.run_dts(P, Wk, dts)
    assert rel_linf(got, ref) <= TOL


def test_spray_2048_full_size_bench_config():
    """Two steps of the 2048^2 spray workload in the benchmark's launch
    configuration against the oracle with the same dts."""
    pre = inputs.SPRAY_2048
    W, ug = inputs.spray_state(pre.nx, pre.ny, 0)
    p = params_from(pre, layout=_lib.FVM_LAYOUT_ROWS)
    s = Solver(p, ug=ug)
    s.set_state(W)
    print(f"spray 2048 bench tiling {s.autotune(TUNING)}", flush=True)
    dts = s.run(2, record_dt=True).cpu().numpy()
    got = gpu_state(s)
    P = oparams(p)
    orc.set_threads(16)
    ref = orc.run_dts(P, W, dts, ug=ug)
    assert rel_linf(got, ref) <= TOL
    _, _, odt = orc.cfl(P, W)
    assert ulps(dts[0], odt) <= DT_ULP


def test_batch_256_full_workload_bench_config():
    """The 256-grid workload as the benchmark runs it (128-byte pitches, row
    storage, tuned persistent tiling): 3 steps, the largest, a middle and the
    smallest grid against the oracle, every grid's dts against its own
    single-grid run's."""
    sizes = inputs.batch_sizes(inputs.BATCH_COUNT, 0)
    plist = [params_from(inputs.BATCH_256, nx=n, ny=n, ld=aligned_pitch(n),
                         layout=_lib.FVM_LAYOUT_ROWS) for n in sizes]
    states = [inputs.riemann_state(n, n, k) for k, n in enumerate(sizes)]
    b = Batch(plist)
    b.set_states(states)
    b.autotune(TUNING)
    b.set_states(states)
    dts = b.run(3, record_dt=True).cpu().numpy()
    got = b.states()
    order = sorted(range(len(sizes)), key=lambda k: sizes[k])
    orc.set_threads(16)
    for k in (order[-1], order[len(order) // 2], order[0]):
        print(f"batch grid {k} n={sizes[k]}", flush=True)
        ref = orc.run_dts(oparams(plist[k]), states[k], dts[:, k])
        assert rel_linf(got[k].cpu().numpy(), ref) <= TOL, k
        _, _, odt = orc.cfl(oparams(plist[k]), states[k])
        assert ulps(dts[0, k], odt) <= DT_ULP, k


def test_adjoint_1024_full_size_step():
    """One adjoint step of the 1024^2 workload's state in the benchmark's
    storage layout against the oracle."""
    pre = inputs.ADJOINT_1024
    W = inputs.riemann_state(pre.nx, pre.ny, 0)
    p = params_from(pre, layout=_lib.FVM_LAYOUT_ROWS)
    lam = np.random.default_rng(3).standard_normal(W.shape)
    P = oparams(p)
    orc.set_threads(16)
    _, _, dt = orc.cfl(P, W)
    got = Solver(p).adjoint_step(W, dt, lam)
    torch.cuda.synchronize()
    ref = orc.adjoint_step(P, W, dt, lam)
    assert rel_linf(got[:, :, :pre.nx].cpu().numpy(), ref) <= TOL
