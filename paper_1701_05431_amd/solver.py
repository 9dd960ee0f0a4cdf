"""Python front end over the C ABI: single grids, batches of grids, and the
differentiable run (torch.autograd.Function over the hand-written adjoint).

PyTorch only provides device memory and the stream; all arithmetic of the
method runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import struct

import numpy as np
import torch

from . import _lib
from ._lib import check, lib


def params_from(preset=None, **kw) -> _lib.Params:
    """fvm_params from a workload preset (or keyword arguments)."""
    d = dict(model=None, bc=_lib.FVM_PERIODIC, nx=None, ny=None, npart_x=1, npart_y=1,
             ld=None, layout=_lib.FVM_LAYOUT_PLANES, lx=1.0, ly=1.0, gamma=1.4, ax=0.0,
             ay=0.0, K=1.0, theta=0.1, s_eps=0.01, cfl=0.45, dt_max=0.0,
             closure=_lib.FVM_CLOSURE_LOGNORMAL)
    if preset is not None:
        for k in ("model", "bc", "nx", "ny", "npart_x", "npart_y", "lx", "ly", "gamma", "ax",
                  "ay", "K", "theta", "s_eps", "cfl", "dt_max"):
            d[k] = getattr(preset, k)
    d.update(kw)
    if d["ld"] is None:
        d["ld"] = d["nx"]
    p = _lib.Params()
    for k, v in d.items():
        setattr(p, k, v)
    return p


def aligned_pitch(nx: int, align: int = 16) -> int:
    """The smallest row pitch (in doubles) >= nx that is a multiple of align:
    with the default 16, every row of every variable starts on a 128-byte
    line, so a wave's row of a strip touches no line it does not use."""
    return (nx + align - 1) // align * align


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def storage_shape(p: _lib.Params, nv: int):
    """Shape of the contiguous tensor that holds one field of nv variables in
    the grid's layout: (nv, Ny, ld) for planes, (Ny, nv, ld) for rows."""
    if p.layout == _lib.FVM_LAYOUT_ROWS:
        return (p.ny, nv, p.ld)
    return (nv, p.ny, p.ld)


def logical(p: _lib.Params, t: torch.Tensor) -> torch.Tensor:
    """The (nVar, Ny, ld) view of a storage tensor (strided for rows)."""
    return t.permute(1, 0, 2) if p.layout == _lib.FVM_LAYOUT_ROWS else t


class Solver:
    """One grid: two ping-pong state buffers (float64, nVar * Ny * ld each,
    in the layout of p.layout), the spray gas velocity if any, and the
    scratch, all allocated by torch. States go in and come out as
    (nVar, Ny, Nx) or (nVar, Ny, ld) tensors whatever the layout."""

    def __init__(self, p: _lib.Params, device="cuda", ug=None):
        L = lib()
        check(L.fvm_validate(C.byref(p)), "fvm_validate")
        self.p = p
        self.device = torch.device(device)
        self.nv = L.fvm_nvar(p.model)
        shape = storage_shape(p, self.nv)
        self.wa = torch.zeros(shape, dtype=torch.float64, device=self.device)
        self.wb = torch.zeros(shape, dtype=torch.float64, device=self.device)
        self.ug = None
        if p.model == _lib.FVM_SPRAY:
            if ug is None:
                raise ValueError("the spray model needs the gas velocity field ug")
            self.ug = self._as_state(ug, 2)
        nbytes = int(L.fvm_scratch_bytes(C.byref(p)))
        self.scratch = torch.zeros(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.scratch.data_ptr()) % 256
        self.scratch_view = self.scratch[off:off + nbytes]
        h = C.c_void_p()
        check(L.fvm_create(C.byref(p), C.byref(h)), "fvm_create")
        self.h = h
        check(L.fvm_bind(self.h, _ptr(self.wa), _ptr(self.wb), _ptr(self.ug),
                         _ptr(self.scratch_view), _stream_handle(self.device)), "fvm_bind")

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                lib().fvm_destroy(h)
            except Exception:
                pass
            self.h = None

    # ---- state -------------------------------------------------------------
    def _as_state(self, W, nv=None) -> torch.Tensor:
        """A storage tensor (grid layout, contiguous) holding W, given as
        (nv, Ny, Nx) or (nv, Ny, ld)."""
        nv = self.nv if nv is None else nv
        p = self.p
        if isinstance(W, np.ndarray):
            W = torch.from_numpy(np.ascontiguousarray(W, dtype=np.float64))
        W = W.to(device=self.device, dtype=torch.float64)
        if W.shape not in ((nv, p.ny, p.nx), (nv, p.ny, p.ld)):
            raise ValueError(f"state shape {tuple(W.shape)} does not match ({nv}, {p.ny}, {p.ld})")
        if W.shape[2] == p.ld and p.layout == _lib.FVM_LAYOUT_PLANES:
            return W.contiguous()
        out = torch.zeros(storage_shape(p, nv), dtype=torch.float64, device=self.device)
        logical(p, out)[:, :, :W.shape[2]].copy_(W)
        return out

    def set_boundary_states(self, ghost) -> None:
        """Dirichlet ghost states, shape (4, nVar): west, east, south, north."""
        g = np.ascontiguousarray(np.asarray(ghost, dtype=np.float64).reshape(4, self.nv))
        check(lib().fvm_set_boundary_states(self.h, g.ctypes.data_as(C.c_void_p)),
              "fvm_set_boundary_states")

    def set_halo_rows(self, south=None, north=None) -> None:
        """Rows j = -1 and j = ny from device tensors of shape (nVar, ld)
        (contiguous float64), or None for the boundary condition."""
        for t in (south, north):
            if t is not None and (t.dtype != torch.float64 or not t.is_contiguous()
                                  or tuple(t.shape) != (self.nv, self.p.ld)):
                raise ValueError("halo rows must be contiguous float64 of shape (nVar, ld)")
        self._halo = (south, north)  # keep them alive while the plan reads them
        check(lib().fvm_set_halo_rows(self.h, _ptr(south), _ptr(north)), "fvm_set_halo_rows")

    def _bind_stream(self):
        lib().fvm_set_stream(self.h, _stream_handle(self.device))

    def set_state(self, W) -> None:
        src = self._as_state(W)
        self._bind_stream()
        check(lib().fvm_set_state(self.h, _ptr(src), 1), "fvm_set_state")
        self._keep = src  # keep the source alive until the copy has run

    def current_storage(self) -> torch.Tensor:
        """The buffer holding the current state, in the grid's layout."""
        ptr = C.c_void_p()
        check(lib().fvm_current(self.h, C.byref(ptr)), "fvm_current")
        return self.wa if ptr.value == self.wa.data_ptr() else self.wb

    def current(self) -> torch.Tensor:
        """The current state as an (nVar, Ny, ld) view of its buffer (the
        next step overwrites the other buffer, not this one)."""
        return logical(self.p, self.current_storage())

    def state(self) -> torch.Tensor:
        """A contiguous copy of the current state, shape (nVar, Ny, Nx)."""
        return self.current()[:, :, :self.p.nx].clone(memory_format=torch.contiguous_format)

    # ---- stepping ------------------------------------------------------------
    def cfl_dt(self):
        """(dt, Sx, Sy) of the current state (synchronises)."""
        self._bind_stream()
        dt, sx, sy = C.c_double(), C.c_double(), C.c_double()
        check(lib().fvm_cfl_dt_host(self.h, C.byref(dt), C.byref(sx), C.byref(sy)), "fvm_cfl_dt")
        return dt.value, sx.value, sy.value

    def step(self, dt: float) -> None:
        self._bind_stream()
        check(lib().fvm_step(self.h, float(dt)), "fvm_step")

    def run(self, nsteps: int, record_dt: bool = False):
        self._bind_stream()
        dts = (torch.zeros(max(nsteps, 1), dtype=torch.float64, device=self.device)
               if record_dt else None)
        check(lib().fvm_run(self.h, int(nsteps), _ptr(dts)), "fvm_run")
        return dts[:nsteps] if record_dt else None

    def run_fixed(self, nsteps: int, dt: float) -> None:
        """nsteps steps of one fixed dt, each checked against the CFL
        condition first (a failed check leaves the state unchanged and is
        reported by sync() as FVM_ECFL)."""
        self._bind_stream()
        check(lib().fvm_run_fixed(self.h, int(nsteps), float(dt)), "fvm_run_fixed")

    def run_dts(self, dts) -> None:
        dts = torch.as_tensor(dts, dtype=torch.float64).to(self.device).contiguous()
        self._bind_stream()
        check(lib().fvm_run_dts(self.h, int(dts.numel()), _ptr(dts)), "fvm_run_dts")
        self._keep = dts

    def run_ckpt(self, nsteps: int, every: int):
        """Adaptive run that stores W^0, W^every, ...; returns (ckpts, dts),
        the checkpoints as storage tensors in the grid's layout."""
        nck = (nsteps + every - 1) // every
        ck = [torch.empty_like(self.wa) for _ in range(nck)]
        dts = torch.zeros(max(nsteps, 1), dtype=torch.float64, device=self.device)
        arr = (C.c_void_p * max(nck, 1))(*[t.data_ptr() for t in ck])
        self._bind_stream()
        check(lib().fvm_run_ckpt(self.h, int(nsteps), int(every), arr, _ptr(dts)), "fvm_run_ckpt")
        return ck, dts[:nsteps]

    def adjoint(self, ckpts, every: int, dts: torch.Tensor, lam: torch.Tensor) -> torch.Tensor:
        """dL/dW^0 from dL/dW^N (lam, shape (nVar, Ny, Nx or ld)) through
        len(dts) steps with the given checkpoints; an (nVar, Ny, ld) view."""
        lam = self._as_state(lam).clone()
        tmp = torch.empty_like(lam)
        seg = torch.empty((max(every - 1, 1),) + tuple(lam.shape), dtype=torch.float64,
                          device=self.device)
        arr = (C.c_void_p * max(len(ckpts), 1))(*[t.data_ptr() for t in ckpts])
        self._bind_stream()
        check(lib().fvm_adjoint_run(self.h, arr, int(every), _ptr(dts), int(dts.numel()),
                                    _ptr(lam), _ptr(tmp), _ptr(seg)), "fvm_adjoint_run")
        self._keep = (tmp, seg)
        return logical(self.p, lam)

    def adjoint_step(self, W, dt: float, lam) -> torch.Tensor:
        W = self._as_state(W)
        lam = self._as_state(lam)
        out = torch.empty_like(lam)
        self._bind_stream()
        check(lib().fvm_adjoint_step(self.h, _ptr(W), float(dt), _ptr(lam), _ptr(out)),
              "fvm_adjoint_step")
        self._keep = (W, lam)
        return logical(self.p, out)

    def sync(self) -> int:
        return int(lib().fvm_sync(self.h))

    def status(self, clear: bool = False) -> int:
        return int(lib().fvm_get_status(self.h, int(clear)))

    def set_tiling(self, rows: int = 0, waves_per_block: int = 0) -> None:
        check(lib().fvm_set_tiling(self.h, int(rows), int(waves_per_block)), "fvm_set_tiling")

    def keep_closure_multipliers(self, enable: bool = True) -> None:
        """Entropy closure: keep every cell's multipliers between steps (a
        4 x Ny x Nx device buffer) so that Newton restarts from them."""
        self._me_lam = (torch.empty(4 * self.p.ny * self.p.nx, dtype=torch.float64,
                                    device=self.device) if enable else None)
        check(lib().fvm_set_closure_buffer(self.h, _ptr(self._me_lam)),
              "fvm_set_closure_buffer")

    def set_adjoint_tiling(self, rows: int = 0, waves_per_block: int = 0,
                           cells_per_lane: int = 0) -> None:
        check(lib().fvm_set_adjoint_tiling(self.h, int(rows), int(waves_per_block),
                                           int(cells_per_lane)), "fvm_set_adjoint_tiling")

    def tiling(self):
        r, w = C.c_int(), C.c_int()
        check(lib().fvm_get_tiling(self.h, C.byref(r), C.byref(w)), "fvm_get_tiling")
        return r.value, w.value

    def set_cells_per_lane(self, cpl: int = 0) -> int:
        """Cells per lane of the step kernel (0 = default); returns the value
        in use."""
        check(lib().fvm_set_cells_per_lane(self.h, int(cpl)), "fvm_set_cells_per_lane")
        return self.cells_per_lane()

    def cells_per_lane(self) -> int:
        return int(lib().fvm_get_cells_per_lane(self.h))

    def set_resident_runs(self, enable: bool = True) -> None:
        """Whole adaptive runs of a grid that fits in one workgroup's LDS in
        one launch (the default), or one launch per step."""
        check(lib().fvm_set_resident_runs(self.h, int(bool(enable))), "fvm_set_resident_runs")

    def autotune(self, cache_path: str | None = None):
        """Times dry-run steps of every tiling and lane layout on this grid,
        applies the fastest (optionally cached in a text file); returns
        (rows, waves_per_block, cells_per_lane)."""
        self._bind_stream()
        path = cache_path.encode() if cache_path else None
        check(lib().fvm_autotune(self.h, path), "fvm_autotune")
        return self.tiling() + (self.cells_per_lane(),)

    def autotune_adjoint(self, W: torch.Tensor, lam_in: torch.Tensor, lam_out: torch.Tensor,
                         cache_path: str | None = None) -> None:
        """Tiles the adjoint kernel by timing dt = 0 steps on these storage
        buffers (one state each; lam_out receives lam_in)."""
        self._bind_stream()
        path = cache_path.encode() if cache_path else None
        check(lib().fvm_autotune_adjoint(self.h, _ptr(W), _ptr(lam_in), _ptr(lam_out), path),
              "fvm_autotune_adjoint")


class Batch:
    """Many independent grids packed in one buffer per ping-pong side, each
    at a 256-byte aligned offset."""

    def __init__(self, plist, device="cuda"):
        L = lib()
        self.device = torch.device(device)
        n = len(plist)
        self.n = n
        self.plist = list(plist)
        self.nv = L.fvm_nvar(plist[0].model)
        offs, o = [], 0
        for p in plist:
            offs.append(o)
            o += self.nv * p.ny * p.ld
            o = (o + 31) // 32 * 32
        self.offsets = offs
        self.total = o
        self.wa = torch.zeros(o, dtype=torch.float64, device=self.device)
        self.wb = torch.zeros(o, dtype=torch.float64, device=self.device)
        parr = (_lib.Params * n)(*plist)
        oarr = (C.c_size_t * n)(*offs)
        h = C.c_void_p()
        check(L.fvm_batch_create(n, parr, oarr, C.byref(h)), "fvm_batch_create")
        self.h = h
        nbytes = int(L.fvm_batch_scratch_bytes(self.h))
        self.scratch = torch.zeros(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.scratch.data_ptr()) % 256
        self.scratch_view = self.scratch[off:off + nbytes]
        check(L.fvm_batch_bind(self.h, _ptr(self.wa), _ptr(self.wb), _ptr(self.scratch_view),
                               _stream_handle(self.device)), "fvm_batch_bind")

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            try:
                lib().fvm_batch_destroy(h)
            except Exception:
                pass
            self.h = None

    def current(self) -> torch.Tensor:
        ptr = C.c_void_p()
        check(lib().fvm_batch_current(self.h, C.byref(ptr)), "fvm_batch_current")
        return self.wa if ptr.value == self.wa.data_ptr() else self.wb

    def view(self, buf: torch.Tensor, k: int) -> torch.Tensor:
        """Grid k of a packed buffer as an (nVar, Ny, ld) view."""
        p = self.plist[k]
        n = self.nv * p.ny * p.ld
        return logical(p, buf[self.offsets[k]:self.offsets[k] + n].view(storage_shape(p, self.nv)))

    def set_states(self, states) -> None:
        cur = self.current()
        for k, W in enumerate(states):
            p = self.plist[k]
            if isinstance(W, np.ndarray):
                W = torch.from_numpy(np.ascontiguousarray(W))
            self.view(cur, k)[:, :, :p.nx].copy_(W.to(self.device, torch.float64))
        # the maxima of the new states are unknown until the next cfl
        check(lib().fvm_batch_cfl(self.h), "fvm_batch_cfl")

    def states(self):
        cur = self.current()
        return [self.view(cur, k)[:, :, :self.plist[k].nx].clone(
            memory_format=torch.contiguous_format) for k in range(self.n)]

    def run(self, nsteps: int, record_dt: bool = False, per_grid: bool = False):
        dts = (torch.zeros(max(nsteps, 1) * self.n, dtype=torch.float64, device=self.device)
               if record_dt else None)
        f = lib().fvm_batch_run_per_grid if per_grid else lib().fvm_batch_run
        check(f(self.h, int(nsteps), _ptr(dts)), "fvm_batch_run")
        return dts[:nsteps * self.n].view(nsteps, self.n) if record_dt else None

    def set_tiling(self, rows: int = 0, waves_per_block: int = 0) -> None:
        check(lib().fvm_batch_set_tiling(self.h, int(rows), int(waves_per_block)),
              "fvm_batch_set_tiling")

    def set_schedule(self, persistent: bool = True, fit_blocks: bool = False) -> None:
        """Persistent workgroups over a work queue, or one workgroup per item;
        fit_blocks: row blocks sized so that strips fill whole workgroups."""
        check(lib().fvm_batch_set_schedule(self.h, int(bool(persistent)), int(bool(fit_blocks))),
              "fvm_batch_set_schedule")

    def set_layout(self, cells_per_lane: int = 2) -> None:
        """2: two cells per lane on every even-pitch grid; 1: one cell per
        lane on every grid."""
        check(lib().fvm_batch_set_layout(self.h, int(cells_per_lane)), "fvm_batch_set_layout")

    def autotune(self, cache_path: str | None = None) -> None:
        """Picks the batched step's tile shape, schedule and lane layout by
        timing dry runs."""
        path = cache_path.encode() if cache_path else None
        check(lib().fvm_batch_autotune(self.h, path), "fvm_batch_autotune")

    def sync(self) -> int:
        return int(lib().fvm_batch_sync(self.h))


SNAPSHOT_HEADER = 64


class AsyncOutput:
    """Non-blocking solution dumps of one grid (Sec. 4.3): `snapshot` enqueues
    the gather of the current state into a device staging buffer on the
    solver's stream, its copy to pinned host memory on a side stream and the
    file write on the library's writer thread, and returns; the time steps
    enqueued after it overlap the copy and the write."""

    def __init__(self, solver: Solver):
        self.solver = solver
        p = solver.p
        n = solver.nv * p.ny * p.nx
        self.staging = torch.empty(n, dtype=torch.float64, device=solver.device)
        self.host = torch.empty(n, dtype=torch.float64, pin_memory=True)
        self.copy_stream = torch.cuda.Stream(device=solver.device)
        solver._bind_stream()
        h = C.c_void_p()
        check(lib().fvm_output_create(solver.h, _ptr(self.staging), _ptr(self.host),
                                      C.c_void_p(self.copy_stream.cuda_stream), C.byref(h)),
              "fvm_output_create")
        self.h = h

    def snapshot(self, path: str, step: int = 0, time: float = 0.0) -> None:
        self.solver._bind_stream()
        check(lib().fvm_output_snapshot(self.h, os.fsencode(path), int(step), float(time)),
              "fvm_output_snapshot")

    def wait(self) -> None:
        check(lib().fvm_output_wait(self.h), "fvm_output_wait")

    def close(self) -> None:
        h, self.h = getattr(self, "h", None), None
        if h is not None and h.value:
            check(lib().fvm_output_destroy(h), "fvm_output_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def read_snapshot(path: str):
    """(header dict, array (nvar, ny, nx)) of a snapshot file."""
    with open(path, "rb") as f:
        head = f.read(SNAPSHOT_HEADER)
        if len(head) != SNAPSHOT_HEADER or head[:8] != b"FVMSNAP1":
            raise ValueError(f"{path}: not a snapshot file")
        model, nvar, nx, ny = struct.unpack_from("<4i", head, 8)
        (step,) = struct.unpack_from("<q", head, 24)
        time, lx, ly = struct.unpack_from("<3d", head, 32)
        npx, npy = struct.unpack_from("<2i", head, 56)
        data = np.fromfile(f, dtype="<f8", count=nvar * ny * nx)
    if data.size != nvar * ny * nx:
        raise ValueError(f"{path}: truncated")
    meta = dict(model=model, nvar=nvar, nx=nx, ny=ny, step=step, time=time, lx=lx, ly=ly,
                npart_x=npx, npart_y=npy)
    return meta, data.reshape(nvar, ny, nx)


class FVRun(torch.autograd.Function):
    """W^N = run(W^0) with adaptive time steps; backward is the hand-written
    discrete adjoint with the forward dts held fixed, recomputing each
    segment of `every` steps from its checkpoint.

    FVRun.apply(W0, solver, nsteps, every) with W0 of shape (nVar, Ny, Nx).
    """

    @staticmethod
    def forward(ctx, W0, solver: Solver, nsteps: int, every: int):
        solver.set_state(W0.detach())
        ck, dts = solver.run_ckpt(nsteps, every)
        ctx.solver = solver
        ctx.every = every
        ctx.ckpts = ck
        ctx.dts = dts
        return solver.state()

    @staticmethod
    def backward(ctx, gN):
        s = ctx.solver
        lam = s.adjoint(ctx.ckpts, ctx.every, ctx.dts, gN.detach().contiguous())
        return lam[:, :, :s.p.nx].clone(memory_format=torch.contiguous_format), None, None, None


def fvrun(W0: torch.Tensor, solver: Solver, nsteps: int, every: int | None = None):
    every = every or max(1, int(round(math.sqrt(nsteps))))
    return FVRun.apply(W0, solver, nsteps, every)
