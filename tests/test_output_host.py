"""The asynchronous output stage without a GPU: argument checks of the C ABI
and the snapshot file format of the header's documentation, read back by
read_snapshot from a file written here field by field."""
import ctypes as C
import struct

import numpy as np
import pytest

from paper_1701_05431_amd import _lib


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_output_calls_reject_missing_arguments(L):
    h = C.c_void_p()
    assert L.fvm_output_create(None, None, None, None, C.byref(h)) == _lib.FVM_EINVAL
    assert not h.value
    assert L.fvm_output_create(None, None, None, None, None) == _lib.FVM_EINVAL
    assert L.fvm_output_snapshot(None, b"x", 0, 0.0) == _lib.FVM_EINVAL
    assert L.fvm_output_wait(None) == _lib.FVM_EINVAL
    assert L.fvm_output_destroy(None) == _lib.FVM_OK


def test_output_needs_a_bound_grid(L):
    from paper_1701_05431_amd.solver import params_from
    p = params_from(model=1, nx=8, ny=8)
    g = C.c_void_p()
    assert L.fvm_create(C.byref(p), C.byref(g)) == _lib.FVM_OK
    buf = (C.c_double * 256)()
    h = C.c_void_p()
    try:
        assert L.fvm_output_create(g, buf, buf, None, C.byref(h)) == _lib.FVM_EINVAL
        assert not h.value
    finally:
        L.fvm_destroy(g)


def test_snapshot_file_format(tmp_path):
    from paper_1701_05431_amd.solver import read_snapshot
    nv, nx, ny = 4, 5, 3
    data = np.arange(nv * ny * nx, dtype=np.float64) * 0.5 - 3.0
    head = (b"FVMSNAP1" + struct.pack("<4i", 1, nv, nx, ny) + struct.pack("<q", 123456789012)
            + struct.pack("<3d", 0.25, 2.0, 1.5) + struct.pack("<2i", 4, 2))
    assert len(head) == 64
    path = tmp_path / "s.bin"
    path.write_bytes(head + data.astype("<f8").tobytes())
    meta, arr = read_snapshot(str(path))
    assert meta == dict(model=1, nvar=nv, nx=nx, ny=ny, step=123456789012, time=0.25, lx=2.0,
                        ly=1.5, npart_x=4, npart_y=2)
    # variable v of cell (i, j) at (v * ny + j) * nx + i
    assert arr.shape == (nv, ny, nx)
    assert arr[2, 1, 3] == data[(2 * ny + 1) * nx + 3]
    path.write_bytes(head + data[:-1].astype("<f8").tobytes())
    with pytest.raises(ValueError):
        read_snapshot(str(path))
    path.write_bytes(b"FVMSNAP0" + head[8:])
    with pytest.raises(ValueError):
        read_snapshot(str(path))
