"""The C ABI without a GPU: the library loads, exports every symbol that
include/fvm.h declares, and rejects invalid parameters on the host."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvm.h")


@pytest.fixture(scope="module")
def L():
    from paper_1701_05431_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1701_05431_amd import build
        build.build()
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fvm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_the_header():
    from paper_1701_05431_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_binding_constants_match_the_header():
    from paper_1701_05431_amd import _lib
    text = open(HEADER).read()
    defines = dict(re.findall(r"#define (FVM_[A-Z_]+) \(?(-?\d+)\)?", text))
    assert len(defines) == 17
    for name, value in defines.items():
        assert getattr(_lib, name) == int(value), name


def test_params_struct_layout():
    from paper_1701_05431_amd import _lib
    # 8 ints, 10 doubles, then the closure int and the tail padding of an
    # 8-byte aligned struct
    assert _lib.Params.closure.offset == 8 * 4 + 10 * 8
    assert C.sizeof(_lib.Params) == 8 * 4 + 10 * 8 + 8


def test_validation_on_host(L):
    from paper_1701_05431_amd import _lib
    from paper_1701_05431_amd.solver import params_from
    ok = params_from(model=1, nx=64, ny=32, npart_x=8, npart_y=4)
    assert L.fvm_validate(ok) == _lib.FVM_OK
    assert L.fvm_scratch_bytes(ok) % 256 == 0 and L.fvm_scratch_bytes(ok) > 0
    cases = [
        dict(npart_x=3),            # unbalanced subdomains
        dict(ld=63),                # pitch below nx
        dict(nx=0),
        dict(model=9),
        dict(bc=5),
        dict(gamma=1.0),
        dict(cfl=0.0),
        dict(cfl=float("nan")),
        dict(lx=-1.0),
        dict(dt_max=-1.0),
        dict(closure=2),
        dict(closure=1),            # the entropy closure is the spray's
        dict(layout=2),             # unknown layout
        dict(layout=1, ld=600_000_000, ny=1, npart_y=1),  # nVar * ld overflows int
    ]
    for c in cases:
        kw = dict(model=1, nx=64, ny=32, npart_x=8, npart_y=4)
        kw.update(c)
        p = params_from(**kw)
        assert L.fvm_validate(p) == _lib.FVM_EINVAL, c
        assert L.fvm_scratch_bytes(p) == 0, c
        h = C.c_void_p()
        assert L.fvm_create(p, C.byref(h)) == _lib.FVM_EINVAL, c
        assert not h.value
    rows = params_from(model=1, nx=64, ny=32, ld=70, layout=_lib.FVM_LAYOUT_ROWS)
    assert L.fvm_validate(rows) == _lib.FVM_OK
    assert L.fvm_validate(params_from(model=1, nx=64, ny=32, bc=_lib.FVM_DIRICHLET)) == _lib.FVM_OK
    assert L.fvm_validate(params_from(model=1, nx=64, ny=32, bc=3)) == _lib.FVM_EINVAL
    sp = params_from(model=2, nx=8, ny=8, theta=0.0)
    assert L.fvm_validate(sp) == _lib.FVM_EINVAL
    sp = params_from(model=2, nx=8, ny=8, s_eps=1.5)
    assert L.fvm_validate(sp) == _lib.FVM_EINVAL


def test_create_destroy_and_unbound_calls(L):
    from paper_1701_05431_amd import _lib
    from paper_1701_05431_amd.solver import params_from
    p = params_from(model=1, nx=64, ny=32)
    h = C.c_void_p()
    assert L.fvm_create(p, C.byref(h)) == _lib.FVM_OK and h.value
    # nothing is bound: every device call is refused before touching HIP
    assert L.fvm_run(h, 3, None) == _lib.FVM_EINVAL
    assert L.fvm_autotune_adjoint(h, None, None, None, None) == _lib.FVM_EINVAL
    assert L.fvm_step(h, 0.1) == _lib.FVM_EINVAL
    assert L.fvm_sync(h) == _lib.FVM_EINVAL
    r, w = C.c_int(), C.c_int()
    assert L.fvm_get_tiling(h, C.byref(r), C.byref(w)) == _lib.FVM_OK
    assert L.fvm_set_tiling(h, 16, 2) == _lib.FVM_OK
    assert L.fvm_set_tiling(h, 16, 3) == _lib.FVM_EINVAL
    assert L.fvm_set_tiling(h, -1, 2) == _lib.FVM_EINVAL
    ghost = (C.c_double * 16)(*([1.0] * 16))
    # ghost states only for Dirichlet boundaries
    assert L.fvm_set_boundary_states(h, ghost) == _lib.FVM_EINVAL
    assert L.fvm_destroy(h) == _lib.FVM_OK
    pd = params_from(model=1, nx=64, ny=32, bc=_lib.FVM_DIRICHLET)
    assert L.fvm_create(pd, C.byref(h)) == _lib.FVM_OK
    assert L.fvm_set_boundary_states(h, ghost) == _lib.FVM_OK
    # halo rows only with periodic or transmissive boundaries (no device access here)
    assert L.fvm_set_halo_rows(h, C.c_void_p(256), None) == _lib.FVM_EUNSUPPORTED
    assert L.fvm_set_halo_rows(h, None, None) == _lib.FVM_OK
    ghost[5] = float("nan")
    assert L.fvm_set_boundary_states(h, ghost) == _lib.FVM_EINVAL
    assert L.fvm_set_boundary_states(h, None) == _lib.FVM_EINVAL
    assert L.fvm_destroy(h) == _lib.FVM_OK
    assert L.fvm_destroy(None) == _lib.FVM_OK
    # the entropy-maximising spray closure: no Dirichlet boundaries, no halo rows
    me = params_from(model=2, nx=8, ny=8, closure=_lib.FVM_CLOSURE_MAXENT)
    assert L.fvm_validate(me) == _lib.FVM_OK
    me_d = params_from(model=2, nx=8, ny=8, bc=_lib.FVM_DIRICHLET,
                       closure=_lib.FVM_CLOSURE_MAXENT)
    assert L.fvm_create(me_d, C.byref(h)) == _lib.FVM_EUNSUPPORTED and not h.value
    assert L.fvm_create(me, C.byref(h)) == _lib.FVM_OK
    assert L.fvm_set_halo_rows(h, C.c_void_p(256), None) == _lib.FVM_EUNSUPPORTED
    assert L.fvm_destroy(h) == _lib.FVM_OK
    assert L.fvm_strerror(-4) == b"non-finite or non-physical state"
    assert L.fvm_nvar(2) == 6 and L.fvm_nvar(7) == 0


def test_batch_create_validation(L):
    from paper_1701_05431_amd import _lib
    from paper_1701_05431_amd.solver import params_from
    ps = [params_from(model=1, bc=1, nx=n, ny=n) for n in (64, 100)]
    arr = (_lib.Params * 2)(*ps)
    h = C.c_void_p()
    assert L.fvm_batch_create(2, arr, (C.c_size_t * 2)(0, 4 * 64 * 64), C.byref(h)) == 0
    assert L.fvm_batch_scratch_bytes(h) % 256 == 0
    # lane layouts: one or two cells per lane (an unbound batch only re-plans)
    assert L.fvm_batch_set_layout(h, 1) == 0
    assert L.fvm_batch_set_layout(h, 2) == 0
    for bad in (0, 3, -1):
        assert L.fvm_batch_set_layout(h, bad) == _lib.FVM_EINVAL
    assert L.fvm_batch_set_layout(None, 1) == _lib.FVM_EINVAL
    assert L.fvm_batch_destroy(h) == 0
    # overlapping grids
    assert L.fvm_batch_create(2, arr, (C.c_size_t * 2)(0, 32), C.byref(h)) == _lib.FVM_EINVAL
    # misaligned offset
    assert (L.fvm_batch_create(2, arr, (C.c_size_t * 2)(0, 4 * 64 * 64 + 8), C.byref(h))
            == _lib.FVM_EINVAL)
    sp = (_lib.Params * 1)(params_from(model=2, nx=8, ny=8))
    assert L.fvm_batch_create(1, sp, (C.c_size_t * 1)(0), C.byref(h)) == _lib.FVM_EUNSUPPORTED
    dp = (_lib.Params * 1)(params_from(model=1, nx=8, ny=8, bc=_lib.FVM_DIRICHLET))
    assert L.fvm_batch_create(1, dp, (C.c_size_t * 1)(0), C.byref(h)) == _lib.FVM_EUNSUPPORTED


def test_noalloc_run_rejects_arguments_on_the_host(L):
    """fvm_run_noalloc refuses invalid arguments before any HIP call (these
    pointers are never dereferenced)."""
    from paper_1701_05431_amd import _lib
    from paper_1701_05431_amd.solver import params_from
    a, b, u = C.c_void_p(4096), C.c_void_p(8192), C.c_void_p(1 << 20)
    f = L.fvm_run_noalloc
    eu = params_from(model=1, nx=64, ny=32)
    assert f(None, a, b, None, 3, None, None, None) == _lib.FVM_EINVAL
    assert f(eu, None, b, None, 3, None, None, None) == _lib.FVM_EINVAL
    assert f(eu, a, None, None, 3, None, None, None) == _lib.FVM_EINVAL
    assert f(eu, a, a, None, 3, None, None, None) == _lib.FVM_EINVAL
    assert f(eu, a, b, None, -1, None, None, None) == _lib.FVM_EINVAL
    assert f(eu, C.c_void_p(4100), b, None, 3, None, None, None) == _lib.FVM_EINVAL
    assert f(eu, a, b, u, 3, None, None, None) == _lib.FVM_EINVAL       # ug for Euler
    assert f(params_from(model=1, nx=64, ny=32, npart_x=3), a, b, None, 3, None, None,
             None) == _lib.FVM_EINVAL
    sp = params_from(model=2, nx=8, ny=8)
    assert f(sp, a, b, None, 3, None, None, None) == _lib.FVM_EINVAL    # spray without ug
    dp = params_from(model=1, nx=64, ny=32, bc=_lib.FVM_DIRICHLET)
    assert f(dp, a, b, None, 3, None, None, None) == _lib.FVM_EUNSUPPORTED
    me = params_from(model=2, nx=8, ny=8, closure=_lib.FVM_CLOSURE_MAXENT)
    assert f(me, a, b, u, 3, None, None, None) == _lib.FVM_EUNSUPPORTED
