"""Host-side checks of the C-ABI library (no GPU needed).

The library loads, exports every function include/lbm.h declares, and
rejects bad arguments on the host before any device work.
"""
import ctypes
import math
import os
import re

import pytest

from paper_2201_11330_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_header_functions_are_exported():
    L = lbm.lib()
    funcs = _header_functions()
    assert len(funcs) >= 12
    for name in funcs:
        assert hasattr(L, name), name
    assert sorted(lbm.EXPORTS) == funcs


def test_header_enums_match_binding():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    for name, val in [("LBM_D2Q9", lbm.D2Q9), ("LBM_D3Q19", lbm.D3Q19), ("LBM_D3Q27", lbm.D3Q27),
                      ("LBM_F64", lbm.F64),
                      ("LBM_F32", lbm.F32), ("LBM_F16_DEV", lbm.F16_DEV),
                      ("LBM_BF16_DEV", lbm.BF16_DEV), ("LBM_E4M11_DEV", lbm.E4M11_DEV),
                      ("LBM_PERIODIC", lbm.PERIODIC),
                      ("LBM_SOLID_ENDS", lbm.SOLID_ENDS), ("LBM_WALLS_OUTSIDE", lbm.WALLS_OUTSIDE),
                      ("LBM_WALLS_NODAL", lbm.WALLS_NODAL),
                      ("LBM_FLAG_AA", lbm.FLAG_AA), ("LBM_FLAG_GRAPH", lbm.FLAG_GRAPH),
                      ("LBM_FLAG_COMPRESSIBLE", lbm.FLAG_COMPRESSIBLE),
                      ("LBM_EINVAL", lbm.EINVAL),
                      ("LBM_ENOTBOUND", lbm.ENOTBOUND), ("LBM_EUNSTABLE", lbm.EUNSTABLE)]:
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == val, name


def _create(lattice=lbm.D3Q19, nx=8, ny=8, nz=8, tau=0.8, force=None, bc=None, storage=lbm.F64,
            flags=0):
    L = lbm.lib()
    h = ctypes.c_void_p()
    F = (ctypes.c_double * 3)(*force) if force is not None else None
    b = ctypes.byref(lbm._BC((ctypes.c_int * 3)(*bc))) if bc is not None else None
    st = L.lbm_create(ctypes.byref(h), lattice, nx, ny, nz, tau, F, b, storage, flags)
    return st, h


@pytest.mark.parametrize("kw", [
    dict(tau=0.5), dict(tau=0.3), dict(tau=float("nan")),
    dict(nx=0), dict(ny=-1), dict(nz=70000),
    dict(lattice=lbm.D2Q9, nz=2), dict(lattice=lbm.D2Q9, nz=1, force=(0, 0, 1e-6)),
    dict(lattice=lbm.D2Q9, nz=1, bc=(0, 0, 1)),
    dict(lattice=7), dict(storage=9), dict(flags=8),
    dict(bc=(0, 1, 0), ny=2), dict(bc=(5, 0, 0)),
    dict(bc=(0, 3, 0), ny=2), dict(bc=(3, 3, 0)), dict(bc=(0, 3, 3)),
    dict(force=(float("inf"), 0, 0)), dict(force=(1e-6, 0, 0), tau=math.inf),
    dict(nx=2048, ny=2048, nz=1024),
])
def test_create_rejects_bad_arguments(kw):
    st, h = _create(**kw)
    assert st == lbm.EINVAL
    assert not h.value
    assert lbm.lib().lbm_last_error()


def test_create_accepts_and_sizes():
    L = lbm.lib()
    for lattice, nz, Q in ((lbm.D2Q9, 1, 9), (lbm.D3Q19, 5, 19), (lbm.D3Q27, 3, 27)):
        for storage, size in ((lbm.F64, 8), (lbm.F32, 4), (lbm.F16_DEV, 2), (lbm.BF16_DEV, 2)):
            st, h = _create(lattice=lattice, nx=7, ny=6, nz=nz, storage=storage)
            assert st == lbm.OK
            N = 7 * 6 * nz
            T = min(4096, 1 << (N - 1).bit_length())  # tile length: power of two, <= 4096
            want = -(-N // T) * T * Q * size
            assert L.lbm_buffer_bytes(h) == -(-want // 256) * 256
            assert L.lbm_buffer_bytes(h) % 256 == 0
            assert L.lbm_adjoint_workspace_bytes(h, 1) > 0
            assert L.lbm_adjoint_workspace_bytes(h, 5) - L.lbm_adjoint_workspace_bytes(h, 4) == \
                L.lbm_buffer_bytes(h)
            assert L.lbm_adjoint_workspace_bytes(h, 0) == 0
            assert L.lbm_steps_taken(h) == 0
            assert L.lbm_destroy(h) == lbm.OK
    st, h = _create(tau=math.inf)  # pure streaming without force is allowed
    assert st == lbm.OK
    L.lbm_destroy(h)
    # nodal walls on one axis, with other wall kinds; the compressible model
    for bc in ((0, 3, 0), (1, 3, 2), (3, 0, 1)):
        st, h = _create(bc=bc, flags=lbm.FLAG_COMPRESSIBLE)
        assert st == lbm.OK
        L.lbm_destroy(h)
    # the compressible adjoint keeps the final state: one more state buffer
    st, h = _create(flags=lbm.FLAG_COMPRESSIBLE)
    st2, h2 = _create()
    assert L.lbm_adjoint_workspace_bytes(h, 3) - L.lbm_adjoint_workspace_bytes(h2, 3) == \
        L.lbm_buffer_bytes(h)
    L.lbm_destroy(h)
    L.lbm_destroy(h2)
    assert L.lbm_destroy(None) == lbm.OK


def test_calls_before_bind_fail_without_device_work():
    L = lbm.lib()
    st, h = _create(bc=(0, 1, 0), force=(1e-6, 0, 0))
    assert st == lbm.OK
    d = ctypes.c_double()
    assert L.lbm_step(h, 1) == lbm.ENOTBOUND
    assert L.lbm_reduce(h, ctypes.byref(d), None, None) == lbm.ENOTBOUND
    assert L.lbm_reduce_noalloc(h, None) == lbm.ENOTBOUND
    assert L.lbm_moments(h, None, None, 0) == lbm.ENOTBOUND
    assert L.lbm_get_populations(h, None) == lbm.ENOTBOUND
    assert L.lbm_set_populations(h, None) == lbm.ENOTBOUND
    assert L.lbm_init_equilibrium(h, None, None, None) == lbm.ENOTBOUND
    assert L.lbm_forward_record(h, 4, 2, None) == lbm.ENOTBOUND
    assert L.lbm_set_solid(h, None) == lbm.ENOTBOUND
    F = (ctypes.c_double * 3)()
    assert L.lbm_wall_force(h, F) == lbm.ENOTBOUND
    assert L.lbm_adjoint(h, 4, 2, None, None, None, None, None, None, None, None) == lbm.ENOTBOUND
    assert b"lbm_bind" in L.lbm_last_error()
    assert L.lbm_step(None, 1) == lbm.EINVAL
    assert L.lbm_destroy(h) == lbm.OK


def test_status_strings():
    L = lbm.lib()
    for st in (lbm.OK, lbm.EINVAL, lbm.ENOTBOUND, lbm.EHIP, lbm.EUNSTABLE, lbm.ESTATE):
        assert L.lbm_status_string(st)
    assert L.lbm_status_string(123) == b"unknown status"


def test_c_example_is_built_and_checks_its_arguments():
    """The C99 driver links against liblbm.so and, given no arguments, prints
    its usage and exits with status 2 before any HIP call."""
    import subprocess
    from paper_2201_11330_amd import build as pkg_build
    exe = pkg_build.EXAMPLE_BIN
    assert os.path.exists(exe)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert res.returncode == 2 and "usage" in res.stderr
