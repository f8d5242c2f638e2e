"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/mplb.h declares, sizes its arena and validates its
parameters (create only validates and records; it touches no device memory)."""
import ctypes
import os
import re

import pytest

from tests.helpers import ROOT

mplb = pytest.importorskip("paper_2101_06769_amd.mplb")
from paper_2101_06769_amd import inputs  # noqa: E402

HEADER = os.path.join(ROOT, "include", "mplb.h")


def lib():
    if not os.path.exists(mplb.LIB_PATH):
        from paper_2101_06769_amd import build

        build.build()
    return mplb.load_library()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mplb_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert L.mplb_version() == 1
    assert L.mplb_arch() == b"gfx950"


def test_params_struct_matches_header_layout():
    # dim, n[3], bc[3] (7 int32 = 28 B, padded to 32), 10 doubles, 4 int32
    assert ctypes.sizeof(mplb.Params) == 32 + 8 * 10 + 16


def case_params(**over):
    p = dict(inputs.rti3d(nx=16, ny=16, nz=32, amp=1.0).params)
    p.update(over)
    return p


def test_state_bytes_scales_with_storage():
    L = lib()
    sizes = {}
    for st in ("fp64", "fp32", "fp16s", "fp16s_all"):
        sizes[st] = mplb.state_bytes(mplb.make_params(case_params(), storage=st))
    n = 16 * 16 * 32
    assert sizes["fp64"] > sizes["fp32"] > sizes["fp16s"] > sizes["fp16s_all"]
    # two ping-pong pairs of 27 planes dominate
    assert sizes["fp32"] >= 2 * 2 * 27 * n * 4
    assert sizes["fp32"] < 2 * 2 * 27 * n * 4 + 64 * n + (1 << 20)
    assert L.mplb_version() == 1


@pytest.mark.parametrize("over,msg", [
    (dict(dim=4), "dim"), (dict(n=(0, 16, 32)), "extent"), (dict(rho_l=0.0), "densities"),
    (dict(nu_h=-1.0), "viscosities"), (dict(W=0.5), "W"), (dict(M=0.0), "mobility"),
    (dict(sigma=-1.0), "surface tension"), (dict(bc=(0, 0, 7)), "boundary"),
])
def test_invalid_parameters_are_rejected(over, msg):
    L = lib()
    p = mplb.make_params(case_params(**over))
    assert L.mplb_state_bytes(ctypes.byref(p)) == 0
    h = ctypes.c_void_p()
    rc = L.mplb_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), 1 << 40, None, ctypes.byref(h))
    assert rc == mplb.EINVAL
    assert msg in L.mplb_last_error().decode()


def test_2d_rejects_out_of_plane_gravity_and_depth():
    L = lib()
    p = mplb.make_params(inputs.rti2d(nx=8, ny=8).params)
    p.gravity[2] = 1e-5
    assert L.mplb_state_bytes(ctypes.byref(p)) == 0
    p.gravity[2] = 0.0
    p.n[2] = 2
    assert L.mplb_state_bytes(ctypes.byref(p)) == 0


def test_create_checks_arena_size_and_alignment_without_touching_it():
    L = lib()
    p = mplb.make_params(case_params())
    need = L.mplb_state_bytes(ctypes.byref(p))
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 30)  # never dereferenced by create
    assert L.mplb_create(ctypes.byref(p), fake, need - 1, None, ctypes.byref(h)) == mplb.ENOMEM
    assert L.mplb_create(ctypes.byref(p), ctypes.c_void_p((1 << 30) + 8), need, None,
                         ctypes.byref(h)) == mplb.EINVAL
    assert L.mplb_create(ctypes.byref(p), fake, need, None, ctypes.byref(h)) == mplb.OK
    # stepping before init is a state error, not a device call
    assert L.mplb_step(h, 1) == mplb.ESTATE
    assert L.mplb_set_block(h, 64, 8, 1) == mplb.EINVAL  # 512 threads
    assert L.mplb_set_block(h, 64, 4, 1) == mplb.OK
    L.mplb_destroy(h)
