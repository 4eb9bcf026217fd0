"""Host-only checks of the C ABI: the library loads, exports every function include/npweno.h
declares, and rejects bad parameters before touching the GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "npweno.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(npw[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1602_00182_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1602_00182_amd import build
        build.build()
    return binding.lib()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for fn in ("npweno_create", "npweno_step", "npweno_solve", "npweno_read", "npweno_destroy"):
        assert fn in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_abi_version_and_strerror(L):
    from paper_1602_00182_amd import binding as B
    assert L.npweno_abi_version() == B.NPW_ABI_VERSION
    for code in (B.OK, B.EINVAL, B.ENOMEM, B.EHIP, B.ENONFINITE, B.ENONPHYSICAL, B.EBUSY, B.ENOTFOUND):
        assert len(L.npweno_strerror(code)) > 0


def test_params_struct_matches_header_defaults(L):
    from paper_1602_00182_amd import binding as B
    p = B.make_params()
    assert p.abi_version == 2 and p.dim == 1 and p.nx == 80 and p.eps_m == 1e-12 and p.eps_weno == 1e-6
    assert p.variables == B.COMPONENTWISE and p.reserved == 0
    assert ctypes.sizeof(B.Params) == 8 * 4 + 8 * 2 + 8 * 11 + 8


@pytest.mark.parametrize("bad", [
    {"nx": 0}, {"flux": 7}, {"flux": 2, "ncomp": 1}, {"ncomp": 3}, {"bc": 5}, {"precision": 3},
    {"cfl": 0.0}, {"cfl": float("nan")}, {"eps_weno": -1.0}, {"eps_m": 0.0}, {"x1": -2.0},
    {"abi_version": 99}, {"recon": 8}, {"recon": 9}, {"switch_mode": 9}, {"dt_fixed": -1.0},
    {"flux": 2, "ncomp": 3, "gamma": 1.0}, {"variables": 1}, {"flux": 2, "ncomp": 3, "variables": 2},
    {"reserved": 1}, {"flux": 2, "ncomp": 3, "nx": 1 << 30}, {"nx": (1 << 31) - (1 << 16) + 1}, {"dim": 2, "nx": 64, "ny": 262141},
])
def test_create_rejects_bad_parameters_before_allocating(L, bad):
    from paper_1602_00182_amd import binding as B
    p = B.make_params(**bad)
    h = ctypes.c_void_p()
    buf = (ctypes.c_double * 1024)()
    rc = L.npweno_create(ctypes.byref(p), ctypes.cast(buf, ctypes.c_void_p), 0, None, ctypes.byref(h))
    assert rc == B.EINVAL
    assert not h.value


def test_null_arguments_rejected(L):
    from paper_1602_00182_amd import binding as B
    p = B.make_params()
    h = ctypes.c_void_p()
    assert L.npweno_create(ctypes.byref(p), None, 0, None, ctypes.byref(h)) == B.EINVAL
    assert L.npweno_create(None, None, 0, None, ctypes.byref(h)) == B.EINVAL
    assert L.npweno_step(None, 1.0, None) == B.EINVAL
    assert L.npweno_solve(None, 1.0, -1, None) == B.EINVAL
    assert L.npweno_read(None, None, 0) == B.EINVAL
    L.npweno_destroy(None)


def test_rhs_noalloc_rejects_bad_arguments_before_touching_the_gpu(L):
    """npweno_rhs_noalloc validates parameters, NULL pointers and overlapping buffers before any
    HIP call (the pointers here are never dereferenced)."""
    from paper_1602_00182_amd import binding as B
    ok = B.make_params(nx=80)
    u, out = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 24)
    assert L.npweno_rhs_noalloc(None, u, out, None, None) == B.EINVAL
    assert L.npweno_rhs_noalloc(ctypes.byref(ok), None, out, None, None) == B.EINVAL
    assert L.npweno_rhs_noalloc(ctypes.byref(ok), u, None, None, None) == B.EINVAL
    for bad in ({"nx": 0}, {"flux": 2, "ncomp": 1}, {"recon": 8}, {"reserved": 1}):
        p = B.make_params(**bad)
        assert L.npweno_rhs_noalloc(ctypes.byref(p), u, out, None, None) == B.EINVAL
    # L_out overlapping u (80 doubles = 640 bytes): rejected; adjacent is fine (not called here)
    assert L.npweno_rhs_noalloc(ctypes.byref(ok), u, ctypes.c_void_p((1 << 20) + 632), None, None) == B.EINVAL
    assert L.npweno_rhs_noalloc(ctypes.byref(ok), ctypes.c_void_p((1 << 20) + 8), u, None, None) == B.EINVAL
    assert len(L.npweno_strerror(B.ESCRATCH)) > 0
