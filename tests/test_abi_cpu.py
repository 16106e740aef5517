"""The C ABI library on a machine without a GPU: it loads, exports every function
include/qiral.h declares, sizes packed fields correctly, and rejects invalid
arguments with the right status before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1401_2039_amd import _lib as L
from paper_1401_2039_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qiral.h")

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built (run __graft_entry__.build())")


def header_functions():
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(qiral_[a-z_A-Z0-9]+)\s*\(", txt)))


def test_exports_match_header():
    lib = L.load()
    names = header_functions()
    assert names and set(names) == set(L.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    lib = L.load()
    for s in range(8):
        assert lib.qiral_status_string(s)
    assert lib.qiral_status_string(99) == b"unknown status"


def test_field_bytes():
    # 4^4: 128 sites per parity -> 2 blocks of 64
    assert api.qiral_field_bytes((4, 4, 4, 4), L.ODD, L.F64) == 128 * 192
    assert api.qiral_field_bytes((4, 4, 4, 4), L.FULL, L.F32, 3) == 2 * 128 * 96 * 3
    assert api.qiral_field_bytes((4, 4, 4, 4), L.EVEN, L.F16S) == 128 * 52
    # 2^4: 8 sites per parity, padded to one block of 64
    assert api.qiral_field_bytes((2, 2, 2, 2), L.EVEN, L.F64) == 64 * 192
    assert api.qiral_field_bytes((24, 24, 24, 48), L.ODD, L.F16S) == 331776 * 52
    # invalid -> 0
    assert api.qiral_field_bytes((3, 4, 4, 4), L.ODD, L.F64) == 0
    assert api.qiral_field_bytes((4, 4, 4, 4), 7, L.F64) == 0
    assert api.qiral_field_bytes((4, 4, 4, 4), L.ODD, 9) == 0
    assert api.qiral_field_bytes((4, 4, 4, 4), L.ODD, L.F64, 0) == 0


def test_gauge_bytes():
    # 4^4: 2 blocks of 64 sites per parity, 8 links (4 directions x 2 parities) per padded site
    n = 8 * 128
    assert api.qiral_gauge_bytes((4, 4, 4, 4), L.F64) == n * 144
    assert api.qiral_gauge_bytes((4, 4, 4, 4), L.F32) == n * 48
    assert api.qiral_gauge_bytes((4, 4, 4, 4), L.F16S) == n * 24
    assert api.qiral_gauge_bytes((24, 24, 24, 48), L.F32) == 8 * 331776 * 48
    # the combinations the library does not build, and invalid dims -> 0
    assert api.qiral_gauge_bytes((4, 4, 4, 4), L.F32, L.RECON18) == 0
    assert api.qiral_gauge_bytes((4, 4, 4, 4), L.F64, L.RECON12) == 0
    assert api.qiral_gauge_bytes((4, 4, 4, 4), L.F64, 7) == 0
    assert api.qiral_gauge_bytes((4, 5, 4, 4), L.F64) == 0


def _create(dims, gauge=1, kappa=0.12, mu=0.0, g64=256, g32=None, g16=None):
    lib = L.load()
    h = ctypes.c_void_p()
    return lib.qiral_lattice_create(ctypes.byref(h), L.dims_arg(dims), kappa, mu, ctypes.c_void_p(gauge),
                                    ctypes.c_void_p(g64), ctypes.c_void_p(g32), ctypes.c_void_p(g16), None), h


def test_create_validation():
    lib = L.load()
    one = ctypes.c_void_p(256)
    assert lib.qiral_lattice_create(None, L.dims_arg((4, 4, 4, 4)), 0.1, 0.0, one, one, None, None, None) == L.ERR_INVALID_ARG
    assert _create((3, 4, 4, 4))[0] == L.ERR_BAD_DIMS
    assert _create((4, 4, 0, 4))[0] == L.ERR_BAD_DIMS
    assert _create((4, 4, 4, 4), gauge=0)[0] == L.ERR_INVALID_ARG
    assert _create((4, 4, 4, 4), g64=None)[0] == L.ERR_INVALID_ARG          # the FP64 store is required
    assert b"gauge_f64" in lib.qiral_last_error()
    assert _create((4, 4, 4, 4), kappa=float("nan"))[0] == L.ERR_INVALID_ARG
    assert _create((4, 4, 4, 4), mu=float("inf"))[0] == L.ERR_INVALID_ARG
    assert _create((4, 4, 4, 4), g32=257)[0] == L.ERR_INVALID_ARG           # misaligned store
    assert _create((4, 4, 4, 4), g32=256)[0] == L.ERR_INVALID_ARG           # the same buffer twice
    st, h = _create((4, 4, 4, 4), g16=512, g32=512)
    assert st == L.ERR_INVALID_ARG and h.value is None


def test_null_handles_rejected():
    lib = L.load()
    one = ctypes.c_void_p(1)
    assert lib.qiral_lattice_destroy(None) == L.ERR_INVALID_ARG
    assert lib.qiral_field_import(None, one, one, L.ODD, L.F64, 1, None) == L.ERR_INVALID_ARG
    assert lib.qiral_field_export(None, one, one, L.ODD, L.F64, 1, None) == L.ERR_INVALID_ARG
    assert lib.qiral_dslash_eo(None, one, one, 0, 0, L.F64, 1, None) == L.ERR_INVALID_ARG
    assert lib.qiral_apply_M(None, one, one, one, L.OP_D, L.F64, 1, None) == L.ERR_INVALID_ARG
    p = api.solve_params()
    info = (L.SolveInfo * 1)()
    ws = ctypes.c_void_p(256)
    assert lib.qiral_solve(None, one, one, 1, ctypes.byref(p), ws, 1 << 20, info, None) == L.ERR_INVALID_ARG
    assert lib.qiral_solve_batch(None, None, None, 1, ctypes.byref(p), ws, 1 << 20, info, None) == L.ERR_INVALID_ARG
    assert lib.qiral_lattice_query(None, None, None) == L.ERR_INVALID_ARG
    assert lib.qiral_tune(None, L.F32, 1, one, one, None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.qiral_nn_create(None, one, 8, one, 1, None) == L.ERR_INVALID_ARG
    assert lib.qiral_nn_destroy(None) == L.ERR_INVALID_ARG
    # size queries answer 0 for invalid arguments
    assert lib.qiral_solve_workspace_bytes(None, ctypes.byref(p), 1) == 0
    assert lib.qiral_solve_batch_workspace_bytes(None, 1, ctypes.byref(p)) == 0
    assert lib.qiral_nn_bytes(None, 8) == 0


def test_solve_params_validation():
    """Parameter checks run before the lattice handle or any HIP call is used, so
    a stand-in handle exercises them on the CPU."""
    lib = L.load()
    one = ctypes.c_void_p(1)
    info = (L.SolveInfo * 1)()

    def solve(**kw):
        p = api.solve_params(**kw)
        return lib.qiral_solve(one, one, one, 1, ctypes.byref(p), ctypes.c_void_p(256), 1 << 20, info, None)

    assert solve(tol=0.0) == L.ERR_INVALID_ARG
    assert solve(maxiter=0) == L.ERR_INVALID_ARG
    assert solve(solver=9) == L.ERR_INVALID_ARG
    assert solve(inner_prec=7) == L.ERR_INVALID_ARG
    assert solve(inner_prec=L.F32, delta=1.5) == L.ERR_INVALID_ARG
    assert solve(solver=L.CRNR_EO, inner_prec=L.F32) == L.ERR_UNSUPPORTED
    assert b"conjugate residual" in lib.qiral_last_error()
    assert solve(solver=L.FCG_NN, precond=1, inner_prec=L.F32) == L.ERR_UNSUPPORTED
    # compositions: the system must be known; CGNR / CRNR take no preconditioner;
    # CRNR runs on the Schur system; the flexible forms run in FP64
    assert solve(system=3) == L.ERR_INVALID_ARG
    assert solve(precond=1) == L.ERR_UNSUPPORTED
    assert solve(solver=L.CRNR_EO, precond=1) == L.ERR_UNSUPPORTED
    assert solve(solver=L.CRNR_EO, system=L.SYSTEM_FULL) == L.ERR_UNSUPPORTED
    assert solve(solver=L.BICGSTAB_EO, precond=1, inner_prec=L.F32) == L.ERR_UNSUPPORTED
    assert solve(solver=L.BICGSTAB_EO, system=L.SYSTEM_FULL, inner_prec=L.F16S) == L.ERR_UNSUPPORTED
    assert solve(system=L.SYSTEM_FULL, inner_prec=L.F32) == L.ERR_UNSUPPORTED
    assert solve(solver=L.FGMRES_NN, system=L.SYSTEM_SCHUR, inner_prec=L.F32) == L.ERR_UNSUPPORTED
    assert solve(solver=L.FGMRES_NN, precond=1, inner_prec=L.F16S) == L.ERR_UNSUPPORTED
    assert solve(solver=L.FGMRES_NN, precond=1, restart=65) == L.ERR_INVALID_ARG
    # an invalid parameter set has no workspace size
    p = api.solve_params(tol=-1.0)
    assert lib.qiral_solve_workspace_bytes(one, ctypes.byref(p), 1) == 0
    assert lib.qiral_solve_workspace_bytes(one, ctypes.byref(api.solve_params()), 0) == 0
    assert lib.qiral_solve_workspace_bytes(one, ctypes.byref(api.solve_params()), 256) == 0


def test_workspace_pointer_checked_before_the_handle():
    """A missing or misaligned workspace is refused before the lattice handle is
    read or any HIP call is made (a stand-in handle would fault if it were)."""
    lib = L.load()
    one = ctypes.c_void_p(1)
    info = (L.SolveInfo * 1)()
    p = api.solve_params()
    assert lib.qiral_solve(one, one, one, 1, ctypes.byref(p), None, 1 << 30, info, None) == L.ERR_WORKSPACE
    assert b"qiral_solve_workspace_bytes" in lib.qiral_last_error()
    assert lib.qiral_solve(one, one, one, 1, ctypes.byref(p), ctypes.c_void_p(4096 + 16), 1 << 30, info,
                           None) == L.ERR_INVALID_ARG
    assert b"aligned" in lib.qiral_last_error()
    arr = (ctypes.c_void_p * 1)(1)
    assert lib.qiral_solve_batch(arr, arr, arr, 1, ctypes.byref(p), None, 1 << 30, info, None) == L.ERR_WORKSPACE


def test_batch_rejects_learned_solvers():
    """FGMRES, FCG and the preconditioned or full-system forms take one lattice:
    the batch entry refuses them before it reads the lattice table."""
    lib = L.load()
    info = (L.SolveInfo * 1)()
    arr = (ctypes.c_void_p * 1)(1)
    for kw in (dict(solver=L.FGMRES_NN, precond=1), dict(solver=L.FCG_NN), dict(solver=L.BICGSTAB_EO, precond=1),
               dict(solver=L.CGNR_EO, system=L.SYSTEM_FULL)):
        p = api.solve_params(**kw)
        assert lib.qiral_solve_batch(arr, arr, arr, 1, ctypes.byref(p), ctypes.c_void_p(256), 1 << 20, info,
                                     None) == L.ERR_UNSUPPORTED
        assert b"one lattice" in lib.qiral_last_error()

