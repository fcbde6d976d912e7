"""The C ABI library loads and exports every function its header declares (CPU only)."""
import ctypes

import pytest

from paper_2506_20350_amd import abi


def test_header_declares_the_core_calls():
    names = abi.header_symbols()
    for core in ["mlfft_create", "mlfft_set_blocks", "mlfft_matvec", "mlfft_precond_apply"]:
        assert core in names


def test_library_exports_every_declared_symbol():
    L = abi.lib()
    missing = [n for n in abi.header_symbols() if not hasattr(L, n)]
    assert not missing, f"symbols declared in include/mlfft.h but not exported: {missing}"


def test_every_exported_call_has_a_binding_signature():
    for n in abi.header_symbols():
        assert n in abi._SIGNATURES, n


def test_create_rejects_null_out_pointer_and_missing_allocator_without_touching_a_gpu():
    alloc = abi.ALLOC_FN(lambda n, u: None)
    free = abi.FREE_FN(lambda p, u: None)
    st = abi.lib().mlfft_create(0, None, alloc, free, None, None)
    assert st == abi.MLFFT_E_ARG
    assert b"NULL" in abi.lib().mlfft_last_error(None)
    h = ctypes.c_void_p()
    st = abi.lib().mlfft_create(0, None, abi.ALLOC_FN(), free, None, ctypes.byref(h))
    assert st == abi.MLFFT_E_ARG and not h.value
    assert b"alloc_fn" in abi.lib().mlfft_last_error(None)


def test_calls_on_null_context_are_argument_errors():
    L = abi.lib()
    assert L.mlfft_destroy(None) == abi.MLFFT_OK
    assert L.mlfft_matvec(None, 0, 1, None, None, 0) == abi.MLFFT_E_ARG
    assert L.mlfft_set_blocks(None, 0, 1, 1, 1, None, 0) == abi.MLFFT_E_ARG


def test_default_solve_options_fill_exactly_the_binding_layout():
    """mlfft_solve_default_opts writes every field of the header's struct and nothing past
    the binding's copy of it (a field added on one side only would show here)."""
    n = ctypes.sizeof(abi.SolveOpts)
    buf = (ctypes.c_ubyte * (n + 64))(*([0xA5] * (n + 64)))
    assert abi.lib().mlfft_solve_default_opts(ctypes.cast(buf, ctypes.POINTER(abi.SolveOpts))) == abi.MLFFT_OK
    assert bytes(buf[n:]) == b"\xa5" * 64
    o = abi.SolveOpts.from_buffer(buf)
    assert (o.restart, o.max_restarts, o.tol, o.inner_prec, o.max_outer, o.precond, o.orth) == \
        (30, 100, 1e-6, abi.MLFFT_FP32, 10, 1, 2)
    assert (o.x0_given, o.record_history, o.use_graph, o.mode, o.pc_bf16) == (0, 0, 0, 0, 0)


def test_no_device_allocation_call_in_the_library_sources():
    """Every device buffer comes from the caller's allocator: no hipMalloc / hipFree in csrc/."""
    import glob
    import os
    srcs = glob.glob(os.path.join(abi.PKG, "csrc", "*.cpp")) + glob.glob(os.path.join(abi.PKG, "csrc", "*.hip")) + \
        glob.glob(os.path.join(abi.PKG, "csrc", "*.h"))
    for f in srcs:
        txt = open(f).read()
        for bad in ("hipMalloc(", "hipMallocAsync", "hipFree(", "hipExtMalloc", "hipMallocManaged"):
            assert bad not in txt, (f, bad)
