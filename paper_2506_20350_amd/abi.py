"""ctypes binding of the C ABI in include/mlfft.h.

Argument marshalling only: every function here forwards to the function of the
same name in libmlfft.so.  Device buffers are passed as raw pointers (for
PyTorch tensors, ``tensor.data_ptr()``); streams as ``hipStream_t`` values
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if the
library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libmlfft.so")
HEADERS = [os.path.join(os.path.dirname(PKG), "include", "mlfft.h")]

MLFFT_OK = 0
MLFFT_NOT_CONVERGED = 1
MLFFT_E_ARG = -1
MLFFT_E_NOMEM = -2
MLFFT_E_HIP = -3
MLFFT_E_SINGULAR = -4
MLFFT_E_STATE = -5

MLFFT_FP64 = 0
MLFFT_FP32 = 1
MLFFT_FP32_BF16GEMM = 2

STATUS_NAMES = {0: "MLFFT_OK", 1: "MLFFT_NOT_CONVERGED", -1: "MLFFT_E_ARG", -2: "MLFFT_E_NOMEM",
                -3: "MLFFT_E_HIP", -4: "MLFFT_E_SINGULAR", -5: "MLFFT_E_STATE"}


class MlfftError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ArrayInfo(ctypes.Structure):
    _fields_ = [("Nx", ctypes.c_int), ("Ny", ctypes.c_int), ("b", ctypes.c_int),
                ("Px", ctypes.c_int), ("Py", ctypes.c_int), ("pc_fallbacks", ctypes.c_int),
                ("pc_min_rcond", ctypes.c_double), ("device_bytes", ctypes.c_size_t), ("Nc", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_restarts", ctypes.c_int), ("tol", ctypes.c_double),
                ("inner_prec", ctypes.c_int), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("precond", ctypes.c_int), ("orth", ctypes.c_int), ("x0_given", ctypes.c_int),
                ("record_history", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("mode", ctypes.c_int), ("pc_bf16", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.POINTER(ctypes.c_int)), ("outer", ctypes.POINTER(ctypes.c_int)),
                ("relres", ctypes.POINTER(ctypes.c_double)), ("converged", ctypes.POINTER(ctypes.c_int)),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int),
                ("fallbacks", ctypes.c_int), ("matvecs64", ctypes.c_int), ("matvecs_inner", ctypes.c_int),
                ("precond_applies", ctypes.c_int), ("net_applies", ctypes.c_int), ("pc_switched", ctypes.c_int)]


# device allocator callbacks of mlfft_create
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


_P = ctypes.c_void_p
_I = ctypes.c_int
_ST = ctypes.c_int

_SIGNATURES = {
    "mlfft_create": (_ST, [_I, _P, ALLOC_FN, FREE_FN, _P, ctypes.POINTER(_P)]),
    "mlfft_destroy": (_ST, [_P]),
    "mlfft_last_error": (ctypes.c_char_p, [_P]),
    "mlfft_set_stream": (_ST, [_P, _P]),
    "mlfft_set_blocks": (_ST, [_P, _I, _I, _I, _I, _P, _I]),
    "mlfft_drop_array": (_ST, [_P, _I]),
    "mlfft_array_info": (_ST, [_P, _I, ctypes.POINTER(ArrayInfo)]),
    "mlfft_matvec": (_ST, [_P, _I, _I, _P, _P, _I]),
    "mlfft_matvec_noalloc": (_ST, [_P, _I, _I, _P, _P, _I]),
    "mlfft_matvec_axpby": (_ST, [_P, _I, _I, ctypes.c_double, _P, ctypes.c_double, _P, _P, _I]),
    "mlfft_axpby": (_ST, [_P, ctypes.c_size_t, ctypes.c_double, _P, ctypes.c_double, _P, _I, _P, _I]),
    "mlfft_precond_apply": (_ST, [_P, _I, _I, _I, _P, _P, _I]),
    "mlfft_solve_default_opts": (_ST, [ctypes.POINTER(SolveOpts)]),
    "mlfft_solve": (_ST, [_P, _I, _I, _P, _P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]),
    "mlfft_solve_batch": (_ST, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_P),
                                ctypes.POINTER(_P), ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]),
    "mlfft_net_create": (_ST, [_P, _I, _I, ctypes.c_uint]),
    "mlfft_net_set_weights": (_ST, [_P, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
    "mlfft_net_get_weights": (_ST, [_P, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
    "mlfft_net_num_weights": (ctypes.c_size_t, [_P]),
    "mlfft_net_forward": (_ST, [_P, _I, _I, _I, _P, _P]),
    "mlfft_net_train_step": (_ST, [_P, _I, _I, _I, _P, _P, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]),
    "mlfft_net_grads": (_ST, [_P, _I, _I, _I, _P, _P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "mlfft_net_apply": (_ST, [_P, _I, _I, _P, _P]),
}

_lib = None


def header_symbols() -> list:
    """Every function name declared in include/*.h."""
    names = []
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"\b(mlfft_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2506_20350_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


def check(ctx, status: int, what: str = "") -> int:
    if status < 0:
        msg = lib().mlfft_last_error(ctx)
        raise MlfftError(status, (msg.decode() if msg else "") + (f" ({what})" if what else ""))
    return status


def mlfft_create(device: int, stream: int, alloc_fn: ALLOC_FN, free_fn: FREE_FN, user: int = 0):
    """alloc_fn / free_fn: ALLOC_FN / FREE_FN callbacks; the caller keeps them alive until mlfft_destroy."""
    h = ctypes.c_void_p()
    st = lib().mlfft_create(device, stream or None, alloc_fn, free_fn, user or None, ctypes.byref(h))
    if st != MLFFT_OK:
        raise MlfftError(st, lib().mlfft_last_error(None).decode())
    return h


def mlfft_destroy(ctx):
    return check(ctx, lib().mlfft_destroy(ctx))


def mlfft_set_stream(ctx, stream: int):
    return check(ctx, lib().mlfft_set_stream(ctx, stream or None))


def mlfft_set_blocks(ctx, array_id: int, Nx: int, Ny: int, b: int, blocks_ptr: int, on_device: bool):
    return check(ctx, lib().mlfft_set_blocks(ctx, array_id, Nx, Ny, b, blocks_ptr, int(on_device)))


def mlfft_drop_array(ctx, array_id: int):
    return check(ctx, lib().mlfft_drop_array(ctx, array_id))


def mlfft_array_info(ctx, array_id: int) -> ArrayInfo:
    info = ArrayInfo()
    check(ctx, lib().mlfft_array_info(ctx, array_id, ctypes.byref(info)))
    return info


def mlfft_matvec(ctx, array_id: int, W: int, x_ptr: int, y_ptr: int, prec: int):
    return check(ctx, lib().mlfft_matvec(ctx, array_id, W, x_ptr, y_ptr, prec))


def mlfft_matvec_noalloc(ctx, array_id: int, W: int, x_ptr: int, y_ptr: int, prec: int):
    return check(ctx, lib().mlfft_matvec_noalloc(ctx, array_id, W, x_ptr, y_ptr, prec))


def mlfft_matvec_axpby(ctx, array_id: int, W: int, alpha: float, x_ptr: int, beta: float, v_ptr, y_ptr: int,
                       prec: int):
    return check(ctx, lib().mlfft_matvec_axpby(ctx, array_id, W, alpha, x_ptr, beta, v_ptr or None, y_ptr, prec))


def mlfft_axpby(ctx, n: int, alpha: float, x_ptr: int, beta: float, y_ptr, in_prec: int, out_ptr: int,
                out_prec: int):
    return check(ctx, lib().mlfft_axpby(ctx, n, alpha, x_ptr, beta, y_ptr or None, in_prec, out_ptr, out_prec))


def mlfft_precond_apply(ctx, array_id: int, kind: int, W: int, r_ptr: int, z_ptr: int, prec: int):
    return check(ctx, lib().mlfft_precond_apply(ctx, array_id, kind, W, r_ptr, z_ptr, prec))


def mlfft_solve_default_opts() -> SolveOpts:
    o = SolveOpts()
    st = lib().mlfft_solve_default_opts(ctypes.byref(o))
    if st != MLFFT_OK:
        raise MlfftError(st, "mlfft_solve_default_opts")
    return o


def mlfft_solve(ctx, array_id: int, W: int, V_ptr: int, I_ptr: int, opts: SolveOpts, info: SolveInfo) -> int:
    return check(ctx, lib().mlfft_solve(ctx, array_id, W, V_ptr, I_ptr, ctypes.byref(opts),
                                        ctypes.byref(info) if info is not None else None))


def mlfft_solve_batch(ctx, array_ids, Ws, V_ptrs, I_ptrs, opts: SolveOpts, info: SolveInfo) -> int:
    n = len(array_ids)
    ids = (ctypes.c_int * n)(*array_ids)
    ws = (ctypes.c_int * n)(*Ws)
    vp = (ctypes.c_void_p * n)(*V_ptrs)
    ip = (ctypes.c_void_p * n)(*I_ptrs)
    return check(ctx, lib().mlfft_solve_batch(ctx, n, ids, ws, vp, ip, ctypes.byref(opts),
                                              ctypes.byref(info) if info is not None else None))


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("prec", ctypes.c_int), ("launches", ctypes.c_long),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


_SIGNATURES["mlfft_profile_enable"] = (_ST, [_P, _I])
_SIGNATURES["mlfft_profile_read"] = (_ST, [_P, ctypes.POINTER(KernelStat), _I, ctypes.POINTER(_I)])


def mlfft_profile_enable(ctx, enable: bool):
    return check(ctx, lib().mlfft_profile_enable(ctx, int(enable)))


def mlfft_profile_read(ctx) -> list:
    buf = (KernelStat * 32)()
    n = ctypes.c_int(0)
    check(ctx, lib().mlfft_profile_read(ctx, buf, 32, ctypes.byref(n)))
    return [dict(name=buf[i].name.decode(), prec=buf[i].prec, launches=buf[i].launches, ms=buf[i].ms,
                 bytes=buf[i].bytes, flops=buf[i].flops) for i in range(min(n.value, 32))]


def mlfft_net_create(ctx, b: int, hidden: int, seed: int = 0):
    return check(ctx, lib().mlfft_net_create(ctx, b, hidden, seed))


def mlfft_net_num_weights(ctx) -> int:
    return int(lib().mlfft_net_num_weights(ctx))


def mlfft_net_set_weights(ctx, w):
    import numpy as np
    w = np.ascontiguousarray(w, dtype=np.float32)
    return check(ctx, lib().mlfft_net_set_weights(ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size))


def mlfft_net_get_weights(ctx):
    import numpy as np
    n = mlfft_net_num_weights(ctx)
    w = np.zeros(n, dtype=np.float32)
    check(ctx, lib().mlfft_net_get_weights(ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n))
    return w


def mlfft_net_forward(ctx, W: int, H: int, Wd: int, x_ptr: int, out_ptr: int):
    return check(ctx, lib().mlfft_net_forward(ctx, W, H, Wd, x_ptr, out_ptr))


def mlfft_net_apply(ctx, array_id: int, W: int, y_ptr: int, z_ptr: int):
    return check(ctx, lib().mlfft_net_apply(ctx, array_id, W, y_ptr, z_ptr))


def mlfft_net_grads(ctx, W: int, H: int, Wd: int, y_ptr: int, e_ptr: int, want_grads: bool = True):
    import numpy as np
    g = np.zeros(mlfft_net_num_weights(ctx), dtype=np.float32) if want_grads else None
    loss = ctypes.c_float(0.0)
    gp = g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if want_grads else None
    check(ctx, lib().mlfft_net_grads(ctx, W, H, Wd, y_ptr, e_ptr, gp, ctypes.byref(loss)))
    return g, float(loss.value)


def mlfft_net_train_step(ctx, W: int, H: int, Wd: int, y_ptr: int, e_ptr: int, lr: float) -> float:
    loss = ctypes.c_float(0.0)
    check(ctx, lib().mlfft_net_train_step(ctx, W, H, Wd, y_ptr, e_ptr, lr, ctypes.byref(loss)))
    return float(loss.value)


_L = ctypes.c_long
_D = ctypes.c_double
_SIGNATURES["mlfft_set_border"] = (_ST, [_P, _I, _I, _P, _P, _I])


def mlfft_set_border(ctx, array_id: int, Nc: int, ZB_ptr, ZC_ptr, on_device: bool):
    return check(ctx, lib().mlfft_set_border(ctx, array_id, Nc, ZB_ptr or None, ZC_ptr or None, int(on_device)))


_SIGNATURES["mlfft_spectrum"] = (_ST, [_P, _I, _I, _I, _P, _I, ctypes.POINTER(ctypes.c_double)])


def mlfft_spectrum(ctx, array_id: int, kind: int, l: int, Omega_ptr: int, power_iters: int = 0):
    """Largest singular values (descending numpy array of l values) of P^{-1} Z."""
    import numpy as np
    out = np.zeros(l, dtype=np.float64)
    check(ctx, lib().mlfft_spectrum(ctx, array_id, kind, l, Omega_ptr, power_iters,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


_SIGNATURES["mlfft_direct_solve"] = (_ST, [_P, _I, _I, _P, _P, ctypes.POINTER(_D), ctypes.POINTER(_D)])
_SIGNATURES["mlfft_dense_gemm"] = (_ST, [_P, _I, _I, _I, _I, _D, _D, _P, _L, _P, _L, _D, _D, _P, _L])
_SIGNATURES["mlfft_dense_solve"] = (_ST, [_P, _I, _P, _L, _P, _L, _I])
_SIGNATURES["mlfft_dense_gemm_ah"] = (_ST, [_P, _I, _I, _I, _D, _D, _P, _L, _P, _L, _D, _D, _P, _L])
_SIGNATURES["mlfft_dense_gen_eig"] = (_ST, [_P, _I, _P, _P, ctypes.POINTER(_D)])


def mlfft_dense_gemm_ah(ctx, M: int, N: int, K: int, alpha: complex, A_ptr: int, lda: int, B_ptr: int, ldb: int,
                        beta: complex, C_ptr: int, ldc: int):
    alpha, beta = complex(alpha), complex(beta)
    return check(ctx, lib().mlfft_dense_gemm_ah(ctx, M, N, K, alpha.real, alpha.imag, A_ptr, lda, B_ptr, ldb,
                                                beta.real, beta.imag, C_ptr, ldc))


def mlfft_dense_gen_eig(ctx, l: int, G_ptr: int, M_ptr: int):
    import numpy as np
    out = np.zeros(l, dtype=np.float64)
    check(ctx, lib().mlfft_dense_gen_eig(ctx, l, G_ptr, M_ptr, out.ctypes.data_as(ctypes.POINTER(_D))))
    return out


def mlfft_direct_solve(ctx, array_id: int, W: int, V_ptr: int, I_ptr: int):
    """Returns (smallest rcond of the recursion's inverses, flops executed)."""
    rc = ctypes.c_double(0.0)
    fl = ctypes.c_double(0.0)
    check(ctx, lib().mlfft_direct_solve(ctx, array_id, W, V_ptr, I_ptr, ctypes.byref(rc), ctypes.byref(fl)))
    return rc.value, fl.value


def mlfft_dense_gemm(ctx, prec: int, M: int, N: int, K: int, alpha: complex, A_ptr: int, lda: int, B_ptr: int,
                     ldb: int, beta: complex, C_ptr: int, ldc: int):
    alpha, beta = complex(alpha), complex(beta)
    return check(ctx, lib().mlfft_dense_gemm(ctx, prec, M, N, K, alpha.real, alpha.imag, A_ptr, lda, B_ptr, ldb,
                                             beta.real, beta.imag, C_ptr, ldc))


def mlfft_dense_solve(ctx, n: int, A_ptr: int, lda: int, B_ptr: int, ldb: int, ncols: int):
    return check(ctx, lib().mlfft_dense_solve(ctx, n, A_ptr, lda, B_ptr, ldb, ncols))


_SIGNATURES["mlfft_autotune"] = (_ST, [_P, _I, _I, _I, _I])
_SIGNATURES["mlfft_tune_report"] = (_ST, [_P, _I, ctypes.c_char_p, ctypes.c_size_t])
_SIGNATURES["mlfft_tune_import"] = (_ST, [_P, ctypes.c_char_p])


def mlfft_autotune(ctx, array_id: int, W: int, prec: int, reps: int = 3):
    return check(ctx, lib().mlfft_autotune(ctx, array_id, W, prec, reps))


def mlfft_tune_report(ctx, array_id: int) -> str:
    buf = ctypes.create_string_buffer(1 << 16)
    check(ctx, lib().mlfft_tune_report(ctx, array_id, buf, len(buf)))
    return buf.value.decode()


def mlfft_tune_import(ctx, text: str):
    return check(ctx, lib().mlfft_tune_import(ctx, text.encode()))
