"""PyTorch-facing wrapper of the C ABI.

PyTorch only provides device memory and the stream here; every step of the
solver path runs in libmlfft.so.  Tensors are passed by pointer after their
dtype, device, size and contiguity are checked, so that the library never sees
a buffer of the wrong shape.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import abi

PREC = {"fp64": abi.MLFFT_FP64, "fp32": abi.MLFFT_FP32, "bf16": abi.MLFFT_FP32_BF16GEMM}
PREC_DTYPE = {abi.MLFFT_FP64: torch.complex128, abi.MLFFT_FP32: torch.complex64,
              abi.MLFFT_FP32_BF16GEMM: torch.complex64}


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


class Context:
    """One library context on one device, enqueueing on the current PyTorch stream.

    Every device buffer the library holds comes from PyTorch's caching allocator
    (on the stream the context enqueues on), so it shows in
    torch.cuda.memory_allocated() and is returned to PyTorch's pool when the
    library frees it.
    """

    def __init__(self, device: int = 0, max_bytes: int = None):
        """max_bytes: optional cap on the device memory the library may hold at once; an
        allocation beyond it is refused and the call reports MLFFT_E_NOMEM."""
        self.device = device
        self.torch_device = torch.device("cuda", device)
        self._stream = torch.cuda.current_stream(self.torch_device)
        self._live = {}
        self.max_bytes = max_bytes
        self.alloc_calls = 0           # allocations the library asked for (granted or refused)

        def alloc(nbytes, user):
            self.alloc_calls += 1
            if self.max_bytes is not None and self.library_bytes() + int(nbytes) > self.max_bytes:
                return None
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self._stream)
            except Exception:          # out of memory: the library reports MLFFT_E_NOMEM
                return None
            self._live[p] = (int(nbytes), self._stream)
            return p

        def free(p, user):
            rec = self._live.pop(p, None)
            if rec is None:
                return
            # PyTorch reuses a freed block for later work on the stream it was allocated on;
            # if the context has moved to another stream since, the library's work on the
            # block is only ordered on the new stream, so wait for it first
            if rec[1] != self._stream:
                self._stream.synchronize()
            torch.cuda.caching_allocator_delete(p)

        # the callbacks must outlive the context
        self._alloc_cb = abi.ALLOC_FN(alloc)
        self._free_cb = abi.FREE_FN(free)
        self.h = abi.mlfft_create(device, self._stream.cuda_stream, self._alloc_cb, self._free_cb)
        self.arrays = {}

    def library_bytes(self) -> int:
        """Device bytes the library currently holds (all drawn from PyTorch's allocator)."""
        return int(sum(n for n, _ in self._live.values()))

    def close(self):
        if self.h is not None:
            abi.mlfft_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync_stream(self):
        self._stream = torch.cuda.current_stream(self.torch_device)
        abi.mlfft_set_stream(self.h, self._stream.cuda_stream)

    # ---------------------------------------------------------------- arrays
    def set_blocks(self, array_id: int, blocks) -> None:
        """blocks: complex128 array (2Ny-1, 2Nx-1, b, b), host (numpy / CPU tensor) or device tensor."""
        self.sync_stream()
        if isinstance(blocks, np.ndarray):
            blocks = torch.from_numpy(np.ascontiguousarray(blocks, dtype=np.complex128))
        if blocks.dtype != torch.complex128 or blocks.dim() != 4:
            raise ValueError("blocks must be a complex128 tensor of shape (2Ny-1, 2Nx-1, b, b)")
        blocks = blocks.contiguous()
        py, qx, b, b2 = blocks.shape
        if b != b2 or py % 2 == 0 or qx % 2 == 0:
            raise ValueError("blocks must have shape (2Ny-1, 2Nx-1, b, b)")
        Nx, Ny = (qx + 1) // 2, (py + 1) // 2
        on_dev = blocks.is_cuda
        abi.mlfft_set_blocks(self.h, array_id, Nx, Ny, b, blocks.data_ptr(), on_dev)
        self.arrays[array_id] = (Nx, Ny, b)

    def set_border(self, array_id: int, ZB=None, ZC=None) -> None:
        """Border blocks of the full matrix (Z_B: (Nc, N), Z_C: (Nc, Nc) complex128, host or device);
        None removes the border.  Vectors of the array then have N + Nc entries per column."""
        self.sync_stream()
        if ZB is None:
            abi.mlfft_set_border(self.h, array_id, 0, None, None, False)
            Nx, Ny, b = self.arrays[array_id][:3]
            self.arrays[array_id] = (Nx, Ny, b)
            return
        if isinstance(ZB, np.ndarray):
            ZB = torch.from_numpy(np.ascontiguousarray(ZB, dtype=np.complex128))
        if isinstance(ZC, np.ndarray):
            ZC = torch.from_numpy(np.ascontiguousarray(ZC, dtype=np.complex128))
        ZB, ZC = ZB.contiguous(), ZC.contiguous()
        Nx, Ny, b = self.arrays[array_id][:3]
        Nc = ZC.shape[0]
        if ZB.dtype != torch.complex128 or ZC.dtype != torch.complex128 or tuple(ZB.shape) != (Nc, Nx * Ny * b) \
                or tuple(ZC.shape) != (Nc, Nc) or ZB.is_cuda != ZC.is_cuda:
            raise ValueError("ZB must be complex128 (Nc, N) and ZC complex128 (Nc, Nc), on the same device")
        self.arrays[array_id] = (Nx, Ny, b)          # the library drops the old border first
        abi.mlfft_set_border(self.h, array_id, Nc, ZB.data_ptr(), ZC.data_ptr(), ZB.is_cuda)
        self.arrays[array_id] = (Nx, Ny, b, Nc)

    def vec_len(self, array_id: int) -> int:
        a = self.arrays[array_id]
        return a[0] * a[1] * a[2] + (a[3] if len(a) > 3 else 0)

    def info(self, array_id: int) -> abi.ArrayInfo:
        return abi.mlfft_array_info(self.h, array_id)

    def _check_vec(self, array_id: int, t: torch.Tensor, prec: int, name: str) -> int:
        n = self.vec_len(array_id)
        if not t.is_cuda or t.device.index != self.device:
            raise ValueError(f"{name} must be on cuda:{self.device}")
        if t.dtype != PREC_DTYPE[prec]:
            raise ValueError(f"{name} must be {PREC_DTYPE[prec]} for this precision")
        if not t.is_contiguous() or t.dim() != 2 or t.shape[1] != n:
            raise ValueError(f"{name} must be a contiguous (W, {n}) tensor")
        return t.shape[0]

    # ---------------------------------------------------------------- operators
    def matvec(self, array_id: int, x: torch.Tensor, y: torch.Tensor = None, prec="fp64") -> torch.Tensor:
        p = _prec(prec)
        W = self._check_vec(array_id, x, p, "x")
        if y is None:
            y = torch.empty_like(x)
        if self._check_vec(array_id, y, p, "y") != W:
            raise ValueError("x and y must have the same number of columns")
        self.sync_stream()
        abi.mlfft_matvec(self.h, array_id, W, x.data_ptr(), y.data_ptr(), p)
        return y

    def precond_apply(self, array_id: int, r: torch.Tensor, z: torch.Tensor = None, kind: int = 1,
                      prec="fp64") -> torch.Tensor:
        p = _prec(prec)
        W = self._check_vec(array_id, r, p, "r")
        if z is None:
            z = torch.empty_like(r)
        if self._check_vec(array_id, z, p, "z") != W:
            raise ValueError("r and z must have the same number of columns")
        self.sync_stream()
        abi.mlfft_precond_apply(self.h, array_id, kind, W, r.data_ptr(), z.data_ptr(), p)
        return z

    def spectrum(self, array_id: int, Omega: torch.Tensor, kind: int = 1, power_iters: int = 1) -> np.ndarray:
        """Largest singular values of P^{-1} Z from the l test vectors Omega (complex128 (l, N))."""
        l = self._check_vec(array_id, Omega, abi.MLFFT_FP64, "Omega")
        self.sync_stream()
        return abi.mlfft_spectrum(self.h, array_id, kind, l, Omega.data_ptr(), power_iters)

    def direct_solve(self, array_id: int, V: torch.Tensor, I: torch.Tensor = None):
        """Z I = V by block Rybicki (with a border: the Schur complement); returns (I, (rcond, flops))."""
        W = self._check_vec(array_id, V, abi.MLFFT_FP64, "V")
        if I is None:
            I = torch.empty_like(V)
        self._check_vec(array_id, I, abi.MLFFT_FP64, "I")
        self.sync_stream()
        return I, abi.mlfft_direct_solve(self.h, array_id, W, V.data_ptr(), I.data_ptr())

    # ---------------------------------------------------------------- solve
    @staticmethod
    def make_opts(**kw) -> abi.SolveOpts:
        o = abi.mlfft_solve_default_opts()
        for k, v in kw.items():
            if k == "inner_prec":
                v = _prec(v)
            if not hasattr(o, k):
                raise ValueError(f"unknown solve option {k}")
            setattr(o, k, v)
        return o

    @staticmethod
    def _info(Wt: int, history_len: int):
        arrs = dict(iters=np.zeros(Wt, np.int32), outer=np.zeros(Wt, np.int32), relres=np.zeros(Wt),
                    converged=np.zeros(Wt, np.int32),
                    history=np.zeros(max(history_len, 1) * Wt))
        info = abi.SolveInfo()
        info.iters = arrs["iters"].ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        info.outer = arrs["outer"].ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        info.relres = arrs["relres"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        info.converged = arrs["converged"].ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        info.history = arrs["history"].ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if history_len else None
        info.history_len = history_len
        return info, arrs

    @staticmethod
    def _pack(info, arrs, status, Wt, history_len):
        out = dict(status=status, iters=arrs["iters"].copy(), outer=arrs["outer"].copy(),
                   relres=arrs["relres"].copy(), converged=arrs["converged"].astype(bool),
                   fallbacks=info.fallbacks, matvecs64=info.matvecs64, matvecs_inner=info.matvecs_inner,
                   precond_applies=info.precond_applies, net_applies=info.net_applies,
                   pc_switched=info.pc_switched)
        if history_len:
            out["history"] = arrs["history"].reshape(history_len, Wt).copy()
        return out

    def solve(self, array_id: int, V: torch.Tensor, I: torch.Tensor = None, history_len: int = 0, **opts):
        """Solve Z I = V (complex128 device tensors of shape (W, N)); returns (I, info dict)."""
        W = self._check_vec(array_id, V, abi.MLFFT_FP64, "V")
        if I is None:
            I = torch.zeros_like(V)
        self._check_vec(array_id, I, abi.MLFFT_FP64, "I")
        o = self.make_opts(record_history=1 if history_len else 0, **opts)
        info, arrs = self._info(W, history_len)
        self.sync_stream()
        st = abi.mlfft_solve(self.h, array_id, W, V.data_ptr(), I.data_ptr(), o, info)
        return I, self._pack(info, arrs, st, W, history_len)

    def solve_batch(self, array_ids, Vs, Is=None, history_len: int = 0, **opts):
        """One batched solve over several arrays; returns (list of I, info dict over the concatenated columns)."""
        Ws = [self._check_vec(a, v, abi.MLFFT_FP64, "V") for a, v in zip(array_ids, Vs)]
        if Is is None:
            Is = [torch.zeros_like(v) for v in Vs]
        for a, i in zip(array_ids, Is):
            self._check_vec(a, i, abi.MLFFT_FP64, "I")
        o = self.make_opts(record_history=1 if history_len else 0, **opts)
        Wt = sum(Ws)
        info, arrs = self._info(Wt, history_len)
        self.sync_stream()
        st = abi.mlfft_solve_batch(self.h, list(array_ids), Ws, [v.data_ptr() for v in Vs],
                                   [i.data_ptr() for i in Is], o, info)
        return Is, self._pack(info, arrs, st, Wt, history_len)
