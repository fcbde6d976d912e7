"""The allocation-free MLFFT product (mlfft_matvec_noalloc) against mlfft_matvec and the oracle,
through the C ABI: two calls in a row, the second with a smaller input, and the size limit."""
import gc

import numpy as np
import pytest
import torch

from oracle import toeplitz as tp
from paper_2506_20350_amd import abi, synth
from paper_2506_20350_amd.api import Context
from tests.gpu_util import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {abi.MLFFT_FP64: 1e-12, abi.MLFFT_FP32: 1e-5, abi.MLFFT_FP32_BF16GEMM: 2e-2}
DT = {abi.MLFFT_FP64: torch.complex128, abi.MLFFT_FP32: torch.complex64, abi.MLFFT_FP32_BF16GEMM: torch.complex64}


@pytest.mark.parametrize("prec", [abi.MLFFT_FP64, abi.MLFFT_FP32, abi.MLFFT_FP32_BF16GEMM])
def test_noalloc_matvec_equals_matvec_on_two_calls(prec):
    c = Context(0)
    cases = [(10, 10, 64, 100, 0), (5, 7, 12, 9, 1)]       # the second call is smaller
    for aid, (Nx, Ny, b, W, seed) in enumerate(cases):
        blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=seed)
        c.set_blocks(aid, blocks)
        X = synth.random_vectors(Nx * Ny * b, W, seed=seed + 3)
        x = to_dev(X, DT[prec])
        y_ref = torch.empty_like(x)
        y = torch.full_like(x, float("nan"))
        c.sync_stream()
        abi.mlfft_matvec(c.h, aid, W, x.data_ptr(), y_ref.data_ptr(), prec)
        held, calls = c.library_bytes(), c.alloc_calls
        gc.collect()
        torch.cuda.synchronize()
        mem = torch.cuda.memory_allocated()
        abi.mlfft_matvec_noalloc(c.h, aid, W, x.data_ptr(), y.data_ptr(), prec)
        torch.cuda.synchronize()
        # the library asked its allocator for nothing, and no device memory was taken
        assert c.alloc_calls == calls and c.library_bytes() == held
        assert torch.cuda.memory_allocated() <= mem
        assert torch.equal(y, y_ref), (aid, prec)          # same kernels, same arithmetic
        assert relerr(to_host(y), tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)) <= TOL[prec]
    c.close()


def test_noalloc_matvec_rejects_products_beyond_its_scratch():
    c = Context(0)
    Nx, Ny, b = 10, 10, 64
    c.set_blocks(0, synth.green_blocks(Nx, Ny, b, np.pi, seed=0))
    W = 164                                   # 4*100*64*164*16 bytes > 64 MiB in FP64
    x = torch.zeros((W, Nx * Ny * b), dtype=torch.complex128, device="cuda")
    y = torch.full_like(x, 3.0)
    c.sync_stream()
    with pytest.raises(abi.MlfftError) as e:
        abi.mlfft_matvec_noalloc(c.h, 0, W, x.data_ptr(), y.data_ptr(), abi.MLFFT_FP64)
    assert e.value.status == abi.MLFFT_E_ARG and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool(torch.all(y == 3.0))
    # the same W fits in FP32 (half the bytes per complex value)
    x32, y32 = x.to(torch.complex64), torch.empty((W, Nx * Ny * b), dtype=torch.complex64, device="cuda")
    c.sync_stream()
    abi.mlfft_matvec_noalloc(c.h, 0, W, x32.data_ptr(), y32.data_ptr(), abi.MLFFT_FP32)
    torch.cuda.synchronize()
    assert bool(torch.all(y32 == 0))
    c.close()
