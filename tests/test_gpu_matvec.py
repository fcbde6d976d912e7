"""GPU parity of the MLFFT matvec and the preconditioner apply against the oracle.

Bars, per column (the largest relative error over the W columns): FP64 1e-12,
FP32 1e-5, block product
with bf16 inputs 2e-2 (its own bound: bf16 keeps 8 significant bits, so one
rounding of G and of the transformed vector costs ~2^-9 relative each).
"""
import numpy as np
import pytest
import torch

from oracle import direct
from oracle import precond as opc
from oracle import toeplitz as tp
from paper_2506_20350_amd import abi, synth
from tests.gpu_util import ctx, relerr, to_dev, to_host  # noqa: F401

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 2e-2}
DT = {"fp64": torch.complex128, "fp32": torch.complex64, "bf16": torch.complex64}

# (Nx, Ny, b, W, generator): single cell, ragged W over one 64-column tile, b not a
# multiple of 8, prime grid sizes, the largest grid, large and maximal b
CASES = [
    (1, 1, 3, 2, "random"),
    (3, 2, 5, 3, "random"),
    (4, 4, 24, 1, "green"),
    (5, 7, 12, 70, "random"),
    (13, 11, 17, 5, "green"),
    (10, 10, 64, 100, "green"),
    (32, 32, 8, 3, "random"),
    (2, 3, 200, 2, "green"),
    (3, 2, 256, 1, "random"),
    (7, 1, 9, 4, "random"),
    (1, 6, 10, 4, "random"),
    (19, 17, 8, 3, "green"),
]


def make_blocks(Nx, Ny, b, kind, seed=0):
    if kind == "green":
        return synth.green_blocks(Nx, Ny, b, np.pi, seed=seed)
    return synth.random_blocks(Nx, Ny, b, seed=seed + 17)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:4])) + c[4][0])
def test_matvec_matches_oracle(ctx, case, prec):
    Nx, Ny, b, W, kind = case
    blocks = make_blocks(Nx, Ny, b, kind)
    ctx.set_blocks(1, blocks)
    X = synth.random_vectors(Nx * Ny * b, W, seed=3)
    ref = tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)
    y = ctx.matvec(1, to_dev(X, DT[prec]), prec=prec)
    err = relerr(to_host(y), ref)
    assert err <= TOL[prec], err


@pytest.mark.parametrize("case", [(3, 2, 5, 3, "random"), (4, 4, 24, 2, "green")], ids=str)
def test_matvec_fp64_matches_dense(ctx, case):
    Nx, Ny, b, W, kind = case
    blocks = make_blocks(Nx, Ny, b, kind)
    ctx.set_blocks(2, blocks)
    X = synth.random_vectors(Nx * Ny * b, W, seed=5)
    ref = tp.matvec_dense(tp.dense_Z(blocks), X)
    y = ctx.matvec(2, to_dev(X))
    assert relerr(to_host(y), ref) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", [(4, 4, 24, 3), (5, 7, 12, 70), (13, 11, 17, 5), (10, 10, 64, 100), (1, 1, 4, 2),
                                  (32, 32, 8, 2), (6, 5, 200, 2), (19, 12, 24, 3), (16, 19, 48, 2)], ids=str)
def test_block_circulant_apply_matches_oracle(ctx, case, prec):
    Nx, Ny, b, W = case
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=1)
    ctx.set_blocks(3, blocks)
    R = synth.random_vectors(Nx * Ny * b, W, seed=2)
    ref = opc.strang_apply(opc.strang_inverse_spectrum(blocks), R)
    z = ctx.precond_apply(3, to_dev(R, DT[prec]), kind=1, prec=prec)
    assert relerr(to_host(z), ref) <= TOL[prec] * 10
    assert ctx.info(3).pc_fallbacks == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_self_block_apply_matches_oracle(ctx, prec):
    Nx, Ny, b, W = 5, 3, 20, 7
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=4)
    ctx.set_blocks(4, blocks)
    R = synth.random_vectors(Nx * Ny * b, W, seed=6)
    ref = opc.kindt_apply(blocks, R)
    z = ctx.precond_apply(4, to_dev(R, DT[prec]), kind=2, prec=prec)
    assert relerr(to_host(z), ref) <= TOL[prec] * 10


def test_periodic_operator_is_inverted_exactly_by_block_circulant(ctx):
    Nx, Ny, b, W = 6, 4, 8, 3
    blocks = synth.periodic_blocks(Nx, Ny, b, seed=2)
    ctx.set_blocks(5, blocks)
    X = synth.random_vectors(Nx * Ny * b, W, seed=1)
    y = ctx.matvec(5, to_dev(X))
    z = ctx.precond_apply(5, y, kind=1)
    assert relerr(to_host(z), X) <= 1e-12


def test_matvec_is_deterministic(ctx):
    Nx, Ny, b, W = 10, 10, 64, 100
    ctx.set_blocks(6, synth.green_blocks(Nx, Ny, b, np.pi, seed=0))
    x = to_dev(synth.random_vectors(Nx * Ny * b, W, seed=9), torch.complex64)
    y1 = ctx.matvec(6, x, prec="fp32").clone()
    y2 = ctx.matvec(6, x, prec="fp32")
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


def test_set_blocks_rejects_bad_input(ctx):
    blocks = synth.green_blocks(3, 3, 4, np.pi, seed=0)
    bad = blocks.copy()
    bad[1, 2, 0, 3] = np.nan
    with pytest.raises(abi.MlfftError) as e:
        ctx.set_blocks(7, bad)
    assert e.value.status == abi.MLFFT_E_ARG
    with pytest.raises(abi.MlfftError) as e:
        ctx.set_blocks(7, to_dev(bad))
    assert e.value.status == abi.MLFFT_E_ARG
    too_big = np.zeros((1, 65, 1, 1), dtype=np.complex128)
    with pytest.raises(abi.MlfftError):
        ctx.set_blocks(7, too_big)
    singular = np.zeros((1, 1, 2, 2), dtype=np.complex128)
    with pytest.raises(abi.MlfftError) as e:
        ctx.set_blocks(7, singular)
    assert e.value.status == abi.MLFFT_E_SINGULAR
    with pytest.raises(abi.MlfftError) as e:
        abi.mlfft_matvec(ctx.h, 12345, 1, 0, 0, 0)
    assert e.value.status == abi.MLFFT_E_STATE


def test_blocks_from_device_memory(ctx):
    Nx, Ny, b, W = 4, 5, 6, 3
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=3)
    ctx.set_blocks(8, to_dev(blocks))
    X = synth.random_vectors(Nx * Ny * b, W, seed=4)
    y = ctx.matvec(8, to_dev(X))
    assert relerr(to_host(y), tp.matvec_fft(blocks, X)) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_30x30_b120_sampled_columns(ctx, prec):
    """30x30 array, b = 120, W = 900 in one launch; 3 sampled columns checked one by one."""
    Nx = Ny = 30
    b, W = 120, 900
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    ctx.set_blocks(9, blocks)
    V = synth.port_rhs(Nx, Ny, b)
    X = V + 0.1 * synth.random_vectors(Nx * Ny * b, W, seed=11)
    y = to_host(ctx.matvec(9, to_dev(X, DT[prec]), prec=prec))
    cols = [0, 451, 899]
    ref = tp.matvec_fft(blocks, X[cols], 2 * Ny, 2 * Nx)
    assert relerr(y[cols], ref) <= TOL[prec]
    assert np.all(np.isfinite(y))


@pytest.mark.parametrize("b", [8, 24, 120, 200, 13, 97, 112, 250])
@pytest.mark.parametrize("shape", ["4 32 1", "8 64 1", "4 64 0", "8 32 0", "8 32 2", "8 16 2", "4 16 2", "8 16 4"])
def test_block_product_shapes_match_oracle(ctx, b, shape):
    """Every launch shape the autotuner can pick, including the three-product FP32 forms (form 4,
    the flat kernel with direct-to-LDS tiles, runs for even b with at least seven 16-row slices:
    112, 120, 200, 250; the others fall back).  W = 70 leaves a partial last tile."""
    Nx, Ny, W = 3, 4, 70
    blocks = synth.random_blocks(Nx, Ny, b, seed=b)
    ctx.set_blocks(50, blocks)
    bp = (b + 7) // 8 * 8
    waves, nt, m3 = shape.split()
    abi.mlfft_tune_import(ctx.h, f"gemm 1 {bp} {waves} {nt} {m3}\n")
    try:
        X = synth.random_vectors(Nx * Ny * b, W, seed=4)
        y = ctx.matvec(50, to_dev(X, torch.complex64), prec="fp32")
        assert relerr(to_host(y), tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)) <= TOL["fp32"]
    finally:
        abi.mlfft_tune_import(ctx.h, f"gemm 1 {bp} 0 0 0\n")


@pytest.mark.parametrize("b", [112, 200, 250])
def test_direct_tile_product_serves_the_fp32_preconditioner(ctx, b):
    """With form 4 tuned for the MLFFT product, the FP32 preconditioner product (900 frequencies
    of a 30x30 torus here, a few columns) runs the same kernel; it matches the oracle, and the
    flat kernel with register-staged tiles to FP32 rounding (the two sum in different orders)."""
    Nx, Ny, W = 30, 30, 19
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=b)
    ctx.set_blocks(55, blocks)
    bp = (b + 7) // 8 * 8
    R = synth.random_vectors(Nx * Ny * b, W, seed=5)
    Rd = to_dev(R, torch.complex64)
    z = {}
    try:
        for form in ("8 16 2", "8 16 4"):
            abi.mlfft_tune_import(ctx.h, f"gemm 1 {bp} {form}\n")
            z[form] = to_host(ctx.precond_apply(55, Rd, kind=1, prec="fp32"))
    finally:
        abi.mlfft_tune_import(ctx.h, f"gemm 1 {bp} 0 0 0\n")
    assert relerr(z["8 16 4"], opc.strang_apply(opc.strang_inverse_spectrum(blocks), R)) <= 1e-4
    assert relerr(z["8 16 4"], z["8 16 2"]) <= 1e-5


def test_direct_tile_product_in_a_batch_with_an_odd_b(ctx):
    """Arrays with b = 114 and b = 119 pad to the same reduction length (120) and share a launch:
    form 4 needs every b even, so the launch falls back to the flat kernel; alone, the b = 114
    array runs form 4.  Both products match the oracle."""
    specs = [(3, 3, 114, 0), (2, 4, 119, 1)]
    abi.mlfft_tune_import(ctx.h, "gemm 1 120 8 16 4\n")
    try:
        ids, Vs, refs = [], [], []
        for i, (Nx, Ny, b, seed) in enumerate(specs):
            blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=seed)
            ctx.set_blocks(62 + i, blocks)
            V = synth.port_rhs(Nx, Ny, b)
            ids.append(62 + i)
            Vs.append(to_dev(V))
            refs.append(direct.lu_solve(tp.dense_Z(blocks), V))
            X = synth.random_vectors(Nx * Ny * b, 20, seed=3)
            y = ctx.matvec(62 + i, to_dev(X, torch.complex64), prec="fp32")
            assert relerr(to_host(y), tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)) <= TOL["fp32"]
        Is, info = ctx.solve_batch(ids, Vs, tol=1e-10, inner_prec="fp32", precond=1)
        assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-10)
        for I, ref in zip(Is, refs):
            assert relerr(to_host(I), ref) <= 1e-8
    finally:
        abi.mlfft_tune_import(ctx.h, "gemm 1 120 0 0 0\n")


def test_autotuned_shapes_keep_parity(ctx):
    Nx, Ny, b, W = 10, 10, 64, 100
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    ctx.set_blocks(51, blocks)
    for prec in (0, 1):
        abi.mlfft_autotune(ctx.h, 51, W, prec, 1)
    rep = abi.mlfft_tune_report(ctx.h, 51)
    assert "gemm 1 64" in rep and "fftshape 1 1 0 10 10 64" in rep and "fftshape 1 1 1 10 10 64" in rep
    X = synth.random_vectors(Nx * Ny * b, W, seed=8)
    ref = tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)
    for prec in ("fp64", "fp32"):
        y = ctx.matvec(51, to_dev(X, DT[prec]), prec=prec)
        assert relerr(to_host(y), ref) <= TOL[prec]
    R = synth.random_vectors(Nx * Ny * b, W, seed=9)
    z = ctx.precond_apply(51, to_dev(R, DT["fp32"]), kind=1, prec="fp32")
    assert relerr(to_host(z), opc.strang_apply(opc.strang_inverse_spectrum(blocks), R)) <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("Nx,Ny,b,W", [(30, 30, 13, 3), (7, 5, 24, 5), (1, 9, 40, 4), (16, 12, 8, 6), (17, 4, 6, 3),
                                        (5, 23, 10, 2), (31, 19, 4, 2)])
def test_fft_tile_kinds_and_chunks_keep_parity(ctx, prec, Nx, Ny, b, W):
    """Every tile kind (one-pass, half-height) and m-chunk of the padded transforms, forced per
    direction through tuning lines, against the oracle: the product and its fused epilogue
    (alpha Z x + beta v, the true residual's form).  Ragged b leaves a partial last m-chunk;
    Nx = 1 and the prime 17 (direct DFT; its half-height kernels run under a 256-thread bound)
    are included."""
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=5)
    ctx.set_blocks(52, blocks)
    X = synth.random_vectors(Nx * Ny * b, W, seed=6)
    Vv = synth.random_vectors(Nx * Ny * b, W, seed=7)
    ref = tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)
    p = 0 if prec == "fp64" else 1
    Xd, Vd = to_dev(X, DT[prec]), to_dev(Vv, DT[prec])
    try:
        for half in (0, 1):
            for cm in (1, 2, 4, 8, 16, 32):
                abi.mlfft_tune_import(ctx.h, "".join(f"fftshape {p} 1 {d} {Nx} {Ny} {b} {cm} {half}\n" for d in (0, 1)))
                assert relerr(to_host(ctx.matvec(52, Xd, prec=prec)), ref) <= TOL[prec], (half, cm)
                y = torch.empty_like(Xd)
                ctx.sync_stream()
                abi.mlfft_matvec_axpby(ctx.h, 52, W, -1.0, Xd.data_ptr(), 1.0, Vd.data_ptr(), y.data_ptr(), p)
                assert relerr(to_host(y), Vv - ref) <= TOL[prec], (half, cm)
    finally:
        abi.mlfft_tune_import(ctx.h, "".join(f"fftshape {p} 1 {d} {Nx} {Ny} {b} 0 -1\n" for d in (0, 1)))


def test_fft_shape_lines_are_validated(ctx):
    for bad in ("fftshape 2 1 0 4 4 8 4 0", "fftshape 0 0 0 4 4 8 4 1", "fftshape 0 1 2 4 4 8 4 0",
                "fftshape 0 1 0 4 4 8 65 0", "fftshape 0 1 0 4 4 8 4 2"):
        with pytest.raises(abi.MlfftError) as e:
            abi.mlfft_tune_import(ctx.h, bad + "\n")
        assert e.value.status == abi.MLFFT_E_ARG


@pytest.mark.parametrize("form", [2, 4])
@pytest.mark.parametrize("b", [24, 120, 200, 13, 40, 33, 201, 256])
def test_fp64_flat_three_product_matches_oracle(ctx, b, form):
    """The FP64 three-product block product with the flat (frequency, slice) assignment: form 2
    stages X tiles through registers, form 4 loads half-reduction tiles straight into LDS (from
    b = 33, three slices; b = 13 and 24 fall back).  Odd b (33, 201) leaves a partial last
    slice and unequal halves; W = 37 a partial last tile."""
    Nx, Ny, W = 3, 4, 37
    blocks = synth.random_blocks(Nx, Ny, b, seed=b + 1)
    ctx.set_blocks(52, blocks)
    bp = (b + 7) // 8 * 8
    abi.mlfft_tune_import(ctx.h, f"gemm 0 {bp} 4 16 {form}\n")
    try:
        X = synth.random_vectors(Nx * Ny * b, W, seed=5)
        y = ctx.matvec(52, to_dev(X), prec="fp64")
        assert relerr(to_host(y), tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)) <= TOL["fp64"]
        # the preconditioner product uses the same kernel (fixed shape)
        R = synth.random_vectors(Nx * Ny * b, W, seed=6)
        z = ctx.precond_apply(52, to_dev(R), kind=1, prec="fp64")
        assert relerr(to_host(z), opc.strang_apply(opc.strang_inverse_spectrum(blocks), R)) <= 1e-10
    finally:
        abi.mlfft_tune_import(ctx.h, f"gemm 0 {bp} 0 0 0\n")


def test_empty_and_overlapping_arguments(ctx):
    Nx, Ny, b = 3, 3, 4
    ctx.set_blocks(53, synth.green_blocks(Nx, Ny, b, np.pi, seed=0))
    assert abi.mlfft_matvec(ctx.h, 53, 0, 0, 0, abi.MLFFT_FP64) == abi.MLFFT_OK
    assert abi.mlfft_precond_apply(ctx.h, 53, 1, 0, 0, 0, abi.MLFFT_FP32) == abi.MLFFT_OK
    x = to_dev(synth.random_vectors(Nx * Ny * b, 2, seed=1))
    with pytest.raises(abi.MlfftError) as e:
        abi.mlfft_matvec(ctx.h, 53, 2, x.data_ptr(), x.data_ptr() + 16, abi.MLFFT_FP64)
    assert e.value.status == abi.MLFFT_E_ARG
    with pytest.raises(abi.MlfftError) as e:
        abi.mlfft_matvec(ctx.h, 53, 2, x.data_ptr(), x.data_ptr(), 7)
    assert e.value.status == abi.MLFFT_E_ARG


@pytest.mark.parametrize("shape", ["8 32 2", "4 16 2"])
@pytest.mark.parametrize("b", [40, 64, 97, 112, 200, 255, 256])
def test_bf16_flat_block_product_matches_oracle_and_eight_row_kernel(ctx, b, shape):
    """The flat bf16 block product (16-row slices; eight waves with 32-column tiles for b >= 97,
    four waves with 16-column tiles for b >= 33): against the oracle at the bf16 bound, against
    the eight-row bf16 kernel on the same bf16 inputs to FP32 accumulation accuracy, and in the
    preconditioner product.  W = 70 spans several tiles with a ragged tail; odd b takes the
    single-value stores."""
    Nx, Ny, W = 3, 4, 70
    blocks = synth.random_blocks(Nx, Ny, b, seed=b + 2)
    ctx.set_blocks(54, blocks)
    X = synth.random_vectors(Nx * Ny * b, W, seed=7)
    ref = tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)
    bp = (b + 15) // 16 * 16
    R = synth.random_vectors(Nx * Ny * b, W, seed=6)
    abi.mlfft_tune_import(ctx.h, f"gemm 2 {bp} {shape}\n")
    try:
        y_flat = to_host(ctx.matvec(54, to_dev(X, torch.complex64), prec="bf16"))
        z = to_host(ctx.precond_apply(54, to_dev(R, torch.complex64), kind=1, prec="bf16"))
        abi.mlfft_tune_import(ctx.h, f"gemm 2 {bp} 8 64 0\n")
        y_rows = to_host(ctx.matvec(54, to_dev(X, torch.complex64), prec="bf16"))
    finally:
        abi.mlfft_tune_import(ctx.h, f"gemm 2 {bp} 8 32 2\n")
    assert relerr(y_flat, ref) <= TOL["bf16"]
    assert relerr(y_flat, y_rows) <= 1e-6
    assert relerr(z, opc.strang_apply(opc.strang_inverse_spectrum(blocks), R)) <= TOL["bf16"]


def test_bf16_flat_block_product_in_a_batched_solve(ctx):
    """Two arrays whose b pad to the same bf16 reduction length (112) share one flat launch
    (two tasks); the bf16 inner solve with FP64 refinement still meets LU."""
    specs = [(3, 3, 100, 0), (2, 4, 110, 1)]
    ids, Vs, refs = [], [], []
    for i, (Nx, Ny, b, seed) in enumerate(specs):
        blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=seed)
        ctx.set_blocks(60 + i, blocks)
        V = synth.port_rhs(Nx, Ny, b)
        ids.append(60 + i)
        Vs.append(to_dev(V))
        refs.append(direct.lu_solve(tp.dense_Z(blocks), V))
    Is, info = ctx.solve_batch(ids, Vs, tol=1e-10, inner_prec="bf16", precond=1)
    assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-10)
    for I, ref in zip(Is, refs):
        assert relerr(to_host(I), ref) <= 1e-8


@pytest.mark.parametrize("Nx,Ny,b,W", [(6, 5, 24, 7), (5, 4, 64, 33), (4, 4, 100, 70), (4, 3, 120, 45),
                                        (4, 3, 161, 11), (30, 30, 200, 40), (3, 3, 208, 5)])
def test_bf16_preconditioner_frequency_kernel_matches_flat_kernel_and_oracle(ctx, Nx, Ny, b, W):
    """The bf16 preconditioner product that stages each X tile once for all row slices of its
    frequency, with the tiles of one frequency per workgroup (form 3) and with all tiles split
    evenly over about one workgroup per CU, ranges crossing frequencies (form 5), against the
    flat kernel (form 2), each forced through a tuning line (form 5 is the default for padded
    b in 112..208, form 2 elsewhere).  Forms 3 and 5 run the same arithmetic per tile, so they
    agree bit for bit; with even b, form 5 reads the spectrum that the forward transform stored
    as bf16 pairs (form 3 rounds an FP32 spectrum as it stages it), so this also pins the bf16
    spectrum path.  The flat kernel rounds the same operands to bf16 and accumulates in FP32
    in another order.  Ragged b (24, 100, 120) leaves padded reduction rows and partial
    16-row slices; W = 5, 7, 11, 33, 45, 70 leave partial 32-column tiles."""
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=3)
    ctx.set_blocks(9, blocks)
    R = synth.random_vectors(Nx * Ny * b, W, seed=4)
    Rd = to_dev(R, torch.complex64)
    bp = (b + 15) // 16 * 16
    z = {}
    for form in (2, 3, 5):
        abi.mlfft_tune_import(ctx.h, f"gemmpc 2 {bp} 8 32 {form}\n")
        try:
            z[form] = to_host(ctx.precond_apply(9, Rd, kind=1, prec="bf16"))
        finally:
            abi.mlfft_tune_import(ctx.h, f"gemmpc 2 {bp} 0 0 0\n")
    z_default = to_host(ctx.precond_apply(9, Rd, kind=1, prec="bf16"))
    assert np.array_equal(z_default, z[5 if 112 <= bp <= 208 else 2])
    assert np.array_equal(z[3], z[5])
    assert relerr(z[3], z[2]) <= 1e-5
    assert relerr(z[3], opc.strang_apply(opc.strang_inverse_spectrum(blocks), R)) <= TOL["bf16"]


def test_bf16_preconditioner_shape_lines_are_validated(ctx):
    for bad in ("gemmpc 2 224 8 32 3", "gemmpc 2 200 8 32 3", "gemmpc 1 208 8 32 3", "gemmpc 2 208 4 16 3",
                "gemmpc 2 224 8 32 5", "gemmpc 2 208 4 16 5", "gemmpc 2 208 8 32 4", "gemmpc 2 208 8 32 6",
                "gemmpcwg 0"):
        with pytest.raises(abi.MlfftError) as e:
            abi.mlfft_tune_import(ctx.h, bad + "\n")
        assert e.value.status == abi.MLFFT_E_ARG
