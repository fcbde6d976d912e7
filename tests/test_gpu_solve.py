"""GPU solves (GMRES with FP64 refinement) against the oracle's direct solutions.

Bars: the final solution matches the LU solution (or, where a dense Z does not
fit, the oracle's FP64 GMRES solution at 1e-12) to 1e-6 relative after
refinement; parity runs refine to a tighter residual than the metric's 1e-6 so
that the error bound ||e|| <= cond(Z) ||r|| leaves room (cond ~ 1.3-1.7 for the
Green's-function generator).
"""
import numpy as np
import pytest
import torch

from oracle import direct, krylov, precond
from oracle import toeplitz as tp
from paper_2506_20350_amd import abi, learned, synth
from tests.gpu_util import ctx, relerr, to_dev, to_host  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("orth", [2, 1])
def test_c1_plain_fp64_gmres_matches_lu_and_oracle_iterations(ctx, orth):
    """4x4 array, b = 24, kd = pi, centre port, GMRES(30), no preconditioner, tol 1e-8;
    classical Gram-Schmidt twice (the second projection from the Gram matrix) and once,
    against the oracle's modified Gram-Schmidt."""
    Nx = Ny = 4
    b = 24
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    V = synth.port_rhs(Nx, Ny, b, cols=[synth.centre_element(Nx, Ny)])
    ctx.set_blocks(10, blocks)
    I, info = ctx.solve(10, to_dev(V), tol=1e-8, inner_prec="fp64", precond=0, history_len=40, orth=orth)
    assert info["status"] == abi.MLFFT_OK and info["converged"].all()
    Z = tp.dense_Z(blocks)
    ref = direct.lu_solve(Z, V)
    assert relerr(to_host(I), ref) <= 1e-7
    assert info["relres"][0] <= 1e-8
    mv = lambda X: tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)
    ores = krylov.gmres_columns(mv, V, None, tol=1e-8 * 0.9)[0]
    assert info["iters"][0] == ores.iters
    h = info["history"][:info["iters"][0], 0]
    # classical Gram-Schmidt applied once loses orthogonality at the 1e-10 level
    # in FP64 here, which shifts its smallest residual estimates by that much
    np.testing.assert_allclose(h, ores.history, rtol=1e-6, atol=0.0 if orth == 2 else 1e-9)


@pytest.mark.parametrize("inner", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("pc", [0, 1, 2])
def test_small_array_all_ports_match_lu(ctx, inner, pc):
    Nx, Ny, b = 5, 7, 12
    blocks = synth.green_blocks(Nx, Ny, b, 2 * np.pi / 3, seed=1)
    V = synth.port_rhs(Nx, Ny, b)
    ctx.set_blocks(11, blocks)
    I, info = ctx.solve(11, to_dev(V), tol=1e-10, inner_prec=inner, precond=pc)
    assert info["status"] == abi.MLFFT_OK, info
    ref = direct.lu_solve(tp.dense_Z(blocks), V)
    assert relerr(to_host(I), ref) <= 1e-8
    assert np.all(info["relres"] <= 1e-10)
    if inner != "fp64":
        assert info["outer"].max() >= 2          # refinement actually worked


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("pc", [1, 2])
def test_bf16_preconditioner_product_matches_lu(ctx, pc, mode):
    """FP32 inner solve with the preconditioner's block product in bf16 (pc_bf16 = 1): the
    solution still meets LU after refinement, the option really changes the preconditioned
    directions (results differ from the FP32 product's), and the iteration count stays within
    two of the FP32 product's (bf16 rounding perturbs the approximate inverse by ~2^-9)."""
    Nx, Ny, b = 10, 10, 64
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    V = synth.port_rhs(Nx, Ny, b)
    ctx.set_blocks(31, blocks)
    ref = direct.lu_solve(tp.dense_Z(blocks), V)
    out = {}
    for pc_bf16 in (0, 1):
        I, info = ctx.solve(31, to_dev(V), tol=1e-10, inner_prec="fp32", precond=pc, mode=mode, pc_bf16=pc_bf16)
        assert info["status"] == abi.MLFFT_OK, info
        assert np.all(info["relres"] <= 1e-10)
        assert relerr(to_host(I), ref) <= 1e-8
        out[pc_bf16] = (to_host(I), info)
    assert not np.array_equal(out[0][0], out[1][0])
    assert out[1][1]["iters"].max() <= out[0][1]["iters"].max() + 2


def test_bf16_preconditioner_product_under_the_learned_correction(ctx):
    """Flexible GMRES with a (small, random) learned correction of the block-circulant output,
    whose block product runs in bf16 (b = 100: the flat bf16 kernel): the refined solution meets
    LU, and it differs from the FP32-product solve, so the option reached the flexible path."""
    Nx, Ny, b = 3, 3, 100
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=2)
    V = synth.port_rhs(Nx, Ny, b)
    ctx.set_blocks(33, blocks)
    abi.mlfft_net_create(ctx.h, b, 16, 4)
    ws = abi.mlfft_net_get_weights(ctx.h)
    ws[-16 * 2 * b * 9:] = np.random.default_rng(5).standard_normal(16 * 2 * b * 9).astype(np.float32) * 0.01
    abi.mlfft_net_set_weights(ctx.h, ws)
    ref = direct.lu_solve(tp.dense_Z(blocks), V)
    out = {}
    for pc_bf16 in (0, 1):
        I, info = ctx.solve(33, to_dev(V), tol=1e-10, inner_prec="fp32", precond=3, pc_bf16=pc_bf16)
        assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-10), info
        assert info["net_applies"] > 0
        assert relerr(to_host(I), ref) <= 1e-8
        out[pc_bf16] = to_host(I)
    assert not np.array_equal(out[0], out[1])


@pytest.mark.parametrize("use_graph", [0, 1])
def test_bf16_preconditioner_product_in_a_batch_of_three_kernels(ctx, use_graph):
    """An uneven batch whose preconditioner products run in bf16 through all three kernels
    (b = 24: the eight-row kernel; b = 64: the four-wave flat kernel; b = 100: the eight-wave
    flat kernel), eagerly and with graph-captured steps (graphs must equal the eager solve bit
    for bit); every array meets its LU solution."""
    specs = [(4, 3, 24, 2), (4, 3, 64, 3), (3, 3, 100, 4)]
    ids, Vs, refs = [], [], []
    for i, (Nx, Ny, b, seed) in enumerate(specs):
        blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=seed)
        ctx.set_blocks(34 + i, blocks)
        V = synth.port_rhs(Nx, Ny, b)
        ids.append(34 + i)
        Vs.append(to_dev(V))
        refs.append(direct.lu_solve(tp.dense_Z(blocks), V))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        I0, info0 = ctx.solve_batch(ids, Vs, tol=1e-10, inner_prec="fp32", precond=1, pc_bf16=1)
        assert info0["status"] == abi.MLFFT_OK and np.all(info0["relres"] <= 1e-10)
        for I, ref in zip(I0, refs):
            assert relerr(to_host(I), ref) <= 1e-8
        if use_graph:
            for rep in range(3):
                I1, info1 = ctx.solve_batch(ids, Vs, tol=1e-10, inner_prec="fp32", precond=1, pc_bf16=1,
                                            use_graph=1)
                side.synchronize()
                assert info1["status"] == abi.MLFFT_OK, rep
                for a, b in zip(I1, I0):
                    assert torch.equal(a, b), rep


def test_bf16_preconditioner_tiles_split_over_two_arrays_in_one_launch(ctx):
    """Two arrays of one padded b (120 and 122 pad to 128) share each bf16 preconditioner
    launch, whose (frequency, tile) items are split evenly over about one workgroup per CU
    with each array taking a share of workgroups proportional to its items; ragged W (9 and
    12 ports) leaves partial tiles.  Every array meets its LU solution and agrees with the
    array solved alone (where its launches hold one task) to the refinement tolerance."""
    specs = [(3, 3, 120, 5), (4, 3, 122, 6)]
    ids, Vs, refs = [], [], []
    for i, (Nx, Ny, b, seed) in enumerate(specs):
        blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=seed)
        ctx.set_blocks(40 + i, blocks)
        V = synth.port_rhs(Nx, Ny, b)
        ids.append(40 + i)
        Vs.append(to_dev(V))
        refs.append(direct.lu_solve(tp.dense_Z(blocks), V))
    I0, info0 = ctx.solve_batch(ids, Vs, tol=1e-10, inner_prec="fp32", precond=1, pc_bf16=1)
    assert info0["status"] == abi.MLFFT_OK and np.all(info0["relres"] <= 1e-10)
    for i, (I, ref) in enumerate(zip(I0, refs)):
        assert relerr(to_host(I), ref) <= 1e-8
        Ia, _ = ctx.solve(ids[i], Vs[i], tol=1e-10, inner_prec="fp32", precond=1, pc_bf16=1)
        assert relerr(to_host(Ia), to_host(I)) <= 1e-9, i


def test_bf16_preconditioner_option_is_validated(ctx):
    blocks = synth.green_blocks(3, 3, 8, np.pi, seed=0)
    ctx.set_blocks(32, blocks)
    V = synth.port_rhs(3, 3, 8)
    with pytest.raises(abi.MlfftError, match="pc_bf16") as e:
        ctx.solve(32, to_dev(V), tol=1e-8, inner_prec="fp32", precond=1, pc_bf16=2)
    assert e.value.status == abi.MLFFT_E_ARG


def test_c2_fp32_refined_block_circulant_matches_lu(ctx):
    """10x10 array, b = 64, 100 port excitations, FP32 inner + FP64 refinement to 1e-8."""
    Nx = Ny = 10
    b = 64
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    V = synth.port_rhs(Nx, Ny, b)
    ctx.set_blocks(12, blocks)
    I, info = ctx.solve(12, to_dev(V), tol=1e-8, inner_prec="fp32", precond=1)
    assert info["status"] == abi.MLFFT_OK
    ref = direct.lu_solve(tp.dense_Z(blocks), V)
    assert relerr(to_host(I), ref) <= 1e-6
    assert np.all(info["relres"] <= 1e-8)


def test_batch_of_uneven_arrays_matches_per_array_lu(ctx):
    shapes = [(4, 6, 24, 0.6 * np.pi), (7, 3, 16, np.pi), (5, 5, 40, 0.8 * np.pi)]
    ids, Vs, refs = [], [], []
    for i, (Nx, Ny, b, kd) in enumerate(shapes):
        blocks = synth.green_blocks(Nx, Ny, b, kd, seed=1000 + i)
        ctx.set_blocks(20 + i, blocks)
        V = synth.port_rhs(Nx, Ny, b)
        ids.append(20 + i)
        Vs.append(to_dev(V))
        refs.append(direct.lu_solve(tp.dense_Z(blocks), V))
    Is, info = ctx.solve_batch(ids, Vs, tol=1e-10, inner_prec="fp32", precond=1)
    assert info["status"] == abi.MLFFT_OK
    for I, ref in zip(Is, refs):
        assert relerr(to_host(I), ref) <= 1e-8
    assert info["relres"].shape[0] == sum(v.shape[0] for v in Vs)


def test_initial_guess_and_zero_columns(ctx):
    Nx, Ny, b = 4, 4, 8
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=3)
    ctx.set_blocks(13, blocks)
    V = synth.port_rhs(Nx, Ny, b, cols=[0, 5, 9])
    V[1] = 0.0                                  # an all-zero excitation
    ref = direct.lu_solve(tp.dense_Z(blocks), V)
    I, info = ctx.solve(13, to_dev(V), to_dev(ref), tol=1e-8, x0_given=1, inner_prec="fp64")
    assert info["status"] == abi.MLFFT_OK and np.all(info["iters"] == 0)
    I2, info2 = ctx.solve(13, to_dev(V), tol=1e-10, inner_prec="fp32")
    out = to_host(I2)
    assert np.all(out[1] == 0) and info2["iters"][1] == 0
    assert relerr(out, ref) <= 1e-8


def test_periodic_operator_converges_in_one_iteration(ctx):
    Nx, Ny, b = 6, 4, 8
    blocks = synth.periodic_blocks(Nx, Ny, b, seed=5)
    ctx.set_blocks(14, blocks)
    V = synth.random_vectors(Nx * Ny * b, 4, seed=2)
    I, info = ctx.solve(14, to_dev(V), tol=1e-10, inner_prec="fp64", precond=1)
    assert info["status"] == abi.MLFFT_OK
    assert np.all(info["iters"] == 1)
    assert relerr(to_host(I), direct.lu_solve(tp.dense_Z(blocks), V)) <= 1e-10


def test_limits_report_not_converged(ctx):
    Nx, Ny, b = 5, 5, 16
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0, alpha=0.3)
    ctx.set_blocks(15, blocks)
    V = synth.port_rhs(Nx, Ny, b, cols=[0, 12])
    I, info = ctx.solve(15, to_dev(V), tol=1e-12, inner_prec="fp64", precond=0, restart=2, max_restarts=1,
                        max_outer=1)
    assert info["status"] == abi.MLFFT_NOT_CONVERGED
    assert np.all(info["relres"] > 1e-12) and np.all(np.isfinite(info["relres"]))
    assert not info["converged"].any()


def test_solve_rejects_bad_arguments(ctx):
    Nx, Ny, b = 3, 3, 4
    ctx.set_blocks(16, synth.green_blocks(Nx, Ny, b, np.pi, seed=0))
    V = to_dev(synth.port_rhs(Nx, Ny, b))
    with pytest.raises(abi.MlfftError) as e:
        ctx.solve(16, V, restart=40)
    assert e.value.status == abi.MLFFT_E_ARG
    with pytest.raises(abi.MlfftError) as e:
        ctx.solve(16, V, precond=3)
    assert e.value.status in (abi.MLFFT_E_STATE, abi.MLFFT_E_ARG)
    bad = V.clone()
    bad[0, 0] = float("nan")
    with pytest.raises(abi.MlfftError) as e:
        ctx.solve(16, bad)
    assert e.value.status == abi.MLFFT_E_ARG
    for g in (-1, 9):
        with pytest.raises(abi.MlfftError) as e:
            ctx.solve(16, V, use_graph=g)
        assert e.value.status == abi.MLFFT_E_ARG


@pytest.mark.parametrize("kd", [2 * np.pi / 3, np.pi])
def test_full_size_30x30_b120_sampled_columns(ctx, kd):
    """30x30 array, b = 120, all 900 ports in one solve (FP32 inner, FP64 refinement), with the
    preconditioner's block product in FP32 and in bf16 (the benchmark's setting); three columns
    checked against the oracle's FP64 GMRES solution at 1e-12."""
    Nx = Ny = 30
    b = 120
    blocks = synth.green_blocks(Nx, Ny, b, kd, seed=0)
    ctx.set_blocks(17, blocks)
    V = synth.port_rhs(Nx, Ny, b)
    cols = [0, 465, 899]
    mv = lambda X: tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)
    Sinv = precond.strang_inverse_spectrum(blocks)
    pc = lambda X: precond.strang_apply(Sinv, X)
    ref = np.array([r.x for r in krylov.gmres_columns(mv, V[cols], pc, tol=1e-12)])
    for pc_bf16 in (0, 1):
        I, info = ctx.solve(17, to_dev(V), tol=1e-8, inner_prec="fp32", precond=1, pc_bf16=pc_bf16)
        assert info["status"] == abi.MLFFT_OK
        assert np.all(info["relres"] <= 1e-8)
        assert relerr(to_host(I)[cols], ref) <= 1e-6


@pytest.mark.timeout(400)
def test_full_uneven_batch_of_64_arrays_against_oracle(ctx):
    """All 64 arrays of the uneven-batch recipe (11 785 ports) in one batched FP32 + FP64-refined
    solve at the benchmark's tol 1e-6; the centre port of every array is checked against the
    oracle's FP64 GMRES solution at 1e-12 (relres <= 1e-6 and cond(Z) < 2 bound the error)."""
    specs = synth.c4_arrays(64, master_seed=0)
    ids, Vs, blocks_all = [], [], []
    for i, sp in enumerate(specs):
        blocks = synth.green_blocks(sp["Nx"], sp["Ny"], sp["b"], sp["kd"], seed=sp["seed"])
        ctx.set_blocks(200 + i, blocks)
        ids.append(200 + i)
        Vs.append(to_dev(synth.port_rhs(sp["Nx"], sp["Ny"], sp["b"])))
        blocks_all.append(blocks)
    Is, info = ctx.solve_batch(ids, Vs, tol=1e-6, inner_prec="fp32", precond=1, pc_bf16=1)
    assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-6)
    assert info["relres"].size == sum(sp["Nx"] * sp["Ny"] for sp in specs)
    for i, sp in enumerate(specs):
        Nx, Ny, b = sp["Nx"], sp["Ny"], sp["b"]
        col = (Ny // 2) * Nx + Nx // 2
        V = synth.port_rhs(Nx, Ny, b, cols=[col])
        Gh = tp.spectra(blocks_all[i], 2 * Ny, 2 * Nx)
        Sinv = precond.strang_inverse_spectrum(blocks_all[i])
        ref = krylov.gmres_columns(lambda X: tp.matvec_spectral(Gh, X, Nx, Ny), V,
                                   lambda X: precond.strang_apply(Sinv, X), tol=1e-12)[0].x
        assert relerr(to_host(Is[i])[col], ref) <= 2e-6, (i, sp)
    for i in ids:
        abi.mlfft_drop_array(ctx.h, i)


def test_uneven_batch_like_c4_sampled_against_oracle(ctx):
    """The first 12 arrays of the uneven-batch recipe (Nx, Ny in [4, 24], b in {24, 48, 64, 96},
    kd in [pi/2, pi]) in one batched FP32 + FP64-refined solve; one column of every third array is
    checked against the oracle's FP64 GMRES solution at 1e-12."""
    specs = synth.c4_arrays(12, master_seed=0)
    ids, Vs, blocks_all = [], [], []
    for i, sp in enumerate(specs):
        blocks = synth.green_blocks(sp["Nx"], sp["Ny"], sp["b"], sp["kd"], seed=sp["seed"])
        ctx.set_blocks(60 + i, blocks)
        ids.append(60 + i)
        Vs.append(to_dev(synth.port_rhs(sp["Nx"], sp["Ny"], sp["b"])))
        blocks_all.append(blocks)
    Is, info = ctx.solve_batch(ids, Vs, tol=1e-9, inner_prec="fp32", precond=1)
    assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-9)
    for i in range(0, len(specs), 3):
        sp = specs[i]
        Nx, Ny, b = sp["Nx"], sp["Ny"], sp["b"]
        col = (Nx * Ny) // 2
        V = synth.port_rhs(Nx, Ny, b, cols=[col])
        mv = lambda X: tp.matvec_fft(blocks_all[i], X, 2 * Ny, 2 * Nx)
        Sinv = precond.strang_inverse_spectrum(blocks_all[i])
        ref = krylov.gmres_columns(mv, V, lambda X: precond.strang_apply(Sinv, X), tol=1e-12)[0].x
        got = to_host(Is[i])[col]
        assert relerr(got, ref) <= 1e-7, (i, sp)


def _graph_case(ctx, aid, precond, seed):
    Nx, Ny, b = 6, 5, 24
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=seed)
    ctx.set_blocks(aid, blocks)
    return blocks, to_dev(synth.port_rhs(Nx, Ny, b))


@pytest.mark.parametrize("precond,steps", [(1, 1), (3, 1), (1, 4), (3, 3)])
def test_graph_captured_steps_match_eager_on_every_replay(ctx, precond, steps):
    """use_graph = 1, 3 or 4 Krylov steps per graph on a side stream: the first solve runs eagerly,
    the second captures the steps, the later ones replay the graphs.  Eager library work and host
    synchronisations run between the solves; every solve must equal the eager solve bit for bit
    (the steps a multi-step graph spends after the last column retired change nothing)."""
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        if precond == 3:
            abi.mlfft_net_create(ctx.h, 24, 16, 4)
            ws = abi.mlfft_net_get_weights(ctx.h)
            ws[-16 * 48 * 9:] = np.random.default_rng(5).standard_normal(16 * 48 * 9).astype(np.float32) * 0.01
            abi.mlfft_net_set_weights(ctx.h, ws)
        blocks, V = _graph_case(ctx, 70, precond, seed=6)
        I0, info0 = ctx.solve(70, V, tol=1e-10, inner_prec="fp32", precond=precond)
        assert info0["status"] == abi.MLFFT_OK
        for rep in range(4):
            I, info = ctx.solve(70, V, tol=1e-10, inner_prec="fp32", precond=precond, use_graph=steps)
            y = ctx.matvec(70, I)                  # eager work between the replays
            side.synchronize()
            assert info["status"] == abi.MLFFT_OK, rep
            assert torch.equal(I, I0), rep
            assert np.array_equal(info["iters"], info0["iters"]) and np.array_equal(info["relres"], info0["relres"])
            assert relerr(to_host(y), to_host(V)) <= 1e-9
    ref = direct.lu_solve(tp.dense_Z(blocks), to_host(V))
    assert relerr(to_host(I0), ref) <= 1e-8


def test_graph_replays_follow_the_workspace_layout_and_refinement_scale(ctx):
    """Captured Krylov steps hold raw workspace addresses, which move between a solve in place
    (V and I separate), a staged one (I aliasing V) and a staged batch, and the rotations read
    the scale of the inner right-hand side (||V|| at x = 0, ||r|| in later refinement steps).
    Alternating those solves with use_graph = 1, several times each, must reproduce the eager
    solutions, iteration counts and residual histories bit for bit."""
    Nx, Ny, b = 6, 5, 24
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=8)
    blocks2 = synth.green_blocks(4, 6, 16, 0.7 * np.pi, seed=9)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ctx.set_blocks(76, blocks)
        ctx.set_blocks(77, blocks2)
        V = to_dev(synth.port_rhs(Nx, Ny, b))
        V2 = to_dev(synth.port_rhs(4, 6, 16))
        kinds = {
            "in_place": lambda g: ctx.solve(76, V, torch.zeros_like(V), tol=1e-10, inner_prec="fp32", use_graph=g),
            "aliased": lambda g: (lambda Vc: ctx.solve(76, Vc, Vc, tol=1e-10, inner_prec="fp32", use_graph=g))(
                V.clone()),
            "batch": lambda g: ctx.solve_batch([76, 77], [V, V2], tol=1e-10, inner_prec="fp32", use_graph=g),
            "bf16_refined": lambda g: ctx.solve(76, V, torch.zeros_like(V), tol=1e-10, inner_prec="bf16",
                                                use_graph=g, history_len=40),
        }
        eager = {}
        for k, f in kinds.items():
            I, info = f(0)
            side.synchronize()
            eager[k] = ([to_host(x) for x in I] if isinstance(I, list) else to_host(I), info)
        assert eager["bf16_refined"][1]["outer"].max() >= 2
        for rep in range(3):
            for k, f in kinds.items():
                I, info = f(1)
                side.synchronize()
                got = [to_host(x) for x in I] if isinstance(I, list) else to_host(I)
                ref, rinfo = eager[k]
                assert info["status"] == abi.MLFFT_OK, (rep, k)
                if isinstance(got, list):
                    assert all(np.array_equal(a, c) for a, c in zip(got, ref)), (rep, k)
                else:
                    assert np.array_equal(got, ref), (rep, k)
                assert np.array_equal(info["iters"], rinfo["iters"]), (rep, k)
                assert np.array_equal(info["relres"], rinfo["relres"]), (rep, k)
                if "history" in rinfo:
                    assert np.array_equal(info["history"], rinfo["history"]), (rep, k)
    ref = direct.lu_solve(tp.dense_Z(blocks), synth.port_rhs(Nx, Ny, b))
    assert relerr(eager["in_place"][0], ref) <= 1e-8


def test_graph_batch_matches_eager_and_null_stream_runs_eagerly(ctx):
    shapes = [(4, 6, 24, 0.6 * np.pi), (7, 3, 16, np.pi)]
    ids, Vs = [], []
    for i, (Nx, Ny, b, kd) in enumerate(shapes):
        ctx.set_blocks(72 + i, synth.green_blocks(Nx, Ny, b, kd, seed=1100 + i))
        ids.append(72 + i)
        Vs.append(to_dev(synth.port_rhs(Nx, Ny, b)))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        Is0, info0 = ctx.solve_batch(ids, Vs, tol=1e-10, inner_prec="fp32", precond=1)
        for rep in range(3):
            Is, info = ctx.solve_batch(ids, Vs, tol=1e-10, inner_prec="fp32", precond=1, use_graph=1)
            side.synchronize()
            assert all(torch.equal(a, b) for a, b in zip(Is, Is0)), rep
            assert np.array_equal(info["iters"], info0["iters"])
    # on the NULL stream the option is accepted and the steps run eagerly
    torch.cuda.synchronize()
    Is, info = ctx.solve_batch(ids, Vs, tol=1e-10, inner_prec="fp32", precond=1, use_graph=1)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(Is, Is0))


@pytest.mark.parametrize("pc", [0, 1])
def test_global_mode_matches_oracle_global_gmres(ctx, pc):
    """mode = 1: one Krylov space for all port columns (eq. ZIVvec).  The FP64 residual history of
    the first inner solve equals the oracle's global GMRES history; the solution matches LU."""
    Nx, Ny, b = 5, 4, 6
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=2)
    ctx.set_blocks(80, blocks)
    V = synth.port_rhs(Nx, Ny, b)
    I, info = ctx.solve(80, to_dev(V), tol=1e-10, inner_prec="fp64", precond=pc, mode=1, history_len=60)
    assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-10)
    mv = lambda X: tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)
    pcf = None
    if pc:
        Sinv = precond.strang_inverse_spectrum(blocks)
        pcf = lambda X: precond.strang_apply(Sinv, X)
    ores = krylov.gmres_global(mv, V, pcf, tol=0.9e-10)
    k = ores.iters
    assert np.all(info["iters"] >= k)
    np.testing.assert_allclose(info["history"][:k, 0], ores.history, rtol=1e-6)
    assert np.all(info["history"][:k] == info["history"][:k, :1])      # one history for all columns
    assert relerr(to_host(I), direct.lu_solve(tp.dense_Z(blocks), V)) <= 1e-8


def test_global_mode_fp32_refined_batch_matches_lu(ctx):
    shapes = [(6, 5, 24, np.pi), (4, 7, 16, 0.7 * np.pi)]
    ids, Vs, refs = [], [], []
    for i, (Nx, Ny, b, kd) in enumerate(shapes):
        blocks = synth.green_blocks(Nx, Ny, b, kd, seed=1200 + i)
        ctx.set_blocks(82 + i, blocks)
        V = synth.port_rhs(Nx, Ny, b)
        ids.append(82 + i)
        Vs.append(to_dev(V))
        refs.append(direct.lu_solve(tp.dense_Z(blocks), V))
    Is, info = ctx.solve_batch(ids, Vs, tol=1e-9, inner_prec="fp32", precond=1, mode=1)
    assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-9)
    for I, ref in zip(Is, refs):
        assert relerr(to_host(I), ref) <= 1e-7
    assert len(set(info["iters"].tolist())) == 1


@pytest.mark.parametrize("precond", [1, 4])
def test_global_mode_drives_every_column_below_tol_on_a_weakly_loaded_array(ctx, precond):
    """Global GMRES reaches the Frobenius target ||R||_F <= f tol ||V||_F with some columns still
    above their own tol (16 x 16, b = 48, loading 1x); the next outer step then aims below
    f tol min ||V_w||, so every column converges (the Frobenius target alone would ask the
    next inner solve for no reduction and the outer loop would stall)."""
    Nx, Ny, b = 16, 16, 48
    ctx.set_blocks(85, synth.green_blocks(Nx, Ny, b, np.pi, seed=0, alpha=1.0))
    V = to_dev(synth.port_rhs(Nx, Ny, b))
    _, info = ctx.solve(85, V, tol=1e-6, inner_prec="fp64", precond=precond, mode=1)
    assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-6)


def test_mode_rejects_unknown_value(ctx):
    Nx, Ny, b = 3, 3, 4
    ctx.set_blocks(84, synth.green_blocks(Nx, Ny, b, np.pi, seed=0))
    with pytest.raises(abi.MlfftError) as e:
        ctx.solve(84, to_dev(synth.port_rhs(Nx, Ny, b)), mode=2)
    assert e.value.status == abi.MLFFT_E_ARG


def test_full_size_30x30_b200_autotuned_sampled_columns(ctx):
    """The benchmark configuration: 30x30 array, b = 200, all 900 ports, autotuned launch shapes,
    FP32 inner + FP64 refinement to the metric's 1e-6; nine columns (the four corner ports, the
    four edge midpoints and the centre) checked against the oracle's FP64 GMRES solution at 1e-12,
    and the matvec of the same launch shape on the same columns."""
    Nx = Ny = 30
    b = 200
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    ctx.set_blocks(18, blocks)
    for prec in (0, 1):
        abi.mlfft_autotune(ctx.h, 18, Nx * Ny, prec, 1)
    V = synth.port_rhs(Nx, Ny, b)
    cols = [iy * Nx + ix for iy, ix in [(0, 0), (0, 29), (29, 0), (29, 29), (0, 15), (15, 0), (15, 29), (29, 15),
                                       (15, 15)]]
    Gh = tp.spectra(blocks, 2 * Ny, 2 * Nx)
    mv = lambda X: tp.matvec_spectral(Gh, X, Nx, Ny)
    Sinv = precond.strang_inverse_spectrum(blocks)
    ref = np.array([r.x for r in krylov.gmres_columns(mv, V[cols], lambda X: precond.strang_apply(Sinv, X),
                                                      tol=1e-12)])
    # the preconditioner's block product in FP32 and in bf16 (both benchmark options)
    for pc_bf16 in (0, 1):
        I, info = ctx.solve(18, to_dev(V), tol=1e-6, inner_prec="fp32", precond=1, pc_bf16=pc_bf16)
        assert info["status"] == abi.MLFFT_OK and np.all(info["relres"] <= 1e-6)
        assert relerr(to_host(I)[cols], ref) <= 2e-6   # relres <= 1e-6 and cond(Z) ~ 1.5
    # the same tuned block-product shape in a plain FP32 matvec, sampled columns against the oracle
    y = to_host(ctx.matvec(18, to_dev(V, torch.complex64), prec="fp32"))
    assert relerr(y[cols], mv(V[cols])) <= 1e-5


def test_in_place_and_staged_solves_agree_bitwise(ctx):
    """The solve works in V and I directly when the batch's columns lie back to back in both
    (no staging copies) and stages them otherwise (separate tensors, or V and I overlapping);
    the arithmetic is the same, so the three solutions agree bit for bit.  I starts as NaN:
    without an initial guess the solve must not read it."""
    shapes = [(4, 6, 24, 0.6 * np.pi), (5, 5, 16, np.pi)]
    ids, Vh, refs = [], [], []
    for i, (Nx, Ny, b, kd) in enumerate(shapes):
        blocks = synth.green_blocks(Nx, Ny, b, kd, seed=2000 + i)
        ctx.set_blocks(40 + i, blocks)
        V = synth.port_rhs(Nx, Ny, b, cols=list(range(0, Nx * Ny, 3)))
        ids.append(40 + i)
        Vh.append(V)
        refs.append(direct.lu_solve(tp.dense_Z(blocks), V))
    opts = dict(tol=1e-10, inner_prec="fp32", precond=1)
    sizes = [v.size for v in Vh]
    # staged: the arrays' slices of V and of I are one element apart (not back to back)
    Vgap = to_dev(np.concatenate([np.concatenate([v.ravel(), np.zeros(1)]) for v in Vh]))
    Igap = torch.full_like(Vgap, float("nan"))
    goffs = np.cumsum([0] + [n + 1 for n in sizes])
    Vs_s = [Vgap[goffs[k]:goffs[k] + sizes[k]].view(v.shape) for k, v in enumerate(Vh)]
    Is_s = [Igap[goffs[k]:goffs[k] + sizes[k]].view(v.shape) for k, v in enumerate(Vh)]
    _, info_s = ctx.solve_batch(ids, Vs_s, Is_s, **opts)
    # in place: one tensor for all V, one for all I, sliced per array
    Vflat = to_dev(np.concatenate([v.ravel() for v in Vh]))
    Iflat = torch.full_like(Vflat, float("nan"))
    offs = np.cumsum([0] + sizes)
    Vs_p = [Vflat[offs[k]:offs[k + 1]].view(v.shape) for k, v in enumerate(Vh)]
    Is_p = [Iflat[offs[k]:offs[k + 1]].view(v.shape) for k, v in enumerate(Vh)]
    _, info_p = ctx.solve_batch(ids, Vs_p, Is_p, **opts)
    assert info_s["status"] == info_p["status"] == abi.MLFFT_OK
    for a, b_, ref in zip(Is_s, Is_p, refs):
        assert torch.equal(a, b_)
        assert relerr(to_host(b_), ref) <= 1e-8
    assert np.array_equal(info_s["iters"], info_p["iters"])
    # V and I the same buffer: staged, the solution overwrites the excitation
    X = to_dev(Vh[0])
    _, info_x = ctx.solve(ids[0], X, X, **opts)
    assert info_x["status"] == abi.MLFFT_OK
    assert torch.equal(X, Is_s[0])


def test_batch_with_an_all_zero_array_and_two_refinement_steps(ctx):
    """An array whose excitations are all zero is converged at x = 0 and drops out of the
    first Krylov steps; the next FP64 residual must still cover every array.  The FP32 inner
    solve cannot reach 1e-11 in one refinement step, so a second one runs."""
    shapes = [(4, 4, 16, np.pi), (3, 5, 8, 0.7 * np.pi)]
    ids, Vs, refs = [], [], []
    for i, (Nx, Ny, b, kd) in enumerate(shapes):
        blocks = synth.green_blocks(Nx, Ny, b, kd, seed=2100 + i)
        ctx.set_blocks(50 + i, blocks)
        V = synth.port_rhs(Nx, Ny, b, cols=[0, 3, 7])
        if i == 1:
            V[:] = 0.0
        ids.append(50 + i)
        Vs.append(V)
        refs.append(direct.lu_solve(tp.dense_Z(blocks), V))
    Is = [torch.full(v.shape, float("nan"), dtype=torch.complex128, device="cuda") for v in Vs]
    Is, info = ctx.solve_batch(ids, [to_dev(v) for v in Vs], Is, tol=1e-11, inner_prec="fp32", precond=1)
    assert info["status"] == abi.MLFFT_OK
    assert int(info["outer"].max()) >= 2
    assert np.all(info["outer"][3:] == 0) and np.all(info["iters"][3:] == 0)
    assert torch.count_nonzero(Is[1]) == 0
    assert relerr(to_host(Is[0]), refs[0]) <= 1e-9
    assert np.all(info["relres"] <= 1e-11)


@pytest.mark.parametrize("pc", [0, 1])
def test_fp32_restarted_inner_solve_matches_lu(ctx, pc):
    """GMRES(3) in FP32: the inner solve restarts, so its restart residual r - Z d runs
    through the FP32 inverse transform's y = alpha Z x + beta addend epilogue."""
    Nx, Ny, b = 6, 5, 16
    blocks = synth.green_blocks(Nx, Ny, b, 0.9 * np.pi, seed=21)
    V = synth.port_rhs(Nx, Ny, b, cols=[0, 7, 14, 29])
    ctx.set_blocks(60, blocks)
    I, info = ctx.solve(60, to_dev(V), tol=1e-10, inner_prec="fp32", precond=pc, restart=3)
    assert info["status"] == abi.MLFFT_OK
    assert info["iters"].max() > 3                  # more than one cycle
    ref = direct.lu_solve(tp.dense_Z(blocks), V)
    assert relerr(to_host(I), ref) <= 1e-8
    assert np.all(info["relres"] <= 1e-10)
