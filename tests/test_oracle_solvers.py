"""Pins of the oracle's direct solvers, preconditioners and GMRES (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import direct, krylov, precond
from oracle import toeplitz as tp
from paper_2506_20350_amd import synth


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ----------------------------------------------------------------- direct

@pytest.mark.parametrize("Nx,Ny,b,kind", [(4, 4, 24, "green"), (3, 5, 8, "green"), (6, 6, 8, "green"),
                                          (3, 4, 5, "random"), (2, 7, 3, "random")])
def test_rybicki_matches_lu(Nx, Ny, b, kind):
    if kind == "green":
        blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    else:
        blocks = synth.random_blocks(Nx, Ny, b, seed=5)
        blocks[Ny - 1, Nx - 1] += 6 * np.sqrt(Nx * Ny * b) * np.eye(b)
    V = synth.port_rhs(Nx, Ny, b)
    Z = tp.dense_Z(blocks)
    I_lu = direct.lu_solve(Z, V)
    I_ry = direct.rybicki_solve_array(blocks, V)
    assert relerr(I_ry, I_lu) <= 1e-10
    assert np.linalg.norm(tp.matvec_dense(Z, I_lu) - V) <= 1e-12 * np.linalg.norm(V) * np.linalg.cond(Z)


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_rybicki_scalar_matches_scipy_solve_toeplitz(n):
    rng = np.random.default_rng(n)
    t = {j: complex(rng.standard_normal(), rng.standard_normal()) for j in range(-(n - 1), n)}
    t[0] += 4.0
    R = {p: np.array([[t[p]]]) for p in t}
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xs = direct.rybicki_solve(R, [np.array([[v]]) for v in y])
    got = np.array([v[0, 0] for v in xs])
    col = np.array([t[j] for j in range(n)])
    row = np.array([t[-j] for j in range(n)])
    ref = sla.solve_toeplitz((col, row), y)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.linalg.norm(ref))


def test_rybicki_reports_singular_leading_section():
    b = 2
    blocks = np.zeros((3, 1, b, b), dtype=np.complex128)   # Nx = 1, Ny = 2
    blocks[1, 0] = np.array([[1.0, 2.0], [2.0, 4.0]])     # R_0 singular
    blocks[0, 0] = np.eye(b)
    blocks[2, 0] = np.eye(b)
    with pytest.raises(direct.SingularSection):
        direct.rybicki_solve_array(blocks, np.ones((1, 2 * b)))


# ----------------------------------------------------------------- preconditioners

def test_strang_lag_weights():
    assert precond.strang_lag_weights(4) == {-1: 1.0, 0: 1.0, 1: 1.0, -2: 0.5, 2: 0.5}
    assert precond.strang_lag_weights(5) == {-2: 1.0, -1: 1.0, 0: 1.0, 1: 1.0, 2: 1.0}
    assert precond.strang_lag_weights(1) == {0: 1.0}


@pytest.mark.parametrize("Nx,Ny,b", [(4, 4, 3), (3, 5, 2), (1, 6, 4), (5, 1, 2), (2, 2, 3)])
def test_strang_exact_for_periodic_operator(Nx, Ny, b):
    blocks = synth.periodic_blocks(Nx, Ny, b, seed=11)
    Z = tp.dense_Z(blocks)
    np.testing.assert_allclose(precond.strang_dense(blocks), Z, rtol=0, atol=1e-14)
    Sinv = precond.strang_inverse_spectrum(blocks)
    X = synth.random_vectors(Nx * Ny * b, 2, seed=3)
    back = precond.strang_apply(Sinv, tp.matvec_dense(Z, X))
    assert relerr(back, X) <= 1e-13
    res = krylov.gmres(lambda v: Z @ v, X[0], lambda r: precond.strang_apply(Sinv, r[None])[0], tol=1e-12)
    assert res.converged and res.iters == 1


@pytest.mark.parametrize("Nx,Ny,b", [(4, 4, 3), (3, 5, 2), (4, 2, 2)])
def test_strang_apply_equals_explicit_inverse(Nx, Ny, b):
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=2)
    S = precond.strang_dense(blocks)
    np.testing.assert_allclose(S, S.T, rtol=0, atol=1e-15 * np.abs(S).max())   # reciprocity kept
    Sinv = precond.strang_inverse_spectrum(blocks)
    R = synth.random_vectors(Nx * Ny * b, 2, seed=9)
    ref = np.linalg.solve(S, R.T).T
    assert relerr(precond.strang_apply(Sinv, R), ref) <= 1e-12


def test_kindt_and_row_preconditioners():
    Nx, Ny, b = 3, 2, 4
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=6)
    R = synth.random_vectors(Nx * Ny * b, 2, seed=1)
    PK = sla.block_diag(*[blocks[Ny - 1, Nx - 1]] * (Nx * Ny))
    np.testing.assert_allclose(precond.kindt_apply(blocks, R), np.linalg.solve(PK, R.T).T, rtol=1e-12)
    T0 = tp.level1_blocks(blocks)[0]
    PZ = sla.block_diag(*[T0] * Ny)
    np.testing.assert_allclose(precond.row_apply(blocks, R), np.linalg.solve(PZ, R.T).T, rtol=1e-12)


# ----------------------------------------------------------------- GMRES

def _nonsym_matrix(n, seed, shift=3.0):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    return A + shift * np.eye(n)


def test_givens_zeroes_second_entry():
    for a, b in [(1 + 2j, 3 - 1j), (0, 2j), (1.5, 0), (-2 + 0.5j, 1e-3)]:
        cs, sn = krylov.givens(a, b)
        G = np.array([[cs, sn], [-np.conj(sn), cs]])
        r = G @ np.array([a, b])
        assert abs(r[1]) <= 1e-15 * (abs(a) + abs(b))
        np.testing.assert_allclose(G.conj().T @ G, np.eye(2), atol=1e-15)


def test_gmres_unrestarted_is_exact_in_n_steps():
    n = 12
    A = _nonsym_matrix(n, 1, shift=0.5)
    v = np.arange(1, n + 1) * (1 + 0.5j)
    res = krylov.gmres(lambda z: A @ z, v, restart=n, tol=1e-13, max_restarts=1)
    assert res.iters <= n
    np.testing.assert_allclose(res.x, np.linalg.solve(A, v), rtol=0, atol=1e-10 * np.linalg.norm(res.x))


def test_gmres_residual_monotone_and_matches_lu_and_scipy():
    n = 60
    A = _nonsym_matrix(n, 2)
    v = np.random.default_rng(3).standard_normal(n) + 0j
    res = krylov.gmres(lambda z: A @ z, v, restart=10, tol=1e-10)
    assert res.converged
    h = np.array(res.history)
    for c in range(0, len(h), 10):                  # monotone inside every cycle
        seg = h[c:c + 10]
        assert np.all(np.diff(seg) <= 1e-15)
    ref = np.linalg.solve(A, v)
    kappa = np.linalg.cond(A)
    assert relerr(res.x, ref) <= 10 * kappa * 1e-10
    xs, info = spla.gmres(A, v, rtol=1e-12, restart=10, maxiter=200)
    assert info == 0 and relerr(res.x, xs) <= 1e-8


def test_right_and_flexible_preconditioning_agree():
    n = 40
    A = _nonsym_matrix(n, 4, shift=2.5)
    M = np.diag(np.diag(A)) + 0.1 * np.triu(A, 1)
    pc = lambda r: np.linalg.solve(M, r)
    v = np.ones(n, dtype=np.complex128)
    r1 = krylov.gmres(lambda z: A @ z, v, pc, restart=8, tol=1e-11)
    r2 = krylov.gmres(lambda z: A @ z, v, pc, restart=8, tol=1e-11, flexible=True)
    assert r1.converged and r2.converged and r1.iters == r2.iters
    np.testing.assert_allclose(r1.history, r2.history, rtol=1e-6, atol=1e-13)
    assert relerr(r1.x, r2.x) <= 1e-9


@pytest.mark.parametrize("use_pc", [False, True])
def test_gmres_on_green_array_matches_lu(use_pc):
    Nx, Ny, b = 4, 4, 24
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    Z = tp.dense_Z(blocks)
    V = synth.port_rhs(Nx, Ny, b, cols=[synth.centre_element(Nx, Ny), 0])
    ref = direct.lu_solve(Z, V)
    mv = lambda X: tp.matvec_fft(blocks, X, 2 * Ny, 2 * Nx)
    pc = None
    if use_pc:
        Sinv = precond.strang_inverse_spectrum(blocks)
        pc = lambda X: precond.strang_apply(Sinv, X)
    out = krylov.gmres_columns(mv, V, pc, tol=1e-10)
    X = np.array([r.x for r in out])
    assert all(r.converged for r in out)
    assert relerr(X, ref) <= 1e-9
    assert np.all(krylov.true_relres(mv, X, V) <= 1e-10)


def test_global_gmres_matches_lu():
    Nx, Ny, b = 3, 3, 6
    blocks = synth.green_blocks(Nx, Ny, b, np.pi, seed=0)
    Z = tp.dense_Z(blocks)
    V = synth.port_rhs(Nx, Ny, b)
    mv = lambda X: tp.matvec_dense(Z, X)
    res = krylov.gmres_global(mv, V, tol=1e-11)
    assert res.converged
    assert relerr(res.x, direct.lu_solve(Z, V)) <= 1e-9


def test_zero_rhs_gives_zero_solution():
    res = krylov.gmres(lambda z: 2 * z, np.zeros(5, dtype=np.complex128))
    assert res.converged and res.iters == 0 and not res.x.any()
