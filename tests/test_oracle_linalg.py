"""Pins of the FP64 oracle's sparse kernels: SpMV (Figures 20-21),
ILU(0) / block ILU(0) and the triangular solves of eq. (3).

Every check compares the oracle with something other than itself: dense
products, dense LU and triangular solves, exact integer arithmetic, and
structural facts of 7-point stencils."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import reservoir_inputs as ri
from tests._helpers import dense, lu_dense_from_factor, relerr, bsr_from_dense


def _systems():
    return [ri.scalar_system(4, 4, 4, seed=1),
            ri.blackoil_system(4, 4, 4, seed=2),
            ri.blackoil_system(5, 3, 2, seed=3)]


# ---- C1 SpMV ---------------------------------------------------------------
@pytest.mark.parametrize("k", range(3))
def test_spmv_matches_dense(k):
    s = _systems()[k]
    A = oracle.Matrix.from_system(s)
    x = np.random.default_rng(k).standard_normal(A.n)
    D = dense(s)
    assert relerr(oracle.spmv(A, x), D @ x) < 1e-14
    y = np.random.default_rng(k + 9).standard_normal(A.n)
    for a, b in [(1.0, 0.0), (-1.0, 1.0), (2.5, -0.5)]:
        assert relerr(oracle.amxpby(A, a, x, b, y), a * (D @ x) + b * y) < 1e-14


def test_spmv_integer_exact():
    rng = np.random.default_rng(0)
    s = ri.blackoil_system(5, 4, 3, seed=4)
    s["val"] = rng.integers(-8, 9, size=s["val"].shape).astype(np.float64)
    A = oracle.Matrix.from_system(s)
    x = rng.integers(-5, 6, size=A.n).astype(np.float64)
    D = dense(s)
    assert np.array_equal(oracle.spmv(A, x), D @ x)


# ---- C2/C3 ILU(0) --------------------------------------------------------------
@pytest.mark.parametrize("k", range(3))
def test_ilu_product_equals_a_on_pattern(k):
    s = _systems()[k]
    A = oracle.Matrix.from_system(s)
    rc, lu = oracle.bilu0(A)
    assert rc == 0
    bs = A.bs
    L, U = lu_dense_from_factor(A.rowptr, A.col, lu, bs)
    P = L @ U
    D = dense(s)
    absprod = np.abs(L) @ np.abs(U)
    for i in range(A.nb):
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            j = A.col[p]
            sl = np.s_[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs]
            assert np.all(np.abs(P[sl] - D[sl]) <= 1e-14 * absprod[sl] + 1e-300)


@pytest.mark.parametrize("k", range(3))
def test_ilu_seven_point_changes_only_diagonal_blocks(k):
    # A 3D Cartesian grid has no triangles, so no fill lands in the
    # pattern: the strictly upper blocks of U equal those of A, and
    # L_ik = A_ik U_kk^-1.
    s = _systems()[k]
    A = oracle.Matrix.from_system(s)
    rc, lu = oracle.bilu0(A)
    bs = A.bs
    a = A.val.reshape(-1, bs, bs)
    f = lu.reshape(-1, bs, bs)
    diag = {}
    for i in range(A.nb):
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            if A.col[p] == i:
                diag[i] = f[p]
    for i in range(A.nb):
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            j = A.col[p]
            if j > i:
                assert np.array_equal(f[p], a[p])
            elif j < i:
                assert np.allclose(f[p] @ diag[j], a[p], rtol=1e-13, atol=1e-13 * np.abs(a[p]).max())


@pytest.mark.parametrize("bs", [1, 3])
def test_ilu_exact_on_tridiagonal(bs):
    s = ri.scalar_system(40, 1, 1, seed=5) if bs == 1 else ri.blackoil_system(30, 1, 1, seed=5)
    A = oracle.Matrix.from_system(s)
    rc, lu = oracle.bilu0(A)
    b = np.random.default_rng(1).standard_normal(A.n)
    x = oracle.bilu0_solve(A, lu, b)
    assert relerr(x, np.linalg.solve(dense(s), b)) < 1e-12


def test_bilu_block_diagonal_is_exact_inverse():
    rng = np.random.default_rng(3)
    D = np.zeros((18, 18))
    for i in range(6):
        D[3*i:3*i+3, 3*i:3*i+3] = rng.standard_normal((3, 3)) + 3 * np.eye(3)
    s = bsr_from_dense(D, 3)
    A = oracle.Matrix.from_system(s)
    rc, lu = oracle.bilu0(A)
    b = rng.standard_normal(18)
    assert relerr(oracle.bilu0_solve(A, lu, b), np.linalg.solve(D, b)) < 1e-13


def test_ilu_zero_pivot_reported():
    D = np.array([[0.0, 1.0], [1.0, 2.0]])
    s = bsr_from_dense(D, 1)
    rc, _ = oracle.bilu0(oracle.Matrix.from_system(s))
    assert rc == oracle.ERR_ZERO_PIVOT
    D3 = np.zeros((3, 3))
    D3[0, 0] = 1.0
    s = bsr_from_dense(D3, 3)
    rc, _ = oracle.bilu0(oracle.Matrix.from_system(s))
    assert rc == oracle.ERR_ZERO_PIVOT


# ---- C4 triangular solves ---------------------------------------------------
@pytest.mark.parametrize("k", range(3))
def test_triangular_solves_match_dense(k):
    s = _systems()[k]
    A = oracle.Matrix.from_system(s)
    rc, lu = oracle.bilu0(A)
    L, U = lu_dense_from_factor(A.rowptr, A.col, lu, A.bs)
    b = np.random.default_rng(k).standard_normal(A.n)
    y = oracle.bilu0_solve(A, lu, b, "lower")
    assert relerr(y, sla.solve_triangular(L, b, lower=True, unit_diagonal=True)) < 1e-13
    x = oracle.bilu0_solve(A, lu, y, "upper")
    # U is block upper triangular: full diagonal blocks when bs > 1
    ref = sla.solve_triangular(U, y, lower=False) if A.bs == 1 else np.linalg.solve(U, y)
    assert relerr(x, ref) < 1e-12
    assert relerr(oracle.bilu0_solve(A, lu, b), np.linalg.solve(L @ U, b)) < 1e-11


def test_bf16_rounding_closed_forms():
    # bfloat16 keeps 7 explicit mantissa bits: spacing 2^-7 at 1
    assert oracle.bf16_round(1.0) == 1.0
    assert oracle.bf16_round(1.0 + 2.0**-8) == 1.0              # tie -> even
    assert oracle.bf16_round(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6  # tie -> even
    assert oracle.bf16_round(1.0 + 2.0**-8 + 2.0**-20) == 1.0 + 2.0**-7
    assert oracle.bf16_round(-3.0) == -3.0
