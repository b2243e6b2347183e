"""Pins of the oracle's Krylov solvers: restarted GMRES(m) (Algorithm 1),
flexible GMRES and BiCGSTAB.  Checked against dense solves, finite
termination (n steps; k+1 steps for identity plus rank k), exact
preconditioners (1 step), residual monotonicity and manufactured
solutions."""
import numpy as np
import pytest

import oracle
import reservoir_inputs as ri
from tests._helpers import bsr_from_dense, dense, relerr


@pytest.mark.parametrize("which", ["scalar", "block"])
def test_unrestarted_gmres_terminates_within_n(which):
    s = ri.scalar_system(4, 4, 4, seed=1) if which == "scalar" else ri.blackoil_system(4, 4, 4, seed=1)
    A = oracle.Matrix.from_system(s)
    pc = oracle.PC(A, "none")
    r = oracle.gmres(A, pc, s["b"], restart=A.n, maxit=A.n, rtol=1e-12)
    assert r["status"] == 0
    assert r["iters"] <= A.n
    assert relerr(r["x"], np.linalg.solve(dense(s), s["b"])) < 1e-8


def test_gmres_identity_plus_rank_k():
    rng = np.random.default_rng(4)
    n, k = 40, 3
    D = np.eye(n) + rng.standard_normal((n, k)) @ rng.standard_normal((k, n)) / n
    s = bsr_from_dense(D, 1)
    A = oracle.Matrix.from_system(s)
    b = rng.standard_normal(n)
    r = oracle.gmres(A, oracle.PC(A, "none"), b, restart=30, maxit=30, rtol=1e-12)
    assert r["status"] == 0 and r["iters"] <= k + 1
    assert relerr(r["x"], np.linalg.solve(D, b)) < 1e-10


@pytest.mark.parametrize("bs", [1, 3])
def test_exact_preconditioner_one_step(bs):
    s = ri.scalar_system(30, 1, 1, seed=2) if bs == 1 else ri.blackoil_system(20, 1, 1, seed=2)
    A = oracle.Matrix.from_system(s)
    pc = oracle.PC(A, "bilu0")
    r = oracle.gmres(A, pc, s["b"], restart=30, maxit=50, rtol=1e-10)
    assert r["iters"] == 1 and r["status"] == 0
    r = oracle.gmres(A, pc, s["b"], restart=30, maxit=50, rtol=1e-10, flexible=True)
    assert r["iters"] == 1 and r["status"] == 0
    r = oracle.bicgstab(A, pc, s["b"], maxit=50, rtol=1e-10)
    assert r["iters"] == 1 and r["status"] == 0


def test_gmres_estimate_monotone_within_cycle_and_true_residual_across_restarts():
    s = ri.blackoil_system(8, 8, 8, seed=3)
    A = oracle.Matrix.from_system(s)
    pc = oracle.PC(A, "bilu0")
    m = 10
    r = oracle.gmres(A, pc, s["b"], restart=m, maxit=60, rtol=1e-12, hist=True)
    h = r["hist"]
    for c in range(len(h) // m):
        seg = h[1 + c * m: 1 + (c + 1) * m]
        assert np.all(np.diff(seg) <= 1e-12 * seg[0])
    prev = np.inf
    for cycles in range(1, 6):
        rr = oracle.gmres(A, pc, s["b"], restart=m, maxit=cycles * m, rtol=0.0,
                          fixed_iters=True)
        assert rr["relres"] <= prev * (1 + 1e-12)
        prev = rr["relres"]


def test_gmres_estimate_equals_true_residual_right_preconditioned():
    # with right preconditioning the Arnoldi estimate |g_{j+1}| is the
    # unpreconditioned residual of the current iterate
    s = ri.blackoil_system(6, 6, 6, seed=4)
    A = oracle.Matrix.from_system(s)
    pc = oracle.PC(A, "bilu0")
    for k in [3, 7, 12]:
        r = oracle.gmres(A, pc, s["b"], restart=30, maxit=k, rtol=0.0,
                         fixed_iters=True, hist=True)
        bn = np.linalg.norm(s["b"])
        assert abs(r["hist"][-1] / bn - r["relres"]) < 1e-9 * max(r["relres"], 1e-12) + 1e-14


@pytest.mark.parametrize("solver", ["gmres", "fgmres", "left", "bicgstab"])
def test_solution_matches_dense_solve(solver):
    s = ri.blackoil_system(5, 4, 4, seed=6)
    A = oracle.Matrix.from_system(s)
    pc = oracle.PC(A, "bilu0")
    if solver == "bicgstab":
        r = oracle.bicgstab(A, pc, s["b"], maxit=500, rtol=1e-12)
    else:
        r = oracle.gmres(A, pc, s["b"], restart=30, maxit=500, rtol=1e-12,
                         flexible=solver == "fgmres", left=solver == "left")
    assert r["status"] == 0 and r["relres"] <= 1e-12
    xd = np.linalg.solve(dense(s), s["b"])
    assert relerr(r["x"], xd) < 1e-8
    assert relerr(r["x"], s["x_true"]) < 1e-8


def test_fgmres_equals_right_gmres_with_fixed_preconditioner():
    s = ri.blackoil_system(8, 8, 4, seed=7)
    A = oracle.Matrix.from_system(s)
    pc = oracle.PC(A, "bilu0")
    for k in [5, 30, 45]:
        a = oracle.gmres(A, pc, s["b"], restart=30, maxit=k, rtol=0.0, fixed_iters=True)
        b = oracle.gmres(A, pc, s["b"], restart=30, maxit=k, rtol=0.0, fixed_iters=True, flexible=True)
        assert relerr(b["x"], a["x"]) < 1e-10


def test_manufactured_solution_error_bounded_by_conditioning():
    s = ri.blackoil_system(6, 5, 4, seed=8)
    A = oracle.Matrix.from_system(s)
    r = oracle.gmres(A, oracle.PC(A, "bilu0"), s["b"], restart=30, maxit=1000, rtol=1e-8)
    kappa = np.linalg.cond(dense(s))
    assert r["status"] == 0 and r["relres"] <= 1e-8
    assert relerr(r["x"], s["x_true"]) <= kappa * 1e-8


def test_bicgstab_diagonal_system():
    d = np.linspace(1.0, 10.0, 12)
    s = bsr_from_dense(np.diag(d), 1)
    A = oracle.Matrix.from_system(s)
    b = np.arange(1.0, 13.0)
    r = oracle.bicgstab(A, oracle.PC(A, "none"), b, maxit=100, rtol=1e-12)
    assert r["status"] == 0 and r["iters"] <= 12
    assert relerr(r["x"], b / d) < 1e-10


def test_bicgstab_breakdown_restart_on_orthogonal_shadow():
    # b chosen so that the first rho of the second iteration vanishes is
    # hard to construct; instead a rotation matrix makes <rhat, A p> = 0 on
    # the first step and forces the restart path, which must still solve.
    R = np.array([[0.0, -1.0], [1.0, 0.0]])
    s = bsr_from_dense(R, 1)
    A = oracle.Matrix.from_system(s)
    b = np.array([1.0, 0.0])
    r = oracle.bicgstab(A, oracle.PC(A, "none"), b, maxit=10, rtol=1e-12)
    # v = A b is orthogonal to rhat = b: <rhat, v> = 0 -> breakdown, which
    # the solver reports through its restart count and iteration cap
    assert r["restarts"] >= 1
    assert r["status"] != 0


def test_maxit_reports_not_converged_with_results_filled():
    s = ri.blackoil_system(8, 8, 8, seed=9)
    A = oracle.Matrix.from_system(s)
    r = oracle.gmres(A, oracle.PC(A, "bilu0"), s["b"], restart=30, maxit=3, rtol=1e-12)
    assert r["status"] == oracle.NOT_CONVERGED and r["iters"] == 3
    assert 0 < r["relres"] < 1


def test_zero_rhs_returns_zero():
    s = ri.scalar_system(4, 4, 4, seed=1)
    A = oracle.Matrix.from_system(s)
    r = oracle.gmres(A, oracle.PC(A, "bilu0"), np.zeros(A.n), rtol=1e-8)
    assert r["status"] == 0 and r["iters"] == 0 and np.all(r["x"] == 0)


# ---- LGMRES (Section 3 names it with aug_k) and PCG (Algorithm 2) --------------
def _dense_minv(A, kind="bilu0"):
    from tests._helpers import lu_dense_from_factor
    rc, lu = oracle.bilu0(A)
    assert rc == 0
    L, U = lu_dense_from_factor(A.rowptr, A.col, lu, A.bs)
    return np.linalg.inv(L @ U), L @ U


def _orth(cols):
    q, _ = np.linalg.qr(np.column_stack(cols))
    return q


def test_lgmres_without_augmentation_is_fgmres():
    s = ri.blackoil_system(6, 5, 4, seed=3)
    A = oracle.Matrix.from_system(s)
    pc = oracle.PC(A, "bilu0")
    a = oracle.lgmres(A, pc, s["b"], restart=5, aug_k=0, maxit=15, fixed_iters=True)
    b = oracle.gmres(A, pc, s["b"], restart=5, maxit=15, flexible=True, fixed_iters=True)
    assert relerr(a["x"], b["x"]) < 1e-12


@pytest.mark.parametrize("k", [1, 2])
def test_lgmres_cycles_minimize_over_augmented_space(k):
    """Each cycle's iterate is x + argmin ||r - A d|| over d in
    M^-1 K_m(A M^-1, r) + span(stored corrections), built here from an
    explicit (orthonormalized) power basis and a dense least-squares solve;
    the stored corrections are this test's own previous cycle updates."""
    s = ri.blackoil_system(3, 3, 2, seed=4)
    A = oracle.Matrix.from_system(s)
    D = dense(s)
    Minv, _ = _dense_minv(A)
    b = s["b"]
    m = 4
    x = np.zeros(A.n)
    Z = []
    steps = 0
    pc = oracle.PC(A, "bilu0")
    for c in range(4):
        r = b - D @ x
        cols = [r]
        for _ in range(m - 1):
            cols.append(D @ (Minv @ _orth(cols)[:, -1]))
        Kb = _orth(cols)
        Ub = np.column_stack([Minv @ Kb] + Z)
        d = np.linalg.lstsq(D @ Ub, r, rcond=None)[0]
        dx = Ub @ d
        x = x + dx
        Z = ([dx / np.linalg.norm(dx)] + Z)[:k]
        steps += m + min(c, k)
        got = oracle.lgmres(A, pc, b, restart=m, aug_k=k, maxit=steps, fixed_iters=True)
        assert got["restarts"] == c + 1
        assert relerr(got["x"], x) < 1e-8, (c, relerr(got["x"], x))


def test_lgmres_converges_where_restarted_gmres_stalls():
    s = ri.blackoil_system(6, 5, 4, seed=3)
    A = oracle.Matrix.from_system(s)
    pc = oracle.PC(A, "bilu0")
    a = oracle.lgmres(A, pc, s["b"], restart=5, aug_k=2, maxit=1000, rtol=1e-10)
    g = oracle.gmres(A, pc, s["b"], restart=5, maxit=1000, rtol=1e-10, flexible=True)
    assert a["status"] == 0 and a["relres"] <= 1e-10
    assert a["iters"] < 0.5 * g["iters"]


def test_ilu0_of_symmetric_matrix_is_symmetric():
    # U = D L^T when A is symmetric, so M = L U is symmetric: a valid CG
    # preconditioner (IC(0) in LU form)
    s = ri.scalar_system(4, 4, 3, seed=2)
    A = oracle.Matrix.from_system(s)
    _, M = _dense_minv(A)
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    assert np.linalg.eigvalsh(M).min() > 0


def test_pcg_iterates_minimize_energy_error_over_krylov_space():
    """x_k = x_0 + B c with B a basis of K_k(M^-1 A, M^-1 r_0) and
    (B^T A B) c = B^T r_0 (the Galerkin condition, solved densely)."""
    s = ri.scalar_system(4, 4, 3, seed=2)
    A = oracle.Matrix.from_system(s)
    D = dense(s)
    Minv, _ = _dense_minv(A)
    b = s["b"]
    pc = oracle.PC(A, "ilu0")
    z0 = Minv @ b
    cols = [z0]
    for k in range(1, 7):
        B = _orth(cols)
        c = np.linalg.solve(B.T @ D @ B, B.T @ b)
        ref = B @ c
        got = oracle.pcg(A, pc, b, maxit=k, fixed_iters=True)
        assert relerr(got["x"], ref) < 1e-9, (k, relerr(got["x"], ref))
        cols.append(Minv @ (D @ B[:, -1]))


def test_cg_exact_after_as_many_steps_as_distinct_eigenvalues():
    # SPD with eigenvalues {1, 4, 9}: the error lies in a 3-dimensional
    # Krylov space, so CG is exact after 3 steps and not after 2
    rng = np.random.default_rng(6)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    D = Q @ np.diag([1.0] * 4 + [4.0] * 4 + [9.0] * 4) @ Q.T
    D = (D + D.T) / 2
    st = bsr_from_dense(D, 1)
    A = oracle.Matrix.from_system(st)
    b = rng.standard_normal(12)
    pc = oracle.PC(A, "none")
    assert oracle.pcg(A, pc, b, maxit=3, fixed_iters=True)["relres"] < 1e-12
    assert oracle.pcg(A, pc, b, maxit=2, fixed_iters=True)["relres"] > 1e-3


def test_pcg_reports_breakdown_on_indefinite_matrix():
    D = np.diag([2.0, -1.0, 3.0, 1.0])
    D[0, 1] = D[1, 0] = 0.5
    st = bsr_from_dense(D, 1)
    A = oracle.Matrix.from_system(st)
    # b along the negative-curvature direction: (p, A p) < 0 at the first step
    got = oracle.pcg(A, oracle.PC(A, "none"), np.array([0.0, 1.0, 0.0, 0.0]), maxit=10, rtol=1e-12)
    assert got["status"] == oracle.ERR_BREAKDOWN


def test_openmp_build_solves_like_the_serial_oracle():
    # the OpenMP build times the CPU leg of the benchmark: its parallel sums
    # round differently, so it must reach the same solve, not the same bits
    import shutil
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    try:
        lib_omp = oracle.load(oracle.build_omp(force=False))
    except Exception as e:       # no OpenMP runtime in this toolchain
        pytest.skip(f"OpenMP build unavailable: {e}")
    s = ri.blackoil_system(16, 12, 10, seed=5)
    A = oracle.Matrix.from_system(s)
    ref = oracle.gmres(A, oracle.PC(A, "bilu0"), s["b"], restart=30, maxit=1000, rtol=1e-10)
    with oracle.using(lib_omp):
        A2 = oracle.Matrix.from_system(s)
        got = oracle.gmres(A2, oracle.PC(A2, "bilu0"), s["b"], restart=30, maxit=1000, rtol=1e-10)
    assert ref["status"] == got["status"] == 0
    assert abs(got["iters"] - ref["iters"]) <= 1
    assert np.linalg.norm(got["x"] - ref["x"]) <= 1e-8 * np.linalg.norm(ref["x"])
    r = s["b"] - oracle.spmv(A, got["x"])
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(s["b"]) * (1 + 1e-9)
