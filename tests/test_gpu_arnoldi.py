"""GPU pins of the Arnoldi step (Algorithm 1's Arnoldi process, with
classical Gram-Schmidt applied twice in place of modified Gram-Schmidt:
CGS2, or for GMRES with a fixed preconditioner its lagged form, whose
second projection of a step's vector runs in the next step's pass):
orthonormality of the basis after a full restart cycle for both forms, the
two forms against each other on a 64^3 black-oil solve, termination in
k + 1 steps on identity plus rank k, and one-step lucky breakdowns on
eigenvectors: one where h_{2,1} is rounding noise of the product A v_1,
and one (A = 4 I) where what the first projection leaves is a rounding
multiple of v_1, the case in which CGS2 takes h_{j+1,j} as an explicit
norm and a norm at the rounding level of the projections counts as zero."""
import numpy as np
import pytest

import oracle
import reservoir_inputs as ri

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1701_05913_amd as K  # noqa: E402
from tests.gpu_helpers import GpuSystem, make_solver, relerr, solve  # noqa: E402


def _csr(dense):
    rp, ci, va = [0], [], []
    for i, row in enumerate(dense):
        nz = np.nonzero(row)[0]
        if i not in nz:
            nz = np.sort(np.append(nz, i))
        ci.extend(nz.tolist())
        va.extend(row[nz].tolist())
        rp.append(len(ci))
    return dict(rowptr=np.array(rp, np.int32), col=np.array(ci, np.int32),
                val=np.array(va), bs=1)


@pytest.mark.parametrize("solver,ortho", [("GMRES", "AUTO"), ("GMRES", "CGS2"), ("FGMRES", "AUTO")])
def test_basis_orthonormal_after_full_cycle_blackoil64(solver, ortho):
    # 64^3 black-oil system, BILU(0), one full cycle of 30 steps (rtol 0):
    # columns 1..30 of V (column 0 holds the next cycle's residual) must be
    # orthonormal to 1e-12, and every column must be a unit vector (GMRES
    # AUTO: the lagged form, whose end-of-cycle pass normalizes v_30)
    s = ri.blackoil_system(64, 64, 64, seed=0)
    g = GpuSystem(s)
    S = make_solver(g, getattr(K, f"KRY_{solver}"), K.KRY_PC_BILU0, rtol=0.0, maxit=30,
                    ortho=getattr(K, f"KRY_ORTHO_{ortho}"))
    try:
        K.SolverAssemble(S)
        bt, bh = g.vec(s["b"])
        xt, xh = g.vec()
        K.SolverSolve(S, bh, xh)
        torch.cuda.synchronize()
        assert K.SolverGetIters(S) == 30
        V = K.SolverGetKrylovBasis(S, 1, 30, g.n)
    finally:
        K.SolverDestroy(S)
        g.close()
    G = V @ V.T
    err = np.abs(G - np.eye(30)).max()
    print(f"max |V^T V - I| over 30 columns: {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("restart", [30, 7])
def test_lagged_gram_schmidt_agrees_with_cgs2_blackoil64(restart):
    # GMRES(m) + BILU(0) to 1e-8 on the 64^3 black-oil system with both
    # forms: the same iteration count, residual estimates equal step by step
    # to 1e-13 of the initial residual (and 1e-6 of each), iterates to 1e-8
    # (both are Algorithm 1 in exact arithmetic and differ by rounding,
    # which restarts carry from cycle to cycle; m = 7 ends many cycles, each
    # with the lagged form's end-of-cycle pass)
    s = ri.blackoil_system(64, 64, 64, seed=0)
    g = GpuSystem(s)
    try:
        lag = solve(g, K.KRY_GMRES, K.KRY_PC_BILU0, rtol=1e-8, maxit=3000, restart=restart)
        cgs = solve(g, K.KRY_GMRES, K.KRY_PC_BILU0, rtol=1e-8, maxit=3000, restart=restart,
                    ortho=K.KRY_ORTHO_CGS2)
    finally:
        g.close()
    print(f"m={restart}: lagged {lag['iters']} its, relres {lag['relres']:.3e}; "
          f"CGS2 {cgs['iters']} its, relres {cgs['relres']:.3e}")
    assert lag["status"] == K.KRY_OK and cgs["status"] == K.KRY_OK
    assert lag["iters"] == cgs["iters"]
    hl, hc = np.asarray(lag["hist"]), np.asarray(cgs["hist"])
    assert hl.shape == hc.shape
    assert np.max(np.abs(hl - hc)) <= 1e-13 * hc[0]
    assert np.max(np.abs(hl - hc) / hc) <= 1e-6
    assert relerr(lag["x"], cgs["x"]) <= 1e-8
    assert lag["relres"] <= 1e-8


def test_identity_plus_rank3_converges_in_four_steps():
    # A = I + U W^T with rank 3: the Krylov space of any b has dimension
    # at most 4, so unpreconditioned GMRES ends within 4 steps (lucky
    # breakdown or the tolerance) with x = A^-1 b
    n = 300
    rng = np.random.default_rng(5)
    U = rng.standard_normal((n, 3)) / np.sqrt(n)
    W = rng.standard_normal((n, 3))
    A = np.eye(n) + U @ W.T
    b = rng.standard_normal(n)
    s = _csr(A)
    s["b"] = b
    g = GpuSystem(s)
    try:
        r = solve(g, K.KRY_GMRES, K.KRY_PC_NONE, rtol=1e-12, maxit=100)
    finally:
        g.close()
    x_ref = np.linalg.solve(A, b)
    assert r["status"] == K.KRY_OK
    assert r["iters"] <= 4, r["iters"]
    assert np.all(np.isfinite(r["x"]))
    assert relerr(r["x"], x_ref) <= 1e-10


@pytest.mark.parametrize("n", [500, 4097])
def test_eigenvector_rhs_lucky_breakdown_one_step(n):
    # 1D Laplacian tridiag(-1, 2, -1): b = sin(pi k i / (n + 1)) is an
    # eigenvector with eigenvalue 2 - 2 cos(pi k / (n + 1)) up to rounding,
    # so w = A v_1 lies in span{v_1} except for rounding: h_{2,1} is the
    # rounding noise of the product, and the step must finish with a finite
    # h_{2,1}, no NaN, and convergence after one step with x = b / lambda
    k = 3
    i = np.arange(1, n + 1)
    lam = 2.0 - 2.0 * np.cos(np.pi * k / (n + 1))
    b = np.sin(np.pi * k * i / (n + 1))
    rp = np.zeros(n + 1, np.int64)
    cols, vals = [], []
    for r in range(n):
        for c, v in ((r - 1, -1.0), (r, 2.0), (r + 1, -1.0)):
            if 0 <= c < n:
                cols.append(c)
                vals.append(v)
        rp[r + 1] = len(cols)
    s = dict(rowptr=rp.astype(np.int32), col=np.array(cols, np.int32), val=np.array(vals), bs=1, b=b)
    g = GpuSystem(s)
    try:
        r = solve(g, K.KRY_GMRES, K.KRY_PC_NONE, rtol=1e-8, maxit=100)
    finally:
        g.close()
    A = oracle.Matrix(s["rowptr"], s["col"], s["val"])
    assert r["status"] == K.KRY_OK
    assert r["iters"] == 1, r["iters"]
    assert np.all(np.isfinite(r["x"])) and np.all(np.isfinite(r["hist"]))
    assert relerr(r["x"], b / lam) <= 1e-10
    assert np.linalg.norm(b - oracle.spmv(A, r["x"])) <= 1e-8 * np.linalg.norm(b)


def test_multiple_of_identity_lucky_breakdown_one_step():
    # A = 4 I: w = A v_1 = 4 v_1 exactly, so whatever the first projection
    # leaves is a rounding multiple of v_1 (the case where ||h2||^2 is
    # comparable to ||w - V h1||^2); one step, x = b / 4, no NaN
    n = 100003
    b = np.random.default_rng(8).standard_normal(n)
    s = dict(rowptr=np.arange(n + 1, dtype=np.int32), col=np.arange(n, dtype=np.int32),
             val=np.full(n, 4.0), bs=1, b=b)
    g = GpuSystem(s)
    try:
        r = solve(g, K.KRY_GMRES, K.KRY_PC_NONE, rtol=1e-10, maxit=100)
    finally:
        g.close()
    assert r["status"] == K.KRY_OK
    assert r["iters"] == 1, r["iters"]
    assert np.all(np.isfinite(r["x"])) and np.all(np.isfinite(r["hist"]))
    assert relerr(r["x"], b / 4.0) <= 1e-14
