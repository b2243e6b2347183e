"""Pins of the oracle's algebraic multigrid (Section 4.2: Algorithms 3 and
4, eq. (4), the defaults of Figure 34): strength on a hand-made matrix,
Ruge-Stueben splitting on a 1D chain worked by hand and its invariants on
random grids, interpolation that keeps constants on zero-row-sum rows and
is exact where an F point sees only C points, truncation that keeps row
sums, the Galerkin product, the V-cycle against a dense restatement of
Algorithm 4 with the smoother as a matrix splitting, and convergence."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import reservoir_inputs as ri
from tests._helpers import bsr_from_dense, dense_from_bsr, relerr


def _csr(D):
    return oracle.Matrix.from_system(bsr_from_dense(np.asarray(D, dtype=float), 1))


def _dense_csr(rp, ci, v, ncols):
    M = np.zeros((len(rp) - 1, ncols))
    for i in range(len(rp) - 1):
        for q in range(rp[i], rp[i + 1]):
            M[i, ci[q]] += v[q]
    return M


def _strong_sets(A, theta=0.5, mrs=0.9):
    srp, sci = oracle.amg_strength(A, theta, mrs)
    return [list(sci[srp[i]:srp[i + 1]]) for i in range(A.nb)]


def _grid_laplacian(grid, seed, acc=0.0, shift_layer0=0.0):
    """7-point finite-volume operator with lognormal transmissibilities;
    acc on every diagonal, shift_layer0 more on the k = 0 layer."""
    s = ri.scalar_system(*grid, seed=seed, acc=acc)
    val = s["val"].copy()
    nx, ny, _ = grid
    for i in range(nx * ny):
        for q in range(s["rowptr"][i], s["rowptr"][i + 1]):
            if s["col"][q] == i:
                val[q] += shift_layer0
    return oracle.Matrix(s["rowptr"], s["col"], val, 1)


# ---- strength ----------------------------------------------------------------
def test_strength_hand_example():
    # theta = 0.5, max_row_sum = 0.9; worked by hand from the definition:
    # row 0: -a = (1, 0.4, 0.6) off the diagonal, max 1: strong {1, 3}
    # row 1: -a = (1, 1, -0.5): the positive coupling is never strong: {0, 2}
    # row 2: -a = (0.4, 1): {1}
    # row 3: |row sum| 9.4 > 0.9 * 10: no strong dependencies
    # row 4: negative diagonal, so +a counts: (0.2, 0.7, 0.3): {3} (0.3 < 0.35)
    D = np.array([[4.0, -1.0, -0.4, -0.6, 0.0],
                  [-1.0, 3.0, -1.0, 0.5, 0.0],
                  [-0.4, -1.0, 2.0, 0.0, 0.0],
                  [-0.6, 0.0, 0.0, 10.0, 0.0],
                  [0.0, 0.2, 0.0, 0.7, -5.0]])
    D[4, 2] = 0.3
    assert _strong_sets(_csr(D)) == [[1, 3], [0, 2], [1], [], [3]]
    # without the row-sum rule row 3 depends on 0; theta 0.3 adds (4, 2)
    assert _strong_sets(_csr(D), 0.5, 1.0)[3] == [0]
    assert _strong_sets(_csr(D), 0.3, 0.9)[4] == [2, 3]


# ---- splitting and interpolation on a 1D chain, worked by hand ---------------
def test_chain_splitting_interpolation_and_galerkin():
    # tridiag(-1, 2, -1), n = 9: every coupling strong; measures 1 2 ... 2 1.
    # Point 1 (largest measure, smallest index) becomes C, 0 and 2 F; 3 then
    # has the largest measure, and so on: C = {1, 3, 5, 7}.  An F point
    # interpolates from its C neighbours with weight -(-1)/2 = 1/2.
    n = 9
    D = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    M = oracle.AMG(_csr(D), max_levels=2, coarse_size=1)
    lv = M.level(0)
    assert list(lv["cf"]) == [0, 1, 0, 1, 0, 1, 0, 1, 0]
    P = _dense_csr(*lv["P"], lv["nc"])
    Pref = np.zeros((9, 4))
    for c, i in enumerate([1, 3, 5, 7]):
        Pref[i, c] = 1.0
        Pref[i - 1, c] += 0.5
        Pref[i + 1, c] += 0.5
    assert np.array_equal(P, Pref)
    Ac = dense_from_bsr(*M.level(1)["A"], 1)
    # P^T A P of linear interpolation: 1/2 tridiag(-1, 2, -1)
    assert np.allclose(Ac, 0.5 * (2 * np.eye(4) - np.eye(4, k=1) - np.eye(4, k=-1)),
                       rtol=0, atol=1e-15)


# ---- invariants on random grids ----------------------------------------------
@pytest.mark.parametrize("grid,seed", [((12, 10, 1), 1), ((8, 7, 6), 2), ((10, 9, 5), 3)])
def test_splitting_invariants(grid, seed):
    A = _grid_laplacian(grid, seed, acc=1e-3)
    M = oracle.AMG(A)
    assert M.nlevels >= 2
    for l in range(M.nlevels - 1):
        lv = M.level(l)
        rp, ci, a = lv["A"]
        Al = oracle.Matrix(rp, ci, a, 1)
        S = _strong_sets(Al)
        cf = lv["cf"]
        assert lv["nc"] == int(cf.sum())
        prp, pci, pv = lv["P"]
        cmap = np.cumsum(cf) - 1
        for i in range(lv["n"]):
            row = list(zip(pci[prp[i]:prp[i + 1]], pv[prp[i]:prp[i + 1]]))
            if cf[i]:
                assert row == [(cmap[i], 1.0)]          # C points are injected
                continue
            Ci = {j for j in S[i] if cf[j]}
            if S[i]:
                assert Ci, (l, i)                       # an F point sees a C point
            for j in S[i]:
                if not cf[j]:                           # strong F-F pairs share one
                    assert Ci & set(S[j]), (l, i, j)
            assert {cmap[j] for j in Ci} >= {c for c, _ in row}


def test_interpolation_keeps_constants_on_zero_row_sums():
    # interior rows of a no-flow operator sum to zero, and so do the coarse
    # rows away from the shifted layer: their weights sum to 1.  On the
    # 7-point level an F point's strong F neighbours share no C point (the
    # stencil has no triangles) and are lumped; the denser coarse levels
    # distribute them.
    grid = (10, 9, 8)
    A = _grid_laplacian(grid, 4, acc=0.0, shift_layer0=1.0)
    M = oracle.AMG(A, max_levels=4)
    checked = [0, 0, 0]
    for l in range(3):
        lv = M.level(l)
        prp, pci, pv = lv["P"]
        rp, ci, a = lv["A"]
        for i in range(lv["n"]):
            if lv["cf"][i] or prp[i] == prp[i + 1]:
                continue
            row = a[rp[i]:rp[i + 1]]
            if abs(row.sum()) > 1e-13 * np.abs(row).max():
                continue
            assert abs(pv[prp[i]:prp[i + 1]].sum() - 1.0) <= 1e-11, (l, i)
            checked[l] += 1
    assert min(checked) > 20, checked


def test_direct_interpolation_where_f_sees_only_c():
    # an F point whose neighbours are all strong C points interpolates with
    # w_ij = -a_ij / a_ii (the ideal -A_FF^-1 A_FC for such a row)
    A = _grid_laplacian((11, 9, 1), 5, acc=1e-3)
    M = oracle.AMG(A, max_levels=2)
    lv = M.level(0)
    S = _strong_sets(A)
    cf, (prp, pci, pv), (rp, ci, a) = lv["cf"], lv["P"], lv["A"]
    cmap = np.cumsum(cf) - 1
    found = 0
    for i in range(A.nb):
        nbrs = [(ci[q], a[q]) for q in range(rp[i], rp[i + 1]) if ci[q] != i]
        aii = a[rp[i]:rp[i + 1]][ci[rp[i]:rp[i + 1]] == i][0]
        if cf[i] or not all(cf[j] and j in S[i] for j, _ in nbrs):
            continue
        w = dict(zip(pci[prp[i]:prp[i + 1]], pv[prp[i]:prp[i + 1]]))
        mx = max(abs(v) for _, v in nbrs) / aii
        want = {cmap[j]: -v / aii for j, v in nbrs if abs(v) / aii >= 1e-2 * mx}
        kept = sum(want.values())
        full = sum(-v / aii for _, v in nbrs)
        for c in want:
            want[c] *= full / kept
        assert set(w) == set(want)
        for c in w:
            assert abs(w[c] - want[c]) <= 1e-15 * abs(want[c]) + 1e-17
        found += 1
    assert found >= 5


def test_truncation_drops_small_weights_and_keeps_row_sums():
    A = _grid_laplacian((10, 8, 6), 6, acc=1e-3)
    full = oracle.AMG(A, max_levels=2, trunc=0.0).level(0)
    cut = oracle.AMG(A, max_levels=2, trunc=0.7).level(0)
    assert np.array_equal(full["cf"], cut["cf"])
    fp, cp = full["P"], cut["P"]
    dropped = 0
    for i in range(A.nb):
        wf = dict(zip(fp[1][fp[0][i]:fp[0][i + 1]], fp[2][fp[0][i]:fp[0][i + 1]]))
        wc = dict(zip(cp[1][cp[0][i]:cp[0][i + 1]], cp[2][cp[0][i]:cp[0][i + 1]]))
        if not wf:
            assert not wc
            continue
        mx = max(abs(v) for v in wf.values())
        assert set(wc) == {c for c, v in wf.items() if abs(v) >= 0.7 * mx}
        dropped += len(wf) - len(wc)
        assert abs(sum(wc.values()) - sum(wf.values())) <= 1e-14 * abs(sum(wf.values()))
        scale = sum(wf.values()) / sum(wf[c] for c in wc)
        for c in wc:
            assert abs(wc[c] - wf[c] * scale) <= 1e-14 * abs(wc[c])
    assert dropped > 0


def test_galerkin_coarse_matrices():
    A = _grid_laplacian((9, 8, 7), 7, acc=1e-3)
    M = oracle.AMG(A)
    for l in range(M.nlevels - 1):
        lv, nxt = M.level(l), M.level(l + 1)
        Al = dense_from_bsr(*lv["A"], 1)
        P = _dense_csr(*lv["P"], lv["nc"])
        Ac = dense_from_bsr(*nxt["A"], 1)
        assert relerr(Ac, P.T @ Al @ P) <= 1e-14


# ---- the V-cycle ----------------------------------------------------------------
def _dense_vcycle(levels, b, chunk, sweeps):
    """Algorithm 4 on dense matrices; hybrid Gauss-Seidel written as the
    splitting A = M - N, M = the diagonal plus the lower triangle inside
    each chunk of rows: x <- x + M^-1 (b - A x)."""
    A, P = levels[0]
    if P is None:
        return np.linalg.solve(A, b)
    n = A.shape[0]
    c = chunk if chunk > 0 else n
    blk = np.arange(n) // c
    Msplit = np.tril(A) * (blk[:, None] == blk[None, :])
    Msplit[np.diag_indices(n)] = np.diag(A)

    def smooth(x):
        for _ in range(sweeps):
            x = x + sla.solve_triangular(Msplit, b - A @ x, lower=True)
        return x

    x = smooth(np.zeros(n))
    xc = _dense_vcycle(levels[1:], P.T @ (b - A @ x), chunk, sweeps)
    return smooth(x + P @ xc)


@pytest.mark.parametrize("chunk,sweeps", [(0, 2), (1, 2), (4, 2), (7, 1), (4, 3)])
def test_vcycle_matches_dense_algorithm4(chunk, sweeps):
    A = _grid_laplacian((8, 7, 6), 8, acc=1e-2)
    M = oracle.AMG(A, gs_chunk=chunk, num_sweeps=sweeps)
    levels = []
    for l in range(M.nlevels):
        lv = M.level(l)
        P = None if lv["P"] is None else _dense_csr(*lv["P"], lv["nc"])
        levels.append((dense_from_bsr(*lv["A"], 1), P))
    b = np.random.default_rng(9).standard_normal(A.n)
    assert relerr(M.vcycle(b), _dense_vcycle(levels, b, chunk, sweeps)) <= 1e-12


def test_single_level_is_exact_solve():
    A = _grid_laplacian((5, 4, 3), 9, acc=1e-2)
    b = np.random.default_rng(10).standard_normal(A.n)
    x = oracle.AMG(A, max_levels=1).vcycle(b)
    assert relerr(x, np.linalg.solve(dense_from_bsr(A.rowptr, A.col, A.val, 1), b)) <= 1e-13


@pytest.mark.parametrize("chunk", [0, 4])
def test_vcycle_converges_on_poisson(chunk):
    # constant-coefficient 7-point Poisson, 16^3: a correct classical AMG
    # reduces the error by well over 3x per cycle
    n = 16
    m = n ** 3
    rows, cols, vals = [], [], []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                r = (k * n + j) * n + i
                for d, ok in ((-n * n, k > 0), (-n, j > 0), (-1, i > 0), (0, True),
                              (1, i < n - 1), (n, j < n - 1), (n * n, k < n - 1)):
                    if ok:
                        rows.append(r)
                        cols.append(r + d)
                        vals.append(6.0 if d == 0 else -1.0)
    order = np.lexsort((cols, rows))
    rp = np.searchsorted(np.array(rows)[order], np.arange(m + 1)).astype(np.int32)
    A = oracle.Matrix(rp, np.array(cols)[order], np.array(vals)[order], 1)
    M = oracle.AMG(A, gs_chunk=chunk)
    b = np.zeros(m)
    x = np.random.default_rng(11).standard_normal(m)
    e0 = np.linalg.norm(x)
    for _ in range(5):
        x = x + M.vcycle(b - oracle.spmv(A, x))
    assert np.linalg.norm(x) / e0 < 0.3 ** 5


def test_amg_preconditioned_gmres_on_scalar_system():
    s = ri.scalar_system(24, 24, 24, seed=0)
    A = oracle.Matrix.from_system(s)
    r_amg = oracle.gmres(A, oracle.PC.amg(A, gs_chunk=4), s["b"], restart=30, maxit=300,
                         rtol=1e-8)
    r_ilu = oracle.gmres(A, oracle.PC(A, "ilu0"), s["b"], restart=30, maxit=3000, rtol=1e-8)
    assert r_amg["status"] == 0 and r_ilu["status"] == 0
    assert r_amg["iters"] <= 15 and r_amg["iters"] * 5 < r_ilu["iters"]
    assert np.linalg.norm(s["b"] - oracle.spmv(A, r_amg["x"])) <= 1e-8 * np.linalg.norm(s["b"]) * (1 + 1e-9)


def test_cpr_with_amg_pressure_stage():
    # the pressure stage is one V-cycle on A_pp; FGMRES still converges
    s = ri.blackoil_system(10, 9, 8, seed=3)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(12).standard_normal(A.n)
    z_amg = oracle.PC.amg(A, "cpr_fpf", gs_chunk=4).apply(v)
    z_ilu = oracle.PC(A, "cpr_fpf").apply(v)
    assert 0 < relerr(z_amg, z_ilu) < 1e-1
    for kind in ("cpr_pf", "cpr_fp", "cpr_fpf", "cpr_ffpf"):
        r = oracle.gmres(A, oracle.PC.amg(A, kind, gs_chunk=4), s["b"], restart=30,
                         maxit=500, rtol=1e-8, flexible=True)
        assert r["status"] == 0 and r["relres"] <= 1e-8


def test_amg_rejects_bad_input():
    s = ri.blackoil_system(3, 3, 2, seed=1)
    A = oracle.Matrix.from_system(s)
    with pytest.raises(RuntimeError):
        oracle.PC.amg(A, "amg")                 # a block matrix
    with pytest.raises(RuntimeError):
        oracle.AMG(_csr(np.eye(3)), max_levels=0)
