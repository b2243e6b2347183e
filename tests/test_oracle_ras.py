"""Pins of the oracle's restricted additive Schwarz preconditioner (Section
4.1; Cai & Sarkis) with block ILU(0) subdomain solves."""
import numpy as np
import pytest

import oracle
import reservoir_inputs as ri
from tests._helpers import bsr_from_dense, dense, lu_dense_from_factor, relerr
from tests.ras_boxes import box_partition


def _ras_dense_sets(s, part, sets, v):
    """RAS assembled densely from explicit subdomain sets: the principal
    submatrix sliced from the dense matrix, its block ILU(0) factor as dense
    L U, the restricted prolongation onto the rows with part == s."""
    bs = s.get("bs", 1)
    D = dense(s)
    part = np.asarray(part)
    z = np.zeros_like(v)
    for sid, idx in enumerate(sets):
        idx = np.sort(np.asarray(idx))
        dofs = (idx[:, None] * bs + np.arange(bs)).reshape(-1)
        Ai = D[np.ix_(dofs, dofs)]
        sub = bsr_from_dense(Ai, bs)
        M = oracle.Matrix.from_system(sub)
        rc, lu = oracle.bilu0(M)
        assert rc == 0
        L, U = lu_dense_from_factor(M.rowptr, M.col, lu, bs)
        xl = np.linalg.solve(L @ U, v[dofs])
        own = part[idx] == sid
        z[dofs.reshape(-1, bs)[own].reshape(-1)] = xl.reshape(-1, bs)[own].reshape(-1)
    return z


def _ras_dense(s, starts, overlap, v):
    """RAS with the overlapped sets grown breadth-first on the block graph of
    the dense matrix from contiguous owned ranges."""
    bs = s.get("bs", 1)
    D = dense(s)
    nb = D.shape[0] // bs
    adj = np.zeros((nb, nb), dtype=bool)
    for i in range(nb):
        for j in range(nb):
            adj[i, j] = np.any(D[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] != 0)
    part = np.empty(nb, dtype=np.int32)
    sets = []
    for sid, (o0, o1) in enumerate(zip(starts[:-1], starts[1:])):
        part[o0:o1] = sid
        inset = np.zeros(nb, dtype=bool)
        inset[o0:o1] = True
        for _ in range(overlap):
            inset = inset | adj[inset].any(axis=0)
        sets.append(np.flatnonzero(inset))
    return _ras_dense_sets(s, part, sets, v)


def test_ras_one_subdomain_is_global_bilu0():
    s = ri.blackoil_system(6, 5, 4, seed=1)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(1).standard_normal(A.n)
    ref = oracle.PC(A, "bilu0").apply(v)
    for ov in (0, 1, 3):
        assert relerr(oracle.PC.ras(A, [0, A.nb], ov).apply(v), ref) == 0.0


@pytest.mark.parametrize("overlap", [0, 1, 2])
@pytest.mark.parametrize("starts", [[0, 12, 24, 36], [0, 5, 23, 36]])
def test_ras_matches_dense_restricted_schwarz(starts, overlap):
    # 4 x 3 x 3 black-oil grid: layer-aligned and ragged owned ranges
    s = ri.blackoil_system(4, 3, 3, seed=2)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(3).standard_normal(A.n)
    got = oracle.PC.ras(A, starts, overlap).apply(v)
    assert relerr(got, _ras_dense(s, starts, overlap, v)) < 1e-12


def test_ras_scalar_pattern():
    s = ri.scalar_system(5, 4, 3, seed=3)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(4).standard_normal(A.n)
    starts = [0, 20, 40, 60]
    assert relerr(oracle.PC.ras(A, starts, 1).apply(v), _ras_dense(s, starts, 1, v)) < 1e-12


def test_ras_exact_for_decoupled_subdomains():
    # no coupling between the owned ranges: every local solve is exact
    # (tridiagonal blocks, ILU(0) = LU), so RAS is A^-1 for any overlap
    rng = np.random.default_rng(5)
    n = 12
    D = np.zeros((n, n))
    for lo, hi in ((0, 5), (5, 12)):
        for i in range(lo, hi):
            D[i, i] = 4.0 + rng.random()
            if i + 1 < hi:
                D[i, i + 1] = -1.0 - rng.random()
                D[i + 1, i] = -1.0 - rng.random()
    st = bsr_from_dense(D, 1)
    A = oracle.Matrix.from_system(st)
    v = rng.standard_normal(n)
    for ov in (0, 1, 2):
        assert relerr(oracle.PC.ras(A, [0, 5, 12], ov).apply(v), np.linalg.solve(D, v)) < 1e-13


def test_ras_rejects_bad_partitions():
    s = ri.blackoil_system(3, 3, 2, seed=1)
    A = oracle.Matrix.from_system(s)
    for bad in ([0, 10], [1, 18], [0, 9, 9, 18], [0, 12, 6, 18]):
        with pytest.raises(RuntimeError):
            oracle.PC.ras(A, bad, 1)


def test_fgmres_with_ras_converges():
    s = ri.blackoil_system(8, 8, 8, seed=1)
    A = oracle.Matrix.from_system(s)
    for nsub in (1, 2, 4):
        starts = [k * 8 // nsub * 64 for k in range(nsub + 1)]
        r = oracle.gmres(A, oracle.PC.ras(A, starts, 1), s["b"], restart=30, maxit=2000,
                         rtol=1e-8, flexible=True)
        assert r["status"] == 0 and r["relres"] <= 1e-8


# ---- explicit subdomain sets: boxes of the grid grown in every direction ----
@pytest.mark.parametrize("parts,overlap", [((2, 2, 1), 1), ((2, 2, 2), 0), ((2, 2, 2), 1),
                                           ((3, 1, 2), 2)])
def test_ras_sets_match_dense_on_boxes(parts, overlap):
    grid = (5, 4, 3)
    s = ri.blackoil_system(*grid, seed=14)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(15).standard_normal(A.n)
    part, sets = box_partition(grid, parts, overlap)
    got = oracle.PC.ras_sets(A, part, sets).apply(v)
    assert relerr(got, _ras_dense_sets(s, part, sets, v)) < 1e-12


@pytest.mark.parametrize("overlap", [0, 1, 2])
def test_ras_boxes_on_slabs_are_graph_overlap(overlap):
    # for z-slabs, growing the box by d cells is d rounds of graph neighbours
    grid = (4, 3, 7)
    s = ri.blackoil_system(*grid, seed=16)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(17).standard_normal(A.n)
    part, sets = box_partition(grid, (1, 1, 3), overlap)
    starts = [q * 7 // 3 * 12 for q in range(4)]
    ref = oracle.PC.ras(A, starts, overlap).apply(v)
    assert np.array_equal(oracle.PC.ras_sets(A, part, sets).apply(v), ref)
    assert np.array_equal(oracle.PC.ras_part(A, part, overlap).apply(v), ref)


def test_ras_sets_exact_for_lower_triangular_stencil():
    # only the -x, -y, -z couplings: ILU(0) of every principal submatrix is
    # its exact LU, so each subdomain solve is a dense solve
    grid = (4, 4, 3)
    nx, ny, nz = grid
    n = nx * ny * nz
    rng = np.random.default_rng(18)
    D = np.zeros((n, n))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = (k * ny + j) * nx + i
                D[r, r] = 2.0 + rng.random()
                for d, ok in ((1, i > 0), (nx, j > 0), (nx * ny, k > 0)):
                    if ok:
                        D[r, r - d] = -0.5 - rng.random()
    st = bsr_from_dense(D, 1)
    A = oracle.Matrix.from_system(st)
    v = rng.standard_normal(n)
    part, sets = box_partition(grid, (2, 2, 1), 1)
    z = np.zeros(n)
    for sid, idx in enumerate(sets):
        xl = np.linalg.solve(D[np.ix_(idx, idx)], v[idx])
        own = part[idx] == sid
        z[idx[own]] = xl[own]
    assert relerr(oracle.PC.ras_sets(A, part, sets).apply(v), z) < 1e-13
    # and the overlap matters: a grown box's local solve sees more of v
    part0, sets0 = box_partition(grid, (2, 2, 1), 0)
    assert relerr(oracle.PC.ras_sets(A, part0, sets0).apply(v), z) > 1e-6


def test_ras_sets_rejects_bad_sets():
    grid = (3, 3, 2)
    s = ri.blackoil_system(*grid, seed=1)
    A = oracle.Matrix.from_system(s)
    part, sets = box_partition(grid, (1, 1, 2), 1)
    missing = [sets[0], sets[1][:-1]]          # a set without one of its owned rows
    outside = [sets[0], np.append(sets[1], 18)]
    for bad in (missing, outside):
        with pytest.raises(RuntimeError):
            oracle.PC.ras_sets(A, part, bad)
    bad_part = part.copy()
    bad_part[0] = 2
    with pytest.raises(RuntimeError):
        oracle.PC.ras_sets(A, bad_part, sets)


# ---- RAS as CPR's full-system stage R(A)^-1 (Algorithms 5-8) -----------------
@pytest.mark.parametrize("kind", ["cpr_pf", "cpr_fp", "cpr_fpf", "cpr_ffpf"])
def test_cpr_with_one_ras_subdomain_is_block_ilu_cpr(kind):
    # one subdomain is the whole matrix: its local block ILU(0) solve is the
    # global one, so the CPR operator is unchanged, bit for bit
    s = ri.blackoil_system(6, 5, 4, seed=21)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(22).standard_normal(A.n)
    one = oracle.PC.ras(A, [0, A.nb], 1)
    assert np.array_equal(oracle.PC.cpr(A, kind, full=one).apply(v), oracle.PC(A, kind).apply(v))
    one = oracle.PC.ras(A, [0, A.nb], 1)
    assert np.array_equal(oracle.PC.cpr(A, kind, amg={"gs_chunk": 4}, full=one).apply(v),
                          oracle.PC.amg(A, kind, gs_chunk=4).apply(v))


def test_cpr_with_ras_full_stage_converges():
    s = ri.blackoil_system(12, 10, 8, seed=23)
    A = oracle.Matrix.from_system(s)
    v = np.random.default_rng(24).standard_normal(A.n)
    part, sets = box_partition((12, 10, 8), (1, 2, 2), 1)
    z_ras = oracle.PC.cpr(A, "cpr_fpf", full=oracle.PC.ras_sets(A, part, sets)).apply(v)
    z_ilu = oracle.PC(A, "cpr_fpf").apply(v)
    assert 1e-8 < relerr(z_ras, z_ilu) < 0.5
    for amg in (None, {"gs_chunk": 4}):
        pc = oracle.PC.cpr(A, "cpr_fpf", amg=amg, full=oracle.PC.ras_sets(A, part, sets))
        r = oracle.gmres(A, pc, s["b"], restart=30, maxit=500, rtol=1e-8, flexible=True)
        assert r["status"] == 0 and r["relres"] <= 1e-8
