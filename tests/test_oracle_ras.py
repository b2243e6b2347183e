"""Pins of the oracle's restricted additive Schwarz preconditioner (Section
4.1; Cai & Sarkis) with block ILU(0) subdomain solves."""
import numpy as np
import pytest

import oracle
import reservoir_inputs as ri
from tests._helpers import bsr_from_dense, dense, lu_dense_from_factor, relerr


def _ras_dense(s, starts, overlap, v):
    """RAS assembled densely: the overlapped set by breadth-first growth on
    the block graph of the dense matrix, the principal submatrix sliced from
    it, its block ILU(0) factor as dense L U, the restricted prolongation."""
    bs = s.get("bs", 1)
    D = dense(s)
    nb = D.shape[0] // bs
    adj = np.zeros((nb, nb), dtype=bool)
    for i in range(nb):
        for j in range(nb):
            adj[i, j] = np.any(D[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] != 0)
    z = np.zeros_like(v)
    for o0, o1 in zip(starts[:-1], starts[1:]):
        inset = np.zeros(nb, dtype=bool)
        inset[o0:o1] = True
        for _ in range(overlap):
            inset = inset | adj[inset].any(axis=0)
        idx = np.flatnonzero(inset)
        dofs = (idx[:, None] * bs + np.arange(bs)).reshape(-1)
        Ai = D[np.ix_(dofs, dofs)]
        sub = bsr_from_dense(Ai, bs)
        M = oracle.Matrix.from_system(sub)
        rc, lu = oracle.bilu0(M)
        assert rc == 0
        L, U = lu_dense_from_factor(M.rowptr, M.col, lu, bs)
        xl = np.linalg.solve(L @ U, v[dofs])
        own = (idx >= o0) & (idx < o1)
        z[dofs.reshape(-1, bs)[own].reshape(-1)] = xl.reshape(-1, bs)[own].reshape(-1)
    return z


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
