"""Seeded input generator: Philox known answers, operator structure, and
b = A x_true (checked with scipy's sparse product, independent of both the
oracle and the GPU path)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import reservoir_inputs as ri

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                rows.append([int(t, 16) for t in ln.split()])
    assert len(rows) == 3
    for r in rows:
        out = ri.philox4x32_10(*r[:6])
        assert [int(o) for o in out] == r[6:]


def test_uniform_and_normal_moments():
    u = ri.uniform01(7, 1, np.arange(200000))
    assert 0.0 < u.min() and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 3e-3
    g = ri.normal01(7, 1, np.arange(200000))
    assert abs(g.mean()) < 1e-2 and abs(g.var() - 1.0) < 1e-2


@pytest.mark.parametrize("grid", [(32, 32, 32), (5, 4, 3), (7, 1, 1)])
def test_scalar_nnz_and_b(grid):
    s = ri.scalar_system(*grid, seed=3)
    nx, ny, nz = grid
    n = nx * ny * nz
    assert s["col"].size == 7 * n - 2 * (ny * nz + nx * nz + nx * ny)
    A = sp.csr_matrix((s["val"], s["col"], s["rowptr"]), shape=(n, n))
    assert np.allclose(A @ s["x_true"], s["b"], rtol=0, atol=1e-12 * np.abs(s["b"]).max())
    # symmetric, diagonally dominant by exactly the accumulation term
    assert abs(A - A.T).max() == 0.0
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    assert np.allclose(d - off, 1e-3)
    if grid == (32, 32, 32):
        assert s["col"].size == 223232


@pytest.mark.parametrize("grid", [(4, 4, 4), (6, 5, 3)])
def test_blackoil_structure_and_b(grid):
    s = ri.blackoil_system(*grid, seed=11)
    nb = s["nb"]
    B = sp.bsr_matrix((s["val"], s["col"], s["rowptr"]), shape=(3 * nb, 3 * nb))
    assert np.allclose(B @ s["x_true"], s["b"], rtol=0, atol=1e-12 * np.abs(s["b"]).max())
    D = B.toarray()
    # block-structurally symmetric, off-diagonal blocks shared (A_ij == A_ji)
    for i in range(nb):
        for p in range(s["rowptr"][i], s["rowptr"][i + 1]):
            j = s["col"][p]
            assert np.array_equal(D[3*i:3*i+3, 3*j:3*j+3], D[3*j:3*j+3, 3*i:3*i+3]) or i == j
    # scalar row sums equal the accumulation block's row sums
    acc_rows = D.sum(axis=1).reshape(nb, 3)
    assert np.all(acc_rows[:, 1:] > 0.999e-3) and np.all(acc_rows[:, 1:] < 1.001e-3)
    assert np.all(acc_rows[:, 0] > 1e-3 + 3e-3 - 1e-12)
    # all off-block-diagonal entries negative (mobility entries in (0.1, 1))
    for i in range(nb):
        for p in range(s["rowptr"][i], s["rowptr"][i + 1]):
            if s["col"][p] != i:
                assert np.all(s["val"][p] < 0)


def test_blackoil64_counts():
    s = ri.blackoil_system(16, 16, 16, seed=0)
    assert s["col"].size == 7 * 4096 - 2 * 3 * 256
    # 64^3: 7*nb - 2*(ny*nz + nx*nz + nx*ny)
    assert 7 * 64**3 - 2 * 3 * 64 * 64 == 1810432


def test_layered_perm_statistics():
    lnkx, lnkz = ri.perm_layered(64, 64, 16, seed=1, sigma2=2.0)
    assert abs(lnkx.var() - 2.0) < 0.3
    assert np.allclose(lnkz - lnkx, np.log(0.1))
    # correlated over 8 cells in x and y, independent between layers
    a = lnkx[:, :, :-1].ravel(); b = lnkx[:, :, 1:].ravel()
    assert np.corrcoef(a, b)[0, 1] > 0.8
    a = lnkx[:-1].ravel(); b = lnkx[1:].ravel()
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.05


def test_channelized_fraction():
    lnkx, _ = ri.perm_channelized(64, 64, 8, seed=2)
    bg, _ = ri.perm_layered(64, 64, 8, seed=2, sigma2=3.0)
    ind = np.abs(lnkx - bg - np.log(1000.0)) < 1e-9
    assert abs(ind.mean() - 0.2) < 1e-3


def test_determinism_by_seed():
    a = ri.blackoil_system(4, 3, 2, seed=5)
    b = ri.blackoil_system(4, 3, 2, seed=5)
    c = ri.blackoil_system(4, 3, 2, seed=6)
    assert np.array_equal(a["val"], b["val"]) and np.array_equal(a["b"], b["b"])
    assert not np.array_equal(a["val"], c["val"])


def test_c_philox_matches_numpy_bit_for_bit():
    # the bulk draws of philox.c against the module's numpy Philox-4x32-10
    if not ri._lib():
        pytest.skip("libphilox.so could not be built")
    idx = np.random.default_rng(0).integers(0, 2 ** 40, size=50000).astype(np.uint64)
    for seed, field, sub in ((0, 1, 0), (3, 7, 5), (2 ** 31 + 5, 3, 8)):
        u1, u2 = ri._uniform_pair(seed, field, idx, sub, True)
        w = ri._words(seed, field, idx, sub)
        assert np.array_equal(u1, ri._u53(w[0], w[1]))
        assert np.array_equal(u2, ri._u53(w[2], w[3]))


def test_blockwise_transpose_is_the_operator_transpose():
    # the learned-stage training builds A^T by transposing every block in
    # place; that is A^T because the generator shares A_ij and A_ji
    s = ri.blackoil_system(5, 4, 3, seed=17)
    nb = s["nb"]
    B = sp.bsr_matrix((s["val"], s["col"], s["rowptr"]), shape=(3 * nb, 3 * nb))
    T = sp.bsr_matrix((np.asarray(s["val"]).transpose(0, 2, 1), s["col"], s["rowptr"]),
                      shape=(3 * nb, 3 * nb))
    assert abs(B.T.toarray() - T.toarray()).max() == 0.0
