"""Test-side helpers: dense views of generated systems and small
hand-made matrices.  Nothing here implements the solver."""
import numpy as np


def dense_from_bsr(rowptr, col, val, bs):
    nb = len(rowptr) - 1
    val = np.asarray(val, dtype=np.float64).reshape(-1, bs, bs)
    D = np.zeros((nb * bs, nb * bs))
    for i in range(nb):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = col[p]
            D[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] = val[p]
    return D


def dense(s):
    return dense_from_bsr(s["rowptr"], s["col"], s["val"], s.get("bs", 1))


def bsr_from_dense(D, bs=1):
    """Block-CSR of a dense matrix keeping every block that has a nonzero
    (and every diagonal block)."""
    nb = D.shape[0] // bs
    rowptr = [0]
    col, val = [], []
    for i in range(nb):
        for j in range(nb):
            blk = D[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs]
            if i == j or np.any(blk != 0):
                col.append(j)
                val.append(blk.copy())
        rowptr.append(len(col))
    return dict(rowptr=np.array(rowptr, dtype=np.int32),
                col=np.array(col, dtype=np.int32),
                val=np.array(val).reshape(-1), bs=bs, nb=nb, n=nb * bs)


def lu_dense_from_factor(rowptr, col, lu, bs):
    """Unit-lower L and upper U (dense) from a combined block factor."""
    nb = len(rowptr) - 1
    n = nb * bs
    lu = np.asarray(lu).reshape(-1, bs, bs)
    L = np.eye(n)
    U = np.zeros((n, n))
    for i in range(nb):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = col[p]
            if j < i:
                L[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] = lu[p]
            else:
                U[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] = lu[p]
    return L, U


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
