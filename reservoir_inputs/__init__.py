"""Seeded synthetic reservoir-shaped linear systems.

This module builds the inputs that both the FP64 CPU oracle and the GPU path
consume: a 7-point finite-volume operator on an nx x ny x nz grid (scalar CSR,
or 3x3-block BSR shaped like a black-oil Jacobian), a manufactured solution
x_true and the right-hand side b = A x_true.  It holds none of the solver's
arithmetic: no SpMV, no factorization, no Krylov step.  b is formed from the
face fluxes directly (acc_i x_i + sum over faces of T_f M_f (x_i - x_j)),
which is how the operator is defined, not by a row-wise matrix-vector product.

The paper's reservoir workloads (refined SPE10 / SPE1 models, Section 5) are
not available; these systems stand in for them with the same shape: one
pressure and two secondary unknowns per cell, a 7-point stencil from
two-point flux approximation, heterogeneous permeability.

Randomness: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed by
(seed, field id), counter = (index lo, index hi, sub-index, 0).  Normals by
Box-Muller.  Every draw is a pure function of (seed, field, index, sub), so
any subset of cells can be regenerated independently.

Cell numbering is natural lexicographic: cell = i + nx*(j + ny*k).

Bulk draws go through philox.c (the same generator in C, compiled on first
use into libphilox.so next to it, threads by OpenMP); the numpy
implementation below gives the same values bit for bit and serves when the
compiler is missing.
"""
from __future__ import annotations

import ctypes as _C
import os
import subprocess

import numpy as np

__all__ = [
    "philox4x32_10", "uniform01", "normal01",
    "perm_iid", "perm_layered", "perm_channelized",
    "scalar_system", "blackoil_system", "grid_config",
    "FIELD_LNK", "FIELD_CHANNEL", "FIELD_MOBILITY", "FIELD_ACCUM",
    "FIELD_XTRUE",
]

# ---------------------------------------------------------------------------
# Philox-4x32-10
# ---------------------------------------------------------------------------
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)

FIELD_LNK = 1        # background log-permeability normals (padded grid)
FIELD_CHANNEL = 2    # channel indicator normals (padded grid)
FIELD_MOBILITY = 3   # 3x3 mobility entries per face (sub = entry 0..8)
FIELD_ACCUM = 4      # pressure-row accumulation coupling per cell (sub 0..2)
FIELD_XTRUE = 5      # manufactured solution per unknown


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Philox-4x32 with 10 rounds on arrays of 32-bit counters.

    Returns four uint32 arrays.  Round: (hi1^c1^k0, lo1, hi0^c3^k1, lo0)
    with (hi0, lo0) = M0*c0 and (hi1, lo1) = M1*c2; the key is bumped by the
    Weyl constants between rounds.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK32
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libphilox.so")
_clib = None


def build(force: bool = True) -> str:
    """Compile philox.c into libphilox.so."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-o", tmp, os.path.join(_HERE, "philox.c")])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _clib
    if _clib is None:
        try:
            if not os.path.exists(_SO):
                build()
            L = _C.CDLL(_SO)
            P, U32, I64, U64 = _C.c_void_p, _C.c_uint32, _C.c_int64, _C.c_uint64
            L.philox_uniforms.argtypes = [U32, U32, P, U64, I64, U32, P, P]
            L.philox_words.argtypes = [U32, U32, P, I64, U32, P]
            _clib = L
        except (OSError, subprocess.CalledProcessError):
            _clib = False
    return _clib


def _uniform_pair(seed: int, field: int, idx, sub: int, both: bool):
    """The two 53-bit uniforms of each index (second one None unless both)."""
    L = _lib()
    if not L:
        w0, w1, w2, w3 = _words(seed, field, idx, sub)
        return _u53(w0, w1), (_u53(w2, w3) if both else None)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64).ravel())
    n = idx.size
    u1 = np.empty(n)
    u2 = np.empty(n) if both else None
    L.philox_uniforms(int(seed) & 0xFFFFFFFF, int(field) & 0xFFFFFFFF,
                      idx.ctypes.data_as(_C.c_void_p), 0, n, int(sub) & 0xFFFFFFFF,
                      u1.ctypes.data_as(_C.c_void_p),
                      u2.ctypes.data_as(_C.c_void_p) if both else None)
    return u1, u2


def _words(seed: int, field: int, idx, sub: int = 0):
    idx = np.asarray(idx, dtype=np.uint64)
    return philox4x32_10(idx & _MASK32, idx >> np.uint64(32),
                         np.uint64(sub), np.uint64(0), seed, field)


def _u53(a, b):
    # 53-bit uniform in the open interval (0, 1)
    a = a.astype(np.float64)
    b = b.astype(np.float64)
    hi = np.floor(a / 32.0)          # a >> 5
    lo = np.floor(b / 64.0)          # b >> 6
    return (hi * 67108864.0 + lo + 0.5) / 9007199254740992.0


def uniform01(seed: int, field: int, idx, sub: int = 0):
    shape = np.shape(idx)
    return _uniform_pair(seed, field, idx, sub, False)[0].reshape(shape)


def normal01(seed: int, field: int, idx, sub: int = 0):
    shape = np.shape(idx)
    u1, u2 = _uniform_pair(seed, field, idx, sub, True)
    return (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).reshape(shape)


# ---------------------------------------------------------------------------
# Permeability fields (natural ordering, arrays of shape (nz, ny, nx))
# ---------------------------------------------------------------------------
def perm_iid(nx, ny, nz, seed, sigma2=1.0):
    """ln k ~ N(0, sigma2) i.i.d. per cell; isotropic (kz = kx)."""
    n = nx * ny * nz
    g = normal01(seed, FIELD_LNK, np.arange(n, dtype=np.uint64))
    lnk = (np.sqrt(sigma2) * g).reshape(nz, ny, nx)
    return lnk, lnk.copy()


def _smoothed(nx, ny, nz, seed, field, wx, wy):
    """i.i.d. N(0,1) on a padded grid, separable moving average of wx cells
    in x and wy cells in y (none in z), rescaled to unit variance."""
    px, py = nx + wx - 1, ny + wy - 1
    g = normal01(seed, field, np.arange(px * py * nz, dtype=np.uint64))
    g = g.reshape(nz, py, px)
    c = np.cumsum(g, axis=2)
    c = np.concatenate([np.zeros((nz, py, 1)), c], axis=2)
    g = (c[:, :, wx:] - c[:, :, :-wx])          # (nz, py, nx)
    c = np.cumsum(g, axis=1)
    c = np.concatenate([np.zeros((nz, 1, nx)), c], axis=1)
    g = (c[:, wy:, :] - c[:, :-wy, :])          # (nz, ny, nx)
    return g / np.sqrt(wx * wy)


def perm_layered(nx, ny, nz, seed, sigma2=2.0, corr=8, kz_ratio=0.1):
    """Layered log-normal: ln kx ~ N(0, sigma2) correlated over `corr` cells
    in x and y and one cell in z; kz = kz_ratio * kx."""
    lnkx = np.sqrt(sigma2) * _smoothed(nx, ny, nz, seed, FIELD_LNK, corr, corr)
    return lnkx, lnkx + np.log(kz_ratio)


def perm_channelized(nx, ny, nz, seed, sigma2=3.0, frac=0.2, contrast=1000.0,
                     kz_ratio=0.1):
    """Layered background (sigma2, 8-cell correlation) plus channels: a
    second field smoothed over 32 cells in x and 4 in y, thresholded at its
    (1-frac) quantile; channel cells get ln(contrast) added."""
    lnkx, _ = perm_layered(nx, ny, nz, seed, sigma2=sigma2)
    ch = _smoothed(nx, ny, nz, seed, FIELD_CHANNEL, 32, 4).ravel()
    order = np.sort(ch)
    thr = order[int(np.floor((1.0 - frac) * ch.size))]
    ind = (ch > thr).reshape(nz, ny, nx)
    lnkx = lnkx + np.log(contrast) * ind
    return lnkx, lnkx + np.log(kz_ratio)


# ---------------------------------------------------------------------------
# Faces and transmissibilities
# ---------------------------------------------------------------------------
def _faces(nx, ny, nz, lnkx, lnkz):
    """Interior faces as arrays (left cell, right cell, T, face id, dir).

    T = 2 k_l k_r / (k_l + k_r) with unit cell sizes; kx for x/y faces and
    kz for z faces.  Face id = 3*left_cell + dir (dir 0=x, 1=y, 2=z)."""
    kx = np.exp(lnkx).ravel()
    kz = np.exp(lnkz).ravel()
    cell = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    out = []
    for d, (sl_l, sl_r, kk) in enumerate([
            ((slice(None), slice(None), slice(0, nx - 1)),
             (slice(None), slice(None), slice(1, nx)), kx),
            ((slice(None), slice(0, ny - 1), slice(None)),
             (slice(None), slice(1, ny), slice(None)), kx),
            ((slice(0, nz - 1), slice(None), slice(None)),
             (slice(1, nz), slice(None), slice(None)), kz)]):
        l = cell[sl_l].ravel()
        r = cell[sl_r].ravel()
        if l.size == 0:
            continue
        t = 2.0 * kk[l] * kk[r] / (kk[l] + kk[r])
        out.append((l, r, t, 3 * l + d))
    if not out:
        e = np.zeros(0, dtype=np.int64)
        return e, e, np.zeros(0), e
    l = np.concatenate([o[0] for o in out])
    r = np.concatenate([o[1] for o in out])
    t = np.concatenate([o[2] for o in out])
    fid = np.concatenate([o[3] for o in out])
    return l, r, t, fid


def _pattern(n, l, r):
    """CSR pattern of the 7-point operator: per row, columns ascending
    (neighbours below, the diagonal, neighbours above).  Returns rowptr,
    col, and for each face the positions of (l,r), (r,l) and the diagonals."""
    rows = np.concatenate([np.arange(n), l, r])
    cols = np.concatenate([np.arange(n), r, l])
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    rows_s = rows[order]
    col = cols[order].astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows_s + 1, 1)
    rowptr = np.cumsum(rowptr)
    pos = np.empty_like(order)
    pos[order] = np.arange(order.size)
    nf = l.size
    return (rowptr.astype(np.int32), col, pos[:n], pos[n:n + nf],
            pos[n + nf:])


def _x_true(seed, n):
    return 2.0 * uniform01(seed, FIELD_XTRUE, np.arange(n, dtype=np.uint64)) - 1.0


def scalar_system(nx, ny, nz, seed=0, perm="iid", sigma2=1.0, acc=1e-3):
    """Scalar 7-point finite-volume operator in CSR (FP64).

    A_ii = sum of face transmissibilities + acc (cell volume 1),
    A_ij = -T_ij.  b = A x_true with x_true ~ U(-1, 1)."""
    if perm == "iid":
        lnkx, lnkz = perm_iid(nx, ny, nz, seed, sigma2)
    elif perm == "layered":
        lnkx, lnkz = perm_layered(nx, ny, nz, seed, sigma2)
    else:
        raise ValueError(perm)
    n = nx * ny * nz
    l, r, t, _ = _faces(nx, ny, nz, lnkx, lnkz)
    rowptr, col, pdiag, plr, prl = _pattern(n, l, r)
    val = np.zeros(col.size)
    diag = np.full(n, acc)
    np.add.at(diag, l, t)
    np.add.at(diag, r, t)
    val[pdiag] = diag
    val[plr] = -t
    val[prl] = -t
    x = _x_true(seed, n)
    b = acc * x
    flux = t * (x[l] - x[r])
    np.add.at(b, l, flux)
    np.add.at(b, r, -flux)
    return dict(kind="csr", grid=(nx, ny, nz), n=n, rowptr=rowptr, col=col,
                val=val, x_true=x, b=b, lnk=lnkx.ravel().copy())


def blackoil_system(nx, ny, nz, seed=0, perm="layered", sigma2=2.0,
                    acc=1e-3, acc_lo=1e-3, acc_hi=1e-2):
    """3x3-block 7-point operator shaped like a black-oil Jacobian (BSR).

    Unknowns per cell: (p, s1, s2), interleaved.  Off-diagonal block
    A_ij = -T_f M_f with one seeded mobility matrix M_f per face, entries
    U(0.1, 1), shared by A_ij and A_ji.  Diagonal block: each scalar row's
    diagonal entry is minus the sum of that row's off-diagonal entries, plus
    the accumulation block acc*I whose pressure row (0,0), (0,1), (0,2) each
    gets += U(acc_lo, acc_hi).  The result is a row-diagonally-dominant
    Z-matrix up to the small pressure-row coupling.  (Summing whole 3x3
    blocks onto the diagonal block instead makes A strongly indefinite,
    since a positive 3x3 matrix has eigenvalues of both signs; no ILU-based
    Krylov solve converges on that operator.)"""
    if perm == "layered":
        lnkx, lnkz = perm_layered(nx, ny, nz, seed, sigma2)
    elif perm == "channelized":
        lnkx, lnkz = perm_channelized(nx, ny, nz, seed, sigma2)
    elif perm == "iid":
        lnkx, lnkz = perm_iid(nx, ny, nz, seed, sigma2)
    else:
        raise ValueError(perm)
    nb = nx * ny * nz
    l, r, t, fid = _faces(nx, ny, nz, lnkx, lnkz)
    rowptr, col, pdiag, plr, prl = _pattern(nb, l, r)
    nf = l.size
    mob = np.empty((nf, 9))
    for e in range(9):
        mob[:, e] = 0.1 + 0.9 * uniform01(seed, FIELD_MOBILITY,
                                           fid.astype(np.uint64), e)
    mob = mob.reshape(nf, 3, 3)
    tm = t[:, None, None] * mob
    val = np.zeros((col.size, 3, 3))
    diag = np.zeros((nb, 3, 3))
    diag[:, 0, 0] = acc
    diag[:, 1, 1] = acc
    diag[:, 2, 2] = acc
    cells = np.arange(nb, dtype=np.uint64)
    for c in range(3):
        diag[:, 0, c] += acc_lo + (acc_hi - acc_lo) * uniform01(
            seed, FIELD_ACCUM, cells, c)
    accb = diag.copy()
    # each scalar row's diagonal entry takes minus the sum of that row's
    # off-diagonal entries (zero row sums before accumulation)
    rs = tm.sum(axis=2)                                  # (nf, 3)
    dflux = np.zeros((nb, 3))
    np.add.at(dflux, l, rs)
    np.add.at(dflux, r, rs)
    diag[:, 0, 0] += dflux[:, 0]
    diag[:, 1, 1] += dflux[:, 1]
    diag[:, 2, 2] += dflux[:, 2]
    val[pdiag] = diag
    val[plr] = -tm
    val[prl] = -tm
    x = _x_true(seed, 3 * nb)
    xb = x.reshape(nb, 3)
    b = np.einsum("nij,nj->ni", accb, xb)
    np.add.at(b, l, rs * xb[l] - np.einsum("fij,fj->fi", tm, xb[r]))
    np.add.at(b, r, rs * xb[r] - np.einsum("fij,fj->fi", tm, xb[l]))
    return dict(kind="bsr", grid=(nx, ny, nz), nb=nb, n=3 * nb, bs=3,
                rowptr=rowptr, col=col, val=val, x_true=x, b=b.ravel(),
                lnk=lnkx.ravel().copy())


def grid_config(name: str, seed: int = 0):
    """The named reservoir-shaped workloads."""
    if name == "scalar32":
        return scalar_system(32, 32, 32, seed=seed, perm="iid", sigma2=1.0)
    if name == "blackoil64":
        return blackoil_system(64, 64, 64, seed=seed, perm="layered", sigma2=2.0)
    if name == "blackoil128x128x64":
        return blackoil_system(128, 128, 64, seed=seed, perm="layered",
                               sigma2=2.0)
    if name == "channelized256x256x128":
        return blackoil_system(256, 256, 128, seed=seed, perm="channelized",
                               sigma2=3.0)
    raise KeyError(name)
