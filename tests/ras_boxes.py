"""Box partitions of an nx x ny x nz grid in natural order for the RAS
tests: box (a, b, c) owns the cells with i in [a nx/px, (a+1) nx/px) (and
likewise in j, k); its overlapped set is the box grown by `overlap` cells in
every direction (edges and corners included), clipped to the grid.  Index
arithmetic only."""
import numpy as np


def _ranges(n, p):
    return [(q * n // p, (q + 1) * n // p) for q in range(p)]


def box_partition(grid, parts, overlap):
    nx, ny, nz = grid
    px, py, pz = parts
    part = np.empty(nx * ny * nz, dtype=np.int32)
    sets = []
    s = 0
    for c, (k0, k1) in enumerate(_ranges(nz, pz)):
        for b, (j0, j1) in enumerate(_ranges(ny, py)):
            for a, (i0, i1) in enumerate(_ranges(nx, px)):
                ii, jj, kk = np.meshgrid(np.arange(i0, i1), np.arange(j0, j1), np.arange(k0, k1),
                                         indexing="ij")
                part[(kk * ny + jj) * nx + ii] = s
                gi = np.arange(max(0, i0 - overlap), min(nx, i1 + overlap))
                gj = np.arange(max(0, j0 - overlap), min(ny, j1 + overlap))
                gk = np.arange(max(0, k0 - overlap), min(nz, k1 + overlap))
                kk, jj, ii = np.meshgrid(gk, gj, gi, indexing="ij")
                sets.append(np.sort(((kk * ny + jj) * nx + ii).reshape(-1)).astype(np.int32))
                s += 1
    return part, sets
