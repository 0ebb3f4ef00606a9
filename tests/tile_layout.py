"""Host-side index maps of the tile layout, for the tests (numpy; no arithmetic
of the method).  Test infrastructure: the product library never uses it.

The tile layout is described in ``include/stiles.h``.  These helpers move
entries between it and the canonical band form used by the input generator:

* :func:`host_pack` -- canonical band form -> tile buffer (same bytes as the
  device ``stiles_pack``);
* :func:`band_part`, :func:`arrow_part`, :func:`corner_part` -- read a tile
  buffer back as band diagonals D[d, j] = X[j+d, j], arrow rows and corner.
"""
from __future__ import annotations

import numpy as np


def _regions(T: np.ndarray, lay):
    b, B, N, ap = lay.tile, lay.bt, lay.nt, lay.arrow_ld
    band = T[lay.off_band: lay.off_arrow].reshape(N, B + 1, b, b)          # [J, d, col, row]
    arrow = T[lay.off_arrow: lay.off_corner].reshape(N, b, ap) if ap else None  # [J, col, row]
    corner = T[lay.off_corner: lay.total_doubles].reshape(ap, ap) if ap else None  # [col, row]
    return band, arrow, corner


def host_pack(ab: np.ndarray, P: np.ndarray, C: np.ndarray, lay) -> np.ndarray:
    """Tile buffer of the matrix given in canonical band form (numpy)."""
    T = np.zeros(lay.total_doubles, dtype=np.float64)
    band, arrow, corner = _regions(T, lay)
    b, N, nb, w, a = lay.tile, lay.nt, lay.nb, lay.w, lay.arrow
    r = np.arange(b)[None, :]   # row in tile
    c = np.arange(b)[:, None]   # col in tile
    for J in range(N):
        for d in range(lay.bt + 1):
            if J + d >= N:
                continue
            i = (J + d) * b + r
            j = J * b + c
            hi, lo = np.maximum(i, j), np.minimum(i, j)
            inside = (i < nb) & (j < nb) & (hi - lo <= w)
            vals = np.zeros((b, b))
            vals[inside] = ab[(hi - lo)[inside], lo[inside]]
            vals[(i == j) & (i >= nb)] = 1.0
            band[J, d] = vals
    if a:
        ap = lay.arrow_ld
        for J in range(N):
            j0, j1 = J * b, min(nb, (J + 1) * b)
            arrow[J, : j1 - j0, :a] = P[:, j0:j1].T
        corner[:a, :a] = C.T
        for k in range(a, ap):
            corner[k, k] = 1.0
    return T


def band_part(T: np.ndarray, lay, maxd: int) -> np.ndarray:
    """D[d, j] = X[j+d, j] for 0 <= d <= maxd, j < nb, read from the band tiles.

    Entries outside the stored tiles (or below row nb) are 0.
    """
    band, _, _ = _regions(T, lay)
    b, N, nb = lay.tile, lay.nt, lay.nb
    D = np.zeros((maxd + 1, nb), dtype=np.float64)
    rr, cc = np.meshgrid(np.arange(b), np.arange(b), indexing="ij")  # rr row, cc col
    for d in range(lay.bt + 1):
        diff = d * b + rr - cc
        for J in range(N - d):
            i = (J + d) * b + rr
            j = J * b + cc
            keep = (diff >= 0) & (diff <= maxd) & (i < nb) & (j < nb)
            D[diff[keep], j[keep]] = band[J, d][cc[keep], rr[keep]]
    return D


def arrow_part(T: np.ndarray, lay) -> np.ndarray:
    """P[r, j] = X[nb+r, j], shape (arrow, nb)."""
    _, arrow, _ = _regions(T, lay)
    a, nb, b = lay.arrow, lay.nb, lay.tile
    if not a:
        return np.zeros((0, nb))
    full = np.transpose(arrow, (2, 0, 1)).reshape(lay.arrow_ld, lay.nt * b)  # [row, J*b+col]
    return np.ascontiguousarray(full[:a, :nb])


def corner_part(T: np.ndarray, lay) -> np.ndarray:
    """The a x a corner block X[nb:, nb:] as stored (row, col)."""
    _, _, corner = _regions(T, lay)
    a = lay.arrow
    if not a:
        return np.zeros((0, 0))
    return np.ascontiguousarray(corner.T[:a, :a])


def band_tile(T: np.ndarray, lay, J: int, d: int) -> np.ndarray:
    """Band tile (J+d, J) as a (row, col) array."""
    band, _, _ = _regions(T, lay)
    return band[J, d].T


def lower_column(T: np.ndarray, lay, j: int):
    """Rows i >= j of column j that the tile pattern stores, and their values.

    For a band column j (tile J = j // b): band tiles (J..J+B, J) below row j
    and inside the matrix, then the arrow rows; for a corner column: the
    corner rows i >= j.
    """
    b, nb, a = lay.tile, lay.nb, lay.arrow
    band, arrow, corner = _regions(T, lay)
    if j < nb:
        J, c = divmod(j, b)
        rows, vals = [], []
        for d in range(lay.bt + 1):
            if J + d >= lay.nt:
                break
            i0 = (J + d) * b
            col = band[J, d][c]               # rows of tile J+d, column c
            ii = i0 + np.arange(b)
            keep = (ii >= j) & (ii < nb)
            rows.append(ii[keep]); vals.append(col[keep])
        if a:
            rows.append(nb + np.arange(a)); vals.append(arrow[J, c, :a])
        return np.concatenate(rows), np.concatenate(vals)
    c = j - nb
    ii = nb + np.arange(c, a)
    return ii, corner[c, c:a].copy()
