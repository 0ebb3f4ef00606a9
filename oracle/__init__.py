"""Oracle: plain CPU FP64 reference of the selected-inversion hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does, and
this package imports nothing from the product (it takes plain numpy arrays).

Functions (element level, see ``stiles_oracle.c`` for the storage and the
passages of the paper each one follows):

* :func:`cholesky`     -- A = L L^T and log det A = 2 sum log L_jj.
* :func:`selinv`       -- Sigma = A^{-1} on the tile pattern of L (Sec. III-A/B).
* :func:`sigma_column` -- one column of A^{-1} by two triangular solves.

The input is the canonical band form produced by the input generator:
``ab`` of shape (w+1, nb) with ab[d, j] = A[j+d, j]; ``P`` of shape (a, nb)
with P[r, j] = A[nb+r, j]; ``C`` of shape (a, a), lower triangle read.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    lib.oracle_cholesky.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_cholesky.restype = ctypes.c_int
    lib.oracle_selinv.argtypes = [_i64, _i64, _i64, _i64, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_selinv.restype = ctypes.c_int
    lib.oracle_sigma_band_rows.argtypes = [_i64, _i64, _i64, _i64]
    lib.oracle_sigma_band_rows.restype = _i64
    lib.oracle_sigma_column.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, _i64, _dp]
    lib.oracle_sigma_column.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(x: np.ndarray):
    assert x.dtype == np.float64 and x.flags.c_contiguous
    return x.ctypes.data_as(_dp)


def _dummy():
    return np.zeros(1, dtype=np.float64)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


@dataclass
class Factor:
    """Oracle Cholesky factor in its own element storage.

    Lr[i, t] = L[i, i-w+t] (t = w is the diagonal), LP[r, k] = L[nb+r, k],
    LC[r, c] = L[nb+r, nb+c] (lower).  ``w`` is the clamped half-bandwidth.
    """
    nb: int
    w: int
    a: int
    Lr: np.ndarray
    LP: np.ndarray
    LC: np.ndarray
    logdet: float
    info: int

    def diag(self) -> np.ndarray:
        d = [self.Lr[:, self.w]] if self.nb else []
        if self.a:
            d.append(np.diag(self.LC))
        return np.concatenate(d) if d else np.zeros(0)


def clamp_w(nb: int, w: int) -> int:
    return max(0, min(int(w), max(int(nb) - 1, 0)))


def cholesky(ab: np.ndarray, P: np.ndarray, C: np.ndarray) -> Factor:
    """Cholesky factor and log det of the band-plus-arrowhead matrix."""
    lib = _load()
    nb = ab.shape[1]
    a = P.shape[0] if P is not None else 0
    w = clamp_w(nb, ab.shape[0] - 1)
    abc = np.ascontiguousarray(ab[: w + 1], dtype=np.float64)
    Pc = np.ascontiguousarray(P, dtype=np.float64) if a else _dummy()
    Cc = np.ascontiguousarray(C, dtype=np.float64) if a else _dummy()
    Lr = np.zeros((nb, w + 1), dtype=np.float64)
    LP = np.zeros((a, nb), dtype=np.float64) if a else _dummy()
    LC = np.zeros((a, a), dtype=np.float64) if a else _dummy()
    ld = ctypes.c_double(0.0)
    info = lib.oracle_cholesky(nb, w, a, _ptr(abc), _ptr(Pc), _ptr(Cc), _ptr(Lr), _ptr(LP),
                               _ptr(LC), ctypes.byref(ld))
    if info < 0:
        raise ValueError(f"oracle_cholesky: bad argument ({info})")
    if not a:
        LP = np.zeros((0, nb))
        LC = np.zeros((0, 0))
    return Factor(nb, w, a, Lr, LP, LC, float(ld.value), int(info))


@dataclass
class Selinv:
    """Selected inverse in the oracle's element storage.

    Sb[d, j] = Sigma[j+d, j] for selected rows (0 elsewhere), d = 0..Wp;
    SP[r, j] = Sigma[nb+r, j]; SC = corner block, full symmetric.
    """
    Sb: np.ndarray
    SP: np.ndarray
    SC: np.ndarray
    tile: int
    bt: int


def tile_halfband(nb: int, w: int, b: int) -> int:
    nt = -(-nb // b) if nb else 0
    bt = -(-clamp_w(nb, w) // b)
    return max(0, min(bt, nt - 1)) if nt else 0


def selinv(f: Factor, b: int) -> Selinv:
    """Sigma = A^{-1} on the tile pattern of L for tile size b."""
    lib = _load()
    if f.info != 0:
        raise ValueError("selinv needs a successful factorization")
    nb, w, a = f.nb, f.w, f.a
    rows = int(lib.oracle_sigma_band_rows(nb, w, a, b))
    Sb = np.zeros((rows, nb), dtype=np.float64)
    SP = np.zeros((a, nb), dtype=np.float64) if a else _dummy()
    SC = np.zeros((a, a), dtype=np.float64) if a else _dummy()
    LP = f.LP if a else _dummy()
    LC = f.LC if a else _dummy()
    Lr = f.Lr if nb else _dummy()
    Sbp = Sb if nb else _dummy()
    rc = lib.oracle_selinv(nb, w, a, b, _ptr(Lr), _ptr(LP), _ptr(LC), _ptr(Sbp), _ptr(SP), _ptr(SC))
    if rc != 0:
        raise RuntimeError(f"oracle_selinv failed ({rc})")
    if not a:
        SP = np.zeros((0, nb))
        SC = np.zeros((0, 0))
    return Selinv(Sb, SP, SC, b, tile_halfband(nb, w, b))


def sigma_column(f: Factor, j: int) -> np.ndarray:
    """Column j of A^{-1} (length n = nb + a) by L y = e_j, L^T x = y."""
    lib = _load()
    n = f.nb + f.a
    x = np.zeros(n, dtype=np.float64)
    LP = f.LP if f.a else _dummy()
    LC = f.LC if f.a else _dummy()
    Lr = f.Lr if f.nb else _dummy()
    rc = lib.oracle_sigma_column(f.nb, f.w, f.a, _ptr(Lr), _ptr(LP), _ptr(LC), int(j), _ptr(x))
    if rc != 0:
        raise RuntimeError(f"oracle_sigma_column failed ({rc})")
    return x


def selected_rows_last(nb: int, w: int, b: int, j: int) -> int:
    """Last selected band row of band column j (the tile pattern of L)."""
    bt = tile_halfband(nb, w, b)
    return min(nb - 1, (j // b + bt + 1) * b - 1)
