"""Seeded synthetic inputs: symmetric positive-definite band-plus-arrowhead matrices.

This module only draws inputs; it holds none of the method's arithmetic.  Both
the HIP path (through :mod:`paper_2504_19171_amd.stiles`) and the CPU oracle
consume what it returns.

The matrices stand in for the arrowhead matrices of INLA-type models the paper
evaluates (Sec. IV, Tables II-III: a band of random effects plus a few dense
rows/columns of fixed effects).  The paper's own matrices and their generator
are not published, so the entries are drawn as follows (one
``numpy.random.default_rng(seed)`` stream, in this order):

1. for d = 1..w: ``standard_normal(nb - d)`` gives A[j+d, j] = A[j, j+d];
2. ``standard_normal((a, nb))`` gives the arrow rows A[nb+r, j] (mirrored);
3. ``standard_normal((a, a))``, strictly lower part, mirrored, gives the corner;
4. A_ii = sum_{j != i} |A_ij| + 1 (strict diagonal dominance, so A is SPD with
   lambda_min >= 1 by Gershgorin).

The result is returned in the *canonical band form*: ``ab`` (w+1, nb) with
ab[d, j] = A[j+d, j]; ``P`` (a, nb) with P[r, j] = A[nb+r, j]; ``C`` (a, a) full
symmetric.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class BandArrow:
    nb: int      # order of the band part
    w: int       # half-bandwidth of the band part (elements)
    a: int       # arrow width
    ab: np.ndarray
    P: np.ndarray
    C: np.ndarray

    @property
    def n(self) -> int:
        return self.nb + self.a

    def dense(self) -> np.ndarray:
        """Dense symmetric n x n matrix (small sizes only)."""
        n, nb = self.n, self.nb
        A = np.zeros((n, n))
        for d in range(min(self.w, max(nb - 1, 0)) + 1):
            idx = np.arange(nb - d)
            A[idx + d, idx] = self.ab[d, : nb - d]
            A[idx, idx + d] = self.ab[d, : nb - d]
        if self.a:
            A[nb:, :nb] = self.P
            A[:nb, nb:] = self.P.T
            A[nb:, nb:] = self.C
        return A


def arrowhead_spd(nb: int, w: int, a: int, seed: int, diag_shift: float = 1.0) -> BandArrow:
    """Draw one seeded SPD band-plus-arrowhead matrix (see module docstring)."""
    nb, w, a = int(nb), int(w), int(a)
    if nb < 0 or w < 0 or a < 0 or nb + a < 1:
        raise ValueError("need nb >= 0, w >= 0, a >= 0 and nb + a >= 1")
    we = min(w, max(nb - 1, 0))
    rng = np.random.default_rng(seed)
    ab = np.zeros((we + 1, nb), dtype=np.float64)
    rowsum = np.zeros(nb, dtype=np.float64)
    for d in range(1, we + 1):
        v = rng.standard_normal(nb - d)
        ab[d, : nb - d] = v
        av = np.abs(v)
        rowsum[: nb - d] += av   # row j, entry (j, j+d)
        rowsum[d:] += av         # row j+d, entry (j+d, j)
    P = rng.standard_normal((a, nb)) if a else np.zeros((0, nb))
    C = np.zeros((a, a))
    if a:
        Z = rng.standard_normal((a, a))
        Lo = np.tril(Z, -1)
        C = Lo + Lo.T
        rowsum += np.abs(P).sum(axis=0)
        csum = np.abs(P).sum(axis=1) + np.abs(C).sum(axis=1)
        C[np.arange(a), np.arange(a)] = csum + diag_shift
    if nb:
        ab[0, :] = rowsum + diag_shift
    return BandArrow(nb, w, a, ab, np.ascontiguousarray(P), np.ascontiguousarray(C))


# Configurations of the workloads (band order nb, half-bandwidth w, arrow a,
# tile size b, seed).  "small": n = 2,000 + 20, w = 32, tile 64.  "large":
# n = 100,000 + 100, w = 1,024, tile 256 (the compute-bound regime).
WORKLOADS = {
    "small": dict(nb=2000, w=32, a=20, tile=64, seed=0),
    "large": dict(nb=100000, w=1024, a=100, tile=256, seed=1),
}


# The batched workload: 64 independent matrices whose band order is uniform
# on [5,000, 50,000], half-bandwidth drawn from {32, 128, 512} and arrow
# width uniform on [10, 200]; the shapes come from one seeded stream and
# matrix k is drawn with seed base + k.
BATCH = dict(count=64, nb_range=(5000, 50000), widths=(32, 128, 512), a_range=(10, 200), seed=2, base=2000)


def batch_shapes(count: int = BATCH["count"], seed: int = BATCH["seed"], nb_range=BATCH["nb_range"],
                 widths=BATCH["widths"], a_range=BATCH["a_range"]):
    """[(nb, w, a, seed_k)] of a seeded batch of matrices (see BATCH)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nb = int(rng.integers(nb_range[0], nb_range[1] + 1))
        w = int(widths[int(rng.integers(0, len(widths)))])
        a = int(rng.integers(a_range[0], a_range[1] + 1))
        out.append((nb, w, a, BATCH["base"] + k))
    return out
