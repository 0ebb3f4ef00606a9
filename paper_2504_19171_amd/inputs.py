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


# The served workload: a stream of jobs whose total order n is log-uniform on
# [2,000, 200,000], half-bandwidth log-uniform on [16, 1,024] (rounded) and
# arrow width uniform on [0, 500]; the shapes come from one seeded stream and
# job k is drawn with seed base + k.
SERVE = dict(n_range=(2000, 200000), w_range=(16, 1024), a_range=(0, 500), seed=3, base=3000)


def serve_shapes(count: int, seed: int = SERVE["seed"]):
    """[(nb, w, a, seed_k)] of the first `count` jobs of the seeded served stream."""
    rng = np.random.default_rng(seed)
    lo, hi = SERVE["n_range"]
    wl, wh = SERVE["w_range"]
    out = []
    for k in range(count):
        n = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        w = int(round(np.exp(rng.uniform(np.log(wl), np.log(wh)))))
        a = int(rng.integers(SERVE["a_range"][0], SERVE["a_range"][1] + 1))
        a = min(a, n - 1)
        out.append((n - a, w, a, SERVE["base"] + k))
    return out


def arrowhead_spd_device(nb: int, w: int, a: int, seed: int, device, diag_shift: float = 1.0):
    """The same construction as arrowhead_spd, drawn on the device with a seeded
    torch generator (a different random stream from the numpy one), for
    workloads too large to draw on the host.  Returns (ab, P, C) device
    tensors in the canonical band form (P, C None when a == 0)."""
    import torch
    nb, w, a = int(nb), int(w), int(a)
    we = min(w, max(nb - 1, 0))
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    ab = torch.zeros((we + 1, nb), dtype=f64, device=device)
    rowsum = torch.zeros(nb, dtype=f64, device=device)
    if we:
        ab[1:] = torch.randn((we, nb), generator=g, dtype=f64, device=device)
        col = torch.arange(nb, device=device)
        d = torch.arange(1, we + 1, device=device)[:, None]
        ab[1:].masked_fill_(col[None, :] >= nb - d, 0.0)    # A[j+d, j] exists for j < nb - d
        av = ab[1:].abs()
        rowsum += av.sum(0)                                # row j, entries (j, j+d)
        for dd in range(1, we + 1):                         # row j+d, entries (j+d, j)
            rowsum[dd:] += av[dd - 1, : nb - dd]
    P = C = None
    if a:
        P = torch.randn((a, nb), generator=g, dtype=f64, device=device)
        Z = torch.randn((a, a), generator=g, dtype=f64, device=device)
        Lo = torch.tril(Z, -1)
        C = Lo + Lo.T
        rowsum += P.abs().sum(0)
        C.diagonal().copy_(P.abs().sum(1) + C.abs().sum(1) + diag_shift)
    if nb:
        ab[0] = rowsum + diag_shift
    return ab, P, C
