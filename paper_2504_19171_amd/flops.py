"""Operation counts of the hot path (host logic, no device code).

Flop convention (algorithmic, tile level, true arrow width a; every output
entry counted once, symmetric outputs by their lower half):
    POTRF, TRTRI, LAUUM on a b x b tile   b^3 / 3
    TRSM, TRMM of an m x b panel           m b^2
    SYRK of a b x b tile                   b^3
    GEMM m x n x k                         2 m n k
    diagonal update of Phase 2 (m x b)     m b^2
For tile column J with s = min(B, N-1-J) band tiles below the diagonal the
panel height is m = s b + a; the factor then costs b^3/3 + m b^2 + m^2 b and
the selected inversion exactly twice that (b^3/3 + m b^2 + b^3/3 for Phase 1,
2 m^2 b + m b^2 for Phase 2); the a x a corner adds a^3/3 and 2 a^3/3.

The tile-GEMM count of Phase 2 (Sec. III-E, Table I, App. A) is
sum_J (|S(J)| + |S(J)|^2), S(J) being the non-zero tiles below tile J.
"""
from __future__ import annotations


def _halfband(nb: int, w: int, b: int) -> tuple[int, int]:
    N = -(-nb // b)
    w = min(w, max(nb - 1, 0))
    B = min(-(-w // b), N - 1) if N else 0
    return N, max(B, 0)


def factor_flops(nb: int, w: int, a: int, b: int) -> float:
    N, B = _halfband(nb, w, b)
    tot = 0.0
    for J in range(N):
        s = min(B, N - 1 - J)
        m = s * b + a
        tot += b ** 3 / 3 + m * b * b + m * m * b
    return tot + a ** 3 / 3


def selinv_flops(nb: int, w: int, a: int, b: int) -> float:
    N, B = _halfband(nb, w, b)
    tot = 0.0
    for J in range(N):
        s = min(B, N - 1 - J)
        m = s * b + a
        tot += b ** 3 / 3 + m * b * b + b ** 3 / 3      # Phase 1: TRTRI, TRMM, LAUUM
        tot += 2 * m * m * b + m * b * b                # Phase 2: GEMMs, diagonal
    return tot + 2 * a ** 3 / 3


def phase2_kernel_flops(nb: int, w: int, a: int, b: int) -> float:
    """Flops of Phase 2 alone (off-diagonal GEMMs + diagonal updates)."""
    N, B = _halfband(nb, w, b)
    tot = 0.0
    for J in range(N):
        s = min(B, N - 1 - J)
        m = s * b + a
        tot += 2 * m * m * b + m * b * b
    return tot


def phase2_tile_gemms(N: int, B: int, arrow_tiles: int = 0) -> int:
    """Number of tile GEMMs of Phase 2: sum_J |S(J)| + |S(J)|^2.

    S(J) holds the band tiles J+1..min(J+B, N-1) and the arrow tiles.
    """
    tot = 0
    for J in range(N):
        s = min(B, N - 1 - J) + arrow_tiles
        tot += s + s * s
    return tot


def appendix_a_gemms(N: int, B: int) -> int:
    """App. A closed form (first, unexpanded form), B counting every tile of the band."""
    return (N - B) * B + B * (B - 1) // 2 + B * B * (N - B - 1) + B * (B + 1) * (2 * B + 1) // 6
