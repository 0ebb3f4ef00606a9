"""Operation-count pins: Table I / App. A of the paper and the flop convention."""
import json
import os

import pytest

from paper_2504_19171_amd import flops

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_gemm_counts.json")


def test_table1_gemm_counts():
    g = json.load(open(GOLD))
    N = g["N"]
    for row in g["rows"]:
        B = row["B"]
        # B tiles of band (a full matrix has B >= N-1)
        assert flops.phase2_tile_gemms(N, min(B, N - 1)) == row["gemm_ops"]
        # the same count with the last tile read as the arrow tile
        if B < N:
            assert flops.phase2_tile_gemms(N - 1, B - 1, arrow_tiles=1) == row["gemm_ops"]
        assert flops.appendix_a_gemms(N, B) == row["gemm_ops"]


@pytest.mark.parametrize("N", [3, 6, 10, 57])
@pytest.mark.parametrize("B", [1, 2, 3, 5])
def test_appendix_a_matches_enumeration(N, B):
    if B >= N:
        pytest.skip("band wider than the matrix")
    assert flops.appendix_a_gemms(N, B) == flops.phase2_tile_gemms(N, B)
    # expanded form with the constant term 2B^3/3 + B^2 + B/3
    expanded = (B * B + B) * N - (2 * B ** 3 + 3 * B * B + B) / 3
    assert flops.appendix_a_gemms(N, B) == pytest.approx(expanded)


@pytest.mark.parametrize("nb,w,a,b", [(2000, 32, 20, 64), (100000, 1024, 100, 256), (777, 100, 33, 128),
                                      (500, 499, 0, 64), (100, 0, 0, 64)])
def test_selinv_is_twice_factor(nb, w, a, b):
    assert flops.selinv_flops(nb, w, a, b) == pytest.approx(2 * flops.factor_flops(nb, w, a, b), rel=1e-15)


def test_workload_totals():
    small = flops.factor_flops(2000, 32, 20, 64) + flops.selinv_flops(2000, 32, 20, 64)
    large = flops.factor_flops(100000, 1024, 100, 256) + flops.selinv_flops(100000, 1024, 100, 256)
    assert small == pytest.approx(8.271e7, rel=1e-3)
    assert large == pytest.approx(4.689e11, rel=1e-3)
