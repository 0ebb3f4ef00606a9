"""Selection: the selected inverse restricted to the closure of a selection
(stiles_selinv_range) equals the whole one on every tile it computes, bit for
bit; selected entries read with stiles_gather match the oracle; pairs outside
L's tile pattern go through the full inverse."""
import numpy as np
import pytest

from paper_2504_19171_amd import inputs
import tile_layout as lo

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case(oracle_mod):
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from gpu_util import to_device
    from paper_2504_19171_amd import stiles as st
    st.load()
    nb, w, a, b = 1000, 100, 20, 64
    M = inputs.arrowhead_spd(nb, w, a, seed=21)
    lay = st.layout(M.n, w, a, b)
    L, _, info = st.factor(st.pack(*to_device(M, "cuda:0"), lay), lay)
    S, sinfo = st.selinv(L, lay)
    torch.cuda.synchronize()
    assert int(info.item()) == 0 and int(sinfo.item()) == 0
    return dict(M=M, lay=lay, L=L, S=S.cpu().numpy(), f=oracle_mod.cholesky(M.ab, M.P, M.C))


@pytest.mark.parametrize("first", [0, 1, 7, 15, 16])
def test_range_equals_whole_on_its_tiles(case, first):
    import torch
    from paper_2504_19171_amd import stiles as st
    lay = case["lay"]
    Sr, info = st.selinv_range(case["L"], lay, first)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Sr = Sr.cpu().numpy()
    for J in range(first, lay.nt):
        for d in range(min(lay.bt, lay.nt - 1 - J) + 1):
            assert np.array_equal(lo.band_tile(Sr, lay, J, d), lo.band_tile(case["S"], lay, J, d)), (J, d)
    A0 = lay.off_arrow + first * lay.arrow_ld * lay.tile
    assert np.array_equal(Sr[A0:], case["S"][A0:])     # arrow tiles from `first` on, and the corner


def test_select_in_pattern_matches_whole_and_oracle(case, oracle_mod):
    import torch
    from paper_2504_19171_amd import stiles as st
    lay, f = case["lay"], case["f"]
    pairs = [(500, 400), (400, 500), (1005, 300), (1010, 1003), (999, 999), (700, 650), (640, 512)]
    vals, info = st.select(case["L"], lay, pairs)
    vals = vals.cpu().numpy()
    assert int(info.item()) == 0
    ij = torch.tensor(pairs, dtype=torch.int64, device="cuda:0")
    whole = st.gather(torch.from_numpy(case["S"]).to("cuda:0"), lay, ij).cpu().numpy()
    assert np.array_equal(vals, whole)
    for (i, j), v in zip(pairs, vals):
        x = oracle_mod.sigma_column(f, j)
        assert abs(v - x[i]) <= 1e-12 * np.sqrt(abs(oracle_mod.sigma_column(f, i)[i] * x[j]))


def test_select_outside_pattern_uses_the_full_inverse(case, oracle_mod):
    import torch
    from paper_2504_19171_amd import stiles as st
    lay, f = case["lay"], case["f"]
    pairs = [(900, 100), (10, 999), (500, 400)]
    ij = torch.tensor(pairs, dtype=torch.int64, device="cuda:0")
    g = st.gather(torch.from_numpy(case["S"]).to("cuda:0"), lay, ij).cpu().numpy()
    assert np.isnan(g[0]) and np.isnan(g[1]) and np.isfinite(g[2])   # outside L's tile pattern: NaN
    vals, info = st.select(case["L"], lay, pairs)
    vals = vals.cpu().numpy()
    for (i, j), v in zip(pairs, vals):
        x = oracle_mod.sigma_column(f, j)
        assert abs(v - x[i]) <= 1e-12 * np.sqrt(abs(oracle_mod.sigma_column(f, i)[i] * x[j]))
