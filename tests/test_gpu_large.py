"""Parity at the full size of the large workload (n = 100,000 + 100,
half-bandwidth 1,024, arrow 100, tile 256, seed 1) in the launch
configuration the benchmark times.  The oracle factors the matrix once
(seconds on the host cores); log det is compared whole, and sampled columns
of L and of Sigma one by one (a column of Sigma = A^{-1} by two triangular
solves with the oracle's factor)."""
import numpy as np
import pytest

from paper_2504_19171_amd import inputs

pytestmark = pytest.mark.gpu

NB, W, A, B = 100000, 1024, 100, 256
# first/last columns of tiles, a column in the middle, the last real band
# column (ragged last tile), the first and last arrow columns
COLS = [0, 255, 256, 40000 + 77, 99840 - 1, 99840, NB - 1, NB, NB + A - 1]


@pytest.fixture(scope="module")
def large_run(oracle_mod):
    import torch
    from gpu_util import to_device
    from paper_2504_19171_amd import stiles as st
    assert torch.cuda.is_available(), "no HIP device"
    st.load()
    M = inputs.arrowhead_spd(NB, W, A, seed=1)
    lay = st.layout(M.n, W, A, B)
    print(f"large workload nb={NB} w={W} a={A} b={B}", flush=True)
    T = st.pack(*to_device(M, "cuda:0"), lay)
    L, logdet, info = st.factor(T, lay)
    S, sinfo = st.selinv(L, lay)
    torch.cuda.synchronize()
    out = dict(M=M, lay=lay, L=L.cpu().numpy(), S=S.cpu().numpy(), logdet=float(logdet.item()),
               info=int(info.item()), sinfo=int(sinfo.item()))
    del T, L, S
    torch.cuda.empty_cache()
    print("  oracle factor ...", flush=True)
    out["f"] = oracle_mod.cholesky(M.ab, M.P, M.C)
    return out


def test_large_status_and_logdet(large_run):
    from gpu_util import logdet_error, LOGDET_TOL
    r = large_run
    assert r["info"] == 0 and r["sinfo"] == 0
    assert r["f"].info == 0
    err = logdet_error(r["logdet"], r["f"])
    print(f"  log det {r['logdet']:.12e} vs oracle {r['f'].logdet:.12e}: scaled error {err:.2e}", flush=True)
    assert err <= LOGDET_TOL


@pytest.mark.parametrize("j", COLS)
def test_large_sampled_columns(large_run, oracle_mod, j):
    """Column j of L and of Sigma on the tile pattern against the oracle."""
    from gpu_util import column_errors, L_TOL, SIGMA_TOL
    r = large_run
    lerr, outside, serr, nrows = column_errors(r["L"], r["S"], r["lay"], r["f"], r["M"], oracle_mod, j)
    print(f"  column {j}: {nrows} rows, L err {lerr:.2e} (outside band {outside:.1e}), Sigma err {serr:.2e}",
          flush=True)
    assert lerr <= L_TOL
    assert outside == 0.0
    assert serr <= SIGMA_TOL
