"""Parity at the full size of the large workload (n = 100,000 + 100,
half-bandwidth 1,024, arrow 100, tile 256, seed 1) in the launch
configuration the benchmark times (pack into L, factor in place, selected
inverse).

* Every stored entry of L and of Sigma (band, arrow and corner tiles) is
  compared with the oracle's factor and selected inverse, and log det whole
  (the oracle takes seconds on the host cores at this size).
* A second run writes into buffers filled with NaN beforehand (a separate L,
  Sigma and both workspaces): every output entry must be written, and nothing
  may be read before it is written.  It must equal the first run bit for bit
  (L, Sigma and log det): the persistent kernels hand data between
  workgroups, and a stale read would show as a difference.
* Sampled columns of Sigma are also checked against columns of A^{-1} from two
  triangular solves with the oracle's factor (a second, independent route).
"""
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
    dev = torch.device("cuda:0")
    print(f"large workload nb={NB} w={W} a={A} b={B}: run 1 (in place, as benchmarked)", flush=True)
    ab, P, C = to_device(M, dev)
    L1 = st.pack(ab, P, C, lay)
    _, ld1, info1 = st.factor(L1, lay, out=L1)
    S1, sinfo1 = st.selinv(L1, lay)
    torch.cuda.synchronize()
    print("  run 2 (separate outputs and workspaces filled with NaN)", flush=True)
    T = st.pack(ab, P, C, lay)
    nan = float("nan")
    L2 = torch.full_like(T, nan)
    S2 = torch.full_like(T, nan)
    wsf = torch.full((lay.factor_workspace_bytes,), 0xFF, dtype=torch.uint8, device=dev)
    wss = torch.full((lay.selinv_workspace_bytes,), 0xFF, dtype=torch.uint8, device=dev)
    _, ld2, info2 = st.factor(T, lay, out=L2, workspace=wsf)
    _, sinfo2 = st.selinv(L2, lay, out=S2, workspace=wss)
    torch.cuda.synchronize()
    same = dict(L=bool(torch.equal(L1, L2)), S=bool(torch.equal(S1, S2)),
                logdet=float(ld1.item()) == float(ld2.item()),
                nan_L=int(torch.isnan(L2).sum().item()), nan_S=int(torch.isnan(S2).sum().item()))
    out = dict(M=M, lay=lay, L=L1.cpu().numpy(), S=S1.cpu().numpy(), logdet=float(ld1.item()),
               info=(int(info1.item()), int(info2.item())), sinfo=(int(sinfo1.item()), int(sinfo2.item())),
               same=same)
    del T, L1, L2, S1, S2, wsf, wss, ab, P, C
    torch.cuda.empty_cache()
    print("  oracle factor and selected inverse ...", flush=True)
    out["f"] = oracle_mod.cholesky(M.ab, M.P, M.C)
    out["ref"] = oracle_mod.selinv(out["f"], B)
    return out


def test_large_status_and_logdet(large_run):
    from gpu_util import logdet_error, LOGDET_TOL
    r = large_run
    assert r["info"] == (0, 0) and r["sinfo"] == (0, 0)
    assert r["f"].info == 0
    err = logdet_error(r["logdet"], r["f"])
    print(f"  log det {r['logdet']:.12e} vs oracle {r['f'].logdet:.12e}: scaled error {err:.2e}", flush=True)
    assert err <= LOGDET_TOL


def test_large_every_entry_of_L(large_run):
    """Every stored entry of L (band tiles, arrow, corner) against the oracle's factor."""
    from gpu_util import factor_error, L_TOL
    r = large_run
    err, outside = factor_error(r["L"], r["lay"], r["f"], r["M"])
    print(f"  L: max scaled error {err:.2e}, largest entry outside the element band {outside:.1e}", flush=True)
    assert err <= L_TOL
    assert outside == 0.0


def test_large_every_entry_of_sigma(large_run):
    """Every entry of Sigma on the tile pattern against the oracle's selected inverse."""
    from gpu_util import sigma_error, SIGMA_TOL
    r = large_run
    err, diag_rel = sigma_error(r["S"], r["lay"], r["ref"])
    print(f"  Sigma: correlation-scaled max error {err:.2e}, diagonal relative {diag_rel:.2e}", flush=True)
    assert err <= SIGMA_TOL
    assert diag_rel <= SIGMA_TOL


def test_large_poisoned_rerun_is_bitwise_equal(large_run):
    s = large_run["same"]
    print(f"  rerun into NaN-filled buffers: {s}", flush=True)
    assert s["nan_L"] == 0 and s["nan_S"] == 0, "an output entry was not written"
    assert s["L"] and s["S"] and s["logdet"], "the rerun differs from the first run"


@pytest.mark.parametrize("j", COLS)
def test_large_sampled_columns(large_run, oracle_mod, j):
    """Column j of L and of Sigma on the tile pattern against the oracle's
    column of A^{-1} from two triangular solves."""
    from gpu_util import column_errors, L_TOL, SIGMA_TOL
    r = large_run
    lerr, outside, serr, nrows = column_errors(r["L"], r["S"], r["lay"], r["f"], r["M"], oracle_mod, j)
    print(f"  column {j}: {nrows} rows, L err {lerr:.2e} (outside band {outside:.1e}), Sigma err {serr:.2e}",
          flush=True)
    assert lerr <= L_TOL
    assert outside == 0.0
    assert serr <= SIGMA_TOL
