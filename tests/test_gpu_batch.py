"""The batched form (stiles_factor_batched / stiles_selinv_batched): every
matrix of a mixed batch comes out bit for bit as from the single-matrix calls,
and within tolerance of the oracle; a matrix that is not positive definite
fails alone; a workspace is reusable across batches of different sizes."""
import math

import numpy as np
import pytest

from paper_2504_19171_amd import inputs

pytestmark = pytest.mark.gpu

# (nb, w, a, b): tile sizes, bandwidths and arrow widths mixed in one batch,
# with a single-tile matrix, a diagonal one, a dense band, an arrow wider than
# 256 (blocked corner) and matrices of very different tile-column counts
MIX = [
    (2000, 32, 20, 64),
    (777, 100, 33, 128),
    (60, 10, 5, 64),
    (1300, 300, 0, 256),
    (900, 64, 300, 64),
    (513, 130, 1, 192),
    (1000, 0, 0, 64),
    (500, 499, 0, 64),
    (3100, 200, 77, 128),
]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from paper_2504_19171_amd import stiles as st
    st.load()
    return torch


def _inputs(cases, seed0, dev="cuda:0"):
    from gpu_util import to_device
    from paper_2504_19171_amd import stiles as st
    Ms, lays, As = [], [], []
    for k, (nb, w, a, b) in enumerate(cases):
        M = inputs.arrowhead_spd(nb, w, a, seed=seed0 + k)
        lay = st.layout(M.n, w, a, b)
        Ms.append(M)
        lays.append(lay)
        As.append(st.pack(*to_device(M, dev), lay))
    return Ms, lays, As


def _plain(As, lays):
    from paper_2504_19171_amd import stiles as st
    out = []
    for A, lay in zip(As, lays):
        L, ld, info = st.factor(A, lay)
        S, sinfo = st.selinv(L, lay)
        out.append((L, S, ld, info, sinfo))
    return out


def _batched(As, lays, ws=None):
    from paper_2504_19171_amd import stiles as st
    Ls, ld, info = st.factor_batched(As, lays, workspace=ws)
    Ss, info = st.selinv_batched(Ls, lays, workspace=ws, info=info)
    return Ls, Ss, ld, info


@pytest.fixture(scope="module")
def mix_run(torch_cuda):
    torch = torch_cuda
    Ms, lays, As = _inputs(MIX, 300)
    print(f"batch of {len(MIX)}: {MIX}", flush=True)
    plain = _plain(As, lays)
    Ls, Ss, ld, info = _batched(As, lays)
    torch.cuda.synchronize()
    return dict(Ms=Ms, lays=lays, As=As, plain=plain, Ls=Ls, Ss=Ss, ld=ld.cpu().numpy(), info=info.cpu().numpy())


def test_batched_equals_single_bitwise(mix_run, torch_cuda):
    torch = torch_cuda
    r = mix_run
    for k, (L, S, ld, info, sinfo) in enumerate(r["plain"]):
        assert int(info.item()) == 0 and int(sinfo.item()) == 0
        assert tuple(r["info"][k]) == (0, 0), k
        assert torch.equal(r["Ls"][k], L), f"L of matrix {k} {MIX[k]}"
        assert torch.equal(r["Ss"][k], S), f"Sigma of matrix {k} {MIX[k]}"
        assert r["ld"][k] == float(ld.item()), k


@pytest.mark.parametrize("cols", ["1", "3", "16"])
def test_columns_per_launch_bitwise(mix_run, torch_cuda, monkeypatch, cols):
    """The batched factor launches several tile columns at a time (STILES_KB_COLS,
    default 8), the columns of one launch chained through per-block update
    counters.  Every count gives the same L and log det, bit for bit, as the
    default run (and so as the single-matrix calls)."""
    torch = torch_cuda
    from paper_2504_19171_amd import stiles as st
    monkeypatch.setenv("STILES_KB_COLS", cols)
    print(f"batched factor, {cols} tile columns per launch", flush=True)
    Ls, ld, info = st.factor_batched(mix_run["As"], mix_run["lays"])
    torch.cuda.synchronize()
    assert (info.cpu().numpy()[:, 0] == 0).all(), cols
    for k in range(len(MIX)):
        assert torch.equal(Ls[k], mix_run["Ls"][k]), (cols, k, MIX[k])
    assert np.array_equal(ld.cpu().numpy(), mix_run["ld"]), cols


def test_batched_matches_oracle(mix_run, oracle_mod):
    from gpu_util import factor_error, sigma_error, logdet_error, SIGMA_TOL, LOGDET_TOL, L_TOL
    r = mix_run
    for k, (nb, w, a, b) in enumerate(MIX):
        M, lay = r["Ms"][k], r["lays"][k]
        f = oracle_mod.cholesky(M.ab, M.P, M.C)
        S = oracle_mod.selinv(f, b)
        lerr, outside = factor_error(r["Ls"][k].cpu().numpy(), lay, f, M)
        serr, drel = sigma_error(r["Ss"][k].cpu().numpy(), lay, S)
        lderr = logdet_error(float(r["ld"][k]), f)
        print(f"  matrix {k} {MIX[k]}: L {lerr:.2e}, Sigma {serr:.2e}, diag {drel:.2e}, logdet {lderr:.2e}",
              flush=True)
        assert lerr <= L_TOL and outside == 0.0
        assert serr <= SIGMA_TOL and drel <= SIGMA_TOL
        assert lderr <= LOGDET_TOL


def test_batched_failure_stays_in_its_matrix(torch_cuda, oracle_mod):
    """Matrix 1 of 3 is not positive definite: its info names the column, its
    log det is NaN; the other two are untouched by it."""
    torch = torch_cuda
    from gpu_util import to_device
    from paper_2504_19171_amd import stiles as st
    cases = [(700, 40, 10, 64), (900, 60, 12, 64), (650, 100, 0, 128)]
    Ms, lays, As = _inputs(cases, 900)
    Ms[1].ab[0, 333] = -1.0
    As[1] = st.pack(*to_device(Ms[1], "cuda:0"), lays[1])
    plain = _plain(As, lays)
    Ls, Ss, ld, info = _batched(As, lays)
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert info[1, 0] == 334 and int(plain[1][3].item()) == 334
    assert math.isnan(float(ld[1].item()))
    for k in (0, 2):
        assert tuple(info[k]) == (0, 0)
        assert torch.equal(Ls[k], plain[k][0]) and torch.equal(Ss[k], plain[k][1])


def test_workspace_reused_by_a_smaller_batch(torch_cuda):
    """Two batched calls in a row on one workspace, the second with fewer and
    different matrices: both equal the single-matrix results."""
    torch = torch_cuda
    from paper_2504_19171_amd import stiles as st
    first = [(1500, 128, 50, 128), (800, 32, 8, 64), (400, 20, 200, 64)]
    second = [(1200, 64, 30, 64)]
    Ms1, lays1, As1 = _inputs(first, 500)
    Ms2, lays2, As2 = _inputs(second, 600)
    ws = torch.empty(max(st.batch_workspace_bytes(lays1), st.batch_workspace_bytes(lays2)), dtype=torch.uint8,
                     device="cuda:0")
    for As, lays in ((As1, lays1), (As2, lays2)):
        plain = _plain(As, lays)
        Ls, Ss, ld, info = _batched(As, lays, ws=ws)
        torch.cuda.synchronize()
        for k in range(len(As)):
            assert torch.equal(Ls[k], plain[k][0]) and torch.equal(Ss[k], plain[k][1])
            assert float(ld[k].item()) == float(plain[k][2].item())


def test_batched_repeatable(mix_run, torch_cuda):
    """The mixed batch again, three times: bit for bit the first result each
    time (the batch puts the diagonal-tile factorizations under the heaviest
    concurrent load, where an ordering fault would show)."""
    torch = torch_cuda
    r = mix_run
    for rep in range(3):
        Ls, Ss, ld, info = _batched(r["As"], r["lays"])
        torch.cuda.synchronize()
        for k in range(len(MIX)):
            assert torch.equal(Ls[k], r["Ls"][k]) and torch.equal(Ss[k], r["Ss"][k]), (rep, k)


def test_graph_replay_equals_eager(torch_cuda):
    """The batched pass (pack + factor + selinv) captured in a HIP graph from
    the enqueue-only calls, replayed three times with other device work and
    host synchronizations in between and the outputs filled with NaN before
    each replay: every replay equals the eager batched pass bit for bit."""
    torch = torch_cuda
    from gpu_util import to_device
    from paper_2504_19171_amd import autotune
    from paper_2504_19171_amd import stiles as st
    cases = [(2000, 32, 20), (777, 100, 33), (60, 10, 5), (900, 64, 300), (1300, 300, 0)]
    mats, shapes = [], []
    for k, (nb, w, a) in enumerate(cases):
        M = inputs.arrowhead_spd(nb, w, a, seed=7000 + k)
        ab, P, C = to_device(M, "cuda:0")
        mats.append((ab, P, C))
        shapes.append((M.n, w, a))
    print(f"graph replay: {len(cases)} matrices, tile 64", flush=True)
    ref = autotune.batch_buffers(mats, shapes, 64)
    ref["mats"] = mats
    ld0, info0 = autotune.run_batched(ref)
    torch.cuda.synchronize()
    assert (info0.cpu().numpy() == 0).all()
    buf = autotune.batch_buffers(mats, shapes, 64)
    buf["mats"] = mats
    g = autotune.capture_batched(buf)
    for rep in range(3):
        for x in buf["Ls"] + buf["Ss"]:
            x.fill_(float("nan"))
        buf["ld"].fill_(float("nan"))
        # other device work on the same buffers' stream between replays
        other = st.factor(ref["As"][0], ref["lays"][0])[0]
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert (buf["info"].cpu().numpy() == 0).all(), rep
        for k in range(len(cases)):
            assert torch.equal(buf["Ls"][k], ref["Ls"][k]), (rep, k, "L")
            assert torch.equal(buf["Ss"][k], ref["Ss"][k]), (rep, k, "Sigma")
        assert torch.equal(buf["ld"], ld0), rep
        del other
