"""The serving loop: jobs that arrive while others run are admitted into
concurrent batches within the HBM budget, and every job's result is the same,
bit for bit, as when it is run alone with the single-matrix calls."""
import math

import numpy as np
import pytest

from paper_2504_19171_amd import inputs

pytestmark = pytest.mark.gpu

# (nb, w, a): mixed sizes, bandwidths and arrows (one arrow wider than 256)
STREAM = [(1500, 40, 12), (700, 200, 0), (2600, 16, 300), (900, 64, 7), (1200, 128, 45),
          (400, 399, 3), (3000, 30, 100), (800, 90, 60), (1700, 250, 20), (600, 10, 500)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no HIP device"
    from paper_2504_19171_amd import stiles as st
    st.load()
    return torch


def _jobs(arrivals, seed0=4000):
    from gpu_util import to_device
    from paper_2504_19171_amd import serve
    out = []
    for k, ((nb, w, a), t) in enumerate(zip(STREAM, arrivals)):
        M = inputs.arrowhead_spd(nb, w, a, seed=seed0 + k)
        ab, P, C = to_device(M, "cuda:0")
        out.append(serve.Job(k, nb, w, a, float(t), ab=ab, P=P, C=C))
    return out


def _alone(job, tile):
    from gpu_util import to_device
    from paper_2504_19171_amd import stiles as st
    M = inputs.arrowhead_spd(job.nb, job.w, job.a, seed=4000 + job.jid)
    lay = st.layout(job.n, job.w, job.a, tile)
    A = st.pack(*to_device(M, "cuda:0"), lay)
    L, ld, info = st.factor(A, lay)
    S, sinfo = st.selinv(L, lay)
    return L, S, float(ld.item()), (int(info.item()), int(sinfo.item()))


@pytest.mark.parametrize("budget_jobs", [100, 2])
def test_served_results_equal_alone(torch_cuda, budget_jobs):
    """Arrivals in three bursts, two lanes, at most three jobs per batch; with
    a budget of about two jobs the admission waits for memory."""
    torch = torch_cuda
    from paper_2504_19171_amd import serve
    tile = 64
    arrivals = [0.0] * 4 + [0.002] * 3 + [0.004] * 3
    jobs = _jobs(arrivals)
    big = max(serve.job_bytes(__import__("paper_2504_19171_amd.stiles", fromlist=["x"]).layout(j.n, j.w, j.a, tile))
              for j in jobs)
    got = {}

    def consume(j):    # results read while resident; the server then frees them
        got[j.jid] = (j.L.cpu().numpy(), j.Sigma.cpu().numpy())
    srv = serve.Server(budget=budget_jobs * big, tile=tile, lanes=2, max_batch=3, on_done=consume)
    peak = [0]
    orig = srv._launch

    def spy(lane, batch, ev, t0):
        peak[0] = max(peak[0], srv.in_use)
        return orig(lane, batch, ev, t0)
    srv._launch = spy
    print(f"serving {len(jobs)} jobs, budget {budget_jobs} x the largest job", flush=True)
    done = srv.run(jobs)
    torch.cuda.synchronize()
    assert len(done) == len(jobs)
    assert peak[0] <= srv.budget
    for j in done:
        assert j.info == (0, 0), j.jid
        assert j.done >= j.arrival
        L, S, ld, info = _alone(j, tile)
        assert info == (0, 0)
        assert np.array_equal(got[j.jid][0], L.cpu().numpy()), f"L of job {j.jid}"
        assert np.array_equal(got[j.jid][1], S.cpu().numpy()), f"Sigma of job {j.jid}"
        assert j.logdet == ld and math.isfinite(ld)
        assert j.L is None
    assert srv.in_use == 0


def test_plain_fifo_matches_too(torch_cuda):
    torch = torch_cuda
    from paper_2504_19171_amd import serve
    jobs = _jobs([0.0] * len(STREAM))[:4]
    out = serve.serve_plain(jobs, 64, keep_results=True)
    for j in out:
        L, S, ld, info = _alone(j, 64)
        assert j.info == info == (0, 0)
        assert torch.equal(j.L, L) and torch.equal(j.Sigma, S) and j.logdet == ld
    assert all(b.done >= a.done for a, b in zip(out, out[1:]))
