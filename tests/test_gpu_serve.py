"""The serving loop: jobs that arrive while others run are admitted into
concurrent batches within the HBM budget, and every job's result is the same,
bit for bit, as when it is run alone with the single-matrix calls, and within
the stated tolerances of the oracle's factor, log det and selected inverse."""
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
def test_served_results_equal_alone(torch_cuda, oracle_mod, budget_jobs):
    """Arrivals in three bursts, two lanes, at most three jobs per batch; with
    a budget of about two jobs the admission waits for memory.  Every job:
    bit for bit the single-matrix result, and within tolerance of the oracle."""
    torch = torch_cuda
    from gpu_util import factor_error, sigma_error, logdet_error, L_TOL, SIGMA_TOL, LOGDET_TOL
    from paper_2504_19171_amd import serve
    from paper_2504_19171_amd import stiles as st
    tile = 64
    arrivals = [0.0] * 4 + [0.002] * 3 + [0.004] * 3
    jobs = _jobs(arrivals)
    big = max(serve.job_bytes(st.layout(j.n, j.w, j.a, tile)) +
              st.batch_workspace_bytes([st.layout(j.n, j.w, j.a, tile)]) for j in jobs)
    got = {}

    def consume(j):    # results read while resident; the server then frees them
        got[j.jid] = (j.L.cpu().numpy(), j.Sigma.cpu().numpy())
    srv = serve.Server(budget=budget_jobs * big, tile=tile, lanes=2, max_batch=3, on_done=consume)
    print(f"serving {len(jobs)} jobs, budget {budget_jobs} x the largest job", flush=True)
    done = srv.run(jobs)
    torch.cuda.synchronize()
    assert len(done) == len(jobs)
    assert srv.peak <= srv.budget
    for j in done:
        assert j.info == (0, 0), j.jid
        assert j.done >= j.arrival
        L, S, ld, info = _alone(j, tile)
        assert info == (0, 0)
        assert np.array_equal(got[j.jid][0], L.cpu().numpy()), f"L of job {j.jid}"
        assert np.array_equal(got[j.jid][1], S.cpu().numpy()), f"Sigma of job {j.jid}"
        assert j.logdet == ld and math.isfinite(ld)
        assert j.L is None
        # the oracle, on the same seeded matrix
        M = inputs.arrowhead_spd(j.nb, j.w, j.a, seed=4000 + j.jid)
        f = oracle_mod.cholesky(M.ab, M.P, M.C)
        ref = oracle_mod.selinv(f, tile)
        lerr, outside = factor_error(got[j.jid][0], j.lay, f, M)
        serr, drel = sigma_error(got[j.jid][1], j.lay, ref)
        lderr = logdet_error(j.logdet, f)
        print(f"  job {j.jid} (n={j.n}, w={j.w}, a={j.a}): L {lerr:.1e}, Sigma {serr:.1e}, log det {lderr:.1e}",
              flush=True)
        assert lerr <= L_TOL and outside == 0.0
        assert serr <= SIGMA_TOL and drel <= SIGMA_TOL
        assert lderr <= LOGDET_TOL
    srv.close()
    assert srv.in_use == 0


def test_inputs_made_at_admission(torch_cuda):
    """Jobs whose inputs are drawn on the device when they are admitted (on
    the lane's stream) give the same results as the same matrices drawn up
    front and run alone."""
    torch = torch_cuda
    from paper_2504_19171_amd import serve
    from paper_2504_19171_amd import stiles as st
    tile = 64
    shapes = [(1500, 40, 12), (700, 200, 0), (2600, 16, 300), (900, 64, 7), (600, 10, 500)]
    jobs = []
    for k, (nb, w, a) in enumerate(shapes):
        mk = (lambda nb=nb, w=w, a=a, k=k: inputs.arrowhead_spd_device(nb, w, a, 5000 + k, "cuda:0"))
        jobs.append(serve.Job(k, nb, w, a, 0.001 * k, make=mk))
    srv = serve.Server(budget=8 << 30, tile=tile, lanes=2, max_batch=2, keep_results=True)
    done = srv.run(jobs)
    torch.cuda.synchronize()
    for j in done:
        assert j.info == (0, 0)
        ab, P, C = inputs.arrowhead_spd_device(j.nb, j.w, j.a, 5000 + j.jid, "cuda:0")
        A = st.pack(ab, P, C, j.lay)
        L, ld, _ = st.factor(A, j.lay)
        S, _ = st.selinv(L, j.lay)
        assert torch.equal(L, j.L) and torch.equal(S, j.Sigma) and float(ld.item()) == j.logdet
        srv.release(j)
    srv.close()
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
