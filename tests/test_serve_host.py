"""Host logic of the serving loop (no GPU): admission order and budget."""
from paper_2504_19171_amd import serve


def jobs(sizes):
    out = []
    for k, b in enumerate(sizes):
        j = serve.Job(k, 100, 4, 1, float(k))
        j.nbytes = b
        out.append(j)
    return out


def test_admission_takes_the_head_while_it_fits():
    q = jobs([10, 20, 30, 5])
    batch = serve.admit(q, 60, 8)
    assert [j.jid for j in batch] == [0, 1, 2]
    assert [j.jid for j in q] == [3]


def test_admission_never_lets_a_job_overtake():
    q = jobs([10, 50, 5])
    batch = serve.admit(q, 40, 8)          # job 1 does not fit, so job 2 waits behind it
    assert [j.jid for j in batch] == [0]
    assert [j.jid for j in q] == [1, 2]


def test_admission_caps_the_batch():
    q = jobs([1] * 10)
    assert len(serve.admit(q, 100, 3)) == 3 and len(q) == 7
    assert serve.admit(jobs([5]), 4, 3) == []


def test_admission_charges_the_workspace_growth():
    """A lane holding a workspace of 12 bytes; a batch of k jobs needs 10 k of
    workspace: the growth beyond 12 counts against the room."""
    held = 12
    growth = lambda batch: max(0, 10 * len(batch) - held)
    q = jobs([5, 5, 5, 5])
    # 1 job: 5 + 0; 2 jobs: 10 + 8 = 18; 3 jobs: 15 + 18 = 33 > 30
    batch = serve.admit(q, 30, 8, growth)
    assert [j.jid for j in batch] == [0, 1]
    # a lane with nothing held: the first job alone needs 5 + 10 = 15
    held = 0
    assert serve.admit(jobs([5]), 14, 8, growth) == []


def test_job_bytes_cover_results_and_input():
    from paper_2504_19171_amd import stiles as st
    lay = st.layout(20000, 128, 40, 128)
    nbytes = serve.job_bytes(lay)
    inp = 8 * (129 * lay.nb + 40 * lay.nb + 40 * 40)
    assert nbytes == 2 * 8 * lay.total_doubles + inp
