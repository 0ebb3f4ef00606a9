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


def test_job_bytes_cover_results_and_workspace():
    from paper_2504_19171_amd import stiles as st
    lay = st.layout(20000, 128, 40, 128)
    nbytes = serve.job_bytes(lay)
    assert nbytes >= 2 * 8 * lay.total_doubles + lay.selinv_workspace_bytes
