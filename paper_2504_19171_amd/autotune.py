"""Tile-size autotuner: the tile size b is picked by timing, on the device,
the factorization and selected inversion of the actual matrices with each
candidate b (no model of the cost).

The tile size is a free parameter of the method (the paper tunes it per
platform, Sec. IV-D); for a batch the tile-column launches run in step
across the matrices, so one b serves the whole batch.  Every timed run is the
library's own HIP path; the candidates' buffers are released between runs.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

from . import stiles as st

CANDIDATES = (64, 128, 256)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def batch_buffers(mats, shapes, tile, in_place: bool = False):
    """Layouts, packed inputs and output buffers of a batch at one tile size.

    mats: [(ab, P, C)] device tensors (canonical band form, P and C None
    without an arrow); shapes: [(n, w, a)].  in_place: each matrix is packed
    straight into its L buffer and factored there (the As are the Ls), as the
    single-matrix step does; otherwise the factor first copies A into L."""
    import torch
    lays = [st.layout(n, w, a, tile) for (n, w, a) in shapes]
    As = [st.pack(ab, P, C, lay) for (ab, P, C), lay in zip(mats, lays)]
    dev = As[0].device
    Ls = As if in_place else [torch.empty_like(x) for x in As]
    Ss = [torch.empty_like(x) for x in As]
    ws = torch.empty(st.batch_workspace_bytes(lays), dtype=torch.uint8, device=dev)
    return dict(lays=lays, As=As, Ls=Ls, Ss=Ss, ws=ws, tile=tile)


def run_batched(buf):
    """pack + batched factor + batched selinv, enqueued on the current stream."""
    for (A, lay), (ab, P, C) in zip(zip(buf["As"], buf["lays"]), buf["mats"]):
        st.pack(ab, P, C, lay, out=A)
    _, ld, info = st.factor_batched(buf["As"], buf["lays"], outs=buf["Ls"], workspace=buf["ws"])
    _, info = st.selinv_batched(buf["Ls"], buf["lays"], outs=buf["Ss"], workspace=buf["ws"], info=info)
    return ld, info


def capture_batched(buf):
    """pack + batched factor + batched selinv of this batch captured in a HIP
    graph (torch.cuda.CUDAGraph): the tables of the batched calls are copied
    once (stiles_batch_upload) and the graph holds device work only, so
    g.replay() repeats the whole pass.  buf gains the log det and info tensors
    the graph writes ("ld", "info")."""
    import torch
    n = len(buf["lays"])
    dev = buf["As"][0].device
    buf["ld"] = torch.empty(n, dtype=torch.float64, device=dev)
    buf["info"] = torch.zeros((n, 2), dtype=torch.int32, device=dev)
    st.batch_upload(buf["lays"], buf["As"], buf["Ls"], buf["Ss"], buf["ld"], buf["info"], buf["ws"])

    def body():
        for (A, lay), (ab, P, C) in zip(zip(buf["As"], buf["lays"]), buf["mats"]):
            st.pack(ab, P, C, lay, out=A)
        st.factor_batched(buf["As"], buf["lays"], outs=buf["Ls"], workspace=buf["ws"], info=buf["info"],
                          logdet=buf["ld"], enqueue_only=True)
        st.selinv_batched(buf["Ls"], buf["lays"], outs=buf["Ss"], workspace=buf["ws"], info=buf["info"],
                          As=buf["As"], logdet=buf["ld"], enqueue_only=True)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        body()          # one eager pass on a side stream before the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        body()
    return g


def time_batched(mats, shapes, tile, reps: int = 1) -> Tuple[float, dict]:
    """Milliseconds of one batched pass at this tile size (after one untimed pass);
    each matrix is packed into its L and factored in place."""
    import torch
    buf = batch_buffers(mats, shapes, tile, in_place=True)
    buf["mats"] = mats
    run_batched(buf)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for _ in range(reps):
        run_batched(buf)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, buf


def time_plain(mats, shapes, tile) -> List[float]:
    """Milliseconds of pack + factor + selinv of each matrix alone (its own launches;
    packed into L and factored in place, as in the batched pass)."""
    import torch
    out = []
    for (ab, P, C), (n, w, a) in zip(mats, shapes):
        lay = st.layout(n, w, a, tile)
        L = torch.empty(lay.total_doubles, dtype=torch.float64, device=ab.device)
        S = torch.empty_like(L)
        wf = torch.empty(lay.factor_workspace_bytes, dtype=torch.uint8, device=ab.device)
        wsl = torch.empty(lay.selinv_workspace_bytes, dtype=torch.uint8, device=ab.device)

        def once():
            st.pack(ab, P, C, lay, out=L)
            st.factor(L, lay, out=L, workspace=wf)
            st.selinv(L, lay, out=S, workspace=wsl)
        once()
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        once()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
        del L, S, wf, wsl
    return out


def tune_batch(mats, shapes, candidates: Sequence[int] = CANDIDATES) -> Tuple[int, Dict[int, float]]:
    """(fastest tile size, {tile: ms of one batched pass})."""
    import torch
    ms = {}
    for b in candidates:
        t, buf = time_batched(mats, shapes, b)
        ms[b] = t
        del buf
        torch.cuda.empty_cache()
    return min(ms, key=ms.get), ms
