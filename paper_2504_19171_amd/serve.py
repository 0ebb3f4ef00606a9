"""Serving loop: factor + selected-inversion jobs of mixed n, bandwidth and
arrow, admitted by an HBM budget, their work overlapped on the device.

Jobs wait in arrival order.  Whenever one of the lanes is free (a lane is a
stream with its own batch workspace), the jobs at the head of the queue that
fit the free part of the budget form a batch and go to that lane as one
`stiles_factor_batched` + `stiles_selinv_batched` sequence; jobs that arrive
while batches run are admitted as lanes and memory free up, so their work
overlaps the running batches.  Each job's L and Sigma stay on the device
(`Job.L`, `Job.Sigma`) until the caller drops them; the budget counts them
while they are held.  Results do not depend on the mix: every matrix of a
batch comes out as from the single-matrix calls, bit for bit.

The budget counts every device buffer the server holds:
  * each job's results (L, factored in place over its packed input, and
    Sigma) and its input in canonical band form, from admission until the
    results are released;
  * each lane's batch workspace, while the lane holds it: a batch is admitted
    only if its results plus the growth of the lane's workspace fit, and idle
    lanes give their workspaces back when the head of the queue would not fit
    otherwise.

A job's input is either given (device tensors) or made on the lane's stream
when the job is admitted (`Job.make`, e.g. drawn on the device from its seed),
and dropped once packed.

Host logic only (admission, queue, clocks); every step of the computation
runs in the library's HIP kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

from . import stiles as st


@dataclass
class Job:
    """One request: the matrix in canonical band form on the device, given
    (ab, P, C) or made at admission by `make()` -> (ab, P, C)."""
    jid: int
    nb: int
    w: int
    a: int
    arrival: float                 # seconds on the server's clock
    ab: object = None              # device tensors (inputs)
    P: object = None
    C: object = None
    make: Optional[Callable[[], tuple]] = None
    lay: Optional[st.Layout] = None
    L: object = None               # results, device-resident
    Sigma: object = None
    logdet: float = float("nan")
    info: tuple = (None, None)
    done: float = float("nan")     # completion time on the server's clock
    nbytes: int = 0                # bytes charged to the budget while held

    @property
    def n(self) -> int:
        return self.nb + self.a


def job_bytes(lay: st.Layout) -> int:
    """Device bytes a job holds from admission until its results are released:
    L (factored in place over its packed input), Sigma, and its input in
    canonical band form (dropped once packed, counted until release)."""
    w = min(lay.bandwidth, max(lay.nb - 1, 0))
    inp = 8 * ((w + 1) * lay.nb + lay.arrow * lay.nb + lay.arrow * lay.arrow)
    return 2 * 8 * lay.total_doubles + inp


def admit(queue: List[Job], room: int, max_batch: int,
          extra: Optional[Callable[[List[Job]], int]] = None) -> List[Job]:
    """Take the next batch off the head of the queue, in arrival order: jobs
    join while the batch's bytes -- its jobs' `nbytes` plus `extra(batch)` (the
    growth of the lane's workspace the batch would need) -- fit the free bytes
    `room`, and the batch has fewer than `max_batch` jobs; the first job that
    does not fit stops the batch (no job overtakes an earlier one)."""
    batch: List[Job] = []
    held = 0
    while queue and len(batch) < max_batch:
        cand = batch + [queue[0]]
        need = held + queue[0].nbytes + (extra(cand) if extra is not None else 0)
        if need > room:
            break
        held += queue[0].nbytes
        batch.append(queue.pop(0))
    return batch


@dataclass
class _Lane:
    stream: object
    jobs: List[Job] = field(default_factory=list)
    ws: object = None
    ws_bytes: int = 0
    ev_done: object = None
    logdet: object = None
    info: object = None


class Server:
    """Continuous admission over `lanes` concurrent batches within `budget` bytes."""

    def __init__(self, budget: int, tile: int, lanes: int = 2, max_batch: int = 32, keep_results: bool = False,
                 on_done: Optional[Callable[[Job], None]] = None):
        import torch
        self.budget = int(budget)
        self.tile = int(tile)
        self.max_batch = int(max_batch)
        self.keep = keep_results
        self.on_done = on_done       # called with each finished job while its results are on the device
        self.lanes = [_Lane(torch.cuda.Stream()) for _ in range(lanes)]
        self.in_use = 0              # bytes held: admitted jobs until released, lane workspaces
        self.peak = 0
        self.finished: List[Job] = []

    def _ws_growth(self, lane: _Lane) -> Callable[[List[Job]], int]:
        def growth(batch: List[Job]) -> int:
            return max(0, st.batch_workspace_bytes([j.lay for j in batch]) - lane.ws_bytes)
        return growth

    def _charge(self, nbytes: int) -> None:
        self.in_use += nbytes
        self.peak = max(self.peak, self.in_use)

    def _launch(self, lane: _Lane, batch: List[Job], clock_ev, t0: float):
        import torch
        with torch.cuda.stream(lane.stream):
            As = []
            for j in batch:
                if j.make is not None:
                    j.ab, j.P, j.C = j.make()
                As.append(st.pack(j.ab, j.P, j.C, j.lay, stream=lane.stream))
                for x in (j.ab, j.P, j.C):       # inputs released once packed
                    if x is not None:
                        x.record_stream(lane.stream)
                j.ab = j.P = j.C = None
            lays = [j.lay for j in batch]
            need = st.batch_workspace_bytes(lays)
            if need > lane.ws_bytes:
                lane.ws = None
                lane.ws = torch.empty(need, dtype=torch.uint8, device=As[0].device)
                self._charge(need - lane.ws_bytes)
                lane.ws_bytes = need
            Ls, ld, info = st.factor_batched(As, lays, outs=As, workspace=lane.ws, stream=lane.stream)
            Ss, info = st.selinv_batched(Ls, lays, workspace=lane.ws, info=info, stream=lane.stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(lane.stream)
        for j, L, S in zip(batch, Ls, Ss):
            j.L, j.Sigma = L, S
        lane.jobs, lane.ev_done, lane.logdet, lane.info = batch, ev, ld, info

    def _retire(self, lane: _Lane, clock_ev, t0: float):
        ldh = lane.logdet.cpu().tolist()
        infoh = lane.info.cpu().tolist()
        t_done = t0 + clock_ev.elapsed_time(lane.ev_done) / 1e3
        for j, ld, inf in zip(lane.jobs, ldh, infoh):
            j.logdet, j.info, j.done = ld, tuple(inf), t_done
            if self.on_done is not None:
                self.on_done(j)
            if not self.keep:
                self.release(j)
            self.finished.append(j)
        lane.jobs, lane.ev_done = [], None

    def _shrink_idle(self) -> bool:
        """Give back the workspaces of idle lanes; True if any was held."""
        freed = False
        for lane in self.lanes:
            if not lane.jobs and lane.ws_bytes:
                lane.stream.synchronize()
                lane.ws = None
                self.in_use -= lane.ws_bytes
                lane.ws_bytes = 0
                freed = True
        return freed

    def release(self, job: Job) -> None:
        """Drop a finished job's device results and give its bytes back to the budget."""
        if job.nbytes and job.L is not None:
            job.L = job.Sigma = None
            self.in_use -= job.nbytes

    def close(self) -> None:
        """Give back every lane workspace (after the last run)."""
        for lane in self.lanes:
            lane.stream.synchronize()
            self.in_use -= lane.ws_bytes
            lane.ws, lane.ws_bytes = None, 0

    def run(self, jobs: List[Job], clock: Callable[[], float] = time.perf_counter) -> List[Job]:
        """Serve `jobs` (sorted by arrival; arrival times on `clock`, in seconds
        from the call).  Returns them in completion order, with their results."""
        import torch
        for j in jobs:
            j.lay = st.layout(j.n, j.w, j.a, self.tile)
            j.nbytes = job_bytes(j.lay)
            alone = j.nbytes + st.batch_workspace_bytes([j.lay])
            if alone > self.budget:
                raise ValueError(f"job {j.jid} needs {alone} bytes, over the budget of {self.budget}")
        clock_ev = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        clock_ev.record()
        t_base = clock()
        t0 = 0.0
        queue: List[Job] = []
        nxt = 0
        while nxt < len(jobs) or queue or any(l.jobs for l in self.lanes):
            now = clock() - t_base
            while nxt < len(jobs) and jobs[nxt].arrival <= now:
                queue.append(jobs[nxt])
                nxt += 1
            progressed = False
            for lane in self.lanes:
                if lane.jobs and lane.ev_done.query():
                    self._retire(lane, clock_ev, t0)
                    progressed = True
            for lane in self.lanes:
                if lane.jobs or not queue:
                    continue
                batch = admit(queue, self.budget - self.in_use, self.max_batch, self._ws_growth(lane))
                if batch:
                    self._charge(sum(j.nbytes for j in batch))
                    self._launch(lane, batch, clock_ev, t0)
                    progressed = True
            if queue and not any(l.jobs for l in self.lanes):
                # nothing runs and the head does not fit: idle workspaces go back first
                if not progressed and not self._shrink_idle():
                    raise RuntimeError("the budget is held by results not released (Server.release)")
                continue
            if not progressed:
                time.sleep(2e-4)
        return self.finished


def serve_plain(jobs: List[Job], tile: int, clock: Callable[[], float] = time.perf_counter,
                keep_results: bool = False) -> List[Job]:
    """The plain FIFO for comparison: one job at a time, in arrival order, with
    the single-matrix calls on one stream."""
    import torch
    clock_ev = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    clock_ev.record()
    t_base = clock()
    for j in jobs:
        while clock() - t_base < j.arrival:
            time.sleep(2e-4)
        j.lay = st.layout(j.n, j.w, j.a, tile)
        if j.make is not None:
            j.ab, j.P, j.C = j.make()
        A = st.pack(j.ab, j.P, j.C, j.lay)
        j.ab = j.P = j.C = None
        L, ld, info = st.factor(A, j.lay, out=A)
        S, sinfo = st.selinv(L, j.lay)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        ev.synchronize()
        j.done = clock_ev.elapsed_time(ev) / 1e3
        j.logdet, j.info = float(ld.item()), (int(info.item()), int(sinfo.item()))
        if keep_results:
            j.L, j.Sigma = L, S
    return jobs
