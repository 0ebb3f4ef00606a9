#!/usr/bin/env python3
"""Throughput of the FP64 hot path on one MI355X: pack + tile Cholesky with
log det + selected inversion (Sigma on the tile pattern of L), on a seeded
synthetic band-plus-arrowhead SPD matrix already resident in HBM.

Prints one JSON line.  ``value`` is algorithmic GFLOP/s of one step (the flop
convention of ``paper_2504_19171_amd/flops.py``); ``roofline`` reports the
kernel kind that takes the most time, timed with HIP events inside the timed
region; ``cpu_baseline`` is the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 factor+selinv GFLOP/s & solves/s, batched vs plain; p50/p99 latency"
PEAK_F64_TFLOPS = 78.6    # MI355X dense FP64 (matrix and vector)

# HBM bytes per launch of the dominant kernel kind, from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs scaled by a copy of known size (profiles/k_factor_all_large_hbm_traffic.md),
# valid only for the kernel sources they were taken with (sha256 prefix of csrc/*)
# and the workload named.
MEASURED_TRAFFIC = {("factor", "large"): {"bytes_per_launch": 13.133e9, "sources": "a0004f271920e463"}}
# FP64 matrix-core counters of the same launch (SQ_INSTS_VALU_MFMA_MOPS_F64 x 512 flops and
# SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE x SIMDs; profiles/mfma_f64_large_counters.md),
# valid for the kernel sources they were taken with.
MEASURED_MFMA = {("factor", "large"): {"mfma_flops_per_launch": 2.034e11, "mfma_busy": 0.075,
                                        "sources": "a0004f271920e463"}}


def sources_hash() -> str:
    """sha256 prefix of the kernel sources with // comments and blank lines removed."""
    import glob
    import hashlib
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for f in sorted(glob.glob(os.path.join(here, "paper_2504_19171_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]
PEAK_HBM_GBS = 8000.0


def kernel_flops(nb, w, a, b):
    """Algorithmic flops per step for each timing kind of the library.  The
    diagonal-tile POTRFs, panel TRSMs and trailing updates of the band all run
    inside the factor's single launch (kind "factor"); kind "potrf" is the
    corner's Cholesky alone (its own launch)."""
    from paper_2504_19171_amd import flops as fl
    N, B = fl._halfband(nb, w, b)
    ap = -(-a // 16) * 16
    k = dict(potrf=0.0, trsm=0.0, update=0.0, phase1=0.0, phase2=0.0, factor=0.0, other=0.0)
    for J in range(N):
        s = min(B, N - 1 - J)
        m = s * b + a
        k["phase1"] += b ** 3 / 3 + m * b * b + b ** 3 / 3
        k["phase2"] += 2 * m * m * b + m * b * b
        k["factor"] += b ** 3 / 3 + m * b * b + m * m * b   # the factor's single launch (k_factor_all)
    if ap <= 256:
        k["potrf"] += a ** 3 / 3          # corner factor: one POTRF launch
    else:
        k["potrf"] += 256 ** 3 / 3 + (a - 256) ** 3 / 3   # its two diagonal blocks; TRSM + SYRK in "other"
        k["other"] += (a - 256) * 256 ** 2 + (a - 256) ** 2 * 256
    k["phase1"] += 2 * a ** 3 / 3     # corner TRTRI + LAUUM
    return k


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE_ONE = r"""
import sys, time, json
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2504_19171_amd import inputs
nb, w, a, b, seed = (int(x) for x in sys.argv[2:7])
M = inputs.arrowhead_spd(nb, w, a, seed=seed)
t0 = time.perf_counter()
f = oracle.cholesky(M.ab, M.P, M.C)
oracle.selinv(f, b)
print(json.dumps({"seconds": time.perf_counter() - t0, "threads": oracle.num_threads()}))
"""


def cpu_baseline(w, a, b, nb_sample, seed, nb_single):
    """The oracle (as it stands) on the host cores: on all of them (OpenMP) over
    nb_sample band rows, and on one core over nb_single band rows (a child
    process with OMP_NUM_THREADS=1), with the same w, a, b as the workload."""
    import subprocess
    import oracle
    from paper_2504_19171_amd import flops as fl
    from paper_2504_19171_amd import inputs
    M = inputs.arrowhead_spd(nb_sample, w, a, seed=seed)
    t0 = time.perf_counter()
    f = oracle.cholesky(M.ab, M.P, M.C)
    oracle.selinv(f, b)
    dt = time.perf_counter() - t0
    del M, f
    flop = fl.factor_flops(nb_sample, w, a, b) + fl.selinv_flops(nb_sample, w, a, b)
    out = {"value": round(flop / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
           "kind": "oracle", "seconds": round(dt, 3), "cpu_model": cpu_model(),
           "sample": f"n = {nb_sample:,} + {a}, w = {w}, tile {b} (same band, arrow and tile as the "
                     f"workload, {nb_sample / WORK['nb']:.0%} of its length); factor + selected inverse"}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-c", _ORACLE_ONE, ROOT, str(nb_single), str(w), str(a), str(b),
                          str(seed)], capture_output=True, text=True, env=env, timeout=600)
    if res.returncode == 0:
        one = json.loads(res.stdout.strip().splitlines()[-1])
        fl1 = fl.factor_flops(nb_single, w, a, b) + fl.selinv_flops(nb_single, w, a, b)
        out["single_thread"] = {"value": round(fl1 / one["seconds"] / 1e9, 3), "unit": "GFLOP/s",
                                "cores": one["threads"], "seconds": round(one["seconds"], 3),
                                "sample": f"n = {nb_single:,} + {a}, w = {w}, tile {b}"}
    else:
        out["single_thread"] = {"error": res.stderr[-400:]}
    return out


WORKLOADS = {
    "large": dict(nb=100000, w=1024, a=100, b=256, seed=1, cpu_nb=100000, cpu_nb1=12000),
    "small": dict(nb=2000, w=32, a=20, b=64, seed=0, cpu_nb=2000, cpu_nb1=2000),
    "batched": dict(),
    "served": dict(),
    "grad": dict(),
}
WORK = WORKLOADS["large"]


def main() -> int:
    global WORK
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="large",
                    help="large (default, the benchmark line), or one other workload alone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="batched: this tile size instead of the autotuner's")
    ap.add_argument("--calib-copy", action="store_true",
                    help="one device copy of a tile buffer (known bytes) before the timed steps, to scale "
                         "hardware byte counters")
    ap.add_argument("--jobs", type=int, default=100, help="served: jobs per arrival rate")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="served: HBM budget of the serving loop")
    ap.add_argument("--lanes", type=int, default=3, help="served: concurrent batches")
    ap.add_argument("--max-batch", type=int, default=8, help="served: jobs per batch at most")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched: skip the plain-form timing and the per-matrix comparison (profiling runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="large: skip the small, batched and served summaries of the default line")
    ap.add_argument("--extra-jobs", type=int, default=200, help="large: jobs of the served summary")
    ap.add_argument("--fracs", default="0.5,0.8,1.5",
                    help="served: arrival rates as fractions of the plain FIFO's capacity")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the batched/served forms shard by instance, see the design notes)", file=sys.stderr)
        return 2

    if args.workload == "batched":
        return main_batched(args)
    if args.workload == "served":
        return main_served(args)
    if args.workload == "grad":
        return main_grad(args)
    if args.workload == "small":
        r = leg_small()
        print(json.dumps(r), flush=True)
        return 0 if r["ok"] else 1

    import numpy as np
    import torch
    from paper_2504_19171_amd import flops as fl
    from paper_2504_19171_amd import inputs
    from paper_2504_19171_amd import stiles as st

    WORK = WORKLOADS[args.workload]
    nb, w, a, b = WORK["nb"], WORK["w"], WORK["a"], WORK["b"]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    M = inputs.arrowhead_spd(nb, w, a, seed=WORK["seed"])
    lay = st.layout(M.n, w, a, b)
    ab = torch.from_numpy(M.ab).to(dev)
    P = torch.from_numpy(M.P).to(dev)
    C = torch.from_numpy(M.C).to(dev)
    L = torch.empty(lay.total_doubles, dtype=torch.float64, device=dev)
    S = torch.empty_like(L)
    wsf = torch.empty(lay.factor_workspace_bytes, dtype=torch.uint8, device=dev)
    wss = torch.empty(lay.selinv_workspace_bytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    print(f"bench: inputs ready in {time.perf_counter() - t0:.1f} s (n={M.n}, w={w}, a={a}, tile={b}, "
          f"{8 * lay.total_doubles / 1e9:.2f} GB per tile buffer)", file=sys.stderr, flush=True)

    def step():
        st.pack(ab, P, C, lay, out=L)                           # packed input, factored in place
        _, ld, info = st.factor(L, lay, out=L, workspace=wsf)
        _, sinfo = st.selinv(L, lay, out=S, workspace=wss)
        return ld, info, sinfo

    if args.calib_copy:
        S.copy_(L)                       # 8 * total_doubles bytes read and written
        torch.cuda.synchronize()
    for i in range(args.warmup):
        ld, info, sinfo = step()
        torch.cuda.synchronize()
        print(f"bench: warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    if args.warmup:
        assert int(info.item()) == 0 and int(sinfo.item()) == 0, "factorization failed"

    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    st.timing_enable(True)
    wall0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        ld, info, sinfo = step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per_kind = st.timing_collect()
    st.timing_enable(False)
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    total_ms = ev[0].elapsed_time(ev[-1])
    ok = int(info.item()) == 0 and int(sinfo.item()) == 0 and np.isfinite(float(ld.item()))
    print(f"bench: timed {args.steps} steps in {wall:.3f} s wall, {total_ms:.1f} ms events; logdet "
          f"{float(ld.item()):.10e}", file=sys.stderr, flush=True)

    flop_step = fl.factor_flops(nb, w, a, b) + fl.selinv_flops(nb, w, a, b)
    ms_step = total_ms / args.steps
    value = flop_step / (ms_step / 1e3) / 1e9

    kf = kernel_flops(nb, w, a, b)
    dom = max((k for k in per_kind if k != "other"), key=lambda k: per_kind[k][0])
    dom_ms, dom_launches = per_kind[dom]
    achieved = kf[dom] * args.steps / (dom_ms / 1e3) / 1e12 if dom_ms > 0 else 0.0
    src = sources_hash()
    mt = MEASURED_TRAFFIC.get((dom, args.workload))
    traffic = mt["bytes_per_launch"] if mt and mt["sources"] == src else None
    mm = MEASURED_MFMA.get((dom, args.workload))
    mm = mm if mm and mm["sources"] == src else None
    # the FP64 matrix-core rate this device sustains (pure-MFMA probe, best of 3)
    peak_meas = None
    try:
        best = 0.0
        for _ in range(3):
            fl, ms = st.mfma_peak(4096)
            best = max(best, fl / (ms / 1e3) / 1e12)
        peak_meas = round(best, 2)
    except Exception as e:   # measurement support only; the step above is the result
        print(f"bench: matrix-core probe failed: {e}", file=sys.stderr, flush=True)
    roofline = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 3), "peak": PEAK_F64_TFLOPS,
                "measured_peak": peak_meas,
                "frac_of_measured_peak": round(achieved / peak_meas, 4) if peak_meas else None,
                "mfma_counters": None if mm is None else {
                    "mfma_flops_per_launch": mm["mfma_flops_per_launch"], "mfma_busy": mm["mfma_busy"]},
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_F64_TFLOPS, 4), "traffic": traffic,
                "launches_per_step": dom_launches // max(args.steps, 1),
                "avg_launch_us": round(dom_ms * 1e3 / max(dom_launches, 1), 2)}
    breakdown = {k: {"ms_per_step": round(v[0] / args.steps, 3),
                     "launches_per_step": v[1] // max(args.steps, 1),
                     "tflops": round(kf[k] / (v[0] / args.steps / 1e3) / 1e12, 3) if v[0] > 0 and kf[k] else None}
                 for k, v in per_kind.items()}

    extras = {}
    if not args.no_extras and args.workload == "large":
        del L, S, wsf, wss, ab, P, C
        torch.cuda.empty_cache()
        _log("bench: small workload (latency)")
        extras["small"] = leg_small()
        _log(f"bench: small {extras['small']}")
        _log("bench: batched workload (bounded: 3 timed passes)")
        extras["batched"] = leg_batched(3, 1, device_inputs=True, log=_log)
        _log(f"bench: served workload (bounded: the first {args.extra_jobs} jobs)")
        extras["served"] = leg_served(args.extra_jobs, fracs=(0.5, 0.8), log=_log)
        ok = ok and extras["small"]["ok"] and extras["batched"]["ok"] and extras["served"]["ok"]

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, a, b, WORK["cpu_nb"], WORK["seed"], WORK["cpu_nb1"])

    srt = sorted(step_ms)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n = {nb:,} + {a}, half-bandwidth {w}, arrow {a}, tile {b}, "
                               "seeded N(0,1) band and arrow, diagonal = row |sum| + 1",
                   "n": nb + a, "bandwidth": w, "arrow": a, "tile": b, "instances": 1,
                   "step": "pack + factor in place (L, log det) + selinv (Sigma on L's tile pattern)",
                   "flops_per_step": flop_step},
        "solves_per_s": round(1e3 / ms_step, 4),
        "latency_ms_p50": round(srt[len(srt) // 2], 4),
        "latency_ms_p99": round(srt[min(len(srt) - 1, int(0.99 * len(srt)))], 4),
        "ok": bool(ok),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": breakdown,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def leg_batched(steps, warmup, tile=0, plain=True, device_inputs=False, log=print):
    """64 uneven matrices (inputs.batch_shapes): the tile size picked by the
    autotuner, then `steps` timed passes of pack + batched factor + batched
    selinv, against the plain form (each matrix alone, its own launches) on the
    same matrices, at the batch's tile size and at each matrix's fastest one.
    device_inputs: draw the matrices on the device from their seeds (the same
    construction, a different random stream) instead of on the host."""
    import numpy as np
    import torch
    from paper_2504_19171_amd import autotune
    from paper_2504_19171_amd import flops as fl
    from paper_2504_19171_amd import inputs
    from paper_2504_19171_amd import stiles as st

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    shapes = inputs.batch_shapes()
    mats, nws = [], []
    for nb, w, a, seed in shapes:
        if device_inputs:
            mats.append(inputs.arrowhead_spd_device(nb, w, a, seed, dev))
        else:
            M = inputs.arrowhead_spd(nb, w, a, seed=seed)
            mats.append((torch.from_numpy(M.ab).to(dev), torch.from_numpy(M.P).to(dev) if a else None,
                         torch.from_numpy(M.C).to(dev) if a else None))
        nws.append((nb + a, w, a))
    torch.cuda.synchronize()
    log(f"bench: {len(shapes)} matrices ready in {time.perf_counter() - t0:.1f} s "
        f"(n {min(s[0] for s in shapes)}..{max(s[0] for s in shapes)}, w in {{32, 128, 512}})")

    if tile:
        tune_ms = None
    else:
        tile, tune_ms = autotune.tune_batch(mats, nws)
        log(f"bench: autotuner ms per batched pass {tune_ms} -> tile {tile}")
    plain_same = plain_best = None
    if plain:
        pt = {b: autotune.time_plain(mats, nws, b) for b in autotune.CANDIDATES}
        plain_same = sum(pt[tile]) if tile in pt else sum(autotune.time_plain(mats, nws, tile))
        plain_best = sum(min(pt[b][k] for b in pt) for k in range(len(shapes)))
        log(f"bench: plain ms per pass {[(b, round(sum(v), 1)) for b, v in pt.items()]}")

    _, buf = autotune.time_batched(mats, nws, tile)
    for i in range(warmup):
        autotune.run_batched(buf)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    st.timing_enable(True)
    ev[0].record(stream)
    for i in range(steps):
        ld, info = autotune.run_batched(buf)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per_kind = st.timing_collect()
    st.timing_enable(False)
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    ms_step = ev[0].elapsed_time(ev[-1]) / steps

    # the same pass replayed from a HIP graph (the outputs land in the same
    # buffers, so the comparison below checks the replayed results)
    graph_ms = None
    try:
        g = autotune.capture_batched(buf)
        g.replay()
        torch.cuda.synchronize()
        ge = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ge[0].record(stream)
        for i in range(steps):
            g.replay()
        ge[1].record(stream)
        torch.cuda.synchronize()
        graph_ms = ge[0].elapsed_time(ge[1]) / steps
        ok_graph = bool((buf["info"].cpu().numpy() == 0).all()) and bool(torch.equal(buf["ld"], ld))
        del g
    except Exception as e:   # reported, not hidden: the line then says the graph pass failed
        log(f"bench: graph capture of the batched pass failed: {e}")
        ok_graph = False
    log(f"bench: batched pass from a HIP graph {graph_ms} ms (eager {ms_step:.3f} ms)")

    # every matrix: batched result == single-matrix result, bit for bit
    same = None if not plain else True
    for k, ((ab, P, C), lay) in enumerate(zip(mats, buf["lays"]) if plain else []):
        A = st.pack(ab, P, C, lay)
        L, ld1, _ = st.factor(A, lay)
        S, _ = st.selinv(L, lay)
        same &= bool(torch.equal(L, buf["Ls"][k]) and torch.equal(S, buf["Ss"][k]))
        same &= float(ld1.item()) == float(ld[k].item())
        del A, L, S
    ok = bool((info.cpu().numpy() == 0).all()) and bool(torch.isfinite(ld).all()) and same is not False and ok_graph
    flop = sum(fl.factor_flops(n - a, w, a, tile) + fl.selinv_flops(n - a, w, a, tile) for (n, w, a) in nws)
    srt = sorted(step_ms)
    del buf, mats
    torch.cuda.empty_cache()
    return {
        "instances": len(shapes), "tile": tile, "autotune_ms": tune_ms,
        "inputs": "drawn on the device" if device_inputs else "drawn on the host",
        "ms_per_pass": round(ms_step, 4), "gflops": round(flop / (ms_step / 1e3) / 1e9, 3),
        "flops_per_pass": flop,
        "solves_per_s": round(len(shapes) * 1e3 / ms_step, 3),
        "pass_ms_p50": round(srt[len(srt) // 2], 4), "pass_ms_p99": round(srt[min(len(srt) - 1, int(0.99 * len(srt)))], 4),
        "ms_per_pass_graph": None if graph_ms is None else round(graph_ms, 4),
        "graph_speedup": None if graph_ms is None else round(ms_step / graph_ms, 4),
        "plain": None if plain_same is None else {
            "ms_same_tile": round(plain_same, 3), "ms_best_tile_each": round(plain_best, 3),
            "solves_per_s_same_tile": round(len(shapes) * 1e3 / plain_same, 3),
            "solves_per_s_best_tile_each": round(len(shapes) * 1e3 / plain_best, 3)},
        "speedup_vs_plain": None if plain_same is None else {
            "same_tile": round(plain_same / ms_step, 2), "best_tile_each": round(plain_best / ms_step, 2)},
        "bitwise_equal_to_single": same,
        "kernels": {k: {"ms_per_pass": round(v[0] / steps, 3), "launches_per_pass": v[1] // max(steps, 1)}
                    for k, v in per_kind.items() if v[1]},
        "ok": ok,
    }


def main_batched(args) -> int:
    r = leg_batched(args.steps, args.warmup, tile=args.tile, plain=not args.no_plain, log=_log)
    out = {
        "metric": METRIC,
        "value": r["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_pass"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batched: {r['instances']} matrices, band order uniform on [5,000, 50,000], "
                               "half-bandwidth in {32, 128, 512}, arrow uniform on [10, 200], seeded N(0,1) "
                               "band and arrow, diagonal = row |sum| + 1",
                   "instances": r["instances"], "tile": r["tile"], "autotune_ms": r["autotune_ms"],
                   "step": "pack + batched factor (L, log det) + batched selinv, all matrices",
                   "flops_per_step": r["flops_per_pass"]},
        "solves_per_s": r["solves_per_s"],
        "plain": r["plain"],
        "speedup_vs_plain": r["speedup_vs_plain"],
        "latency_ms_p50": r["pass_ms_p50"],
        "latency_ms_p99": r["pass_ms_p99"],
        "ok": r["ok"],
        "bitwise_equal_to_single": r["bitwise_equal_to_single"],
        "kernels": r["kernels"],
    }
    print(json.dumps(out), flush=True)
    return 0 if r["ok"] else 1


def main_grad(args) -> int:
    """log det A(theta) and its gradient tr(Sigma dA/dtheta) (autograd, the
    selected inverse in the backward) on the spatio-temporal model: n_t = 50,
    n_s = 2,000, kappa = 0.5, 50 fixed effects, tile 256 (n = 100,050,
    half-bandwidth 2,002); K timed forward + backward evaluations, then a
    central-difference check of the gradient."""
    import torch
    from paper_2504_19171_amd import flops as fl
    from paper_2504_19171_amd import grad

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    model = grad.SpatioTemporal(50, 2000, 0.5, 50, seed=4, device=dev)
    tile = args.tile or 256
    fn = grad.LogDet(model, tile=tile)
    print(f"bench: model n = {model.n}, w = {model.w}, arrow {model.a}, tile {tile} ready in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    theta0 = [0.0, 0.0]

    def evaluate():
        th = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
        ld = fn(th)
        ld.backward()
        return ld, th.grad

    for _ in range(args.warmup):
        evaluate()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t1 = time.perf_counter()
        ld, g = evaluate()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
    h = 1e-5
    fd = []
    for i in range(2):
        tp = torch.tensor(theta0, dtype=torch.float64); tm = tp.clone()
        tp[i] += h; tm[i] -= h
        fd.append((float(fn(tp)) - float(fn(tm))) / (2 * h))
    g = g.tolist()
    rel = [abs(gi - fi) / abs(gi) for gi, fi in zip(g, fd)]
    ok = all(r <= 1e-6 for r in rel) and all(map(lambda x: x == x, g))
    nb, w, a = model.nb, model.w, model.a
    flop = fl.factor_flops(nb, w, a, tile) + fl.selinv_flops(nb, w, a, tile)
    ms = 1e3 * sorted(times)[len(times) // 2]
    out = {
        "metric": METRIC,
        "value": round(flop / (ms / 1e3) / 1e9, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "grad: A(theta) = blockdiag(exp(theta_1) kron(R_t, Q_s), 0) + exp(theta_2) I + Z^T Z, "
                               "Z = [I | X], n_t = 50, n_s = 2,000, kappa = 0.5, X 100,000 x 50 N(0,1); "
                               "log det and its gradient by autograd",
                   "n": model.n, "bandwidth": w, "arrow": a, "tile": tile, "theta": theta0,
                   "step": "assemble + pack + factor (forward); selinv + two trace products (backward)",
                   "flops_per_step": flop},
        "evaluations_per_s": round(1e3 / ms, 4),
        "logdet": float(ld.detach()),
        "gradient": g,
        "central_difference": {"h": h, "values": fd, "rel_diff": rel},
        "ok": bool(ok),
    }
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


def leg_served(njobs, tile=0, budget_gb=64.0, lanes=3, max_batch=8, fracs=(0.5, 0.8, 1.5), log=print):
    """A Poisson stream of the first `njobs` factor + selinv jobs of the served
    workload (inputs.serve_shapes) through the serving loop
    (paper_2504_19171_amd/serve.py) and through the plain FIFO (one job at a
    time), at fractions of the plain FIFO's capacity measured on a prefix of
    the stream; p50/p99 latency and solves/s.  Each job's matrix is drawn on
    the device from its seed when the job is admitted (its upload), and
    dropped once packed: the stream never holds more than the running jobs."""
    import numpy as np
    import torch
    from paper_2504_19171_amd import autotune
    from paper_2504_19171_amd import inputs
    from paper_2504_19171_amd import serve

    dev = torch.device("cuda:0")
    shapes = inputs.serve_shapes(njobs)
    log(f"bench: served stream of {len(shapes)} jobs (n {min(s[0] + s[2] for s in shapes)}.."
        f"{max(s[0] + s[2] for s in shapes)})")
    if tile:
        tune_ms = None
    else:
        k = min(16, len(shapes))
        mats = [inputs.arrowhead_spd_device(nb, w, a, seed, dev) for (nb, w, a, seed) in shapes[:k]]
        tile, tune_ms = autotune.tune_batch(mats, [(nb + a, w, a) for (nb, w, a, _) in shapes[:k]])
        del mats
        torch.cuda.empty_cache()
        log(f"bench: autotuner on the first {k} jobs {tune_ms} -> tile {tile}")

    def jobs_at(arrivals):
        return [serve.Job(k, nb, w, a, float(t),
                          make=(lambda nb=nb, w=w, a=a, seed=seed: inputs.arrowhead_spd_device(nb, w, a, seed, dev)))
                for k, ((nb, w, a, seed), t) in enumerate(zip(shapes, arrivals))]

    def server():
        return serve.Server(budget=int(budget_gb * 2**30), tile=tile, lanes=lanes, max_batch=max_batch)

    # capacities: a prefix of the stream, all arrived at 0
    npre = min(40, len(shapes))
    done = serve.serve_plain(jobs_at([0.0] * npre)[:npre], tile)
    mu = npre / max(j.done for j in done)
    srv = server()
    done = srv.run(jobs_at([0.0] * npre)[:npre])
    srv.close()
    mu_served = npre / max(j.done for j in done)
    log(f"bench: capacity on the first {npre} jobs: plain FIFO {mu:.2f} jobs/s, served {mu_served:.2f} jobs/s")
    rates = {}
    ok = True
    for frac in fracs:
        rng = np.random.default_rng(33)
        arr = np.cumsum(rng.exponential(1.0 / (frac * mu), len(shapes)))
        arr -= arr[0]
        res = {}
        for form in ("served", "plain"):
            jobs = jobs_at(arr)
            if form == "served":
                srv = server()
                out = srv.run(jobs)
                srv.close()
            else:
                out = serve.serve_plain(jobs, tile)
            lat = np.array([j.done - j.arrival for j in out]) * 1e3
            span = max(j.done for j in out) - min(j.arrival for j in out)
            bad = [j for j in out if not (j.info == (0, 0) and np.isfinite(j.logdet))]
            ok &= not bad
            res[form] = {"latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                         "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                         "solves_per_s": round(len(out) / span, 3)}
            if bad:
                # which jobs failed, with their (factor, selinv) status codes
                res[form]["failed"] = len(bad)
                res[form]["failed_jobs"] = [
                    {"job": j.jid, "nb": j.nb, "w": j.w, "a": j.a, "info": list(j.info),
                     "latency_ms": round((j.done - j.arrival) * 1e3, 3)} for j in bad[:10]]
            if form == "served":
                res[form]["peak_bytes_held"] = srv.peak
            for j in jobs:
                j.L = j.Sigma = None
            torch.cuda.synchronize()
            log(f"bench: {form} at {frac} x capacity: {res[form]}")
        rates[str(frac)] = dict(qps=round(frac * mu, 3), **res)
    return {"jobs": len(shapes), "tile": tile, "autotune_ms": tune_ms, "lanes": lanes, "max_batch": max_batch,
            "budget_gb": budget_gb, "rates_are_fractions_of": "the plain FIFO's capacity",
            "capacity_jobs_per_s": {"plain_fifo": round(mu, 3), "served": round(mu_served, 3), "on_jobs": npre},
            "rates": rates, "ok": bool(ok)}


def main_served(args) -> int:
    r = leg_served(args.jobs, tile=args.tile, budget_gb=args.budget_gb, lanes=args.lanes,
                   max_batch=args.max_batch, fracs=tuple(float(x) for x in args.fracs.split(",")), log=_log)
    # the headline rate: 0.8 x capacity when it was run, else the highest rate run
    top = r["rates"]["0.8" if "0.8" in r["rates"] else max(r["rates"], key=float)]["served"]
    out = {
        "metric": METRIC,
        "value": top["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": r["jobs"],
        "warmup": 0,
        "ms_per_step": round(1e3 / top["solves_per_s"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"served: {r['jobs']} jobs of a Poisson stream, n log-uniform on [2,000, 200,000], "
                               "half-bandwidth log-uniform on [16, 1,024], arrow uniform on [0, 500], seeded N(0,1) "
                               "band and arrow drawn on the device at admission, diagonal = row |sum| + 1",
                   "jobs": r["jobs"], "tile": r["tile"], "autotune_ms": r["autotune_ms"], "lanes": r["lanes"],
                   "max_batch": r["max_batch"], "budget_gb": r["budget_gb"],
                   "rates_are_fractions_of": r["rates_are_fractions_of"]},
        "capacity_jobs_per_s": r["capacity_jobs_per_s"],
        "latency_ms_p50": top["latency_ms_p50"],
        "latency_ms_p99": top["latency_ms_p99"],
        "rates": r["rates"],
        "ok": r["ok"],
    }
    print(json.dumps(out), flush=True)
    return 0 if r["ok"] else 1


def leg_small(reps=200, warmup=20):
    """The small workload (n = 2,000 + 20, w = 32, tile 64, seed 0), a latency
    case: `reps` solves of pack + factor + selinv one after another, each
    bracketed by HIP events; microseconds per solve and solves/s."""
    import numpy as np
    import torch
    from paper_2504_19171_amd import inputs
    from paper_2504_19171_amd import stiles as st
    W = WORKLOADS["small"]
    nb, w, a, b = W["nb"], W["w"], W["a"], W["b"]
    dev = torch.device("cuda:0")
    M = inputs.arrowhead_spd(nb, w, a, seed=W["seed"])
    lay = st.layout(M.n, w, a, b)
    ab = torch.from_numpy(M.ab).to(dev)
    P = torch.from_numpy(M.P).to(dev)
    C = torch.from_numpy(M.C).to(dev)
    L = torch.empty(lay.total_doubles, dtype=torch.float64, device=dev)
    S = torch.empty_like(L)
    wsf = torch.empty(lay.factor_workspace_bytes, dtype=torch.uint8, device=dev)
    wss = torch.empty(lay.selinv_workspace_bytes, dtype=torch.uint8, device=dev)

    def step():
        st.pack(ab, P, C, lay, out=L)
        _, ld, info = st.factor(L, lay, out=L, workspace=wsf)
        _, sinfo = st.selinv(L, lay, out=S, workspace=wss)
        return ld, info, sinfo
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    stream = torch.cuda.current_stream()
    for i in range(reps):
        ev[2 * i].record(stream)
        ld, info, sinfo = step()
        ev[2 * i + 1].record(stream)
    torch.cuda.synchronize()
    us = sorted(1e3 * ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(reps))
    span_ms = ev[0].elapsed_time(ev[-1])
    ok = int(info.item()) == 0 and int(sinfo.item()) == 0 and bool(np.isfinite(float(ld.item())))
    return {"workload": f"small: n = {nb:,} + {a}, half-bandwidth {w}, arrow {a}, tile {b}, seed {W['seed']}",
            "reps": reps, "warmup": warmup, "us_per_solve_p50": round(us[len(us) // 2], 2),
            "us_per_solve_p99": round(us[min(len(us) - 1, int(0.99 * len(us)))], 2),
            "solves_per_s": round(reps * 1e3 / span_ms, 2), "ok": bool(ok)}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


if __name__ == "__main__":
    sys.exit(main())
