"""Benchmark: the paper-scale network build on one MI355X.

Workload: N = 800,000 seeded synthetic CDR3-beta strings (80,000 templates +
Poisson(1.5) edits), threshold k = 1, inputs resident in HBM when the timed
region starts.  A step is one whole build through the device entry point
(validate/encode -> length sort -> bucket plan -> pair kernel -> canonical
sorted edge list + degrees).  Prints ONE JSON line.

  value          logical pairs/s = N(N-1)/2 / step time
  roofline       the pair kernel against the 32-bit VALU issue peak of
                 gfx950 (256 CU x 128 lanes x 2.4 GHz = 78.6 T lane-instr/s:
                 two waves of a SIMD issue plain 32-bit ops per 4 clocks);
                 its algorithmic work = the text steps of the sorted-text walk
                 with prefix-group jumps x 64 lanes x 12 VALU instructions per
                 bit-vector step (13 where two 16-bit patterns share a lane;
                 wave steps counted exactly by the CPU work model in
                 bench_model.json)
  cpu_baseline   the CPU oracle (full DP, all host cores) on a bounded sample
                 of rows of the same workload
  serve / batch  the served and batched forms (see their sections)

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pairs/s + edges/s at N=8e5,k=1 vs VALU roofline; p50/p99 query latency"
PEAK_LANE_OPS = 256 * 128 * 2.4e9         # 32-bit VALU lane-instructions per second (dual issue)
WAVE = 64
T_STEP_INSTR = 12                          # gfx950 VALU instructions per Myers/Hyyro step
T_STEP_INSTR_PACKED = 13                   # the same with two 16-bit patterns per lane (one more)
T_STEP_LOGICAL = 17                        # word operations of the published step


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_model(name: str) -> dict:
    with open(os.path.join(ROOT, "bench_model.json")) as f:
        return json.load(f)["workloads"][name]


def source_sha1(files) -> str:
    h = hashlib.sha1()
    for rel in files:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counted_traffic(texts_per_item: int, peq_lds: int):
    """HBM bytes per pair-kernel launch from the committed FETCH_SIZE /
    WRITE_SIZE counts (bench_traffic.json), each scaled by what the same
    counter reads for a device copy of known size; None once the kernel's
    sources, the work-item size or the kernel variant differ from those the
    counters were taken with."""
    path = os.path.join(ROOT, "bench_traffic.json")
    if not os.path.exists(path):
        log("no HBM counter record: traffic not reported")
        return None
    with open(path) as f:
        rec = json.load(f)
    if source_sha1(rec["sources"]) != rec["sources_sha1"]:
        log("pair kernel sources changed since the HBM counters were taken: traffic not reported")
        return None
    if texts_per_item != rec["texts_per_item"]:
        log(f"HBM counters were taken at {rec['texts_per_item']} texts per item: traffic not reported")
        return None
    if peq_lds != rec["peq_lds"]:
        log(f"HBM counters were taken with peq_lds={rec['peq_lds']}: traffic not reported")
        return None
    kib = 1024.0
    return (rec["fetch_kib"] * kib * rec["fetch_scale"] + rec["write_kib"] * kib * rec["write_scale"])


def evaluated_pairs(lengths: np.ndarray, k: int) -> int:
    cnt = np.bincount(lengths, minlength=34).astype(np.int64)
    tot = 0
    for L in range(1, 33):
        tot += int(cnt[L] * (cnt[L] - 1) // 2)
        for d in range(1, k + 1):
            if L + d <= 32:
                tot += int(cnt[L] * cnt[L + d])
    return tot


def plain_build(tn, torch, seqs, k, steps, warmup, ctx):
    dev = torch.device("cuda", 0)
    chars = torch.from_numpy(seqs.chars).to(dev)
    offs = torch.from_numpy(seqs.offsets.astype(np.int64)).to(dev)
    deg = torch.empty(seqs.n, dtype=torch.int32, device=dev)
    cap = max(1 << 16, 4 * seqs.n)
    pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        E = tn.tcrnet_build_device(ctx, chars, offs, k, pairs, deg, stream)
        log(f"warmup {i}: E={E} pair kernel {ctx.last_info()['pair_kernel_ms']:.2f} ms")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        E = tn.tcrnet_build_device(ctx, chars, offs, k, pairs, deg, stream)
        infos.append(ctx.last_info())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {steps} steps: {wall * 1e3 / steps:.2f} ms/step, E={E}")
    return wall / steps, E, infos


def cpu_baseline(seqs, k, target_s: float) -> dict:
    import oracle

    o = oracle.Oracle()
    n = seqs.n
    # the oracle hands rows to its threads in chunks of 16 (OpenMP dynamic
    # schedule), so the sample is a whole number of chunks per thread: one
    # round first, then as many rounds as fit the target time
    chunk = 16 * o.threads()
    rows = min(n, chunk)
    t0 = time.perf_counter()
    o.build(seqs, k, row_lo=0, row_hi=rows)
    dt = time.perf_counter() - t0
    rounds = max(1, int(round(target_s / max(dt, 1e-3))))
    if rounds > 1 and rows < n:
        rows = min(n, chunk * rounds)
        t0 = time.perf_counter()
        o.build(seqs, k, row_lo=0, row_hi=rows)
        dt = time.perf_counter() - t0
    pairs = sum(n - 1 - i for i in range(rows))
    return {"value": pairs / dt, "unit": "pairs/s", "cores": o.threads(), "kind": "oracle",
            "sample": f"rows 0..{rows - 1} of the N={n} k={k} workload against all later rows "
                      f"({pairs} full-DP pairs, {dt:.1f} s)"}


def batch_leg(tn, ctx, reps, k: int = 1) -> dict:
    """Many repertoires in one captured launch sequence vs. one plain build
    per repertoire, back to back, on the same GPU (host inputs and outputs in
    both cases)."""
    tot = sum(r.n for r in reps)
    tn.tcrnet_build_batch(ctx, reps, k)          # warm-up (captures the graph)
    t0 = time.perf_counter()
    gs = tn.tcrnet_build_batch(ctx, reps, k)
    t_batch = time.perf_counter() - t0
    for r in reps[:4]:
        tn.tcrnet_build(ctx, r, k)
    t0 = time.perf_counter()
    plain_edges = 0
    for r in reps:
        plain_edges += len(tn.tcrnet_build(ctx, r, k).pairs)
    t_plain = time.perf_counter() - t0
    batch_edges = sum(len(g.pairs) for g in gs)
    assert batch_edges == plain_edges
    logical = sum(r.n * (r.n - 1) // 2 for r in reps)
    return {"repertoires": len(reps), "total_sequences": tot, "k": k, "edges": batch_edges,
            "batched_ms": t_batch * 1e3, "back_to_back_ms": t_plain * 1e3, "speedup": t_plain / t_batch,
            "batched_pairs_per_s": logical / t_batch, "back_to_back_pairs_per_s": logical / t_plain}


def serve_leg(tn, ctx, rep, n_requests: int, log) -> dict:
    """Resident repertoire; Poisson arrivals of query batches of 1-4,096
    sequences (k in {1, 2}), 20% of them inserts.  Saturation rate first
    (all requests at once), then an open-loop run at half of it."""
    import threading

    import synth

    T = 80000
    idx = tn.tcrnet_index_create(ctx, rep, 1)
    trace = synth.request_trace(n_requests, 1.0)
    qs = [synth.queries(r.size, T, synth.SEED_PAPER, r.qseed) for r in trace]
    # closed loop: everything submitted at once
    t0 = time.perf_counter()
    ts = [tn.tcrnet_submit(idx, q, r.k, r.insert) for q, r in zip(qs, trace)]
    for t in ts:
        tn.tcrnet_wait(idx, t)
    sat = n_requests / (time.perf_counter() - t0)
    log(f"serve: saturation {sat:.1f} requests/s")
    # open loop at half the saturation rate, fresh index
    idx.close()
    idx = tn.tcrnet_index_create(ctx, rep, 1)
    rate = 0.5 * sat
    trace = synth.request_trace(n_requests, rate)
    qs = [synth.queries(r.size, T, synth.SEED_PAPER, r.qseed) for r in trace]
    tickets = [None] * n_requests

    def submitter():
        start = time.perf_counter()
        for i, r in enumerate(trace):
            delay = start + r.t_arrival - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tickets[i] = tn.tcrnet_submit(idx, qs[i], r.k, r.insert)

    th = threading.Thread(target=submitter)
    t0 = time.perf_counter()
    th.start()
    th.join()
    res = [tn.tcrnet_wait(idx, t) for t in tickets]
    wall = time.perf_counter() - t0
    lat = np.array([r.info["latency_ms"] for r in res])
    dev = np.array([r.info["device_ms"] for r in res])
    nq = sum(r.size for r in trace)
    final = idx.size()
    idx.close()
    return {"requests": n_requests, "offered_rate_hz": rate, "saturation_rate_hz": sat,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_device_ms": float(dev.mean()), "requests_per_s": n_requests / wall,
            "query_seqs_per_s": nq / wall, "inserts": int(sum(r.insert for r in trace)),
            "resident_start": rep.n, "resident_end": final, "index_k": 1}


def host_to_host(tn, ctx, seqs, k) -> dict:
    """One build from host strings to host edges and degrees (PCIe copies
    and the host-side validation included)."""
    tn.tcrnet_build(ctx, seqs, k)
    t0 = time.perf_counter()
    g = tn.tcrnet_build(ctx, seqs, k)
    dt = time.perf_counter() - t0
    n = seqs.n
    return {"ms": dt * 1e3, "pairs_per_s": n * (n - 1) // 2 / dt, "edges": int(len(g.pairs))}


def analysis_leg(tn, ctx, seqs, k) -> dict:
    """Network analysis of the built network: components/LCC, the site-
    percolation curve at 21 removal fractions, degree statistics (host edge
    list in, host results out)."""
    g = tn.tcrnet_build(ctx, seqs, k)
    n = seqs.n
    out = {"edges": int(len(g.pairs))}
    tn.tcrnet_components(ctx, g.pairs, n)
    t0 = time.perf_counter()
    labels, sizes, nc, lcc = tn.tcrnet_components(ctx, g.pairs, n)
    out["components_ms"] = (time.perf_counter() - t0) * 1e3
    out["n_components"], out["lcc"] = int(nc), int(lcc)
    order = np.random.default_rng(20211215).permutation(n).astype(np.uint32)   # random removal order
    removed = np.round(np.linspace(0.0, 1.0, 21) * n).astype(np.uint32)
    t0 = time.perf_counter()
    curve = tn.tcrnet_robustness(ctx, g.pairs, n, order, removed)
    out["robustness_ms"] = (time.perf_counter() - t0) * 1e3
    out["lcc_norm2"] = [round(float(x), 6) for x in tn.lcc_norm2(curve, removed, n)]
    t0 = time.perf_counter()
    st = tn.tcrnet_graph_stats(ctx, g.pairs, n)
    out["graph_stats_ms"] = (time.perf_counter() - t0) * 1e3
    out["max_degree"] = int(st["max_degree"])
    out["triangles"] = int(st["triangles"])
    out["assortativity"] = float(st["assortativity"])
    out["avg_clustering"] = float(st["avg_clustering"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-analysis", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the path is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2112_06613_amd as tn
    import synth

    tn.load_library()
    log(f"library {tn.version()}, device {torch.cuda.get_device_name(0)}")
    if args.calib_copy_mib:
        nb = args.calib_copy_mib << 20
        a = torch.empty(nb // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log(f"calibration copy of {args.calib_copy_mib} MiB done")

    k = 1
    seqs = synth.paper_scale()
    n = seqs.n
    model = load_model("paper_n800000_k1")
    ev_pairs = evaluated_pairs(seqs.lengths(), k)
    assert ev_pairs == model["evaluated_pairs"]
    ctx = tn.Context(0)
    if args.autotune:
        tn.tcrnet_autotune(ctx, seqs, k)
    peak_meas, peak_s = tn.tcrnet_valu_peak(ctx)
    log(f"measured VALU issue rate {peak_meas / 1e12:.2f} T lane-instr/s ({peak_s * 1e3:.1f} ms probe)")
    step_s, E, infos = plain_build(tn, torch, seqs, k, args.steps, args.warmup, ctx)
    pk_ms = float(np.mean([i["pair_kernel_ms"] for i in infos]))
    assert all(i["evaluated_pairs"] == ev_pairs for i in infos)
    trav = model["traversal"]
    T_used = infos[-1]["texts_per_item"]
    pack_used = bool(infos[-1]["pack"])
    priced = T_used == trav["texts_per_item"] and pack_used == trav["pack"]
    if not priced:
        log(f"schedule (T={T_used}, pack={pack_used}) differs from the work model's "
            f"(T={trav['texts_per_item']}, pack={trav['pack']}): roofline not priced")
    plain_steps = trav["wave_steps"] - trav["wave_steps_packed"]
    work_instr = WAVE * (plain_steps * T_STEP_INSTR + trav["wave_steps_packed"] * T_STEP_INSTR_PACKED)
    achieved = work_instr / (pk_ms * 1e-3)
    pair_work = ev_pairs * model["mean_exit_steps"] * T_STEP_INSTR
    logical = n * (n - 1) // 2
    out = {
        "metric": METRIC,
        "value": logical / step_s,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "plain network build, N=800,000 synthetic CDR3b (80,000 templates, "
                               "Poisson(1.5) edits, seed 20211215), k=1, inputs resident in HBM",
                   "n": n, "k": k, "seed": synth.SEED_PAPER},
        "edges": int(E),
        "edges_per_s": E / step_s,
        "evaluated_pairs": ev_pairs,
        "evaluated_pairs_per_s": ev_pairs / step_s,
        "pair_kernel_ms": pk_ms,
        "schedule": {kk: infos[-1][kk] for kk in ("texts_per_item", "waves_per_simd", "peq_lds", "pack")},
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12 if priced else None,
            "peak": PEAK_LANE_OPS / 1e12,
            "unit": "T lane-instr/s",
            "frac": achieved / PEAK_LANE_OPS if priced else None,
            "traffic": counted_traffic(T_used, infos[-1]["peq_lds"]),
            "traffic_unit": "B per launch",
            "kernel": "k_pairs",
            "work_per_unit": f"{WAVE} lanes x {T_STEP_INSTR} VALU instr per wave text step "
                             f"({T_STEP_INSTR_PACKED} when two patterns share a lane)",
            "units_per_launch": trav["wave_steps"],
            "units_packed": trav["wave_steps_packed"],
            "visited_wave_texts": trav["visited_texts"],
            # the published step's 17 word operations per pattern and text step
            # (a packed wave step covers 128 patterns)
            "frac_logical_17op": (WAVE * T_STEP_LOGICAL * (plain_steps + 2 * trav["wave_steps_packed"])
                                  / (pk_ms * 1e-3) / PEAK_LANE_OPS) if priced else None,
            "peak_measured": peak_meas / 1e12,
            "frac_of_measured": achieved / peak_meas if priced else None,
            "per_pair_work_lane_instr": pair_work,
            "traversal_saving": pair_work / work_instr,
            # every kept pair priced at its own exit step, per second, over the
            # peak: above 1 because the walk skips most of that work
            "frac_pair_work": pair_work / (pk_ms * 1e-3) / PEAK_LANE_OPS,
        },
    }
    log("host-to-host build ...")
    out["host_to_host"] = host_to_host(tn, ctx, seqs, k)
    if not args.no_analysis:
        log("network analysis ...")
        out["analysis"] = analysis_leg(tn, ctx, seqs, k)
    if not args.no_batch:
        log("batched form (256 repertoires) ...")
        out["batch"] = batch_leg(tn, ctx, synth.batch())
    if not args.no_serve:
        log("served form ...")
        out["serve"] = serve_leg(tn, ctx, seqs, args.serve_requests, log)
        out["serve"]["plain_rebuild_ms"] = step_s * 1e3
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(seqs, k, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
