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
                 its algorithmic work = the wave text steps of its walk x 64
                 lanes x 12 VALU instructions per bit-vector step (13 where
                 two 16-bit patterns share a lane), the steps counted by the
                 kernel's own counting variant at the timed schedule (and
                 checked against the CPU work model in bench_model.json)
  counters       issue, LDS and HBM counter figures of the same launch from
                 bench_counters.json (rocprofv3 runs of this script), reported
                 only while the pair kernel's sources are the ones they were
                 taken with
  medium         N = 50,000 (5,000 templates) at k = 1 and k = 2
  cpu_baseline   the CPU oracle (full DP, all host cores) on a bounded sample
                 of rows of the same workload, with the host's core count
  serve / batch  the served and batched forms (see their sections)

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 2]
       python bench.py --ingest-counters DIR   (rocprofv3 CSVs -> bench_counters.json)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
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
COUNTER_SOURCES = ["paper_2112_06613_amd/csrc/pairs.hip", "paper_2112_06613_amd/csrc/common.h",
                   "paper_2112_06613_amd/csrc/prep.hip"]


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


def evaluated_pairs(lengths: np.ndarray, k: int) -> int:
    cnt = np.bincount(lengths, minlength=34).astype(np.int64)
    tot = 0
    for L in range(1, 33):
        tot += int(cnt[L] * (cnt[L] - 1) // 2)
        for d in range(1, k + 1):
            if L + d <= 32:
                tot += int(cnt[L] * cnt[L + d])
    return tot


# ----------------------------------------------------------------- roofline
def counted_work(tn, seqs, k, info) -> dict:
    """Wave text steps of the pair kernel's walk at the schedule `info` ran
    with, counted by the kernel's counting variant (one extra build outside
    any timed region; the walk depends on the texts per item and packing)."""
    flags = tn.TCRNET_F_COUNT_WORK | tn.TCRNET_F_NO_AUTOTUNE | (0 if info["pack"] else tn.TCRNET_F_NO_PACK)
    with tn.Context(0, texts_per_item=info["texts_per_item"], flags=flags) as c:
        g = tn.tcrnet_build(c, seqs, k)
    gi = g.info
    assert gi["work_counted"] == 1 and gi["texts_per_item"] == info["texts_per_item"]
    return {"wave_steps": gi["wave_steps"], "wave_steps_packed": gi["wave_steps_packed"],
            "visited_texts": gi["visited_texts"], "edges": int(len(g.pairs))}


def roofline(work: dict, pair_ms: float) -> dict:
    plain = work["wave_steps"] - work["wave_steps_packed"]
    instr = WAVE * (plain * T_STEP_INSTR + work["wave_steps_packed"] * T_STEP_INSTR_PACKED)
    achieved = instr / (pair_ms * 1e-3)
    return {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_LANE_OPS / 1e12,
        "unit": "T lane-instr/s",
        "frac": achieved / PEAK_LANE_OPS,
        "kernel": "k_pairs",
        "work_per_unit": f"{WAVE} lanes x {T_STEP_INSTR} VALU instr per wave text step "
                         f"({T_STEP_INSTR_PACKED} when two patterns share a lane)",
        "units_per_launch": work["wave_steps"],
        "units_packed": work["wave_steps_packed"],
        "visited_wave_texts": work["visited_texts"],
        "units_source": "counted by the pair kernel's counting variant at the timed schedule",
        # the published step's 17 word operations per pattern and text step
        # (a packed wave step covers 128 patterns)
        "frac_logical_17op": (WAVE * T_STEP_LOGICAL * (plain + 2 * work["wave_steps_packed"])
                              / (pair_ms * 1e-3) / PEAK_LANE_OPS),
    }


def counter_figures(pair_ms: float, E: int, schedule: dict):
    """Issue, LDS and HBM figures of the timed launch from bench_counters.json
    (None, with the reason logged, once the pair kernel's sources or the
    schedule differ from the ones the counters were taken with)."""
    path = os.path.join(ROOT, "bench_counters.json")
    if not os.path.exists(path):
        log("no counter record: counters not reported")
        return None
    with open(path) as f:
        rec = json.load(f)
    if source_sha1(rec["sources"]) != rec["sources_sha1"]:
        log("pair kernel sources changed since the counters were taken: counters not reported")
        return None
    for key in ("texts_per_item", "peq_lds", "pack", "waves_per_simd"):
        if rec["schedule"].get(key) != schedule.get(key):
            log(f"counters were taken with {key}={rec['schedule'].get(key)}: counters not reported")
            return None
    c = rec["counters"]
    t = pair_ms * 1e-3
    fetch = c["FETCH_SIZE"] * 1024.0 * rec["fetch_scale"]
    write = c["WRITE_SIZE"] * 1024.0 * rec["write_scale"]
    return {
        "F_issue_valu": c["SQ_INSTS_VALU"] * WAVE / t / PEAK_LANE_OPS,
        "valu_per_unit": c["SQ_INSTS_VALU"] / rec["units"],
        "salu_per_unit": c["SQ_INSTS_SALU"] / rec["units"],
        "branch_per_unit": c["SQ_INSTS_BRANCH"] / rec["units"],
        "smem_per_unit": c["SQ_INSTS_SMEM"] / rec["units"],
        "scalar_issue_frac": c["SQ_INSTS_SALU"] * 4.0 / (t * 2.4e9 * 1024),
        "wait_frac": c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"] if c.get("SQ_WAVE_CYCLES") else None,
        "lds_bank_conflict_per_lds_instr": (c["SQ_LDS_BANK_CONFLICT"] / c["SQ_INSTS_LDS"]
                                            if c["SQ_INSTS_LDS"] else 0.0),
        "hbm_read_bytes": fetch,
        "hbm_write_bytes": write,
        "hbm_write_GBps": write / t / 1e9,
        "hbm_write_bytes_per_edge": write / E if E else None,
        "hbm_GBps": (fetch + write) / t / 1e9,
        "record": "bench_counters.json",
    }


def ingest_counters(src: str):
    """Read the rocprofv3 counter CSVs of the profiling passes under `src`
    (one subdirectory per pass, each from `python bench.py --profile-run`),
    average the pair kernel's dispatches and write bench_counters.json."""
    per = {}
    calib = {}
    for f in sorted(glob.glob(os.path.join(src, "**", "*counter_collection.csv"), recursive=True)):
        with open(f) as fh:
            rows = list(csv.DictReader(fh))
        disp = {}
        for r in rows:
            name = r["Kernel_Name"]
            d = disp.setdefault(r["Dispatch_Id"], {"name": name, "c": {}})
            d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        for d in disp.values():
            if "copyBuffer" in d["name"]:
                for k, v in d["c"].items():
                    calib.setdefault(k, []).append(v)
            elif "k_pairs<" in d["name"] and d["name"].split("k_pairs<")[1].split(">")[0].endswith("false"):
                for k, v in d["c"].items():
                    per.setdefault(k, []).append(v)
    if not per:
        sys.exit(f"no pair-kernel dispatches under {src}")
    counters = {k: float(np.mean(v)) for k, v in per.items()}
    with open(os.path.join(src, "run.json")) as f:
        run = json.load(f)
    copy_kib = run["calib_copy_mib"] * 1024.0
    rec = {
        "kernel": run["kernel"],
        "workload": run["workload"],
        "schedule": run["schedule"],
        "units": run["units"],
        "edges": run["edges"],
        "pair_kernel_ms": run["pair_kernel_ms"],
        "sources": COUNTER_SOURCES,
        "sources_sha1": source_sha1(COUNTER_SOURCES),
        "counters": counters,
        "dispatches": {k: len(v) for k, v in per.items()},
        # the calibration copy is the largest copy kernel of the run (the
        # run's other copies move its inputs and are far smaller)
        "fetch_scale": copy_kib / float(np.max(calib["FETCH_SIZE"])),
        "write_scale": copy_kib / float(np.max(calib["WRITE_SIZE"])),
        "calibration": f"one {run['calib_copy_mib']} MiB device-to-device copy: FETCH_SIZE "
                       f"{np.max(calib['FETCH_SIZE']):.1f} KiB, WRITE_SIZE {np.max(calib['WRITE_SIZE']):.1f} KiB "
                       f"for {copy_kib:.0f} KiB read and written",
    }
    with open(os.path.join(ROOT, "bench_counters.json"), "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(rec, indent=1, sort_keys=True))


# ------------------------------------------------------------------- builds
def device_build(tn, torch, seqs, k, steps, warmup, ctx):
    dev = torch.device("cuda", 0)
    chars = torch.from_numpy(seqs.chars).to(dev)
    offs = torch.from_numpy(seqs.offsets.astype(np.int64)).to(dev)
    deg = torch.empty(seqs.n, dtype=torch.int32, device=dev)
    cap = max(1 << 16, 4 * seqs.n)
    pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        E = tn.tcrnet_build_device(ctx, chars, offs, k, pairs, deg, stream)
        log(f"warmup {i}: E={E} pair kernel {ctx.last_info()['pair_kernel_ms']:.3f} ms")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        E = tn.tcrnet_build_device(ctx, chars, offs, k, pairs, deg, stream)
        infos.append(ctx.last_info())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {steps} steps: {wall * 1e3 / steps:.3f} ms/step, E={E}")
    return wall / steps, E, infos


def medium_leg(tn, torch, ctx) -> dict:
    """N = 50,000 at k = 1 and k = 2 (separate runs), device-resident."""
    import synth

    s = synth.medium()
    n = s.n
    out = {"n": n, "seed": synth.SEED_MEDIUM}
    for k in (1, 2):
        step_s, E, infos = device_build(tn, torch, s, k, 20, 3, ctx)
        pk = float(np.median([i["pair_kernel_ms"] for i in infos]))
        work = counted_work(tn, s, k, infos[-1])
        assert work["edges"] == E
        r = roofline(work, pk)
        out[f"k{k}"] = {"ms_per_step": step_s * 1e3, "pair_kernel_ms": pk, "edges": int(E),
                        "logical_pairs_per_s": n * (n - 1) // 2 / step_s,
                        "evaluated_pairs_per_s": infos[-1]["evaluated_pairs"] / step_s,
                        "edges_per_s": E / step_s,
                        "roofline_frac": r["frac"], "units_per_launch": r["units_per_launch"],
                        "schedule": {kk: infos[-1][kk] for kk in ("texts_per_item", "waves_per_simd", "peq_lds",
                                                                   "pack")}}
    return out


def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_count": os.cpu_count(), "affinity_cpus": aff, "cpu_model": model}


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
    out = {"value": pairs / dt, "unit": "pairs/s", "cores": o.threads(), "kind": "oracle",
           "sample": f"rows 0..{rows - 1} of the N={n} k={k} workload against all later rows "
                     f"({pairs} full-DP pairs, {dt:.1f} s)"}
    out.update({"host_" + kk: v for kk, v in host_info().items()})
    out["threads_used"] = o.threads()
    return out


def batch_leg(tn, ctx, reps, k: int = 1) -> dict:
    """Many repertoires in one captured launch sequence, with the schedule
    the autotuner picks for the batch shape, vs. one plain build per
    repertoire, back to back, on the same GPU (host inputs and outputs in
    both cases); the batched pair kernel priced like the plain one."""
    tot = sum(r.n for r in reps)
    t0 = time.perf_counter()
    tn.tcrnet_autotune_batch(ctx, reps, k)
    t_tune = time.perf_counter() - t0
    tuned = tn.tcrnet_autotune_get(ctx, True, tot, k)
    tn.tcrnet_build_batch(ctx, reps, k)          # warm-up (captures the graph)
    # host to host, the median of three calls (the host side -- staging,
    # the per-repertoire result arrays -- varies with the allocator's state)
    t_calls = []
    for _ in range(3):
        gs = None
        t0 = time.perf_counter()
        gs = tn.tcrnet_build_batch(ctx, reps, k)
        t_calls.append(time.perf_counter() - t0)
    t_batch = float(np.median(t_calls))
    binfo = ctx.last_info()
    for r in reps[:4]:
        tn.tcrnet_build(ctx, r, k)
    t0 = time.perf_counter()
    plain_edges = 0
    for r in reps:
        plain_edges += len(tn.tcrnet_build(ctx, r, k).pairs)
    t_plain = time.perf_counter() - t0
    batch_edges = sum(len(g.pairs) for g in gs)
    assert batch_edges == plain_edges
    # work of the batched walk at the schedule it ran with (counting variant)
    flags = tn.TCRNET_F_COUNT_WORK | tn.TCRNET_F_NO_AUTOTUNE | (0 if binfo["pack"] else tn.TCRNET_F_NO_PACK)
    with tn.Context(0, texts_per_item=binfo["texts_per_item"], flags=flags) as c:
        tn.tcrnet_build_batch(c, reps, k)
        ci = c.last_info()
    logical = sum(r.n * (r.n - 1) // 2 for r in reps)
    out = {"repertoires": len(reps), "total_sequences": tot, "k": k, "edges": batch_edges,
           "batched_ms": t_batch * 1e3, "batched_ms_calls": [round(t * 1e3, 3) for t in t_calls],
           "back_to_back_ms": t_plain * 1e3, "speedup": t_plain / t_batch,
           "batched_device_ms": binfo["build_ms"],
           "batched_pairs_per_s": logical / t_batch, "back_to_back_pairs_per_s": logical / t_plain,
           "evaluated_pairs": binfo["evaluated_pairs"],
           "schedule": {kk: binfo[kk] for kk in ("texts_per_item", "waves_per_simd", "peq_lds", "pack", "tuned")},
           "autotune_s": t_tune, "autotuned": tuned}
    work = {"wave_steps": ci["wave_steps"], "wave_steps_packed": ci["wave_steps_packed"],
            "visited_texts": ci["visited_texts"]}
    # the batch's pair kernel time is not separated from its captured launch
    # sequence; pricing the whole device time gives a lower bound of its frac
    r = roofline(work, binfo["build_ms"])
    out["roofline_frac_lower_bound"] = r["frac"]
    out["units_per_launch"] = r["units_per_launch"]
    return out


def serve_leg(tn, ctx, rep, n_requests: int, loads) -> dict:
    """Resident repertoire; Poisson arrivals of query batches of 1-4,096
    sequences (log-uniform sizes, k in {1, 2}), 20% of them inserts.  The
    saturation rate first (all requests at once), then an open-loop run at
    each fraction of it, each on a fresh index."""
    import threading

    import synth

    T = 80000
    # the trace's sizes, thresholds, kinds and query seeds do not depend on
    # the rate (only the arrival times scale), so the queries are drawn once
    trace = synth.request_trace(n_requests, 1.0)
    qs = [synth.queries(r.size, T, synth.SEED_PAPER, r.qseed) for r in trace]

    idx = tn.tcrnet_index_create(ctx, rep, 1)
    t0 = time.perf_counter()
    ts = [tn.tcrnet_submit(idx, q, r.k, r.insert) for q, r in zip(qs, trace)]
    for t in ts:
        tn.tcrnet_wait(idx, t)
    sat = n_requests / (time.perf_counter() - t0)
    idx.close()
    log(f"serve: saturation {sat:.1f} requests/s")
    out = {"requests_per_load": n_requests, "saturation_rate_hz": sat, "resident_start": rep.n, "index_k": 1,
           "loads": {}}
    for frac in loads:
        idx = tn.tcrnet_index_create(ctx, rep, 1)
        trace = synth.request_trace(n_requests, frac * sat)
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
        final = idx.size()
        idx.close()
        lat = np.array([r.info["latency_ms"] for r in res])
        dev = np.array([r.info["device_ms"] for r in res])
        que = np.array([r.info["queue_ms"] for r in res])
        size = np.array([r.size for r in trace])
        ks = np.array([r.k for r in trace])
        ins = np.array([r.insert for r in trace])
        slow = lat >= np.percentile(lat, 99)
        rec = {"offered_rate_hz": frac * sat, "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99)), "mean_device_ms": float(dev.mean()),
               "requests_per_s": n_requests / wall, "query_seqs_per_s": float(size.sum()) / wall,
               "inserts": int(ins.sum()), "resident_end": final,
               # what the slowest 1% were: time in the queue vs on the device,
               # and their size, threshold and kind
               "p99_tail": {"n": int(slow.sum()), "mean_queue_ms": float(que[slow].mean()),
                            "mean_device_ms": float(dev[slow].mean()),
                            "mean_size": float(size[slow].mean()), "frac_k2": float((ks[slow] == 2).mean()),
                            "frac_insert": float(ins[slow].mean())}}
        for name, sel in (("k1", ks == 1), ("k2", ks == 2), ("insert", ins), ("size_lt_64", size < 64),
                          ("size_ge_1024", size >= 1024)):
            if sel.any():
                rec[f"p99_ms_{name}"] = float(np.percentile(lat[sel], 99))
        out["loads"][str(frac)] = rec
        log(f"serve at {frac} x saturation: p50 {rec['p50_ms']:.3f} ms, p99 {rec['p99_ms']:.3f} ms")
    return out


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
    ap.add_argument("--no-medium", action="store_true")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-analysis", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--profile-run", metavar="DIR", default=None,
                    help="only the timed plain builds, after one device copy of --calib-copy-mib MiB "
                         "(HBM counter calibration); the run's schedule and work go to DIR/run.json")
    ap.add_argument("--calib-copy-mib", type=int, default=256)
    ap.add_argument("--ingest-counters", metavar="DIR", default=None)
    ap.add_argument("--batch-only", action="store_true",
                    help="profiling aid: tune the batched form (256 repertoires), then run --steps "
                         "batched launches and print their timings; no bench line")
    args = ap.parse_args()
    if args.ingest_counters:
        ingest_counters(args.ingest_counters)
        return
    if args.gpus != 1:
        print(f"bench.py: the network build runs on one GPU (asked for --gpus {args.gpus}); "
              "the path is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2112_06613_amd as tn
    import synth

    tn.load_library()
    log(f"library {tn.version()}, device {torch.cuda.get_device_name(0)}")
    if args.batch_only:
        reps = synth.batch()
        with tn.Context(0) as bctx:
            tn.tcrnet_autotune_batch(bctx, reps, 1)
            tn.tcrnet_build_batch(bctx, reps, 1)  # warm-up (captures the graph)
            ms = []
            for _ in range(args.steps):
                t0 = time.perf_counter()
                tn.tcrnet_build_batch(bctx, reps, 1)
                ms.append((time.perf_counter() - t0) * 1e3)
            info = bctx.last_info()
        print(json.dumps({"batch_only": True, "repertoires": len(reps), "host_ms": ms,
                          "device_ms": info["build_ms"],
                          "schedule": {kk: info[kk] for kk in ("texts_per_item", "waves_per_simd", "peq_lds",
                                                               "pack", "tuned")}}))
        return

    k = 1
    seqs = synth.paper_scale()
    n = seqs.n
    ev_pairs = evaluated_pairs(seqs.lengths(), k)
    ctx = tn.Context(0)
    if args.profile_run:
        nb = args.calib_copy_mib << 20
        a = torch.empty(nb // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        step_s, E, infos = device_build(tn, torch, seqs, k, args.steps, 0, ctx)
        pk = float(np.mean([i["pair_kernel_ms"] for i in infos]))
        sched = {kk: infos[-1][kk] for kk in ("texts_per_item", "waves_per_simd", "peq_lds", "pack")}
        ctx.close()
        work = counted_work(tn, seqs, k, infos[-1])
        os.makedirs(args.profile_run, exist_ok=True)
        with open(os.path.join(args.profile_run, "run.json"), "w") as f:
            json.dump({"kernel": "k_pairs<%s, %d, false>" % ("true" if sched["peq_lds"] else "false", k),
                       "workload": "plain network build, N=800,000 synthetic CDR3b, k=1",
                       "schedule": sched, "units": work["wave_steps"], "edges": int(E), "pair_kernel_ms": pk,
                       "calib_copy_mib": args.calib_copy_mib}, f, indent=1)
        log(f"profile run: pair kernel {pk:.3f} ms, {work['wave_steps']} wave steps")
        return
    if args.autotune:
        tn.tcrnet_autotune(ctx, seqs, k)
    peak_meas, peak_s = tn.tcrnet_valu_peak(ctx)
    log(f"measured VALU issue rate {peak_meas / 1e12:.2f} T lane-instr/s ({peak_s * 1e3:.1f} ms probe)")
    form_rates = tn.tcrnet_valu_rates(ctx)
    log("issue rate by form (T lane-instr/s): " +
        ", ".join(f"{kk} {v / 1e12:.1f}" for kk, v in form_rates.items()))
    step_s, E, infos = device_build(tn, torch, seqs, k, args.steps, args.warmup, ctx)
    pk_ms = float(np.mean([i["pair_kernel_ms"] for i in infos]))
    assert all(i["evaluated_pairs"] == ev_pairs for i in infos)
    schedule = {kk: infos[-1][kk] for kk in ("texts_per_item", "waves_per_simd", "peq_lds", "pack")}
    log("counting the pair kernel's work ...")
    work = counted_work(tn, seqs, k, infos[-1])
    assert work["edges"] == E
    rl = roofline(work, pk_ms)
    cf = counter_figures(pk_ms, E, schedule)
    rl["traffic"] = (cf["hbm_read_bytes"] + cf["hbm_write_bytes"]) if cf else None
    rl["traffic_unit"] = "B per launch"
    rl["peak_measured"] = peak_meas / 1e12
    rl["frac_of_measured"] = rl["achieved"] * 1e12 / peak_meas
    # per instruction form, in units of one wave64 instruction per SIMD per
    # 4 clocks (39.3 T lane-instr/s): plain 32-bit logic/adds issue near 1.45,
    # packed, 3-operand, min, shift, popcount and compare forms near 0.95
    single = PEAK_LANE_OPS / 2
    rl["issue_rates"] = {kk: round(v / single, 3) for kk, v in form_rates.items()}
    rl["issue_rates_unit"] = "x one wave64 instruction per SIMD per 4 clocks"
    # the CPU work model of the same walk (bench_model.json), where it was
    # computed at this schedule
    model = load_model("paper_n800000_k1")
    assert ev_pairs == model["evaluated_pairs"]
    trav = model["traversal"]
    if trav["texts_per_item"] == schedule["texts_per_item"] and trav["pack"] == bool(schedule["pack"]):
        rl["units_model"] = trav["wave_steps"]
        rl["units_model_agrees"] = trav["wave_steps"] == work["wave_steps"]
    pair_work = ev_pairs * model["mean_exit_steps"] * T_STEP_INSTR
    rl["per_pair_work_lane_instr"] = pair_work
    rl["traversal_saving"] = pair_work / (rl["achieved"] * 1e12 * pk_ms * 1e-3)
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
        "build_device_ms": float(np.mean([i["build_ms"] for i in infos])),
        "schedule": schedule,
        "roofline": rl,
        "counters": cf,
    }
    log("host-to-host build ...")
    out["host_to_host"] = host_to_host(tn, ctx, seqs, k)
    if not args.no_medium:
        log("N = 50,000 at k = 1 and 2 ...")
        out["medium"] = medium_leg(tn, torch, ctx)
    if not args.no_analysis:
        log("network analysis ...")
        out["analysis"] = analysis_leg(tn, ctx, seqs, k)
    if not args.no_batch:
        log("batched form (256 repertoires) ...")
        out["batch"] = batch_leg(tn, ctx, synth.batch())
    if not args.no_serve:
        log("served form ...")
        out["serve"] = serve_leg(tn, ctx, seqs, args.serve_requests, (0.25, 0.5, 0.8))
        out["serve"]["plain_rebuild_ms"] = step_s * 1e3
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(seqs, k, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
