"""Algorithmic-work model of the named workloads -- writes ../bench_model.json.

Test/benchmark infrastructure: it calls only ``oracle/`` and ``synth/``.

For each workload it records
  * evaluated_pairs: pairs (i < j) with |len_i - len_j| <= k (the pairs the
    length filter keeps; counted from the length histogram);
  * mean_exit_steps: the mean, over a seeded uniform sample of those pairs,
    of the text steps the exact final-diagonal early exit needs (rows = the
    longer string; computed from the oracle's full DP table, see
    oracle_exit_step), with its standard error.
The benchmark prices a build as evaluated_pairs * mean_exit_steps * T_step.

Usage: python -m oracle.workload_model [--samples 400000]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "bench_model.json")

WORKLOADS = {
    "small_n2000_k1": (synth.small, 1),
    "medium_n50000_k1": (synth.medium, 1),
    "medium_n50000_k2": (synth.medium, 2),
    "paper_n800000_k1": (synth.paper_scale, 1),
}


def length_pairs(lengths: np.ndarray, k: int):
    """Bucket pairs (L, L2) with L <= L2 <= L + k and their pair counts."""
    cnt = np.bincount(lengths, minlength=34).astype(np.int64)
    out = []
    for L in range(1, 33):
        for d in range(0, k + 1):
            L2 = L + d
            if L2 > 32:
                continue
            c = cnt[L] * (cnt[L] - 1) // 2 if d == 0 else cnt[L] * cnt[L2]
            if c > 0:
                out.append((L, L2, int(c)))
    return out


def sample_pairs(lengths: np.ndarray, k: int, n_samples: int, seed: int):
    bp = length_pairs(lengths, k)
    w = np.array([c for _, _, c in bp], dtype=np.float64)
    rng = np.random.default_rng(seed)
    choice = rng.choice(len(bp), size=n_samples, p=w / w.sum())
    members = {L: np.flatnonzero(lengths == L) for L in range(1, 33)}
    pi = np.empty(n_samples, dtype=np.uint32)
    pj = np.empty(n_samples, dtype=np.uint32)
    for b, (L, L2, _) in enumerate(bp):
        sel = np.flatnonzero(choice == b)
        if not len(sel):
            continue
        a = rng.choice(members[L], size=len(sel))
        c = rng.choice(members[L2], size=len(sel))
        if L == L2:  # redraw self-pairs
            same = a == c
            while same.any():
                c[same] = rng.choice(members[L2], size=int(same.sum()))
                same = a == c
        pi[sel], pj[sel] = a, c
    return pi, pj, int(w.sum())


def model(seqs, k: int, n_samples: int, seed: int = 1) -> dict:
    lengths = seqs.lengths()
    pi, pj, evaluated = sample_pairs(lengths, k, n_samples, seed)
    steps = oracle.Oracle().exit_steps(seqs, pi, pj, k).astype(np.float64)
    n = seqs.n
    return {
        "n": n,
        "k": k,
        "logical_pairs": n * (n - 1) // 2,
        "evaluated_pairs": evaluated,
        "mean_exit_steps": float(steps.mean()),
        "stderr_exit_steps": float(steps.std(ddof=1) / np.sqrt(len(steps))),
        "samples": n_samples,
        "sample_seed": seed,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=400000)
    args = ap.parse_args()
    out = {"note": "written by oracle/workload_model.py; exit steps from the oracle's full DP table",
           "workloads": {}}
    for name, (gen, k) in WORKLOADS.items():
        out["workloads"][name] = model(gen(), k, args.samples)
        print(name, out["workloads"][name])
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
