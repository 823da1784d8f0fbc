"""Algorithmic-work model of the named workloads -- writes ../bench_model.json.

Benchmark infrastructure: it prices the pair kernel's launches for the
roofline; it decides no edge and imports neither the HIP library nor the
test oracle (walk.c computes its own DP distances).

For each workload it records
  * evaluated_pairs: pairs (i < j) with |len_i - len_j| <= k (the pairs the
    length filter keeps; counted from the length histogram);
  * mean_exit_steps: the mean, over a seeded uniform sample of those pairs,
    of the text steps the exact final-diagonal early exit needs (rows = the
    longer string; from a full DP table, see wm_exit_step), with its
    standard error -- the per-pair work;
  * wave_steps: the text steps of the pair kernel's traversal, where a wave
    of 64 patterns walks the lexicographically sorted texts of a work item,
    jumps past every prefix group on which all its lanes ended early, and
    starts each visited text after the residues it shares with the previous
    one (up to RESUME of them)
    (replayed by walk.c over a seeded uniform sample of work items, or all
    items when few), with the number of visited texts and the standard error.
The benchmark prices a build as wave_steps * 64 lanes * T_step.

Usage: python -m workmodel [--samples 400000]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import subprocess

import numpy as np

import synth

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libworkmodel.so")
_lib = None


def build_lib(out: str = LIB_PATH) -> str:
    """Compile walk.c with gcc (OpenMP)."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", os.path.join(_HERE, "walk.c"),
                    "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        lib.wm_exit_step.restype = ctypes.c_int
        lib.wm_exit_step.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        lib.wm_exit_steps.restype = None
        lib.wm_exit_steps.argtypes = [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int, vp]
        lib.wm_items.restype = None
        lib.wm_items.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, vp, vp]
        _lib = lib
    return _lib


def _chars(seqs):
    return np.ascontiguousarray(seqs.chars) if seqs.chars.size else np.zeros(1, np.uint8)


def exit_step(a: str, b: str, k: int) -> tuple[int, int]:
    """(exit step, distance) of one pair from the model's own DP table."""
    a, b = a.encode(), b.encode()
    lev = ctypes.c_int()
    s = _load().wm_exit_step(a, len(a), b, len(b), k, ctypes.byref(lev))
    return s, lev.value


def exit_steps(seqs, pi, pj, k: int) -> np.ndarray:
    pi = np.ascontiguousarray(pi, dtype=np.uint32)
    pj = np.ascontiguousarray(pj, dtype=np.uint32)
    out = np.zeros(max(1, len(pi)), dtype=np.int32)
    chars = _chars(seqs)
    offs = np.ascontiguousarray(seqs.offsets, dtype=np.uint64)
    _load().wm_exit_steps(chars.ctypes.data, offs.ctypes.data, pi.ctypes.data, pj.ctypes.data, len(pi), k,
                          out.ctypes.data)
    return out[:len(pi)]


def work_items(seqs, seq, gend, items, k: int, resume: int):
    """(text steps, texts visited) of each work item (rows of items: gbase,
    np, tb, te, tri, width over sorted positions; seq: sorted position ->
    input id; gend: n x 8 prefix-group ends; resume: steps a visited text
    can take over from the previous one)."""
    seq = np.ascontiguousarray(seq, dtype=np.uint32)
    gend = np.ascontiguousarray(gend, dtype=np.uint32)
    items = np.ascontiguousarray(items, dtype=np.uint32).reshape(-1, 6)
    steps = np.zeros(max(1, len(items)), dtype=np.uint64)
    texts = np.zeros(max(1, len(items)), dtype=np.uint64)
    chars = _chars(seqs)
    offs = np.ascontiguousarray(seqs.offsets, dtype=np.uint64)
    _load().wm_items(chars.ctypes.data, offs.ctypes.data, seq.ctypes.data, gend.ctypes.data, items.ctypes.data,
                     len(items), k, resume, steps.ctypes.data, texts.ctypes.data)
    return steps[:len(items)], texts[:len(items)]


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "bench_model.json")

# (generator, k, texts per work item: the library's default for the size,
# about n / 195 rounded down to a power of two in 512..16384)
WORKLOADS = {
    "small_n2000_k1": (synth.small, 1, 256),
    "medium_n50000_k1": (synth.medium, 1, 256),
    "medium_n50000_k2": (synth.medium, 2, 256),
    "paper_n800000_k1": (synth.paper_scale, 1, 8192),
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


ALPHABET = "ARNDCQEGHILKMFPSTWYV"
SORT_RESIDUES = 8    # residues in the sort key (as many as the prefix-group depths)
DEPTHS = 8           # prefix depths with a group end
RESUME = 6           # text steps a visited text can take over from the previous one
WAVE = 64


def code_matrix(seqs):
    """n x 32 residue codes (0 past the end) and the lengths."""
    lut = np.zeros(256, dtype=np.uint8)
    for i, c in enumerate(ALPHABET):
        lut[ord(c)] = i
    L = seqs.lengths().astype(np.int64)
    n = seqs.n
    M = np.zeros((n, 32), dtype=np.uint8)
    row = np.repeat(np.arange(n), L)
    col = np.arange(len(seqs.chars)) - np.repeat(seqs.offsets[:-1].astype(np.int64), L)
    M[row, col] = lut[seqs.chars]
    return M, L


def sorted_order(M, L):
    """Sorted position -> input id: by length, the first SORT_RESIDUES codes,
    then input position."""
    keys = [np.arange(len(L))] + [M[:, q] for q in reversed(range(SORT_RESIDUES))] + [L]
    return np.lexsort(keys).astype(np.uint32)


def group_ends(M, L, order):
    """gend[s, d-1]: first sorted position after s whose length or first d
    residues differ (n when none)."""
    n = len(order)
    Ms, Ls = M[order], L[order]
    gend = np.empty((n, DEPTHS), dtype=np.uint32)
    same = Ls[1:] == Ls[:-1]
    for d in range(1, DEPTHS + 1):
        same = same & (Ms[1:, d - 1] == Ms[:-1, d - 1])
        start = np.ones(n, dtype=bool)
        start[1:] = ~same
        starts = np.flatnonzero(start)
        gid = np.cumsum(start) - 1
        ends = np.append(starts[1:], n).astype(np.uint32)
        gend[:, d - 1] = ends[gid]
    return gend


PACK_MAX_LEN = 16    # patterns this short run two to a lane (k < 16)


def group_width(m: int, k: int, pack: bool) -> int:
    """Patterns per work item of a bucket pair with pattern length m."""
    return 2 * WAVE if pack and m <= PACK_MAX_LEN and k < 16 else WAVE


def diag_texts(T: int) -> int:
    """Texts per work item of a triangle row block's first T texts."""
    return max(64, T // 8 // 64 * 64)


def plan_items(L_sorted, k: int, T: int, pack: bool = True) -> np.ndarray:
    """The pair kernel's work items of a one-segment build: rows (gbase, np,
    tb, te, tri, width) over sorted positions; width = patterns per item
    (64, or 128 when two patterns share a lane).  A triangle row block's
    first T texts come in chunks of diag_texts(T) (an item there may be
    empty: tb >= te), the rest in chunks of T."""
    cnt = np.bincount(L_sorted, minlength=34)
    off = np.concatenate([[0], np.cumsum(cnt)])
    rows = []
    for m in range(1, 33):
        W = group_width(m, k, pack)
        for delta in range(0, k + 1):
            nl = m - delta
            if nl < 1:
                continue
            npat, ntxt = int(cnt[m]), int(cnt[nl])
            if delta > 0:
                if npat == 0 or ntxt == 0:
                    continue
                g = np.arange((npat + W - 1) // W)
                c = np.arange((ntxt + T - 1) // T)
                G, C = np.meshgrid(g, c, indexing="ij")
                gb = off[m] + W * G
                tb = off[nl] + T * C
                te = np.minimum(off[nl] + ntxt, tb + T)
                npg = np.minimum(W, npat - W * G)
                rows.append(np.stack([gb, npg, tb, te, np.zeros_like(gb), np.full_like(gb, W)], -1).reshape(-1, 6))
            else:
                if npat < 2:
                    continue
                # a row block's first T texts (its diagonal) in chunks of
                # diag_texts(T), the rest in chunks of T
                Td = diag_texts(T)
                for bk in range((npat - 1 + T - 1) // T):
                    nrow = min(T, npat - bk * T)
                    p0 = off[m] + bk * T
                    ntb = npat - bk * T
                    g = np.arange((nrow + W - 1) // W)
                    for t0, nt, Tc in ((p0, min(ntb, T), Td), (p0 + T, ntb - T, T)):
                        if nt <= 0:
                            continue
                        c = np.arange((nt + Tc - 1) // Tc)
                        G, C = np.meshgrid(g, c, indexing="ij")
                        gb = p0 + W * G
                        tb = t0 + Tc * C
                        te = np.minimum(t0 + nt, tb + Tc)
                        tb = np.maximum(tb, gb + 1)
                        npg = np.minimum(W, nrow - W * G)
                        rows.append(np.stack([gb, npg, tb, te, np.ones_like(gb), np.full_like(gb, W)],
                                             -1).reshape(-1, 6))
    if not rows:
        return np.zeros((0, 6), dtype=np.uint32)
    return np.concatenate(rows).astype(np.uint32)


def traversal(seqs, k: int, T: int, max_items: int, seed: int = 1, resume: int = RESUME,
              pack: bool = True) -> dict:
    """Text steps and visited texts of the traversal over all work items
    (exact when the items number at most max_items, else estimated from a
    seeded uniform sample of max_items items)."""
    M, L = code_matrix(seqs)
    order = sorted_order(M, L)
    gend = group_ends(M, L, order)
    items = plan_items(L[order], k, T, pack)
    total = len(items)
    exact = total <= max_items
    if exact:
        pick = items
    else:
        pick = items[np.random.default_rng(seed).choice(total, size=max_items, replace=False)]
    steps, texts = work_items(seqs, order, gend, pick, k, resume)
    steps = steps.astype(np.float64)
    texts = texts.astype(np.float64)
    scale = total / max(1, len(pick))
    packed = pick[:, 5] > WAVE
    out = {"texts_per_item": T, "resume_depth": resume, "pack": bool(pack), "items": total,
           "items_packed": int((items[:, 5] > WAVE).sum()), "items_modelled": int(len(pick)),
           "exact": bool(exact),
           "wave_steps": float(steps.sum() * scale), "visited_texts": float(texts.sum() * scale),
           "wave_steps_packed": float(steps[packed].sum() * scale)}
    out["stderr_wave_steps"] = 0.0 if exact else float(steps.std(ddof=1) * total / np.sqrt(len(pick)))
    return out


def model(seqs, k: int, n_samples: int, seed: int = 1, T: int = 16384, max_items: int = 1 << 20) -> dict:
    lengths = seqs.lengths()
    pi, pj, evaluated = sample_pairs(lengths, k, n_samples, seed)
    steps = exit_steps(seqs, pi, pj, k).astype(np.float64)
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
        "traversal": traversal(seqs, k, T, max_items, seed),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=400000)
    args = ap.parse_args()
    out = {"note": "written by workmodel (python -m workmodel); exit steps from a full DP table; "
                   "traversal = text steps of the sorted-text walk with prefix-group jumps",
           "workloads": {}}
    for name, (gen, k, T) in WORKLOADS.items():
        out["workloads"][name] = model(gen(), k, args.samples, T=T)
        print(name, out["workloads"][name])
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
