"""Seeded synthetic CDR3-beta repertoires (shared input source).

This module only draws strings and workload parameters; it holds none of the
edit-distance arithmetic, so both the test oracle and the GPU library may take
their inputs from it.  The fast path is ``gen.c`` (built into ``libsynth.so``
by ``__graft_entry__.build()``); ``generate_py`` is an equivalent pure-Python
version of the same draws, used by a test to check that both agree byte for
byte.

Workload recipe (a stand-in for the paper's SONIA-generated and empirical
repertoires, which are not available): T templates 'C' + uniform residues + 'F'
of length round(N(14, 2)) clipped to [6, 25]; each sequence is a random
template plus Poisson(1.5) random substitutions / insertions / deletions.
Residues are the 20 amino acids in the order of the paper's Methods section
("Combination of amino acids").
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

ALPHABET = "ARNDCQEGHILKMFPSTWYV"
MAX_LEN = 32
_MASK = (1 << 64) - 1
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")

# Seeds of the named workloads (recorded so that every run draws the same data).
SEED_SMALL = 20211213      # N=2,000, 200 templates
SEED_MEDIUM = 20211214     # N=50,000, 5,000 templates
SEED_PAPER = 20211215      # N=800,000, 80,000 templates
SEED_BATCH = 20211216      # 256 repertoires
SEED_SERVE = 20211217      # request trace


@dataclass
class Seqs:
    """Concatenated ASCII strings with n+1 offsets (uint64)."""

    chars: np.ndarray    # uint8, total length offsets[-1]
    offsets: np.ndarray  # uint64, n+1

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def to_list(self) -> list[str]:
        b = self.chars.tobytes()
        o = self.offsets
        return [b[o[i]:o[i + 1]].decode("ascii") for i in range(self.n)]

    @staticmethod
    def from_list(strs) -> "Seqs":
        enc = [s.encode("ascii") if isinstance(s, str) else bytes(s) for s in strs]
        offs = np.zeros(len(enc) + 1, dtype=np.uint64)
        if enc:
            offs[1:] = np.cumsum([len(e) for e in enc], dtype=np.uint64)
        chars = np.frombuffer(b"".join(enc), dtype=np.uint8).copy()
        return Seqs(chars, offs)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def subset(self, idx) -> "Seqs":
        strs = self.to_list()
        return Seqs.from_list([strs[i] for i in idx])

    def concat(self, other: "Seqs") -> "Seqs":
        offs = np.concatenate([self.offsets, other.offsets[1:] + self.offsets[-1]])
        return Seqs(np.concatenate([self.chars, other.chars]), offs.astype(np.uint64))


# ----------------------------------------------------------------- SplitMix64
class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood 2014), bit-identical to gen.c."""

    def __init__(self, seed: int):
        self.s = seed & _MASK

    def next(self) -> int:
        self.s = (self.s + 0x9E3779B97F4A7C15) & _MASK
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def below(self, n: int) -> int:
        return ((self.next() >> 32) * n) >> 32

    def u01(self) -> float:
        return float(self.next() >> 11) * (1.0 / 9007199254740992.0)


def _poisson15(r: SplitMix64) -> int:
    L = 0.22313016014842982  # exp(-1.5), same literal as gen.c
    n = 0
    p = r.u01()
    while p > L:
        n += 1
        p *= r.u01()
    return n


def _template_len(r: SplitMix64) -> int:
    s = 0
    for _ in range(12):
        s += r.next() >> 40
    L = (2 * s + (2 << 24) + (1 << 23)) >> 24
    return max(6, min(25, L))


def generate_py(tseed: int, n_templates: int, sseed: int, n_seqs: int) -> Seqs:
    """Pure-Python twin of ``synth_generate`` in gen.c (slow; small n only)."""
    tr = SplitMix64(tseed)
    tmpl = []
    for _ in range(n_templates):
        L = _template_len(tr)
        t = [4] + [tr.below(20) for _ in range(L - 2)] + [13]
        tmpl.append(t)
    sr = SplitMix64(sseed)
    out = []
    for _ in range(n_seqs):
        s = list(tmpl[sr.below(n_templates)])
        for _ in range(_poisson15(sr)):
            typ = sr.below(3)
            if typ == 0:
                p = sr.below(len(s))
                c = sr.below(19)
                s[p] = c if c < s[p] else c + 1
            elif typ == 1:
                p = sr.below(len(s) + 1)
                c = sr.below(20)
                if len(s) < MAX_LEN:
                    s.insert(p, c)
            else:
                p = sr.below(len(s))
                if len(s) > 1:
                    del s[p]
        out.append("".join(ALPHABET[c] for c in s))
    return Seqs.from_list(out)


# ------------------------------------------------------------------ C binding
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        lib.synth_generate.restype = ctypes.c_int64
        lib.synth_generate.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                       ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def generate(tseed: int, n_templates: int, sseed: int, n_seqs: int) -> Seqs:
    """Draw n_seqs sequences from n_templates templates (templates from tseed,
    sequences from sseed)."""
    lib = _load()
    chars = np.empty(max(1, n_seqs * MAX_LEN), dtype=np.uint8)
    offs = np.empty(n_seqs + 1, dtype=np.uint64)
    nb = lib.synth_generate(tseed & _MASK, n_templates, sseed & _MASK, n_seqs,
                            chars.ctypes.data, offs.ctypes.data)
    if nb < 0:
        raise ValueError("synth_generate: bad arguments")
    return Seqs(chars[:nb].copy(), offs)


def repertoire(n_seqs: int, n_templates: int, seed: int) -> Seqs:
    """A repertoire: templates from ``seed``, sequences from ``seed + 1``."""
    return generate(seed, n_templates, seed + 1, n_seqs)


def queries(n_seqs: int, n_templates: int, seed: int, qseed: int) -> Seqs:
    """New sequences drawn from the same template set as ``repertoire(.., seed)``."""
    return generate(seed, n_templates, qseed, n_seqs)


# ------------------------------------------------------- named workload shapes
def small(seed: int = SEED_SMALL) -> Seqs:
    return repertoire(2000, 200, seed)


def medium(seed: int = SEED_MEDIUM) -> Seqs:
    return repertoire(50000, 5000, seed)


def paper_scale(seed: int = SEED_PAPER) -> Seqs:
    return repertoire(800000, 80000, seed)


def derive_seed(base: int, r: int) -> int:
    """Seed of sub-stream r (one SplitMix64 output of base + r)."""
    return SplitMix64((base + r * 0x9E3779B97F4A7C15) & _MASK).next()


def batch_sizes(n_reps: int = 256, lo: int = 1000, hi: int = 40000,
                seed: int = SEED_BATCH) -> list[int]:
    """Repertoire sizes log-uniform in [lo, hi]."""
    r = SplitMix64(seed)
    a, b = math.log(lo), math.log(hi)
    return [int(round(math.exp(a + (b - a) * r.u01()))) for _ in range(n_reps)]


def batch(n_reps: int = 256, lo: int = 1000, hi: int = 40000, seed: int = SEED_BATCH) -> list[Seqs]:
    """Independent repertoires of uneven size, each with N/10 templates."""
    out = []
    for i, n in enumerate(batch_sizes(n_reps, lo, hi, seed)):
        s = derive_seed(seed, i)
        out.append(repertoire(n, max(1, int(round(n / 10))), s))
    return out


@dataclass
class Request:
    t_arrival: float     # seconds after trace start
    size: int            # number of query sequences
    k: int               # threshold of the query
    insert: bool         # also insert the sequences into the repertoire
    qseed: int           # seed of the query strings


def request_trace(n_requests: int, rate_hz: float, max_size: int = 4096,
                  p_insert: float = 0.2, ks=(1, 2), seed: int = SEED_SERVE) -> list[Request]:
    """Poisson arrivals; sizes log-uniform in [1, max_size]; k uniform in ks."""
    r = SplitMix64(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += -math.log(1.0 - r.u01()) / rate_hz
        size = int(round(math.exp(math.log(max_size) * r.u01())))
        k = ks[r.below(len(ks))]
        ins = r.u01() < p_insert
        out.append(Request(t, max(1, min(max_size, size)), k, ins, derive_seed(seed, 1000003 + i)))
    return out
