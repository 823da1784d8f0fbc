"""Brute-force checks of the oracle -- TEST INFRASTRUCTURE ONLY.

``bfs_distances`` computes the edit distance straight from its definition in
the paper's Methods ("Levenshtein distance"): the least number of
single-character insertions, deletions and substitutions turning one string
into another.  It runs a breadth-first search over the graph whose nodes are
all strings over a tiny alphabet and whose edges are single edits, so it
involves no recursion or table at all.  An optimal edit script can be reordered
into deletions, then substitutions, then insertions, so no intermediate string
is longer than the longer endpoint; the search universe is capped one longer
than that anyway.
"""
from __future__ import annotations

from collections import deque
from itertools import product


def all_strings(alphabet: str, max_len: int) -> list[str]:
    out = [""]
    for L in range(1, max_len + 1):
        out += ["".join(p) for p in product(alphabet, repeat=L)]
    return out


def _neighbours(s: str, alphabet: str, cap: int):
    for p in range(len(s)):                      # deletions
        yield s[:p] + s[p + 1:]
    for p in range(len(s)):                      # substitutions
        for c in alphabet:
            if c != s[p]:
                yield s[:p] + c + s[p + 1:]
    if len(s) < cap:                             # insertions
        for p in range(len(s) + 1):
            for c in alphabet:
                yield s[:p] + c + s[p:]


def bfs_distances(alphabet: str, max_len: int) -> dict[tuple[str, str], int]:
    """Edit distance between every ordered pair of strings of length <= max_len."""
    cap = max_len + 1
    nodes = all_strings(alphabet, max_len)
    dist = {}
    for src in nodes:
        seen = {src: 0}
        q = deque([src])
        while q:
            u = q.popleft()
            for v in _neighbours(u, alphabet, cap):
                if v not in seen:
                    seen[v] = seen[u] + 1
                    q.append(v)
        for dst in nodes:
            dist[(src, dst)] = seen[dst]
    return dist


def k1_adjacent(a: str, b: str) -> bool:
    """Closed form of lev(a, b) <= 1 (equal; one substitution; one indel)."""
    if len(a) == len(b):
        return sum(x != y for x, y in zip(a, b)) <= 1
    if len(a) < len(b):
        a, b = b, a
    if len(a) != len(b) + 1:
        return False
    return any(a[:p] + a[p + 1:] == b for p in range(len(a)))


def hamming(a: str, b: str) -> int:
    assert len(a) == len(b)
    return sum(x != y for x, y in zip(a, b))
