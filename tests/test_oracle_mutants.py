"""The oracle's pins have teeth: plant plausible mistakes in copies of the
oracle's C source (on the CPU, in a temporary directory) and check that the
pin suite rejects every one of them."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle.checks import bfs_distances

ORACLE_C = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "drop_insertion": ("      if (ins < best) best = ins;\n", ""),
    "drop_deletion": ("      int best = del;\n", "      int best = sub;\n"),
    "sub_cost_always_one": ("(a[i - 1] != b[j - 1] ? 1 : 0)", "1"),
    "sub_cost_never": ("(a[i - 1] != b[j - 1] ? 1 : 0)", "0"),
    "index_shift": ("(a[i - 1] != b[j - 1] ? 1 : 0)", "(a[i - 1] != b[j > 1 ? j - 2 : 0] ? 1 : 0)"),
    "base_case_shift": ("D[i * w + 0] = i;", "D[i * w + 0] = i > 0 ? i - 1 : 0;"),
    "strict_threshold": ("      int l = (int)(offsets[j + 1] - offsets[j]);\n      if (oracle_lev(a, m, b, l) <= k) {",
                         "      int l = (int)(offsets[j + 1] - offsets[j]);\n      if (oracle_lev(a, m, b, l) < k) {"),
    "degree_one_end": ("      degree[(*out_pairs)[2 * e + 1]] += 1;\n", ""),
    "self_pairs": ("for (uint32_t j = (uint32_t)i + 1; j < n; ++j)", "for (uint32_t j = (uint32_t)i; j < n; ++j)"),
    "wrong_corner": ("int r = D[m * (n + 1) + n];", "int r = D[m * (n + 1) + (n > 0 ? n - 1 : 0)];"),
}


def pin_failures(o: "oracle.Oracle") -> list[str]:
    """Run the pins; return the names of those that fail."""
    bad = []
    if o.lev("ACCA", "ACGG") != 2:
        bad.append("worked_example")
    if o.lev("kitten", "sitting") != 3:
        bad.append("kitten")
    dist = bfs_distances("AR", 4)
    if any(o.lev(a, b) != d for (a, b), d in dist.items()):
        bad.append("bfs")
    s = synth.Seqs.from_list(["AAAA", "AAAR", "RAAA", "AWNR", "AANR"])
    e, d = o.build(s, 1)
    if [tuple(x) for x in e.tolist()] != [(0, 1), (0, 2), (1, 4), (3, 4)] or d.tolist() != [2, 2, 1, 1, 2]:
        bad.append("adjacency_example")
    sm = synth.repertoire(400, 40, 3)
    e, d = o.build(sm, 1)
    e1, d1 = o.k1_build(sm)
    if not (np.array_equal(e, e1) and np.array_equal(d, d1)):
        bad.append("k1_witness")
    return bad


def test_unmutated_oracle_passes(orc):
    assert pin_failures(orc) == []


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    src = open(ORACLE_C).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mut = tmp_path / "oracle.c"
    mut.write_text(src.replace(old, new))
    others = [os.path.join(os.path.dirname(ORACLE_C), f) for f in ("k1.c", "graph.c")]
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", str(mut), *others, "-o", str(lib)],
                   check=True)
    o = oracle.Oracle(str(lib))
    assert pin_failures(o), f"mutant {name} passed every pin"
