"""The oracle pins catch plausible mistakes planted in the oracle (CPU only).

Each mutant is a copy of the oracle source with one plausible slip (a dropped
term, a wrong sign, an off-by-one, a wrong comparison), built into a temporary
library; the condensed pin suite below must reject every mutant and accept the
unmodified source.
"""
import os

import numpy as np
import pytest

import codes
from oracle import build as obuild
from oracle import bzref
from paper_2603_29942_amd import synth

MUTANTS = {
    "bound_drops_plus_one": ("int v = g + 1 - (k - kj);", "int v = g - (k - kj);"),
    "bound_uses_rank_wrong": ("int v = g + 1 - (k - kj);", "int v = g + 1 - kj;"),
    "strict_termination": ("(!round_mode || j == m) && Lgj >= U", "(!round_mode || j == m) && Lgj > U"),
    "round_check_first_matrix": ("(!round_mode || j == m) && Lgj >= U", "(!round_mode || j == 1) && Lgj >= U"),
    "round_check_every_matrix": ("(!round_mode || j == m) && Lgj >= U", "(!round_mode || j >= 1) && Lgj >= U"),
    "singleton_off_by_one": ("int U = n - k + 1, L = 1;", "int U = n - k, L = 1;"),
    "elimination_sign": ("(A[i * n + t] + (p - f) * A[rank * n + t]) % p", "(A[i * n + t] + f * A[rank * n + t]) % p"),
    "coefficient_dropped": ("        for (int a = 1; a < p; a++) {\n            for (int t = 0; t < n; t++) next[t]",
                            "        for (int a = 1; a < p - 1; a++) {\n            for (int t = 0; t < n; t++) next[t]"),
    "weight_counts_ones": ("wt += (c[t] != 0);", "wt += (c[t] == 1);"),
    "used_columns_first": ("if (!used[c]) order[nu++] = c;", "if (used[c]) order[nu++] = c;"),
    "brute_force_radix": ("while (i < k && msg[i] == p - 1) msg[i++] = 0;", "while (i < k && msg[i] == p - 2) msg[i++] = 0;"),
    "rows_start_at_last": ("for (int i = last + 1; i < x->k; i++) {", "for (int i = last; i < x->k; i++) {"),
}


def pin_suite(L):
    """Condensed pins; returns the list of failed pin names."""
    failed = []

    def check(name, cond):
        if not cond:
            failed.append(name)

    spec = codes.golden("classical_codes.json")
    G = codes.ternary_golay()
    d, hist = bzref.brute_force(3, G, _L=L)
    check("golay_A", {w: int(c) for w, c in enumerate(hist) if c} ==
          {int(w): c for w, c in spec["ternary_golay_11_6_5"]["weight_distribution"].items()})
    check("golay_d", bzref.min_distance(3, G, _L=L)["d"] == 5)
    r = bzref.min_distance(3, codes.extended_golay(), _L=L)
    check("ext_golay_trace", r["stages"] == [(1, 1, 6, 6, 6, 3), (1, 2, 6, 6, 6, 4),
                                             (2, 1, 30, 6, 6, 5), (2, 2, 30, 6, 6, 6)]
          and r["terminated_by"] == 0)
    tetra = np.array(spec["tetracode_4_2_3"]["generator"], dtype=np.uint8)
    check("tetracode_trace", bzref.min_distance(3, tetra, _L=L)["stages"] == [(1, 1, 2, 3, 3, 3)])
    # round mode (derived traces: only the last matrix of a round ends a run)
    check("tetracode_round_trace", bzref.min_distance(3, tetra, check="round", _L=L)["stages"] ==
          [(1, 1, 2, 3, 3, 3), (1, 2, 2, 3, 3, 4)])
    r = bzref.min_distance(3, codes.extended_golay(), check="round", _L=L)
    check("ext_golay_round_trace", r["stages"] == [(1, 1, 6, 6, 6, 3), (1, 2, 6, 6, 6, 4),
                                                   (2, 1, 30, 6, 6, 5), (2, 2, 30, 6, 6, 6)])
    for n, k in [(7, 3), (6, 4), (7, 5)]:
        check("mds_d", bzref.min_distance(7, codes.reed_solomon(7, n, k), _L=L)["d"] == n - k + 1)
    # histogram identity on small random codes, and d against brute force
    for p, n, k, seed in [(3, 9, 4, 1), (7, 7, 3, 2), (3, 12, 5, 3), (3, 8, 6, 4), (7, 9, 2, 5)]:
        G = synth.random_generator(p, n, k, seed, stream=77)
        if codes.rank_mod_p(G, p) < k:
            continue
        dbf, A = bzref.brute_force(p, G, _L=L)
        check("d_vs_brute", bzref.min_distance(p, G, _L=L)["d"] == dbf)
        r = bzref.min_distance(p, G, no_termination=True, histograms=True, _L=L)
        for j in range(1, r["m"] + 1):
            tot = sum(r["hist"][s] for s, st in enumerate(r["stages"]) if st[1] == j)
            check("hist_identity", all(int(tot[w]) * (p - 1) == int(A[w]) for w in range(1, n + 1)))
    for seed in range(8):
        p, G = synth.config_code(1, seed)
        dbf, _ = bzref.brute_force(p, G, _L=L)
        check("cfg1_vs_brute", bzref.min_distance(p, G, _L=L)["d"] == dbf)
    return failed


def _build_variant(tmp_path, name, old, new):
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, name
    path = os.path.join(tmp_path, name + ".c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    with open(os.path.join(tmp_path, "bzref.h"), "w") as f:
        f.write(open(os.path.join(os.path.dirname(obuild.SRC), "bzref.h")).read())
    return bzref.load(obuild.build(src=path, lib=os.path.join(tmp_path, name + ".so")))


def test_pristine_passes(tmp_path):
    L = bzref.load(obuild.build(lib=os.path.join(tmp_path, "pristine.so")))
    assert pin_suite(L) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_caught(tmp_path, name):
    old, new = MUTANTS[name]
    L = _build_variant(str(tmp_path), name, old, new)
    assert pin_suite(L), f"mutant {name} passed every pin"
