"""CPU-only checks of the GPU library: host logic and the exported C ABI.

No GPU work is launched here: the shared host/device code is compiled with
g++ and run on the CPU, and the HIP library is only loaded and called on
argument-validation paths that return before touching a device.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_29942_amd", "csrc")
HEADER = os.path.join(ROOT, "include", "bz.h")


def test_host_checks(tmp_path):
    exe = os.path.join(str(tmp_path), "host_checks")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-DBZ_HD=inline", "-I", CSRC, "-I",
                    os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host_checks.cpp"), "-o", exe],
                   check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    lines = out.stdout.splitlines()
    assert [l.split(" (")[0] for l in lines] == ["OK top row", "OK bits", "OK blocks", "OK pairs", "OK digits",
                                                   "OK arith", "OK schedule", "OK parallel schedule", "OK unrank"]


SWEEP_MUTANTS = {
    "sweep_skips_first_row": ("for (int L = s + 1; L < k; L += UR) {", "for (int L = s + 2; L < k; L += UR) {"),
    "sweep_drops_last_group_row": ("const int nr = k - L < UR ? k - L : UR;", "const int nr = k - L < UR ? k - L - 1 : UR;"),
    "sweep_repeats_a_row": ("for (int L = s + 1; L < k; L += UR) {", "for (int L = s + 1; L < k; L += UR - 1) {"),
    "sweep_counts_whole_groups": ("done += nr;", "done += UR;"),
}


@pytest.mark.parametrize("name", sorted(SWEEP_MUTANTS))
def test_host_replay_catches_sweep_mutants(tmp_path, name):
    """A row skipped, repeated or miscounted in the last-row sweep (the loop
    the enumeration kernel and the host replay share) fails the replay."""
    old, new = SWEEP_MUTANTS[name]
    root = tmp_path / "tree"
    (root / "pkg" / "csrc").mkdir(parents=True)
    (root / "include").mkdir()
    for f in ("bz_arith.hpp", "bz_state.hpp"):
        src = open(os.path.join(CSRC, f)).read()
        if f == "bz_state.hpp":
            assert src.count(old) == 1, name
            src = src.replace(old, new)
        (root / "pkg" / "csrc" / f).write_text(src)
    (root / "include" / "bz.h").write_text(open(HEADER).read())
    exe = os.path.join(str(tmp_path), "host_checks")
    subprocess.run(["g++", "-std=c++17", "-O1", "-DBZ_HD=inline", "-I", str(root / "pkg" / "csrc"), "-I",
                    str(root / "include"), os.path.join(ROOT, "tests", "host_checks.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode != 0 and "OK unrank" not in out.stdout, name


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(bz_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def bzlib():
    from paper_2603_29942_amd import bz
    if not os.path.exists(bz.LIB_PATH):
        from paper_2603_29942_amd import build
        build.build()
    return bz


def test_exports(bzlib):
    names = _declared()
    assert set(names) == set(bzlib.EXPORTS)
    L = bzlib.lib()
    for name in names:
        assert hasattr(L, name), name
    syms = subprocess.run(["nm", "-D", "--defined-only", bzlib.LIB_PATH], capture_output=True, text=True).stdout
    for name in names:
        assert re.search(rf"\bT {name}$", syms, re.M), name


def test_struct_layout(bzlib, tmp_path):
    """The ctypes mirrors match the C layout that gcc computes from include/bz.h."""
    src = os.path.join(str(tmp_path), "layout.c")
    with open(src, "w") as f:
        f.write('#include <stdio.h>\n#include <stddef.h>\n#include "bz.h"\n'
                'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(bz_stage),'
                ' sizeof(bz_result), offsetof(bz_result, stages), offsetof(bz_result, codewords_total),'
                ' sizeof(bz_options), offsetof(bz_options, max_codewords), offsetof(bz_options, trace_out),'
                ' sizeof(bz_code), offsetof(bz_code, g_offset), sizeof(bz_batch_options),'
                ' offsetof(bz_batch_options, hip_stream), offsetof(bz_batch_options, enum_ms));'
                ' printf("%zu %zu %zu\\n", sizeof(bz_server_options), offsetof(bz_server_options, max_codewords),'
                ' offsetof(bz_server_options, max_n));'
                ' printf("%zu %zu %zu\\n", offsetof(bz_result, info), offsetof(bz_options, no_ahead),'
                ' offsetof(bz_batch_options, code_ms_out));'
                ' printf("%zu %zu %zu\\n", offsetof(bz_server_options, admit_budget), sizeof(bz_server_options),'
                ' offsetof(bz_options, pair_tables));'
                ' return 0;}\n')
    exe = os.path.join(str(tmp_path), "layout")
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    c_vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    py_vals = [ctypes.sizeof(bzlib.bz_stage), ctypes.sizeof(bzlib.bz_result), bzlib.bz_result.stages.offset,
               bzlib.bz_result.codewords_total.offset, ctypes.sizeof(bzlib.bz_options),
               bzlib.bz_options.max_codewords.offset, bzlib.bz_options.trace_out.offset,
               ctypes.sizeof(bzlib.bz_code), bzlib.bz_code.g_offset.offset, ctypes.sizeof(bzlib.bz_batch_options),
               bzlib.bz_batch_options.hip_stream.offset, bzlib.bz_batch_options.enum_ms.offset,
               ctypes.sizeof(bzlib.bz_server_options), bzlib.bz_server_options.max_codewords.offset,
               bzlib.bz_server_options.max_n.offset, bzlib.bz_result.info.offset, bzlib.bz_options.no_ahead.offset,
               bzlib.bz_batch_options.code_ms_out.offset, bzlib.bz_server_options.admit_budget.offset,
               ctypes.sizeof(bzlib.bz_server_options), bzlib.bz_options.pair_tables.offset]
    assert c_vals == py_vals


def test_defaults_and_status_strings(bzlib):
    o = bzlib.bz_default_options()
    assert (o.check, o.no_termination, o.identity_skip, o.histograms, o.max_codewords) == (0, 0, 1, 0, 0)
    for st, text in [(0, "ok"), (-1, "invalid argument"), (-3, "generator matrix has rank < k"),
                     (-6, "work limit reached")]:
        assert bzlib.bz_status_str(st) == text


def test_argument_errors_need_no_device(bzlib):
    G = np.zeros((4, 10), dtype=np.uint8)
    for p, Gx in [(5, G), (2, G), (3, np.zeros((11, 10), dtype=np.uint8)),
                  (3, np.zeros((65, 70), dtype=np.uint8)), (7, np.zeros((2, 129), dtype=np.uint8))]:
        st, _ = bzlib.bz_min_distance(p, Gx)
        assert st == bzlib.ERR_ARG
    o = bzlib.bz_default_options()
    o.check = 5
    st, _ = bzlib.bz_min_distance_ex(3, G, o)
    assert st == bzlib.ERR_ARG


def test_batch_argument_errors_need_no_device(bzlib):
    """An invalid code descriptor rejects the whole batch before any device work."""
    G = np.zeros((4, 10), dtype=np.uint8)
    ok = [(3, G), (7, G)]
    for bad in [(5, G), (3, np.zeros((11, 10), dtype=np.uint8)), (7, np.zeros((65, 70), dtype=np.uint8))]:
        buf, descs = bzlib.pack_batch(ok + [bad])
        st, _, _ = bzlib.bz_min_distance_batch(buf, descs)
        assert st == bzlib.ERR_ARG
    buf, descs = bzlib.pack_batch(ok)
    descs[1].g_offset = buf.size - 8  # generator runs past the buffer
    st, _, _ = bzlib.bz_min_distance_batch(buf, descs)
    assert st == bzlib.ERR_ARG
    buf, descs = bzlib.pack_batch(ok)
    o = bzlib.bz_default_batch_options()
    assert (o.check, o.no_termination, o.identity_skip, o.max_codewords) == (0, 0, 1, 0)
    o.check = 9
    st, _, _ = bzlib.bz_min_distance_batch(buf, descs, o)
    assert st == bzlib.ERR_ARG
    st, res, _ = bzlib.bz_min_distance_batch(buf, (bzlib.bz_code * 0)())
    assert st == bzlib.OK and res == []
    o = bzlib.bz_default_options()
    o.histograms = 1  # without a buffer
    st, _ = bzlib.bz_min_distance_ex(3, G, o)
    assert st == bzlib.ERR_ARG
    L = bzlib.lib()
    assert L.bz_sliced_op(7, bzlib.OP_KAT_ADD, 1, 32, ctypes.c_void_p(8), ctypes.c_void_p(8),
                          ctypes.c_void_p(8), 1, None) == bzlib.ERR_ARG
    assert L.bz_sliced_pack(5, 0, 1, 32, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == bzlib.ERR_ARG


def test_server_option_errors_need_no_device(bzlib):
    import ctypes
    o = bzlib.bz_server_options()
    bzlib.lib().bz_default_server_options(ctypes.byref(o))
    assert (o.slots, o.policy, o.check, o.identity_skip) == (1024, 0, 0, 1)
    h = ctypes.c_void_p()
    for field, value in [("policy", 1), ("slots", -1), ("check", 7), ("max_n", 129), ("blocks_per_cu", -1),
                         ("admit_budget", -1.0)]:
        bad = bzlib.bz_server_options()
        ctypes.pointer(bad)[0] = o
        setattr(bad, field, value)  # policy 1 needs the network's parameters
        assert bzlib.lib().bz_server_start(ctypes.byref(bad), ctypes.byref(h)) == bzlib.ERR_ARG
    assert bzlib.lib().bz_server_submit(None, 3, 10, 4, None, 0) == bzlib.ERR_ARG


def test_noalloc_and_release_argument_errors_need_no_device(bzlib):
    """The entry point that allocates nothing rejects options it does not carry
    and sizes beyond the library's limits before any device work; releasing a
    device that was never set up does nothing."""
    L = bzlib.lib()
    G = ctypes.c_void_p(8)  # never read: every call below fails its argument checks
    out = bzlib.bz_result()
    for field in ("histograms", "timing", "cooperative"):
        o = bzlib.bz_default_options()
        setattr(o, field, 1)
        assert L.bz_min_distance_noalloc(3, 10, 4, G, ctypes.byref(o), ctypes.byref(out)) == bzlib.ERR_ARG
    o = bzlib.bz_default_options()
    o.trace_out = (ctypes.c_uint64 * 4)()
    assert L.bz_min_distance_noalloc(3, 10, 4, G, ctypes.byref(o), ctypes.byref(out)) == bzlib.ERR_ARG
    o = bzlib.bz_default_options()
    for p, n, k in [(3, 129, 4), (7, 100, 65), (5, 10, 4), (3, 10, 11)]:
        assert L.bz_min_distance_noalloc(p, n, k, G, ctypes.byref(o), ctypes.byref(out)) == bzlib.ERR_ARG
    o.device = -1
    assert L.bz_min_distance_noalloc(3, 10, 4, G, ctypes.byref(o), ctypes.byref(out)) == bzlib.ERR_ARG
    assert L.bz_min_distance_noalloc(3, 10, 4, None, None, ctypes.byref(out)) == bzlib.ERR_ARG
    assert L.bz_release(-1) == bzlib.ERR_ARG and L.bz_release(16) == bzlib.ERR_ARG
    assert L.bz_release(3) == bzlib.OK  # never set up
    ms, ops = ctypes.c_float(), ctypes.c_double()
    for op, iters, bpc in [(6, 1, 1), (-1, 1, 1), (0, 0, 1), (0, 1, 9)]:
        assert L.bz_valu_rate(op, iters, bpc, ctypes.c_void_p(8), ctypes.byref(ms), ctypes.byref(ops), None) == bzlib.ERR_ARG


def test_cooperative_launch_is_rejected(bzlib):
    """The reserved cooperative field must be 0 on every entry point that has
    it; the check comes before any device work."""
    G = np.zeros((4, 10), dtype=np.uint8)
    o = bzlib.bz_default_options()
    o.cooperative = 1
    st, _ = bzlib.bz_min_distance_ex(3, G, o)
    assert st == bzlib.ERR_ARG
    buf, descs = bzlib.pack_batch([(3, G)])
    ob = bzlib.bz_default_batch_options()
    ob.cooperative = 1
    st, _, _ = bzlib.bz_min_distance_batch(buf, descs, ob)
    assert st == bzlib.ERR_ARG
    so = bzlib.bz_server_options()
    bzlib.lib().bz_default_server_options(ctypes.byref(so))
    so.cooperative = 1
    h = ctypes.c_void_p()
    assert bzlib.lib().bz_server_start(ctypes.byref(so), ctypes.byref(h)) == bzlib.ERR_ARG
