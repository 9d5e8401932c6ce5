"""GPU parity of the batched path: many codes of different p, n and k in one
decomposition launch and one persistent enumeration launch.  Every code's
result in a batch must equal, field for field, the plain one-code path's and
(where the oracle finishes in seconds) the oracle's: status, d, m, ranks, the
stage trace with its per-stage counts, the termination reason."""
import sys

import numpy as np
import pytest

import codes
from paper_2603_29942_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("status", "d", "m", "ranks", "stages", "terminated_by", "codewords_total")
LIMIT = 1 << 36


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bz():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_2603_29942_amd import bz as _bz
    _bz.lib()
    return _bz


def same(a, b, label):
    for key in KEYS:
        assert a[key] == b[key], (label, key, a[key], b[key])


def mixed_codes():
    """Classical codes, trivial and degenerate codes, config-1 draws and random
    shapes across every word count (n up to 128) and both fields."""
    rng = np.random.default_rng([21, 0])
    out = [(3, codes.ternary_golay()), (3, codes.extended_golay()),
           (3, np.array([[1, 1, 1, 0], [0, 1, 2, 1]], dtype=np.uint8)),
           (7, codes.reed_solomon(7, 7, 3)), (7, codes.reed_solomon(7, 6, 3)),
           (3, codes.hamming(3, 3)), (7, codes.hamming(2, 7)),
           (3, codes.repetition(10, 3)), (7, codes.zero_sum(12, 7)), (3, codes.full_space(5, 3))]
    out += [synth.config_code(1, s) for s in range(6)]
    for p, n, k in [(3, 20, 1), (7, 15, 5), (3, 33, 11), (7, 40, 13), (3, 64, 20), (7, 70, 3),
                    (3, 100, 33), (7, 128, 40), (3, 128, 64), (7, 9, 9), (3, 97, 40), (7, 33, 32)]:
        out.append((p, rng.integers(0, p, size=(k, n), dtype=np.uint8)))
    G = rng.integers(0, 3, size=(6, 30), dtype=np.uint8)
    G[5] = (G[0] + G[1]) % 3  # rank 5 < k
    out.append((3, G))
    G = rng.integers(0, 7, size=(5, 20), dtype=np.uint8)
    G[2, 7] = 7  # entry outside F_7
    out.append((7, G))
    return out


def test_batch_mixed_equals_plain_and_oracle(bz, oracle):
    cs = mixed_codes()
    say(f"case batch mixed: {len(cs)} codes")
    res = bz.min_distance_batch(cs, max_codewords=LIMIT, wait_timeout_s=30)
    assert len(res) == len(cs)
    for i, ((p, G), r) in enumerate(zip(cs, res)):
        plain = bz.min_distance(p, G, max_codewords=LIMIT)
        same(r, plain, f"code {i} p={p} shape={G.shape} vs plain")
        if plain["codewords_total"] < 2e8:
            same(r, oracle.min_distance(p, G, max_codewords=LIMIT), f"code {i} vs oracle")
    statuses = [r["status"] for r in res]
    assert statuses.count(bz.ERR_RANK) == 1 and statuses.count(bz.ERR_VALUE) == 1


@pytest.mark.parametrize("opts", [dict(check="round"), dict(identity_skip=False),
                                  dict(no_termination=True, max_codewords=3_000_000),
                                  pytest.param(dict(cooperative=True), marks=pytest.mark.skip(
                                      reason="cooperative launches are no longer offered (BZ_ERR_ARG): processes "
                                             "that made one ended in a crash inside rocprofv3's shutdown"))])
def test_batch_options_equal_plain(bz, opts):
    import torch
    cs = mixed_codes()[:16] + synth.batch_codes(3, count=16)
    say(f"case batch options {opts}")
    kw = dict(opts)
    kw.setdefault("max_codewords", LIMIT)
    res = bz.min_distance_batch(cs, device=torch.device("cuda:0"), wait_timeout_s=30, **kw)
    for i, ((p, G), r) in enumerate(zip(cs, res)):
        same(r, bz.min_distance(p, G, **kw), f"code {i} {opts}")


def test_batch_config4_equals_plain(bz, oracle):
    """The batched workload: 512 codes, half F_3 and half F_7, n in [30, 90],
    rate 1/2 or 1/3 (F_7 capped at n <= 56 / 63), in one call."""
    import torch
    cs = synth.batch_codes(0)
    say(f"case batch config 4 seed 0: {len(cs)} codes")
    res, ms = bz.min_distance_batch(cs, device=torch.device("cuda:0"), timing=True, wait_timeout_s=30)
    say(f"  decompose {ms['decompose_ms']:.2f} ms, enumerate {ms['enum_ms']:.2f} ms")
    checked = 0
    for i, ((p, G), r) in enumerate(zip(cs, res)):
        plain = bz.min_distance(p, G)
        same(r, plain, f"config-4 code {i} p={p} shape={G.shape}")
        if plain["codewords_total"] < 5e7 and checked < 40:
            same(r, oracle.min_distance(p, G), f"config-4 code {i} vs oracle")
            checked += 1
    assert checked >= 20
    assert all(r["status"] in (0, bz.ERR_RANK) for r in res)


def test_batch_tiling_does_not_change_results(bz):
    import torch
    cs = synth.batch_codes(1, count=48)
    dev = torch.device("cuda:0")
    base = bz.min_distance_batch(cs, device=dev, wait_timeout_s=30)
    for bpc, ops in [(1, 0), (2, 700), (4, 12000)]:
        say(f"case batch tiling blocks_per_cu={bpc} sweep_ops={ops}")
        other = bz.min_distance_batch(cs, device=dev, blocks_per_cu=bpc, sweep_ops=ops or None, wait_timeout_s=30)
        for i, (a, b) in enumerate(zip(base, other)):
            same(a, b, f"code {i} bpc={bpc} ops={ops}")


def test_batch_workspace_reuse(bz):
    """A large batch, then a smaller one, then the large one again (the
    workspace is reused; results must not leak between calls)."""
    big = synth.batch_codes(2, count=96)
    small = big[10:20]
    r1 = bz.min_distance_batch(big, wait_timeout_s=30)
    r2 = bz.min_distance_batch(small, wait_timeout_s=30)
    r3 = bz.min_distance_batch(big, wait_timeout_s=30)
    for i in range(len(big)):
        same(r1[i], r3[i], f"code {i} repeat")
    for i in range(len(small)):
        same(r2[i], r1[10 + i], f"code {10 + i} in the small batch")


def test_autotuner_table(bz, tmp_path):
    """The autotuner picks one candidate per (p, W) group and a grid shape;
    running with its table gives the same results as the defaults."""
    import json
    from paper_2603_29942_amd import autotune
    cs = synth.batch_codes(7, count=24)
    t = autotune.tune(cs, reps=1, sweep_candidates=(1500, 6000), bpc_candidates=(2, 4), log=say)
    assert t["sweep_ops"] and set(t["sweep_ops"].values()) <= {1500, 6000}
    assert t["blocks_per_cu"] in (2, 4)
    path = tmp_path / "table.json"
    path.write_text(json.dumps(t))
    fn, bpc = autotune.load(str(path))
    tuned = bz.min_distance_batch(cs, sweep_ops=fn, blocks_per_cu=bpc, wait_timeout_s=30)
    plain = bz.min_distance_batch(cs, wait_timeout_s=30)
    for i, (a, b) in enumerate(zip(tuned, plain)):
        same(a, b, f"code {i} tuned")
