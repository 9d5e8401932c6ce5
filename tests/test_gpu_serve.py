"""GPU checks of continuous-batching serving: every request's result is the
same alone (the plain path on that code) and in the mix, whatever the order of
arrival, the rounds and yields the server goes through, and the ordering policy
(arrival order, or shortest predicted work first)."""
import sys
import time

import numpy as np
import pytest

import codes
from paper_2603_29942_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("status", "d", "m", "ranks", "stages", "terminated_by", "codewords_total")


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


def requests(seed, count):
    reqs = [(p, G) for _, p, G in synth.serving_requests(seed, count, rate_per_s=1.0)]
    rng = np.random.default_rng([51, seed])
    G = rng.integers(0, 3, size=(6, 30), dtype=np.uint8)
    G[4] = (G[1] + 2 * G[2]) % 3  # rank deficient
    reqs += [(3, codes.extended_golay()), (7, codes.reed_solomon(7, 7, 3)), (3, codes.full_space(5, 3)), (3, G)]
    return reqs


def drain(srv, expect, limit_s=60.0):
    out = {}
    t0 = time.perf_counter()
    while len(out) < expect:
        for tag, r in srv.poll():
            out[tag] = r
        assert time.perf_counter() - t0 < limit_s, f"server stalled with {len(out)}/{expect} results"
    return out


def check_alone(bz, reqs, results, label, oracle=None):
    """Each served result equals the plain path's on that code alone and, for
    the requests with k <= 20 (the oracle finishes those in well under a
    second), the oracle's: Algorithm 6 on that code alone."""
    checked = 0
    for tag, (p, G) in enumerate(reqs):
        alone = bz.min_distance(p, G)
        for key in KEYS:
            assert results[tag][key] == alone[key], (label, tag, key, results[tag][key], alone[key])
        if oracle is not None and G.shape[0] <= 20:
            ref = oracle.min_distance(p, G)
            for key in KEYS:
                assert results[tag][key] == ref[key], (label, tag, key, "oracle", results[tag][key], ref[key])
            checked += 1
    if oracle is not None:
        assert checked >= 20, checked


@pytest.mark.parametrize("policy", ["fifo", "predicted"])
def test_serve_all_at_once_equals_alone(bz, oracle, policy):
    from paper_2603_29942_amd import predictor
    reqs = requests(1, 120)
    say(f"case serve all at once policy={policy}: {len(reqs)} requests")
    params = predictor.load()[0] if policy == "predicted" else None
    srv = bz.Server(policy=policy, mlp_params=params, slots=256, max_n=80, wait_timeout_s=30)
    try:
        for tag, (p, G) in enumerate(reqs):
            srv.submit(p, G, tag)
        res = drain(srv, len(reqs))
        say(f"  {srv.stats()}")
    finally:
        srv.stop()
    check_alone(bz, reqs, res, policy, oracle)


def test_serve_arrivals_during_rounds_equal_alone(bz, oracle):
    """Requests arrive in waves while earlier ones run, more of them than
    slots: rounds yield, slots recycle, results never change."""
    reqs = requests(2, 300)
    say(f"case serve waves: {len(reqs)} requests, 64 slots")
    srv = bz.Server(policy="fifo", slots=64, max_n=80, wait_timeout_s=30)
    res = {}
    try:
        nxt = 0
        t0 = time.perf_counter()
        while len(res) < len(reqs):
            for _ in range(7):
                if nxt < len(reqs):
                    srv.submit(reqs[nxt][0], reqs[nxt][1], nxt)
                    nxt += 1
            for tag, r in srv.poll():
                res[tag] = r
            assert time.perf_counter() - t0 < 120, "server stalled"
        st = srv.stats()
        say(f"  {st}")
        assert st["rounds"] > 1 and st["yields"] >= 1
    finally:
        srv.stop()
    check_alone(bz, reqs, res, "waves", oracle)


def test_serve_rejects_oversize(bz):
    srv = bz.Server(slots=8, max_n=40)
    try:
        with pytest.raises(RuntimeError):
            srv.submit(3, np.zeros((10, 41), dtype=np.uint8), 0)
        srv.submit(3, codes.ternary_golay(), 1)
        res = drain(srv, 1)
        assert res[1]["d"] == 5
    finally:
        srv.stop()
