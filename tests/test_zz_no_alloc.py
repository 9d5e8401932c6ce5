"""GPU check of the entry point that allocates nothing (bz_min_distance_noalloc,
called through the C ABI): on the same device generator its results equal
bz_min_distance_ex's, field for field, on two calls in a row, the second with
a smaller code (the device array the calls share keeps the first call's
contents), with several option sets; and the device's free memory does not
move across its calls."""
import sys

import pytest

import codes
from paper_2603_29942_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("status", "d", "m", "ranks", "stages", "terminated_by", "codewords_total")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def golden(part, seed):
    g = dict(codes.golden("oracle_traces.json")[part][str(seed)])
    g["ranks"] = list(g["ranks"])
    g["stages"] = [tuple(st) for st in g["stages"]]
    return g


def test_noalloc_equals_ex_on_consecutive_calls(oracle):
    import torch
    from paper_2603_29942_amd import bz
    assert torch.cuda.is_available(), "no GPU visible"
    dev = torch.device("cuda:0")
    # (workload, seed): a large code, then a smaller one, in each pair
    pairs = [((2, 3), (1, 4)), ((3, 1), (1, 9)), ((2, 7), (2, 0))]
    opts = [dict(), dict(check=bz.CHECK_ROUND), dict(identity_skip=0), dict(no_ahead=1),
            dict(no_termination=1, max_codewords=20_000_000)]
    for first, second in pairs:
        for kw in opts:
            for cfg, seed in (first, second):
                p, G = synth.config_code(cfg, seed)
                Gd = torch.from_numpy(G).to(dev)
                say(f"case noalloc cfg{cfg} seed={seed} {kw}")
                o1 = bz.bz_default_options()
                o2 = bz.bz_default_options()
                for key, v in kw.items():
                    setattr(o1, key, v)
                    setattr(o2, key, v)
                st1, r1 = bz.bz_min_distance_noalloc(p, Gd, o1)
                st2, r2 = bz.bz_min_distance_ex(p, Gd, o2)
                a, b = bz.result_dict(st1, r1), bz.result_dict(st2, r2)
                for key in KEYS:
                    assert a[key] == b[key], (cfg, seed, kw, key, a[key], b[key])
                if not kw or kw.get("no_ahead"):
                    want = oracle.min_distance(p, G) if cfg == 1 else golden(f"config{cfg}", seed)
                    for key in KEYS:
                        assert a[key] == want[key], (cfg, seed, "oracle", key)
    # no allocation across calls: the device's free memory stays where it is
    p, G = synth.config_code(2, 5)
    Gd = torch.from_numpy(G).to(dev)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info(dev)
    for _ in range(3):
        st, r = bz.bz_min_distance_noalloc(p, Gd)
        assert st == bz.OK
    free1, _ = torch.cuda.mem_get_info(dev)
    assert free1 == free0
    assert bz.result_dict(st, r)["stages"] == golden("config2", 5)["stages"]


def test_noalloc_on_a_user_stream_and_errors():
    import torch
    from paper_2603_29942_amd import bz
    dev = torch.device("cuda:0")
    side = torch.cuda.Stream()
    p, G = synth.config_code(2, 11)
    Gd = torch.from_numpy(G).to(dev)
    torch.cuda.synchronize()
    say("case noalloc user stream")
    with torch.cuda.stream(side):
        st, r = bz.bz_min_distance_noalloc(p, Gd)
    want = golden("config2", 11)
    got = bz.result_dict(st, r)
    for key in KEYS:
        assert got[key] == want[key], key
    o = bz.bz_default_options()
    o.timing = 1
    st, _ = bz.bz_min_distance_noalloc(p, Gd, o)
    assert st == bz.ERR_ARG
