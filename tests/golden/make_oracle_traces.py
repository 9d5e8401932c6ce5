"""Write tests/golden/oracle_traces.json: the oracle's results on the benchmark's
own inputs, so that the GPU tests can compare every benchmarked code with the
oracle without rerunning it (the larger codes take the oracle minutes).

    python tests/golden/make_oracle_traces.py [--part config2|config3|batch0|all]

Calls only the oracle (oracle/bzref.py) on inputs from the seeded generators
(paper_2603_29942_amd/synth.py); nothing here runs or reads the GPU library.

Contents:
  config2, config3  the full result (status, d, m, ranks, stage trace,
                    termination reason, total combinations) of the random
                    F_3 [72,36] and F_7 [48,24] codes of seeds 0..19;
  batch0            every code of the 512-code mixed batch of seed 0, run with
                    a work limit of BATCH_LIMIT combinations (larger codes stop
                    with the LIMIT status and the trace up to the cut): status,
                    d, total combinations and a hash of the whole result.
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bzref  # noqa: E402
from paper_2603_29942_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "oracle_traces.json")
SEEDS = range(20)
BATCH_LIMIT = 50_000_000
KEYS = ("status", "d", "m", "ranks", "stages", "terminated_by", "codewords_total")


def canonical(r):
    """The result as plain JSON values, in KEYS order."""
    return [r["status"], r["d"], r["m"], [int(x) for x in r["ranks"]],
            [[int(v) for v in st] for st in r["stages"]], r["terminated_by"], int(r["codewords_total"])]


def digest(r):
    return hashlib.sha256(json.dumps(canonical(r), separators=(",", ":")).encode()).hexdigest()[:16]


def single(cfg, log):
    out = {}
    for seed in SEEDS:
        p, G = synth.config_code(cfg, seed)
        t = time.perf_counter()
        r = bzref.min_distance(p, G)
        out[str(seed)] = dict(zip(KEYS, canonical(r)))
        log(f"config {cfg} seed {seed}: d = {r['d']}, {r['codewords_total']} combinations, "
            f"{time.perf_counter() - t:.1f} s")
    return out


def batch0(log):
    codes = []
    t = time.perf_counter()
    for i, (p, G) in enumerate(synth.batch_codes(0)):
        r = bzref.min_distance(p, G, max_codewords=BATCH_LIMIT)
        codes.append([r["status"], r["d"], int(r["codewords_total"]), digest(r)])
        if i % 64 == 63:
            log(f"batch 0: {i + 1} codes, {time.perf_counter() - t:.1f} s")
    return {"max_codewords": BATCH_LIMIT, "codes": codes}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--part", default="all", choices=["config2", "config3", "batch0", "all"])
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["about"] = ("Oracle results on the benchmark's inputs, written by tests/golden/make_oracle_traces.py "
                     "(oracle only). Trace rows: g, j, combinations, stage minimum, U after, L_{g,j}. "
                     "batch0 rows: status, d, combinations, hash of the whole result (see digest()).")
    data["nthreads"] = bzref.threads(0)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if args.part in ("config2", "all"):
        data["config2"] = single(2, log)
    if args.part in ("config3", "all"):
        data["config3"] = single(3, log)
    if args.part in ("batch0", "all"):
        data["batch0"] = batch0(log)
    with open(OUT + ".tmp", "w") as f:
        json.dump(data, f, separators=(",", ":"))
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
