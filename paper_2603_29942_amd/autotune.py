"""Autotuner for the batched path: the size of a unit of work per (p, W) and
the workgroups per compute unit of the persistent launch.

    python -m paper_2603_29942_amd.autotune [--seed 100] [--count 256] [--out PATH]

A task of the enumeration kernel gives each lane a block of rows s whose
last-row sweeps add up to about `sweep_ops` VALU operations; small values cut
stages into many short tasks (better balance, more per-task decoding), large
values into few long ones.  The best value depends on the field and on W (the
words per plane a combination takes), so codes are grouped by (p, W) and each
group is timed as its own batch for every candidate (the smallest size within
1% of the fastest is taken); then the grid shape is timed on the whole sample
with the chosen sizes (the most workgroups per CU within 1% of the fastest is
taken).  Results never depend on
these knobs (the tests check it); only time does.

The table is JSON: {"sweep_ops": {"p,W": ops, ...}, "blocks_per_cu": b,
"kernel_source_hash": h, ...}; it is used only while the kernel sources hash
to h (a table taken on other kernels is ignored, and load_checked says so).
The persistent batched kernel fits at most 5 workgroups per compute unit for
W <= 2 (its registers); larger candidates are clamped to that by the library.
"""
import argparse
import hashlib
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning_gfx950.json")
SWEEP_CANDIDATES = (1500, 3000, 6000, 12000, 24000, 48000, 96000, 192000)
BPC_CANDIDATES = (1, 2, 3, 4, 5, 6)
KERNEL_SOURCES = ("bz_kernels.hpp", "bz_arith.hpp", "bz_state.hpp")


def kernel_source_hash():
    """Hash of the device code's sources (tables and profiles taken on other
    kernels no longer apply)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def words(p, n, k, identity_skip=True):
    w = (n - k + 31) // 32 if identity_skip else (n + 31) // 32
    return max(w, 1)


def load(path=TABLE):
    """(sweep_ops function (p, W) -> ops, blocks_per_cu), or defaults when no table exists."""
    if not os.path.exists(path):
        return (lambda p, W: 0), 0
    with open(path) as f:
        t = json.load(f)
    ops = {tuple(int(x) for x in key.split(",")): int(v) for key, v in t["sweep_ops"].items()}
    return (lambda p, W: ops.get((p, W), 0)), int(t.get("blocks_per_cu", 0))


def load_checked(path=TABLE):
    """As load(), but only a table taken on the current kernel sources is used;
    returns (sweep_ops function, blocks_per_cu, a note saying which)."""
    if not os.path.exists(path):
        return (lambda p, W: 0), 0, "defaults (no autotuner table)"
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return (lambda p, W: 0), 0, "defaults (the autotuner table was taken on other kernel sources; ignored)"
    fn, bpc = load(path)
    return fn, bpc, f"autotuner table (kernel sources {t['kernel_source_hash']})"


def _time_batch(bz, codes, dev, reps, **kw):
    best = None
    for _ in range(reps):
        _, ms = bz.min_distance_batch(codes, device=dev, timing=True, **kw)
        t = ms["decompose_ms"] + ms["enum_ms"]
        best = t if best is None else min(best, t)
    return best


def tune(codes, reps=2, sweep_candidates=SWEEP_CANDIDATES, bpc_candidates=BPC_CANDIDATES, log=print):
    import torch
    from . import bz
    dev = torch.device("cuda:0")
    groups = {}
    for p, G in codes:
        k, n = G.shape
        groups.setdefault((p, words(p, n, k)), []).append((p, G))
    bz.min_distance_batch(codes[:8], device=dev)  # warm-up: context, workspace
    chosen, timings = {}, {}
    for key, cs in sorted(groups.items()):
        row = {}
        for ops in sweep_candidates:
            row[ops] = _time_batch(bz, cs, dev, reps, sweep_ops=ops)
        # the smallest size within 1% of the fastest: the times are flat over a
        # wide range, and smaller parts let a serving round yield sooner
        tmin = min(row.values())
        best = min(o for o, t in row.items() if t <= 1.01 * tmin)
        chosen[key] = best
        timings[f"{key[0]},{key[1]}"] = {str(o): round(t, 4) for o, t in row.items()}
        log(f"  p={key[0]} W={key[1]} ({len(cs)} codes): " +
            " ".join(f"{o}:{t:.3f}ms" for o, t in row.items()) + f" -> {best}")
    fn = (lambda p, W: chosen.get((p, W), 0))
    bpc_t = {b: _time_batch(bz, codes, dev, reps, sweep_ops=fn, blocks_per_cu=b) for b in bpc_candidates}
    # the most workgroups per CU within 1% of the fastest: the 256-code sample
    # cannot tell counts that close apart, and on the full 512-code batch
    # five per CU ran 2.3% faster than four (interleaved runs of one build)
    tmin = min(bpc_t.values())
    bpc = max(b for b, t in bpc_t.items() if t <= 1.01 * tmin)
    log("  blocks_per_cu: " + " ".join(f"{b}:{t:.3f}ms" for b, t in bpc_t.items()) + f" -> {bpc}")
    return {"sweep_ops": {f"{p},{W}": ops for (p, W), ops in sorted(chosen.items())},
            "blocks_per_cu": bpc,
            "timings_ms": {"sweep_ops": timings, "blocks_per_cu": {str(b): round(t, 4) for b, t in bpc_t.items()}},
            "sample": f"{len(codes)} codes of the mixed batch distribution",
            "device": torch.cuda.get_device_properties(0).name}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=100)
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    from . import synth
    t0 = time.perf_counter()
    table = tune(synth.batch_codes(args.seed, count=args.count), reps=args.reps)
    table["tuning_seconds"] = round(time.perf_counter() - t0, 1)
    table["kernel_source_hash"] = kernel_source_hash()
    table["command"] = f"python -m paper_2603_29942_amd.autotune --seed {args.seed} --count {args.count}"
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps(table))


if __name__ == "__main__":
    main()
