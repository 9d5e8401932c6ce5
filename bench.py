"""Benchmark: exact minimum distance of random linear codes on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4]

Default workload (config 4): a step is one call of the batched path on 512
random codes of mixed field and size (half F_3, half F_7, n uniform in
[30, 90], rate 1/2 or 1/3; F_7 n <= 56 at rate 1/2 and n <= 63 at rate 1/3),
their generators already resident in GPU memory: one information-set
decomposition launch and one persistent enumeration launch compute every
code's minimum distance (the stages of Algorithm 6 with the isometric last
addition, popcount weights, min-reduce and the L >= U test).  The same codes
then run on the plain path (one call per code), and the two are compared:
combinations evaluated per second and each code's time to d (p50 / p99).

Prints one JSON line: value = combinations evaluated per second by the
batched path over the timed steps (whole job), the plain path on the same
codes, the roofline position of the persistent enumeration kernel (device
time from HIP events on the launch's stream), two sub-blocks with the plain
path on F_3 [72,36] and F_7 [48,24] (20 codes each, each with its own
roofline), and the oracle timed on the host cores on a bounded sample of the
same batch.  --config 1-3 time one workload of the plain path alone, 5 the
serving loop.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X int32 VALU rates from its unit counts and clock: 256 CUs x 4 SIMDs at
# 2.4 GHz.  32-bit bitwise operations and adds issue at the fp32 FMA rate, 32
# lanes per SIMD per clock (the chip's 157.3 TFLOP/s fp32 vector figure is 2
# flops x 128 lanes x 256 CUs x 2.4 GHz): 78.6 T lane-ops/s.  Popcount and min
# issue at half that rate, 16 lanes per SIMD per clock: 39.3 T lane-ops/s (both
# rates checked with an issue-rate probe on the chip: 100 and 58 lane-ops per
# CU per clock against 128 and 64).
FULL_RATE_TOPS = 256 * 128 * 2.4e9 / 1e12
HALF_RATE_TOPS = 256 * 64 * 2.4e9 / 1e12
CONFIG_NAMES = {1: "F_3 [40,10]", 2: "F_3 [72,36]", 3: "F_7 [48,24]"}


def op_mix(p, W):
    """Algorithmic int32 VALU operations per combination for W words per plane,
    as (bitwise, popcount + min): F_3: 2 boolean ops (isometric add or
    subtract) + 1 popcount per word, + 1 min; F_7: 3 boolean + 1 popcount per
    word (xors shared by the add/subtract pair), + 1 min."""
    return (2 * W, W + 1) if p == 3 else (3 * W, W + 1)


def ops_per_codeword(p, W):
    full, half = op_mix(p, W)
    return full + half


def peak_seconds_per_codeword(p, W):
    """Time one combination's algorithmic operations take at the chip's peak
    rates (bitwise at the full rate, popcount and min at half rate)."""
    full, half = op_mix(p, W)
    return full / (FULL_RATE_TOPS * 1e12) + half / (HALF_RATE_TOPS * 1e12)


def peak_tops(p, W):
    """Peak algorithmic operations per second for the op mix of (p, W), in T/s."""
    return ops_per_codeword(p, W) / peak_seconds_per_codeword(p, W) / 1e12


def pct(xs, q):
    xs = sorted(xs)
    i = max(0, min(len(xs) - 1, int(-(-q * len(xs) // 100)) - 1))  # nearest rank
    return xs[i]


def kernel_source_hash():
    from paper_2603_29942_amd import autotune
    return autotune.kernel_source_hash()


def traffic_for(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, only if the
    kernel source has not changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(f"{kernel}/{workload}")
    if not rec or rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    """The host CPU as the kernel reports it: model name, family / model /
    stepping, clock, and the hardware threads this process may use."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if info:
                        break  # the first processor's block is enough
                    continue
                key, val = (x.strip() for x in line.split(":", 1))
                if key in ("vendor_id", "model name", "cpu family", "model", "stepping", "cpu MHz") and key not in info:
                    info[key] = val
                if key == "flags":
                    info["hypervisor"] = "hypervisor" in val.split()
    except OSError:
        pass
    info["logical_cpus"] = os.cpu_count()
    info["usable_cpus"] = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return info


# The paper's own CPU timings of the method (another machine: context only).
PAPER_CPU_CONTEXT = {
    "processor": "AMD EPYC 7F52, 16 cores (the paper's Sec. 5)",
    "F_7 [50,25,13], one core (Table 3)": {"SC8 s": 29.57, "SS64I s": 8.44, "SS64IN s": 5.15},
    "F_7 [52,19,19] (Table 4)": {"SS64IN 1 core s": 21.90, "SS64IN 4 cores s": 5.69},
    "note": "the paper's codes are not published; these figures are not on this workload",
}


def cpu_baseline_codes(codes, gpu, budget_s, budget_1t_s, max_cw, max_cw_1t):
    """The oracle as it stands, on the host cores, over whole codes of the
    benchmark's own workload, in order, skipping codes above max_cw
    combinations (by the GPU's count) until about budget_s seconds have been
    spent: its rate, its time to d per code (p50 / p99) and d equality with the
    GPU.  Then on one thread, codes up to max_cw_1t combinations, for about
    budget_1t_s seconds."""
    from oracle import bzref
    threads = bzref.threads(0)

    def run(nthreads, budget, cap):
        cw, spent, times, used, match = 0, 0.0, [], [], True
        for i, (p, G) in enumerate(codes):
            if gpu[i]["codewords_total"] > cap:
                continue
            t = time.perf_counter()
            r = bzref.min_distance(p, G, nthreads=nthreads)
            dt = time.perf_counter() - t
            spent += dt
            times.append(dt)
            cw += r["codewords_total"]
            used.append(i)
            match &= (r["d"] == gpu[i]["d"] and r["codewords_total"] == gpu[i]["codewords_total"])
            if spent >= budget:
                break
        return cw, spent, times, used, match

    cw, spent, times, used, match = run(threads, budget_s, max_cw)
    cw1, spent1, times1, used1, match1 = run(1, budget_1t_s, max_cw_1t)
    return {"value": cw / spent, "unit": "codewords/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {len(used)} codes of the timed batch of seed 0 with at most {max_cw:.0e} "
                      f"combinations (codes {used[0]}..{used[-1]}), whole runs, {cw} combinations in {spent:.1f} s; "
                      f"oracle d and counts equal the GPU's: {match}",
            "d_match": bool(match and match1),
            "time_to_d_ms": {"p50": pct(times, 50) * 1e3, "p99": pct(times, 99) * 1e3, "codes": len(times)},
            "single_thread": {"value": cw1 / spent1, "unit": "codewords/s", "cores": 1,
                              "time_to_d_ms": {"p50": pct(times1, 50) * 1e3, "p99": pct(times1, 99) * 1e3},
                              "sample": f"the first {len(used1)} codes of the same batch with at most "
                                        f"{max_cw_1t:.0e} combinations, whole runs on one thread: "
                                        f"{cw1} combinations in {spent1:.1f} s"},
            "cpu": cpu_model(), "paper_context": PAPER_CPU_CONTEXT}


def cpu_baseline_plain(cfg, gpu_d, budget_s):
    """The oracle on the host cores over whole codes of a single-code workload
    (seeds 0, 1, ...) for about budget_s seconds."""
    from oracle import bzref
    from paper_2603_29942_amd import synth
    threads = bzref.threads(0)
    cw, spent, seeds, match, times = 0, 0.0, [], True, []
    for seed in range(len(gpu_d)):
        p, G = synth.config_code(cfg, seed)
        t = time.perf_counter()
        r = bzref.min_distance(p, G, nthreads=threads)
        dt = time.perf_counter() - t
        spent += dt
        times.append(dt)
        cw += r["codewords_total"]
        seeds.append(seed)
        match &= (r["d"] == gpu_d[seed])
        if spent >= budget_s:
            break
    return {"value": cw / spent, "unit": "codewords/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(seeds)} whole {CONFIG_NAMES[cfg]} codes (seeds {seeds[0]}..{seeds[-1]}), "
                      f"{cw} combinations in {spent:.1f} s; oracle d equals GPU d: {match}",
            "d_match": match, "time_to_d_ms": {"p50": pct(times, 50) * 1e3, "p99": pct(times, 99) * 1e3},
            "cpu": cpu_model(), "paper_context": PAPER_CPU_CONTEXT}


# The paper's arithmetic benchmark (Sec. 5, Tables 1-2): pairwise addition of
# two sets of 10,000 vectors of 512 symbols, repeated 10,000 times, and its
# single-core times on the AMD EPYC 7F52 (context only, another machine).
MICRO_VARIANTS = [
    # field, label, encoding, op name, boolean ops per 32-symbol word per addition, EPYC seconds
    (3, "F_3 natural encoding, Algorithm 3 (HQ)", "natural", "add", 9, 1.04),
    (3, "F_3 Kawahara et al. encoding, Algorithm 2 (KAT)", "kat", "kat", 6, 0.89),
    (7, "F_7 natural encoding, Algorithm 4 (HQ)", "natural", "add", 22, 2.30),
]


def micro(nvec=10000, nsym=512, reps=10000, passes=2000):
    """Sliced exact addition on the GPU at the paper's sizes.  Chain mode: one
    launch, every thread applies x <- x + b `reps` times to one 32-symbol word
    in registers (the arithmetic alone).  Streaming mode: `passes` single
    additions c = a + b over all vectors, each a launch, captured in one HIP
    graph and replayed (memory and launch bound)."""
    import numpy as np
    import torch
    from paper_2603_29942_amd import bz
    dev = torch.device("cuda:0")
    out = []
    for p, label, enc, opname, ops_word, epyc_s in MICRO_VARIANTS:
        rng = np.random.default_rng([5, p, len(out)])
        a = rng.integers(0, p, (nvec, nsym), dtype=np.uint8)
        b = rng.integers(0, p, (nvec, nsym), dtype=np.uint8)
        e = bz.ENC_KAT if enc == "kat" else bz.ENC_NATURAL
        op = bz.OP_KAT_ADD if opname == "kat" else bz.OP_ADD
        A = bz.bz_sliced_pack(p, torch.from_numpy(a).to(dev), encoding=e)
        B = bz.bz_sliced_pack(p, torch.from_numpy(b).to(dev), encoding=e)
        O = torch.empty_like(A)
        want = (a.astype(np.int64) + reps * b.astype(np.int64)) % p
        bz.bz_sliced_op(p, op, A, B, nsym, reps=reps, out=O)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bz.bz_sliced_op(p, op, A, B, nsym, reps=reps, out=O)
        e1.record()
        torch.cuda.synchronize()
        chain_s = e0.elapsed_time(e1) / 1e3
        ok_chain = bool(np.array_equal(bz.bz_sliced_unpack(p, O, nsym, encoding=e).cpu().numpy(), want))
        # streaming: single additions, captured once and replayed
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                bz.bz_sliced_op(p, op, A, B, nsym, reps=1, out=O)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for _ in range(passes):
                bz.bz_sliced_op(p, op, A, B, nsym, reps=1, out=O)
        graph.replay()
        torch.cuda.synchronize()
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        pass_s = e0.elapsed_time(e1) / 1e3 / passes
        ok_stream = bool(np.array_equal(bz.bz_sliced_unpack(p, O, nsym, encoding=e).cpu().numpy(),
                                        (a.astype(np.int64) + b.astype(np.int64)) % p))
        r = 2 if p == 3 else 3
        words = nvec * ((nsym + 31) // 32)
        adds = nvec * nsym * reps
        stream_bytes = 3 * words * r * 4
        out.append({
            "variant": label, "p": p,
            "chain": {"seconds_for_paper_workload": chain_s, "symbol_additions_per_s": adds / chain_s,
                      "bool_ops_per_s": words * reps * ops_word / chain_s,
                      "frac_of_bitwise_peak": words * reps * ops_word / chain_s / (FULL_RATE_TOPS * 1e12),
                      "correct": ok_chain},
            "streaming": {"us_per_pass": pass_s * 1e6, "seconds_for_paper_workload": pass_s * reps,
                          "hbm_GBps": stream_bytes / pass_s / 1e9, "frac_of_hbm_peak": stream_bytes / pass_s / 8e12,
                          "bytes_per_pass": stream_bytes, "correct": ok_stream},
            "paper_epyc_7f52_1core_s": epyc_s,
        })
    return {"metric": "sliced exact additions, the arithmetic benchmark of Tables 1-2",
            "workload": f"2 x {nvec} vectors x {nsym} symbols, {reps} repeated additions",
            "dtype": "u32", "data": "synthetic", "results": out}


def bench_plain(cfg, K, Wm, blocks_per_cu=0):
    """The plain path on one single-code workload: K codes (seeds 0..K-1), one
    call each, generators resident in HBM, Wm warm-up calls on other seeds.
    The call's arguments are prepared once, as a C caller holding its inputs
    in HBM would: a step is the library call.  The timed pass runs without
    timing events (the call returns when the final check hands the result
    over); a second pass over the same codes with HIP events gives the kernel
    durations for the roofline, and its results must equal the first's."""
    import ctypes
    import numpy as np
    import torch
    from paper_2603_29942_amd import bz, synth
    dev = torch.device("cuda:0")
    p, n, k = synth.CONFIGS[cfg]
    Gt = torch.from_numpy(np.stack([synth.config_code(cfg, s)[1] for s in range(K)])).to(dev)
    Gw = torch.from_numpy(np.stack([synth.config_code(cfg, 10000 + s)[1] for s in range(max(Wm, 1))])).to(dev)
    torch.cuda.synchronize()
    o = bz.bz_default_options()
    o.timing = 0
    o.blocks_per_cu = blocks_per_cu
    o.max_codewords = 1 << 40
    o.hip_stream = bz._stream_of(Gt)
    o.device = dev.index or 0
    out = bz.bz_result()
    fn = bz.lib().bz_min_distance_ex
    o_ref, out_ref = ctypes.byref(o), ctypes.byref(out)
    ptr_t = [ctypes.c_void_p(Gt[i].data_ptr()) for i in range(K)]
    ptr_w = [ctypes.c_void_p(Gw[i].data_ptr()) for i in range(Gw.shape[0])]
    outs = [bz.bz_result() for _ in range(K)]  # one result block per step, read after the loop
    out_refs = [ctypes.byref(r) for r in outs]

    def run(ptr, ref):
        st = fn(p, n, k, ptr, 1, o_ref, ref)
        if st != bz.OK:
            raise RuntimeError(f"bz_min_distance_ex: {bz.bz_status_str(st)}")

    for i in range(Wm):
        run(ptr_w[i], out_ref)
    torch.cuda.synchronize()
    per_step = [0.0] * K
    t0 = time.perf_counter()
    for i in range(K):
        ts = time.perf_counter()
        run(ptr_t[i], out_refs[i])
        per_step[i] = time.perf_counter() - ts
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cws = [r.codewords_total for r in outs]
    # the kernel durations: the same codes again, with HIP events on the stream
    o.timing = 1
    timed = [bz.bz_result() for _ in range(K)]
    for i in range(K):
        run(ptr_t[i], ctypes.byref(timed[i]))
    torch.cuda.synchronize()
    o.timing = 0
    if [(r.d, r.codewords_total) for r in timed] != [(r.d, r.codewords_total) for r in outs]:
        raise RuntimeError("the timed pass and the event pass disagree")
    enum_ms = [r.enum_ms for r in timed]
    dec_ms = [r.decompose_ms for r in timed]
    W = (n - k + 31) // 32  # words per plane over the non-pivot columns
    opc = ops_per_codeword(p, W)
    total_cw = sum(cws)
    achieved = total_cw * opc / (sum(enum_ms) / 1e3) / 1e12
    peak = peak_tops(p, W)
    return {
        "workload": f"one random {CONFIG_NAMES[cfg]} code per step (seeds 0..{K - 1}), plain path, "
                    "generator resident on the GPU",
        "p": p, "n": n, "k": k, "steps": K, "warmup": Wm,
        "value": total_cw / elapsed, "unit": "codewords/s", "ms_per_step": elapsed / K * 1e3,
        "time_to_d_ms": {"p50": pct(per_step, 50) * 1e3, "p99": pct(per_step, 99) * 1e3,
                         "mean": elapsed / K * 1e3},
        "codewords_per_step": {"mean": total_cw / K, "min": min(cws), "max": max(cws)},
        "d": [r.d for r in outs],
        "kernel_ms_per_step": {"decompose": sum(dec_ms) / K, "enum": sum(enum_ms) / K},
        "roofline": {"kernel": "enum_kernel", "bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "T int32 VALU lane-ops/s (algorithmic)", "frac": achieved / peak,
                     "traffic": traffic_for("enum_kernel", f"f{p}_{n}_{k}"),
                     "ops_per_codeword": opc, "op_mix": {"bitwise": op_mix(p, W)[0], "popcount_min": op_mix(p, W)[1]},
                     "peak_note": f"bitwise at {FULL_RATE_TOPS:.1f} T/s, popcount and min at {HALF_RATE_TOPS:.1f} T/s",
                     "avg_launch_ms": sum(enum_ms) / K},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=4, choices=[1, 2, 3, 4, 5],
                    help="4 (default): the 512-code mixed batch per step, batched against plain; "
                         "1-3: one code per step (plain path); 5: serving under Poisson arrivals")
    ap.add_argument("--sub-steps", type=int, default=20, help="config 4: codes of each plain sub-block")
    ap.add_argument("--no-plain", action="store_true", help="config 4: skip the plain path on the batch's codes")
    ap.add_argument("--requests", type=int, default=2000, help="config 5: requests per policy")
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--micro", action="store_true",
                    help="only run the sliced-arithmetic benchmark (Tables 1-2 sizes) and print its JSON line")
    ap.add_argument("--valu-rates", action="store_true",
                    help="only measure the VALU issue rate of the instructions the path uses and print it")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (the known-size copy kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "sharding the stages over several GPUs is designed but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.micro:
        print(json.dumps(micro()), flush=True)
        return
    if args.valu_rates:
        from paper_2603_29942_amd import bz
        props = torch.cuda.get_device_properties(dev)
        clk_hz = 2.4e9
        rates = {}
        for op, name in enumerate(bz.VALU_PROBE_OPS):
            bz.valu_rate(op, iters=256)  # warm-up
            r = max(bz.valu_rate(op) for _ in range(3))
            rates[name] = {"lane_ops_per_s": r,
                           "lane_ops_per_cu_per_clock": r / props.multi_processor_count / clk_hz}
        print(json.dumps({"metric": "VALU issue rate (8 independent chains per thread, 8 waves per SIMD)",
                          "cus": props.multi_processor_count, "clock_hz": clk_hz, "rates": rates,
                          "peak_model": {"bitwise_and_add_lanes_per_cu_per_clock": 128,
                                         "popcount_and_min_lanes_per_cu_per_clock": 64}}), flush=True)
        return
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}), flush=True)
        return
    cfg = args.config
    if cfg == 4:
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if cfg == 5:
        print(json.dumps(bench_serve(args)), flush=True)
        return
    K, Wm = args.steps, args.warmup
    blk = bench_plain(cfg, K, Wm, args.blocks_per_cu)
    line = {
        "metric": "codewords evaluated/s (whole job, plain path: one code per call)",
        "value": blk["value"], "unit": "codewords/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": blk["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": blk["workload"], "p": blk["p"], "n": blk["n"], "k": blk["k"],
                   "identity_skip": True, "blocks_per_cu": args.blocks_per_cu or "occupancy"},
        "time_to_d_ms": blk["time_to_d_ms"], "codewords_per_step": blk["codewords_per_step"],
        "d": {"min": min(blk["d"]), "max": max(blk["d"])}, "kernel_ms_per_step": blk["kernel_ms_per_step"],
        "roofline": blk["roofline"],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_plain(cfg, blk["d"], args.cpu_seconds)
    print(json.dumps(line), flush=True)


def autotune_table():
    from paper_2603_29942_amd import autotune
    return autotune.load()


def bench_serve(args):
    """Serving: Poisson arrivals of random F_3 / F_7 codes (k uniform in
    [10, 40], F_7 k <= 28, n = 2k) at 0.7 x the capacity of the server itself
    (jobs/s with every request of a calibration set submitted at once,
    measured before the run and frozen), through the continuous-batching
    server: arrival order, shortest predicted work first, and the latter with
    a per-round admission budget of predicted work.  The same arrival trace is
    then served by the plain path, one call per request in arrival order.
    Latency is arrival to result as seen by the polling loop."""
    import numpy as np
    import torch
    from paper_2603_29942_amd import bz, predictor, synth
    dev = torch.device("cuda:0")
    params = predictor.load()[0]

    def server(policy, budget=0.0):
        return bz.Server(policy="predicted" if policy != "fifo" else "fifo",
                         mlp_params=params if policy != "fifo" else None, slots=1024, max_n=80,
                         admit_budget=budget)

    def warm(srv):
        for t, (_, p, G) in enumerate(synth.serving_requests(98, 16, 1.0)):
            srv.submit(p, G, 10 ** 9 + t)
        got = 0
        while got < 16:
            got += len(srv.poll())

    # capacity of the server: a calibration set submitted at once
    cal = synth.serving_requests(99, 1000, 1.0)
    srv = server("fifo")
    warm(srv)
    tc = time.perf_counter()
    for t, (_, p, G) in enumerate(cal):
        srv.submit(p, G, t)
    got = 0
    while got < len(cal):
        got += len(srv.poll())
    cap = len(cal) / (time.perf_counter() - tc)
    srv.stop()
    lam = 0.7 * cap
    N = args.requests
    reqs = synth.serving_requests(0, N, lam)
    offered = (N - 1) / (reqs[-1][0] - reqs[0][0])
    out, ds = {}, {}
    budget = 4e10
    for policy in ("fifo", "predicted", "predicted_budget"):
        srv = server(policy, budget if policy == "predicted_budget" else 0.0)
        warm(srv)
        lat, cw, dvals, done_at = np.zeros(N), 0, [0] * N, np.zeros(N)
        t0 = time.perf_counter()
        i, done = 0, 0
        while done < N:
            now = time.perf_counter() - t0
            while i < N and reqs[i][0] <= now:
                srv.submit(reqs[i][1], reqs[i][2], i)
                i += 1
            for tag, r in srv.poll():
                done_at[tag] = time.perf_counter() - t0
                lat[tag] = done_at[tag] - reqs[tag][0]
                cw += r["codewords_total"]
                dvals[tag] = r["d"]
                done += 1
        span = float(done_at.max() - reqs[0][0])
        st = srv.stats()
        srv.stop()
        ds[policy] = dvals
        out[policy] = {"latency_ms": {"p50": pct(lat.tolist(), 50) * 1e3, "p99": pct(lat.tolist(), 99) * 1e3,
                                      "mean": float(lat.mean() * 1e3)},
                       "served_jobs_per_s": N / span, "served_over_offered": (N / span) / offered,
                       "codewords_per_s": cw / span, "seconds": span, **st}
        if policy == "predicted_budget":
            out[policy]["admit_budget_combinations"] = budget
    # the plain path on the same arrival trace: one call per request, in order
    o = bz.bz_default_options()
    lat, dvals, done_at = np.zeros(N), [0] * N, np.zeros(N)
    for _, p, G in synth.serving_requests(98, 8, 1.0):
        bz.bz_min_distance_ex(p, G, o)
    t0 = time.perf_counter()
    for i, (ta, p, G) in enumerate(reqs):
        while time.perf_counter() - t0 < ta:
            pass
        st, r = bz.bz_min_distance_ex(p, G, o)
        done_at[i] = time.perf_counter() - t0
        lat[i] = done_at[i] - ta
        dvals[i] = r.d
    span = float(done_at.max() - reqs[0][0])
    out["plain_same_requests"] = {"latency_ms": {"p50": pct(lat.tolist(), 50) * 1e3,
                                                 "p99": pct(lat.tolist(), 99) * 1e3, "mean": float(lat.mean() * 1e3)},
                                  "served_jobs_per_s": N / span, "served_over_offered": (N / span) / offered,
                                  "seconds": span, "note": "one bz_min_distance_ex call per request at its arrival"}
    ds["plain"] = dvals
    return {
        "metric": "time-to-d under Poisson arrivals (continuous batching), p50/p99",
        "value": out["predicted"]["latency_ms"]["p50"], "unit": "ms", "n_gpus": 1, "steps": N, "warmup": 16,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{N} requests, Poisson arrivals at {lam:.1f}/s = 0.7 x the server's capacity "
                               f"{cap:.1f} jobs/s (1000 requests submitted at once); p uniform in {{3,7}}, k uniform "
                               "in [10,40] (F_7 k <= 28), n = 2k",
                   "slots": 1024, "arrival_rate_per_s": lam, "offered_jobs_per_s": offered,
                   "capacity_jobs_per_s": cap},
        "policies": out,
        "d_equal_between_policies": ds["fifo"] == ds["predicted"] == ds["predicted_budget"] == ds["plain"],
    }


def bench_batch(args):
    """The batched workload: each step is one call on a 512-code mixed batch
    (batch seed = step index), its generators resident in HBM; then the plain
    path (one call per code, arguments prepared once) on the same codes."""
    import ctypes
    import numpy as np
    import torch
    from paper_2603_29942_amd import autotune, bz, synth
    dev = torch.device("cuda:0")
    K, Wm = args.steps, args.warmup
    sweep_fn, bpc_tuned, tune_note = autotune.load_checked()
    bpc = args.blocks_per_cu or bpc_tuned
    batches = [synth.batch_codes(s) for s in range(K)]
    warm = [synth.batch_codes(1000 + s, count=64) for s in range(max(Wm, 1))]
    packed = [bz.pack_batch(b, device=dev) for b in batches]
    for b, descs in packed:
        for i in range(len(descs)):
            d = descs[i]
            descs[i].sweep_ops = int(sweep_fn(d.p, max((d.n - d.k + 31) // 32, 1)))
    for wb in warm[:Wm]:
        bz.min_distance_batch(wb, device=dev, sweep_ops=sweep_fn, blocks_per_cu=bpc)
    torch.cuda.synchronize()
    code_ms = [np.zeros(len(b), dtype=np.float32) for b in batches]
    opts = []
    for i in range(K):
        o = bz.bz_default_batch_options()
        o.timing = 1
        o.blocks_per_cu = bpc
        o.code_ms_out = code_ms[i].ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        opts.append(o)
    times, results = [], []
    t0 = time.perf_counter()
    for i, (buf, descs) in enumerate(packed):
        ts = time.perf_counter()
        st, res, _ = bz.bz_min_distance_batch(buf, descs, opts[i])
        times.append(time.perf_counter() - ts)
        if st != bz.OK:
            raise RuntimeError(f"bz_min_distance_batch: {bz.bz_status_str(st)}")
        results.append(res)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cws = [sum(r.codewords_total for _, r in res) for res in results]
    ops_total, ideal_s = 0.0, 0.0
    for (buf, descs), res in zip(packed, results):
        for i, (_, r) in enumerate(res):
            d = descs[i]
            W = max((d.n - d.k + 31) // 32, 1)
            ops_total += r.codewords_total * ops_per_codeword(d.p, W)
            ideal_s += r.codewords_total * peak_seconds_per_codeword(d.p, W)
    dec = [o.decompose_ms for o in opts]
    enum = [o.enum_ms for o in opts]
    statuses = [s_i for res in results for s_i, _ in res]
    total_cw = sum(cws)
    enum_s = sum(enum) / 1e3
    achieved = ops_total / enum_s / 1e12
    frac = ideal_s / enum_s  # the batch's op mix at the peak rates, against the launches' time
    batched_code_ms = np.concatenate(code_ms).tolist()
    gpu_first = [{"d": r.d, "codewords_total": r.codewords_total} for _, r in results[0]]
    line = {
        "metric": "codewords evaluated/s + time-to-d, batched vs plain (bit-exact d); p50/p99",
        "value": total_cw / elapsed, "unit": "codewords/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": elapsed / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"batched path, 512 random codes per step (batch seeds 0..{K - 1}): 256 over F_3 "
                               "and 256 over F_7 in random order, n uniform in [30,90], rate 1/2 or 1/3 at random "
                               "(k = n//2 or n//3), entries i.i.d. uniform; F_7 codes redrawn above n = 56 "
                               "(rate 1/2) / 63 (rate 1/3); draws are not redrawn for rank (a rank-deficient "
                               "draw, probability below p^-(n-k), returns the RANK status); generators resident "
                               "on the GPU",
                   "codes_per_step": 512, "identity_skip": True, "blocks_per_cu": bpc or 4,
                   "sweep_ops": tune_note, "rank_deficient_codes": sum(1 for x in statuses if x == bz.ERR_RANK)},
        "time_to_d_ms": {"batched_per_code": {"p50": pct(batched_code_ms, 50), "p99": pct(batched_code_ms, 99),
                                              "note": "device time from the start of the batch's decomposition "
                                                      "launch to the check that ended the code"},
                         "batched_call": {"p50": pct(times, 50) * 1e3, "p99": pct(times, 99) * 1e3,
                                          "note": "host time of one 512-code call"}},
        "codewords_per_step": {"mean": total_cw / K, "min": min(cws), "max": max(cws)},
        "kernel_ms_per_step": {"decompose": sum(dec) / K, "enum": sum(enum) / K},
        "roofline": {"kernel": "enum_batch_kernel", "bound": "alu", "achieved": achieved, "peak": achieved / frac,
                     "unit": "T int32 VALU lane-ops/s (algorithmic)", "frac": frac,
                     "traffic": traffic_for("enum_batch_kernel", "mixed_512"),
                     "ops_per_codeword": "3W+1 (F_3: 2W bitwise, W+1 popcount and min), 4W+1 (F_7: 3W bitwise, "
                                         "W+1 popcount and min), W = words over the n-k non-pivot columns",
                     "peak_note": f"the batch's op mix at bitwise {FULL_RATE_TOPS:.1f} T/s, popcount and min "
                                  f"{HALF_RATE_TOPS:.1f} T/s",
                     "avg_launch_ms": sum(enum) / K},
    }
    if not args.no_plain:
        # the plain path on the same codes: one call per code, device pointers
        # and options prepared once; per-code time to d by the host clock
        o = bz.bz_default_options()
        o.blocks_per_cu = 0
        o.device = dev.index or 0
        o.hip_stream = bz._stream_of(packed[0][0])
        fn = bz.lib().bz_min_distance_ex
        o_ref = ctypes.byref(o)
        outs = [bz.bz_result() for _ in range(512)]
        out_refs = [ctypes.byref(r) for r in outs]
        plain_lat, plain_done, plain_cw, equal = [], [], 0, True
        tp = time.perf_counter()
        for bi, (buf, descs) in enumerate(packed):
            base = buf.data_ptr()
            tb = time.perf_counter()
            for ci in range(len(descs)):
                d = descs[ci]
                tc = time.perf_counter()
                st = fn(d.p, d.n, d.k, ctypes.c_void_p(base + d.g_offset), 1, o_ref, out_refs[ci])
                plain_lat.append(time.perf_counter() - tc)
                plain_done.append(time.perf_counter() - tb)
                if st not in (bz.OK, bz.ERR_RANK):
                    raise RuntimeError(f"bz_min_distance_ex: {bz.bz_status_str(st)}")
            torch.cuda.synchronize()
            for ci, (s_i, r) in enumerate(results[bi]):
                q = outs[ci]
                plain_cw += q.codewords_total
                equal &= (q.d == r.d and q.codewords_total == r.codewords_total and q.n_stages == r.n_stages)
        plain_s = time.perf_counter() - tp
        line["plain_same_codes"] = {
            "value": plain_cw / plain_s, "unit": "codewords/s", "seconds": plain_s,
            "time_to_d_ms": {"per_call": {"p50": pct(plain_lat, 50) * 1e3, "p99": pct(plain_lat, 99) * 1e3,
                                          "note": "host time of one call per code"},
                             "per_code_in_job": {"p50": pct(plain_done, 50) * 1e3, "p99": pct(plain_done, 99) * 1e3,
                                                 "note": "time from the start of the batch's 512 calls to the "
                                                         "return of the code's call (codes in batch order), the "
                                                         "plain counterpart of the batched per-code time"}},
            "d_and_counts_equal_batched": bool(equal)}
        line["speedup_vs_plain"] = plain_s / elapsed
    line["sub_blocks"] = {
        "plain_f3_72_36": bench_plain(2, args.sub_steps, 2),
        "plain_f7_48_24": bench_plain(3, args.sub_steps, 2),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_codes(batches[0], gpu_first, args.cpu_seconds, args.cpu_seconds / 2,
                                                  max_cw=3e8, max_cw_1t=2e7)
    return line


if __name__ == "__main__":
    main()
