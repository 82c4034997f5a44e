#!/usr/bin/env python3
"""Benchmark of the MI355X chaotic-iteration PRNG.

One step = one cprng_generate call of the paper-shaped workload: the
neighbour-exchange variant (Algorithm 4) on 2^20 streams x 1,024 uint32
outputs (4 GiB written to HBM), in the interleaved layout out[i * 2^20 + s]
(the collision-free reading of the paper's store index with NumThreads the
number of threads), states seeded from SplitMix64 with seed 1 and already
resident on the device.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-extra] [--no-cpu-baseline]
                    [--no-autotune] [--serving-duration S]
    python bench.py --workload serving [--duration 60]
    python bench.py --workload ragged|ragged_v1|ragged_groups|consume   (one leg alone, for profiling)

Order of the default run: the headline's W + K launches right after idle
(per-launch times in extra.cold_start: the shader clock settles over the
first tens of milliseconds of activity); the serving trace (Poisson 2,000
req/s, 60 s by default); the small plain configuration (1,024 x 1,024, V0 and
V1); the same workload in the stream-major layout out[s * 1024 + i]; the
plain variants V0, V1, V3, V4 in both layouts; batched uneven runs of V0, V1
and V2 groups (each autotuned first, then one hipGraph launch per call);
in-kernel consumption (2^36 numbers) against its instruction-mix ALU
roofline; the VALU issue-rate probes and the store-only fill probe; then the
headline: W untimed and K timed steps (and each launch's duration); then the
autotuner on the headline workload (reported beside it, not used for it) and
the CPU oracle baselines.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
CU, CLOCK_HZ = 256, 2.4e9      # MI355X compute units, peak engine clock
# VALU issue limits of gfx950 from its unit counts, in lanes per CU per
# clock: 4 SIMDs x 16 lanes = 64 for the single-rate instruction classes
# (left shifts, min/max, int<->float conversions, integer multiplies and
# 24-bit multiply-adds, three-operand integer ops, bit-field ops and byte
# permutes, bit counts, 64-bit shifts and adds), and 128 for any VALU
# instruction (the rate behind the published 157.3 TFLOP/s fp32 vector peak;
# xor/and/or/add/sub, right shifts and f32 add/mul/fma reach it).  A kernel
# with N VALU instructions per number, S of them single-rate, produces at most
# CU * clock * 64 / max(N / 2, S) numbers/s.
LANES_FAST, LANES_SHIFT = 128, 64
# (N, S) per generated number, counted in the loop body of each kernel in the
# gfx950 code object (hipcc -S of gen_vN.hip; the unrolled loop of the
# configuration that runs by default).
ALU_MIX = {
    "v0_consume": (201 / 16, 33 / 16),      # k_consume<0, u32, 16>
    "v2_consume": (217 / 16, 33 / 16),      # k_consume<2, u32, 16>
    "v1_generate": (1081 / 32, 400 / 32),   # k_generate_ilv<1, u64, 32, 256, NT>: 14 xor + 7 xor3 + 9 64-bit
                                            # shifts + 2.5 64-bit adds + 1 add3
    "v3_generate": (2181 / 16, 436 / 16),   # k_generate_ilv<3, u32, 16, 512, NT, LDS exchange>
    "v3_consume": (2265 / 16, 449 / 16),    # k_consume<3, u32, 16>
}

# kernels whose loop bodies are integer-only (no f32 instruction to pair with)
INTEGER_ONLY = {"v1_generate"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def headline_launch_key(cfg):
    """The headline's resolved launch configuration as text (which template of
    the kernel runs: tile, round, store mode, buffers, exchange, residency)."""
    return ",".join(f"{k}={cfg[k]}" for k in ("block", "unroll", "store", "waves_per_cu",
                                               "streams_per_lane", "exchange"))


def kernel_source_sha(launch_key=""):
    """Hash of the sources the headline kernel (k_generate_ilv of the exchange
    variant) is built from: its template and launch code, the device helpers,
    the variant's instantiation unit and the kernel-argument struct, plus the
    launch configuration that selects the template's instance."""
    csrc = os.path.join(ROOT, "paper_1112_5239_amd", "csrc")
    h = hashlib.sha256()
    h.update(b"launch\0" + launch_key.encode())
    for name in ("device_common.inc", "gen_kernels.inc", "gen_v2.hip"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(csrc, "internal.h"), "rb") as f:
        text = f.read()
    a = text.index(b"struct GenArgs {")
    h.update(b"GenArgs\0" + text[a:text.index(b"};", a)])
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_tag, launch_key):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was
    taken on the current kernel source and launch configuration; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_sha(launch_key):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def per_launch(torch, fn, count):
    """Device time of each of `count` back-to-back launches (events around each)."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(count)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def cpu_baseline_paper(budget_s=12.0):
    """The oracle, single-threaded, on a bounded sample of the same workload."""
    from oracle import oracle as O
    comb = O.comb_tables(32)
    batch = 8192
    done = 0
    t0 = time.perf_counter()
    O.generate(2, O.seed(2, 1, 0, 32), 16, comb=comb)       # load / warm
    t0 = time.perf_counter()
    elapsed = 0.0
    while elapsed < budget_s and done < (1 << 20):
        st = O.seed(2, 1, done, batch)
        t1 = time.perf_counter()
        O.generate(2, st, 1024, comb=comb)
        elapsed += time.perf_counter() - t1
        done += batch
    return {"value": done * 1024 / elapsed / 1e9, "unit": "Gnumbers/s", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of the 2^20 streams x 1024 outputs (exchange variant, seed 1), "
                      f"{elapsed:.1f} s of single-thread CPU time"}


def cpu_baseline_all_cores(budget_s=8.0):
    """The same oracle run by one thread per host core on disjoint slices of
    exchange groups (ctypes releases the GIL inside the oracle's C code)."""
    import concurrent.futures as cf
    from oracle import oracle as O
    # the host cores this process may use, at most the 16 a GPU's jobs get on
    # a shared host
    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    comb = O.comb_tables(32)
    batch = 2048
    O.generate(2, O.seed(2, 1, 0, 32), 16, comb=comb)
    def work(tid):
        done, first = 0, tid * batch
        t1 = time.perf_counter()
        while time.perf_counter() - t1 < budget_s and first < (1 << 20):
            st = O.seed(2, 1, first, batch)
            O.generate(2, st, 1024, comb=comb)
            done += batch
            first += threads * batch
        return done
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        done = sum(ex.map(work, range(threads)))
    wall = time.perf_counter() - t0
    return {"value": done * 1024 / wall / 1e9, "unit": "Gnumbers/s", "cores": threads, "kind": "oracle",
            "host_cores": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0)),
            "sample": f"{done} of the 2^20 streams x 1024 outputs (exchange variant, seed 1), "
                      f"{threads} threads, {wall:.1f} s wall"}


def run_paper(torch, G, L, args, interleaved, steps=None, warmup=None):
    ns, n = 1 << 20, 1024
    log(f"[bench] paper workload: V2, {ns} streams x {n}, seed 1, "
        f"{'interleaved' if interleaved else 'stream-major'} layout")
    g = G.Generator(ns, "v2", seed=1, interleaved=interleaved)
    shape = (n, ns) if interleaved else (ns, n)
    out = torch.empty(shape, dtype=torch.int32, device="cuda")
    ms, wall = timed(torch, lambda: g.generate(n, out=out), steps or args.steps,
                     args.warmup if warmup is None else warmup)
    numbers = ns * n
    alg_bytes = numbers * 4 + ns * 6 * 4 * 2
    achieved = alg_bytes / (ms / 1e3) / 1e9
    g.close()
    del out
    return ms, wall, numbers, alg_bytes, achieved


def alu_roofline(gn, key):
    """ALU roofline (Gnumbers/s) of a kernel from its per-number VALU mix."""
    n, single = ALU_MIX[key]
    peak = CU * CLOCK_HZ * 64 / max(n / 2, single) / 1e9
    res = {"bound": "alu", "achieved": round(gn, 1), "peak": round(peak, 1), "unit": "Gnumbers/s",
           "frac": round(gn / peak, 4), "valu_per_number": round(n, 3),
           "single_rate_per_number": round(single, 3)}
    if key in INTEGER_ONLY:
        # integer-only mixes holding single-rate shifts issue about one
        # wave64 instruction per CU-clock in total (measured on gfx950)
        peak1 = CU * CLOCK_HZ * 64 / n / 1e9
        res["peak_integer_mix"] = round(peak1, 1)
        res["frac_integer_mix"] = round(gn / peak1, 4)
    return res


def run_plain(torch, G, variant, args, interleaved=False):
    ns, n = 1 << 20, 1024
    words = {"v0": 5, "v1": 23, "v2": 6, "v3": 10, "v4": 4}[variant]
    g = G.Generator(ns, variant, seed=1, interleaved=interleaved)
    shape = (n, ns) if interleaved else (ns, n)
    out = torch.empty(shape, dtype=torch.int32, device="cuda")
    ms, _ = timed(torch, lambda: g.generate(n, out=out), max(5, args.steps // 2), 30)
    g.close()
    del out
    gn = ns * n / (ms / 1e3) / 1e9
    byts = ns * n * 4 + ns * words * 8
    return {"workload": f"{variant}: 2^20 streams x 1024, seed 1, "
                        f"{'interleaved' if interleaved else 'stream-major'} layout",
            "ms": round(ms, 4), "gnumbers_per_s": round(gn, 2), "hbm_gbs": round(byts / (ms / 1e3) / 1e9, 1),
            "frac_hbm_peak": round(byts / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def run_rows_off_lines(torch, G, args):
    """Stream-major rows that start off 128-byte lines (n = 1000: 16-byte
    aligned rows; n = 1001: 4-byte aligned), stored in line-aligned pieces."""
    ns = 1 << 20
    res = {"workload": "2^20 streams, stream-major, default launch, rows of 1000 and 1001 words"}
    for variant, words in (("v0", 5), ("v2", 6)):
        g = G.Generator(ns, variant, seed=1)
        for n in (1000, 1001):
            out = torch.empty((ns, n), dtype=torch.int32, device="cuda")
            ms, _ = timed(torch, lambda: g.generate(n, out=out), max(5, args.steps // 2), 40)
            del out
            byts = ns * n * 4 + ns * words * 8
            res[f"{variant}_n{n}"] = {"ms": round(ms, 4), "hbm_gbs": round(byts / (ms / 1e3) / 1e9, 1),
                                      "frac_hbm_peak": round(byts / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        g.close()
    return res


def _tune_ragged(g, lengths, out, args):
    """Run the batched-launch autotuner unless disabled; returns its record."""
    t0 = time.perf_counter()
    if not args.no_autotune:
        g.autotune_ragged(lengths, out=out)
    cfg = g.resolved_tuning_ragged(lengths)
    return {"tuned": not args.no_autotune, "tune_s": round(time.perf_counter() - t0, 2), "config": cfg}


def run_ragged(torch, G, args, ref_v0_gn):
    """Ratio is against plain V0 in the same (stream-major) layout."""
    from paper_1112_5239_amd import workloads
    lengths = workloads.ragged_lengths()
    ns = lengths.size
    total = int(lengths.sum())
    g = G.Generator(ns, "v0", seed=2)
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    tune = _tune_ragged(g, lengths, out, args)
    ms, _ = timed(torch, lambda: g.generate_ragged(lengths, out=out), max(5, args.steps // 4), 10)
    g.close()
    # The same runs as a device-described subset (cprng_generate_subset):
    # descriptors in device memory, checked, counted and chunked on the device
    # in every call (default tuning: 2048-output chunks).
    gs = G.Generator(ns, "v0", seed=2)
    ids = torch.arange(ns, dtype=torch.int32, device="cuda")
    lens = torch.tensor(lengths.astype(np.int64), device="cuda")
    offs = torch.cumsum(lens, 0) - lens
    ms_sub, _ = timed(torch, lambda: gs.generate_subset(ids, lens, offs, out), max(5, args.steps // 4), 10)
    gs.close()
    del out
    gn = total / (ms / 1e3) / 1e9
    gn_sub = total / (ms_sub / 1e3) / 1e9
    return {"workload": f"4096 streams, log-uniform lengths [1e3,1e7] (total {total}), seed 2, "
                        "one hipGraph launch", "ms": round(ms, 4), "gnumbers_per_s": round(gn, 2),
            "hbm_gbs": round(total * 4 / (ms / 1e3) / 1e9, 1),
            "frac_hbm_peak": round(total * 4 / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "ratio_to_plain_v0": round(gn / ref_v0_gn, 4) if ref_v0_gn else None, **tune,
            "device_subset": {"workload": "the same runs through cprng_generate_subset (descriptors in device "
                                          "memory, planned on the device every call, 2048-output chunks)",
                              "ms": round(ms_sub, 4), "gnumbers_per_s": round(gn_sub, 2),
                              "frac_hbm_peak": round(total * 4 / (ms_sub / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                              "ratio_to_host_planned": round(gn_sub / gn, 4)}}


def run_ragged_groups(torch, G, args, ref_gn):
    """Batched uneven runs of the exchange variant: 128 groups of 32 streams,
    group lengths log-uniform in [1e3, 1e7] (equal within a group), seed 2,
    one hipGraph launch; ratio against plain V2 in the stream-major layout."""
    from paper_1112_5239_amd import workloads
    lengths = workloads.ragged_group_lengths()
    total = int(lengths.sum())
    g = G.Generator(lengths.size, "v2", seed=2)
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    tune = _tune_ragged(g, lengths, out, args)
    ms, _ = timed(torch, lambda: g.generate_ragged(lengths, out=out), max(5, args.steps // 4), 3)
    g.close()
    del out
    gn = total / (ms / 1e3) / 1e9
    return {"workload": f"V2, 128 groups x 32 streams, group lengths log-uniform [1e3,1e7] (total {total}), "
                        "seed 2, one hipGraph launch", "ms": round(ms, 4), "gnumbers_per_s": round(gn, 2),
            "hbm_gbs": round(total * 4 / (ms / 1e3) / 1e9, 1),
            "frac_hbm_peak": round(total * 4 / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "ratio_to_plain_v2_stream_major": round(gn / ref_gn, 4) if ref_gn else None, **tune}


def run_ragged_v1(torch, G, args, ref_gn):
    """Batched uneven runs of V1 on the batched workload's lengths (4,096
    streams, log-uniform [1e3, 1e7], seed 2), one hipGraph launch; ratio
    against plain V1 in the stream-major layout."""
    from paper_1112_5239_amd import workloads
    lengths = workloads.ragged_lengths()
    total = int(lengths.sum())
    g = G.Generator(lengths.size, "v1", seed=2)
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    tune = _tune_ragged(g, lengths, out, args)
    ms, _ = timed(torch, lambda: g.generate_ragged(lengths, out=out), max(5, args.steps // 4), 3)
    g.close()
    del out
    gn = total / (ms / 1e3) / 1e9
    return {"workload": f"V1, 4096 streams, log-uniform lengths [1e3,1e7] (total {total}), seed 2, "
                        "one hipGraph launch", "ms": round(ms, 4), "gnumbers_per_s": round(gn, 2),
            "ratio_to_plain_v1_stream_major": round(gn / ref_gn, 4) if ref_gn else None, **tune}


def run_small(torch, G, args):
    """The small plain configuration: 1,024 streams x 1,024 outputs (4 MiB),
    seed 0, V0 and V1, stream-major: 16 waves, a latency-bound size."""
    res = {"workload": "1024 streams x 1024 uint32 (4 MiB), seed 0, stream-major"}
    for variant in ("v0", "v1"):
        g = G.Generator(1024, variant, seed=0)
        out = torch.empty((1024, 1024), dtype=torch.int32, device="cuda")
        ms, _ = timed(torch, lambda: g.generate(1024, out=out), 200, 20)
        g.close()
        res[variant] = {"ms": round(ms, 5), "gnumbers_per_s": round((1 << 20) / (ms / 1e3) / 1e9, 2),
                        "frac_hbm_peak": round((1 << 22) / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    return res


def run_serving(args):
    from paper_1112_5239_amd import serving
    summary = serving.run_trace(args.serving_duration)
    return {"workload": f"Poisson 2000 req/s for {args.serving_duration:g} s, sizes log-uniform 1 KiB..256 MiB "
                        "of uint32, 10000 resident client streams (V0, seed 4), 64 GiB result budget, "
                        "2 HIP streams; results released as they complete", **summary}


def run_headline_autotuned(torch, G, args, default_ms):
    """The autotuner on the headline workload (interleaved candidates); the
    headline itself is timed on the default configuration before this runs.
    The tuner's pick and the default (as explicit tuning) are then timed in
    alternating rounds, so that slow drifts of the clock hit both alike."""
    ns, n = 1 << 20, 1024
    g = G.Generator(ns, "v2", seed=1, interleaved=True)
    d = G.Generator(ns, "v2", seed=1, interleaved=True)
    # the library's default for this layout: 1,024-stream x 16-step tiles,
    # two tile buffers, non-temporal stores, LDS word exchange
    d.set_tuning(block=1024, unroll=16, store=4, streams_per_lane=2, exchange=2)
    out = torch.empty((n, ns), dtype=torch.int32, device="cuda")
    t0 = time.perf_counter()
    g.autotune(n, scratch=out)
    tune_s = time.perf_counter() - t0
    cfg = g.resolved_tuning(n)
    tuned, default = [], []
    for _ in range(5):
        tuned.append(timed(torch, lambda: g.generate(n, out=out), 10, 2)[0])
        default.append(timed(torch, lambda: d.generate(n, out=out), 10, 2)[0])
    g.close()
    d.close()
    del out
    tm, dm = float(np.median(tuned)), float(np.median(default))
    return {"ms": round(tm, 4), "default_ms_alternating": round(dm, 4), "tune_s": round(tune_s, 2),
            "config": cfg, "ratio_to_default": round(dm / tm, 4)}


def run_copy_probe(torch, L):
    """Two 1 GiB copies by k_copy: the byte counters' calibration in profiled runs."""
    n_words = 1 << 28
    src = torch.zeros(n_words, dtype=torch.int32, device="cuda")
    dst = torch.empty(n_words, dtype=torch.int32, device="cuda")
    for _ in range(2):
        L.cprng_probe_copy(dst, src, n_words, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    del src, dst
    log("[bench] copy probe: 2 x 1 GiB copies (k_copy)")


def run_valu_probes(torch, L):
    """Issue rates (wave64 instructions per CU per clock at the peak clock) of
    the three probe classes, with every CU holding its full complement of waves."""
    n_threads, iters = 1 << 21, 1024
    out = torch.empty(n_threads, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    res = {}
    for kind, name in ((0, "xor"), (1, "shift"), (2, "f32_mul_add"), (3, "shift64"), (4, "add64")):
        ms, _ = timed(torch, lambda: L.cprng_probe_valu(kind, out, n_threads, iters, st), 3, 1)
        rate = n_threads / 64 * iters * 32 / (ms / 1e3)
        res[name] = round(rate / CU / CLOCK_HZ, 3)
    del out
    return {"unit": "wave64 instructions per CU per clock at 2.4 GHz", **res,
            "peak_fast": LANES_FAST / 64, "peak_shift": LANES_SHIFT / 64}


def run_consume(torch, G, args):
    ns, n = 1 << 20, 1 << 16
    res = {}
    for variant in ("v2", "v0", "v3"):
        g = G.Generator(ns, variant, seed=3)
        counts = torch.empty(ns, dtype=torch.int64, device="cuda")
        ms, _ = timed(torch, lambda: g.consume_qc(n, counts=counts), 3, 1)
        g.close()
        gn = ns * n / (ms / 1e3) / 1e9
        res[variant] = {"ms": round(ms, 3), "gnumbers_per_s": round(gn, 1)}
        if f"{variant}_consume" in ALU_MIX:
            res[variant]["roofline"] = alu_roofline(gn, f"{variant}_consume")
    return {"workload": "2^36 uint32 (2^20 streams x 2^16) -> quarter-circle hit counts, seed 3", **res}


def run_dpp_study(torch, G):
    """V2 with the arrays two DPP row rotations implement (groups of 16,
    neighbours j+1 and j+4): the same words through cross-lane reads (1), the
    LDS word buffer (2) and DPP (4), in the consumption kernel (ALU-bound) and
    the interleaved generate kernel (store-bound)."""
    import numpy as np
    c1 = np.array([(j + 1) % 16 for j in range(16)], dtype=np.uint32)
    c2 = np.array([(j + 4) % 16 for j in range(16)], dtype=np.uint32)
    ns = 1 << 20
    res = {"workload": "V2, groups of 16 with the DPP arrays, 2^20 streams, seed 4"}
    g = G.Generator(ns, "v2", seed=4, group=16, comb=(c1, c2))
    counts = torch.empty(ns, dtype=torch.int64, device="cuda")
    for xm in (1, 2, 4):
        g.set_tuning(exchange=xm)
        ms, _ = timed(torch, lambda: g.consume_qc(1 << 16, counts=counts), 3, 1)
        res[f"consume_2^16_xch{xm}_gnumbers_per_s"] = round(ns * 65536 / (ms / 1e3) / 1e9, 1)
    g.close()
    del counts
    g = G.Generator(ns, "v2", seed=4, group=16, comb=(c1, c2), interleaved=True)
    out = torch.empty((1024, ns), dtype=torch.int32, device="cuda")
    for xm in (1, 2, 4):
        g.set_tuning(exchange=xm)
        ms, _ = timed(torch, lambda: g.generate(1024, out=out), 20, 10)
        res[f"interleaved_1024_xch{xm}_ms"] = round(ms, 4)
    g.close()
    del out
    return res


def run_fill_probe(torch, L):
    n_words = 1 << 30
    buf = torch.empty(n_words, dtype=torch.int32, device="cuda")
    ms, _ = timed(torch, lambda: L.cprng_probe_fill(buf, n_words, 7,
                                                      torch.cuda.current_stream().cuda_stream), 10, 2)
    del buf
    return {"bytes": n_words * 4, "ms": round(ms, 4), "gbs": round(n_words * 4 / (ms / 1e3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10, help="untimed steps before the timed ones")
    ap.add_argument("--workload", default="paper",
                    choices=["paper", "ragged", "serving", "consume", "ragged_v1", "ragged_groups"])
    ap.add_argument("--duration", type=float, default=60.0, help="serving: seconds of arrivals")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched legs on the default launch configuration instead of the autotuner's")
    ap.add_argument("--serving-duration", type=float, default=60.0,
                    help="seconds of arrivals of the serving leg in the default run (0: skip it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB copy kernel (hardware byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the streams shard with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    from paper_1112_5239_amd import _lib as L
    from paper_1112_5239_amd import generator as G
    L.lib()

    if args.workload == "serving":
        from paper_1112_5239_amd import serving
        res = serving.bench_line(args)
        print(json.dumps(res), flush=True)
        return
    if args.workload == "consume":
        # The in-kernel consumption kernels alone (ALU-bound), for profiling.
        res = run_consume(torch, G, args)
        log(f"[bench] consume: {res}")
        print(json.dumps({"metric": "in-kernel consumption: Gnumbers/s against the ALU roofline",
                          "value": res["v2"]["gnumbers_per_s"], "unit": "Gnumbers/s", "n_gpus": 1,
                          "ms_per_step": res["v2"]["ms"], "higher_is_better": True, "dtype": "u32",
                          "data": "synthetic", "config": {"workload": res["workload"]},
                          "consume": res}), flush=True)
        return
    if args.workload == "ragged":
        # The batched half of the metric alone, for profiling: uneven streams
        # in one hipGraph launch, against plain V0 (stream-major) timed first.
        ref = run_plain(torch, G, "v0", args, interleaved=False)
        if args.copy_probe:
            run_copy_probe(torch, L)
        res = run_ragged(torch, G, args, ref["gnumbers_per_s"])
        log(f"[bench] ragged: {res}")
        print(json.dumps({"metric": "batched uneven streams: Gnumbers/s and ratio to plain V0",
                          "value": res["gnumbers_per_s"], "unit": "Gnumbers/s", "n_gpus": 1,
                          "ms_per_step": res["ms"], "higher_is_better": True, "dtype": "u32",
                          "data": "synthetic", "config": {"workload": res["workload"]},
                          "plain_v0": ref, "ragged": res}), flush=True)
        return

    if args.workload in ("ragged_v1", "ragged_groups"):
        # Batched uneven runs of V1 (4,096 streams) or of V2 in groups, alone,
        # for profiling, against the plain variant (stream-major) timed first.
        variant = "v1" if args.workload == "ragged_v1" else "v2"
        ref = run_plain(torch, G, variant, args, interleaved=False)
        if args.copy_probe:
            run_copy_probe(torch, L)
        run = run_ragged_v1 if variant == "v1" else run_ragged_groups
        res = run(torch, G, args, ref["gnumbers_per_s"])
        log(f"[bench] {args.workload}: {res}")
        print(json.dumps({"metric": f"batched uneven runs ({variant}): Gnumbers/s and ratio to plain {variant}",
                          "value": res["gnumbers_per_s"], "unit": "Gnumbers/s", "n_gpus": 1,
                          "ms_per_step": res["ms"], "higher_is_better": True, "dtype": "u32",
                          "data": "synthetic", "config": {"workload": res["workload"]},
                          "plain": ref, args.workload: res}), flush=True)
        return

    ns, n = 1 << 20, 1024
    numbers = ns * n
    alg_bytes = numbers * 4 + ns * 6 * 4 * 2        # outputs + the 24-byte state read and written
    log(f"[bench] paper workload: V2, {ns} streams x {n}, seed 1, interleaved layout")
    g = G.Generator(ns, "v2", seed=1, interleaved=True)
    out = torch.empty((n, ns), dtype=torch.int32, device="cuda")
    step = lambda: g.generate(n, out=out)
    extra = {}
    if not args.no_extra:
        # The first launches after the GPU has been idle (host-side seeding just
        # ran): the shader clock settles over ~30-40 ms of activity, and the
        # kernel, store-bound at the settled clock, runs slower meanwhile.  The
        # headline below is timed after the secondary legs, with the clock
        # settled; the same warmup + steps launches from idle are reported here.
        cold = per_launch(torch, step, args.warmup + args.steps)
        win = cold[args.warmup:]
        extra["cold_start"] = {
            "what": "the headline's warmup + steps launches right after idle (before any other leg)",
            "ms_per_launch": [round(x, 4) for x in cold],
            "timed_window_mean_ms": round(sum(win) / len(win), 4),
            "frac_hbm_peak": round(alg_bytes / (sum(win) / len(win) / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"[bench] cold start: window mean {extra['cold_start']['timed_window_mean_ms']} ms")
        if args.serving_duration > 0:
            extra["serving"] = run_serving(args)
            log(f"[bench] serving: {extra['serving']}")
        extra["small"] = run_small(torch, G, args)
        log(f"[bench] small: {extra['small']}")
        sm_ms, _, _, sm_bytes, sm_ach = run_paper(torch, G, L, args, interleaved=False,
                                                  steps=max(5, args.steps // 2), warmup=30)
        extra["v2_stream_major"] = {"workload": "the same run in the stream-major layout out[s * 1024 + i]",
                                    "ms": round(sm_ms, 4), "gnumbers_per_s": round(numbers / (sm_ms / 1e3) / 1e9, 2),
                                    "hbm_gbs": round(sm_ach, 1), "frac_hbm_peak": round(sm_ach / HBM_PEAK_GBS, 4)}
        log(f"[bench] v2 stream-major: {extra['v2_stream_major']}")
        extra["valu_probe"] = run_valu_probes(torch, L)
        log(f"[bench] valu probe: {extra['valu_probe']}")
        for variant in ("v0", "v1", "v3", "v4"):
            for ilv in (True, False):
                key = f"{variant}_{'interleaved' if ilv else 'stream_major'}"
                extra[key] = run_plain(torch, G, variant, args, interleaved=ilv)
                if f"{variant}_generate" in ALU_MIX:
                    extra[key]["roofline"] = alu_roofline(extra[key]["gnumbers_per_s"], f"{variant}_generate")
                log(f"[bench] {key}: {extra[key]}")
        extra["rows_off_lines"] = run_rows_off_lines(torch, G, args)
        log(f"[bench] rows off lines: {extra['rows_off_lines']}")
        extra["ragged"] = run_ragged(torch, G, args, extra["v0_stream_major"]["gnumbers_per_s"])
        log(f"[bench] ragged: {extra['ragged']}")
        extra["ragged_groups_v2"] = run_ragged_groups(torch, G, args, extra["v2_stream_major"]["gnumbers_per_s"])
        log(f"[bench] ragged groups (V2): {extra['ragged_groups_v2']}")
        extra["ragged_v1"] = run_ragged_v1(torch, G, args, extra["v1_stream_major"]["gnumbers_per_s"])
        log(f"[bench] ragged (V1): {extra['ragged_v1']}")
        extra["consume"] = run_consume(torch, G, args)
        log(f"[bench] consume: {extra['consume']}")
        extra["dpp_study"] = run_dpp_study(torch, G)
        log(f"[bench] dpp study: {extra['dpp_study']}")
        extra["fill_probe"] = run_fill_probe(torch, L)
        log(f"[bench] fill probe: {extra['fill_probe']}")

    # Headline: warmup untimed steps, then exactly `steps` timed steps, each
    # launch bracketed by its own events as well (the kernel's duration).
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for a, b in ev:
        a.record()
        step()
        b.record()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    launches = [a.elapsed_time(b) for a, b in ev]
    kernel_ms = sum(launches) / len(launches)
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
    value = numbers / (ms / 1e3) / 1e9
    log(f"[bench] paper: {ms:.4f} ms/step ({kernel_ms:.4f} ms per launch), {value:.1f} Gnumbers/s, "
        f"{achieved:.0f} GB/s")
    extra["headline_launch_ms"] = [round(x, 4) for x in launches]
    launch_key = headline_launch_key(g.resolved_tuning(n))
    log(f"[bench] headline launch: {launch_key}")
    if args.copy_probe:
        run_copy_probe(torch, L)
    g.close()
    del out
    if not args.no_extra and not args.no_autotune:
        extra["headline_autotuned"] = run_headline_autotuned(torch, G, args, ms)
        log(f"[bench] headline autotuned: {extra['headline_autotuned']}")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_paper()
        log(f"[bench] cpu baseline: {cpu}")
        if not args.no_extra:
            extra["cpu_baseline_all_cores"] = cpu_baseline_all_cores()
            log(f"[bench] cpu baseline, all cores: {extra['cpu_baseline_all_cores']}")
    if "fill_probe" in extra:
        extra["headline_vs_fill_probe"] = round(achieved / extra["fill_probe"]["gbs"], 4)
    line = {
        "metric": "Gnumbers/s (uint32 to HBM) at 1 GPU, % HBM write peak; plain vs batched",
        "value": round(value, 3),
        "unit": "Gnumbers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "paper-shaped neighbour-exchange variant (Algorithm 4): 2^20 streams "
                               "x 1024 uint32 outputs (4 GiB), SplitMix64 seed 1, group 32, interleaved "
                               "layout out[i * 2^20 + s]",
                   "n_streams": ns, "n_per_stream": n, "variant": "v2", "layout": "interleaved",
                   "timed_after": "the secondary legs (shader clock settled)" if not args.no_extra
                                  else "the first launches after idle"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile("k_generate_ilv_v2_paper", launch_key),
                     "algorithmic_bytes_per_launch": alg_bytes, "kernel_ms": round(kernel_ms, 5)},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
