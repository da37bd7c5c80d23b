#!/usr/bin/env python3
"""Benchmark of the pre-alignment filter path on one MI355X.

Workload: 10M synthetic (read, reference segment) pairs of 250 bp, 2-bit
packed and resident in HBM, E = 10 (70% unrelated segments, related ones with
k ~ U{0..40} random edits).  One step = one pass of the whole path over the
batch: features and cost model (a cost level per pair), then the compacting
filter (load, map build, SneakySnake traversal, decision and output writes)
with each chunk's pairs taken in level order.  The plain filter (no model) is
timed beside it.

Prints one JSON line.  `roofline` is for the dominant kernel (for the filter,
algorithmic bytes: both packed sequences and the level in, counts and accept
bits out), timed with HIP events on the stream the kernel runs on;
`cpu_baseline` is the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# One wave64 VALU instruction per SIMD every 4 cycles (256 CUs x 4 SIMDs,
# 2.4 GHz): 614.4 G/s.  A model line only: adds and 3-input logic issue
# faster than this (valu_ceiling measures it), funnel shifts and popcounts
# at about this rate.
VALU_PEAK_GIPS = 256 * 4 * 2.4 / 4


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_batch(ctx, w, n, dev, chunk=2_000_000):
    """Generate pairs [0, n) of workload w chunk by chunk and pack them on the GPU."""
    import torch

    import pairgen
    import paper_1910_03936_amd as paf

    m = w.lens[0]
    stride = paf.words_for(m)
    rd = torch.empty(n * stride, dtype=torch.int64, device=dev)
    rf = torch.empty(n * stride, dtype=torch.int64, device=dev)
    first = None
    for a in range(0, n, chunk):
        q = pairgen.generate(w, a, min(chunk, n - a))
        if first is None:
            first = q
        r = ctx.pack(torch.from_numpy(q.reads).to(dev), uniform_len=m, stride_words=stride)
        f = ctx.pack(torch.from_numpy(q.refs).to(dev), uniform_len=m, stride_words=stride)
        rd[a * stride:(a + q.n) * stride] = r
        rf[a * stride:(a + q.n) * stride] = f
        del r, f
    torch.cuda.synchronize()
    ctx.check()
    E = w.fixed_E
    b = paf.Batch(rd, rf, n, stride, uniform_len=m, uniform_E=E, max_len=m, max_E=E)
    return b, first


def ramp(fn, seconds=0.3):
    """Untimed launches of fn for a few hundred ms: the GPU's clocks ramp up
    under load, and a timed region should not start while they do."""
    import torch

    t = time.perf_counter()
    while time.perf_counter() - t < seconds:
        fn()
        torch.cuda.synchronize()


def time_steps(fn, steps, warmup):
    """Per-step HIP event times (ms) on the current stream, plus the total."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(s)
    for a, b in ev:
        a.record(s)
        fn()
        b.record(s)
    t1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per = [a.elapsed_time(b) for a, b in ev]
    return per, t0.elapsed_time(t1), wall


# A kernel's sources: its file and the device headers it includes.  A traffic
# record holds their hash and is used only while it matches.
KERNEL_SOURCES = {"snake_chunk": ("filter.hip", "paf_tile.h", "paf_map.h", "paf_internal.h"),
                  "key_levels": ("mlp.hip", "paf_map.h", "paf_internal.h")}


def kernel_source_hash(kernel: str = "snake_chunk") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1910_03936_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(key: str, path: str | None = None):
    """HBM bytes per launch measured with rocprofv3 counters, if they were taken
    on the current sources of the record's kernel (else None).  Keys name the
    kernel first: `key_levels_...` records hold the levels kernel, the others
    the compacting filter."""
    path = path or os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    r = rec.get(key)
    kernel = "key_levels" if key.startswith("key_levels") else "snake_chunk"
    if not r or r.get("kernel_sha256_16") != kernel_source_hash(kernel):
        return None
    return r


# Chunk-size and pass-width sweep of the compacting filter (the first entry is
# the layout paf_filter picks by itself at max_E 9..15).
LAYOUT_SWEEP = "2,6,2,3;2,8,2,3;2,4,2,3;4,4,2,3;2,3,2,3;2,2,2,3;2,6,3,3"


def parse_layouts(spec: str) -> list:
    """'W,K,F,P;...' -> paf_layout dicts (one lane per pair, full grid)."""
    out = []
    for part in spec.split(";"):
        wpb, k, f, p = (int(x) for x in part.split(","))
        out.append({"lanes_per_pair": 1, "waves_per_block": wpb, "blocks_per_cu": 0, "tiles_per_grab": 1,
                    "chunk_tiles": k, "first_pass_windows": f, "pass_windows": p})
    return out


def layout_tuple(lay: dict) -> list:
    return [lay["waves_per_block"], lay["chunk_tiles"], lay["first_pass_windows"], lay["pass_windows"]]


def counter_run(args):
    """One kind of launch, repeated, for rocprofv3 counter runs: `plain` is the
    compacting filter alone; `keyed` trains the cost model on --train-pairs
    pairs, then runs the cost levels and the keyed filter in turn.  Every
    dispatch of the chosen kernels in such a run is the record's launch."""
    import torch

    import pairgen
    import paper_1910_03936_amd as paf
    from paper_1910_03936_amd import costmodel

    dev = torch.device("cuda", 0)
    ctx = paf.Context(0)
    w = pairgen.FIXED_250BP.with_E(args.E)
    n = args.pairs or w.n_pairs
    batch, _ = build_batch(ctx, w, n, dev)
    out = ctx.alloc_out(n, paf.SNEAKYSNAKE, dev)
    if args.counter_run == "plain":
        step = lambda: ctx.filter(batch, paf.SNEAKYSNAKE, out=out)
    else:
        costmodel.train(ctx, w, n=args.train_pairs, epochs=4, batch=4096, lr=2e-3)
        step = lambda: ctx.filter_keyed(batch, ctx.cost_levels(batch), out=out)
    layouts = parse_layouts(args.layout) if args.layout else [None]
    for lay in layouts:
        # With several layouts the dispatches come in this order, --steps each.
        ctx.set_layout(lay)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
    ctx.set_layout(None)
    ctx.check()
    print(json.dumps({"counter_run": args.counter_run, "n_pairs": n, "E": args.E, "launches": args.steps,
                      "layouts": [layout_tuple(l) for l in layouts if l is not None]}), flush=True)


def _counter_csv(path):
    """Per-dispatch counter sums of a rocprofv3 --pmc output folder:
    {dispatch id: (kernel name, {counter: value})}."""
    import csv
    import glob

    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit(f"expected one counter_collection.csv under {path}, found {len(files)}")
    out = {}
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            name, vals = out.setdefault(d, (r["Kernel_Name"], {}))
            vals[r["Counter_Name"]] = vals.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def record_traffic(args):
    """Writes profiles/hbm_traffic.json (or --record-out) from counter runs under DIR:
    plain_fetch, plain_write, plain_valu, keyed_fetch, keyed_write,
    keyed_valu (bench.py --counter-run plain|keyed under rocprofv3 --pmc
    FETCH_SIZE / WRITE_SIZE / the SQ counters), and cfetch, cwrite (the same
    counters over bench.py --calibrate-copy).  FETCH_SIZE and WRITE_SIZE are
    KiB per dispatch; each is scaled by the ratio of the copy's true bytes to
    what the counter reads for it."""
    d = args.record_traffic
    n = args.pairs or 10_000_000
    gib = 2 << 30
    fs = gib / (max(v["FETCH_SIZE"] for _, v in _counter_csv(os.path.join(d, "cfetch")).values()) * 1024)
    ws = gib / (max(v["WRITE_SIZE"] for _, v in _counter_csv(os.path.join(d, "cwrite")).values()) * 1024)
    # The levels kernel's second template argument picks its form (two tiles
    # of words in flight on uniform batches); either form counts.
    kernels = {"snake_chunk": (f"chunk_kernel<{args.E}, false, false, 1>(",),
               "key_levels": (f"key_kernel<{args.E}>(", f"key_kernel<{args.E}, true>(", f"key_kernel<{args.E}, false>(")}
    rec = {}

    def mean(kind, part, knames):
        rows = [v for name, v in _counter_csv(os.path.join(d, f"{kind}_{part}")).values()
                if any(k in name for k in knames)]
        if not rows:
            return None, 0
        return {k: sum(r.get(k, 0.0) for r in rows) / len(rows) for k in rows[0]}, len(rows)

    for kind in ("plain", "keyed"):
        for label, kname in kernels.items():
            if label == "key_levels" and kind == "plain":
                continue
            fv, nd = mean(kind, "fetch", kname)
            wv, _ = mean(kind, "write", kname)
            vv, _ = mean(kind, "valu", kname)
            if fv is None or wv is None or vv is None:
                raise SystemExit(f"no {kname[0][:-1]} dispatches in the {kind} counter runs")
            fb, wb = fv["FETCH_SIZE"] * 1024 * fs, wv["WRITE_SIZE"] * 1024 * ws
            key = f"{label}_{kind}_250bp_E{args.E}" if label == "snake_chunk" else f"{label}_250bp_E{args.E}"
            rec[key] = {"kernel_sha256_16": kernel_source_hash(label), "kernel": kname[0][:-1], "n_pairs": n,
                        "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                        "bytes_per_launch": fb + wb, "fetch_scale": fs, "write_scale": ws, "dispatches": nd,
                        "waves_per_launch": vv["SQ_WAVES"],
                        "valu_insts_per_launch": vv["SQ_INSTS_VALU"],
                        "valu_lane_util": vv["SQ_THREAD_CYCLES_VALU"] / (64 * vv["SQ_ACTIVE_INST_VALU"]),
                        "mfma_insts_per_launch": vv.get("SQ_INSTS_MFMA", 0.0),
                        "wait_per_wave_cycle": vv["SQ_WAIT_ANY"] / vv["SQ_WAVE_CYCLES"],
                        "gui_active_cycles_per_xcd": vv["GRBM_GUI_ACTIVE"] / 8}
    path = args.record_out or os.path.join(ROOT, "profiles", "hbm_traffic.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    for k, r in rec.items():
        log(f"{k}: {r['dispatches']} dispatches, fetch {r['fetch_bytes_per_launch'] / 1e9:.4f} GB, write "
            f"{r['write_bytes_per_launch'] / 1e9:.4f} GB, VALU {r['valu_insts_per_launch']:.4g}, lanes "
            f"{r['valu_lane_util']:.3f}, wait {r['wait_per_wave_cycle']:.3f}")
    log(f"copy scale: fetch x {fs:.4f}, write x {ws:.4f}; wrote {path}")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample, E, budget_s=10.0, single_budget_s=3.0):
    """The oracle (as is) on host threads over a bounded sample of the workload:
    the first chunk of pairs, passed over repeatedly until about budget_s of
    wall time has been spent on 16 threads (the CPU share of one GPU on the
    benchmark machine; nproc is reported beside it), and a single-thread rate
    on the sample's first 100k pairs."""
    import oracle

    nproc = os.cpu_count() or 1
    threads = max(1, min(16, nproc))

    def rate(reads, refs, lens, th, budget):
        done, reps = 0, 0
        t = time.perf_counter()
        while True:
            oracle.filter_batch(reads, refs, lens, E, oracle.SNEAKYSNAKE, threads=th)
            done += reads.shape[0]
            reps += 1
            dt = time.perf_counter() - t
            if dt >= budget or reps >= 200:
                return done / dt, reps, dt

    k = min(100_000, sample.n)
    one, reps1, dt1 = rate(sample.reads[:k], sample.refs[:k], sample.len[:k], 1, single_budget_s)
    many, reps, dt = rate(sample.reads, sample.refs, sample.len, threads, budget_s)
    return {"value": many, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample.n} pairs of the workload x {reps} passes, SneakySnake only, "
                      f"{dt:.1f} s on {threads} threads; single thread: first {k} pairs x {reps1} passes, "
                      f"{dt1:.1f} s",
            "single_thread": one, "nproc": nproc, "cpu_model": cpu_model(),
            "threads_note": f"{threads} threads = min(16, nproc); 16 is the host CPU share of one GPU on the "
                            f"benchmark machine"}


def calibrate_copy(gib=2.0, reps=5):
    """A plain device-to-device copy of known size: the reference the HBM
    counters (FETCH_SIZE / WRITE_SIZE) of the filter kernel are scaled by."""
    import torch

    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.int64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 8, "reps": reps}), flush=True)


def hbm_ceiling(gib=4.0, reps=3):
    """Measured HBM rates: a streaming read of `gib` GiB (libpaf_calib.so's
    read kernel, 16-byte loads at a grid stride, best over grid sizes) and a
    device-to-device copy of half that size (torch), each the fastest of
    `reps` launches timed with HIP events.  Returns GB/s (1e9 bytes)."""
    import ctypes

    import torch

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1910_03936_amd", "libpaf_calib.so"))
    lib.paf_calib_read.restype = ctypes.c_float
    lib.paf_calib_read.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                   ctypes.c_void_p]
    nbytes = int(gib * (1 << 30))
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    read = {}
    for per_cu in (4, 8, 16, 32):
        ms = lib.paf_calib_read(ctypes.c_void_p(src.data_ptr()), nbytes // 16, cus * per_cu, reps,
                                ctypes.c_void_p(out.data_ptr()))
        if ms <= 0:
            raise RuntimeError(f"read calibration failed (code {ms})")
        read[per_cu] = nbytes / (ms / 1e3) / 1e9
    half = src[: src.numel() // 2]
    dst = torch.empty_like(half)
    best = 1e30
    for r in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(half)
        b.record()
        b.synchronize()
        if r > 0:
            best = min(best, a.elapsed_time(b))
    copy = 2 * half.numel() * 8 / (best / 1e3) / 1e9
    return {"read_GBps": round(max(read.values()), 1), "read_GBps_by_blocks_per_cu": {k: round(v, 1) for k, v in read.items()},
            "copy_GBps_read_plus_write": round(copy, 1), "bytes_read": nbytes}


CALIB_MIXES = ("v_add_u32", "v_bitop3_b32", "v_bcnt_u32_b32", "probe: v_add_u32 + v_bitop3_b32",
               "v_alignbit_b32", "v_pk_add_u16", "map: v_alignbit_b32 + v_bitop3_b32")
PROBE_MIX = 3


def valu_ceiling(mixes=None, waves_per_simd=(8,), iters=20000, reps=3):
    """Measured VALU issue rate (G wave64 instructions/s) of known instruction
    mixes: libpaf_calib.so's kernel runs `iters` turns of 16 inline-asm VALU
    instructions per thread, timed with HIP events.  Returns
    {mix name: {waves per SIMD: rate}}."""
    import ctypes

    import torch

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1910_03936_amd", "libpaf_calib.so"))
    lib.paf_calib_valu.restype = ctypes.c_float
    lib.paf_calib_valu.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p]
    per_turn = lib.paf_calib_per_turn()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    res = {}
    for mix in (range(len(CALIB_MIXES)) if mixes is None else mixes):
        row = {}
        for wps in waves_per_simd:
            blocks = cus * wps            # 256-thread blocks: 4 waves, one per SIMD
            ms = lib.paf_calib_valu(mix, blocks, iters, reps, ctypes.c_void_p(out.data_ptr()))
            if ms <= 0:
                raise RuntimeError(f"VALU calibration failed (code {ms})")
            row[wps] = blocks * 4 * iters * per_turn / (ms / 1e3) / 1e9
        res[CALIB_MIXES[mix]] = row
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=None, help="override the batch size (default 10M)")
    ap.add_argument("--E", type=int, default=10)
    ap.add_argument("--train-pairs", type=int, default=2_000_000)
    ap.add_argument("--no-learned", action="store_true", help="time the plain filter only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="fixed250",
                    choices=["fixed250", "filters", "partitioned", "verify", "accuracy", "uneven", "learned-uneven",
                             "stream", "layouts"],
                    help="fixed250 (default): 10M x 250 bp at E (plain and learned-bucketed); filters: the "
                         "same pairs at E = 0, 5, 10, 25 with SneakySnake, GateKeeper, Shouji and all three "
                         "on one map; uneven: 50M pairs of mixed lengths in the persistent launch, default "
                         "vs autotuned layout; learned-uneven: the same batch, learned-bucketed vs plain; "
                         "stream: 200M pairs streamed from pinned host memory in 8M-pair chunks; "
                         "filters also times MAGNET; partitioned: SneakySnake on sub-mazes of t = 5, 10, 25, 50 columns vs the whole maze "
                         "at E = 0, 5, 10, 25; verify: banded edit distance of the pairs SneakySnake accepts "
                         "(filter + verify) vs verifying every pair, at E = 5, 10, 25; accuracy: false accept "
                         "and false reject rates of every filter against the exact banded distance, at E = 0, 5, "
                         "10, 25; layouts: the plain filter at E under each forced compacting layout (--layout)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain copy kernel of known size (counter calibration)")
    ap.add_argument("--calibrate-hbm", action="store_true",
                    help="only measure the streaming read and copy rates of HBM and print them")
    ap.add_argument("--calibrate-valu", action="store_true",
                    help="only measure the VALU issue rate of known instruction mixes and print it")
    ap.add_argument("--reps", type=int, default=3, help="timed repetitions of each calibration kernel")
    ap.add_argument("--counter-run", choices=["plain", "keyed"], default=None,
                    help="only launch one kind of filter step --steps times (for rocprofv3 counter runs)")
    ap.add_argument("--layout", default=None, metavar="W,K,F,P[;...]",
                    help="forced compacting layouts (waves per block, tiles per chunk, first / later pass "
                         "windows): --counter-run plain launches each in turn, --workload layouts times "
                         "each (default: the chunk-size sweep)")
    ap.add_argument("--record-traffic", metavar="DIR", default=None,
                    help="write profiles/hbm_traffic.json from the counter runs under DIR (no GPU)")
    ap.add_argument("--record-out", metavar="PATH", default=None,
                    help="where --record-traffic writes (default profiles/hbm_traffic.json)")
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(args)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.calibrate_hbm:
        r = hbm_ceiling(reps=args.reps)
        log(f"HBM streaming read {r['read_GBps']} GB/s, copy {r['copy_GBps_read_plus_write']} GB/s")
        print(json.dumps(dict(r, published_peak_GBps=HBM_PEAK_GBS)), flush=True)
        return
    if args.calibrate_valu:
        r = valu_ceiling(waves_per_simd=(1, 2, 4, 8), reps=args.reps)
        for k, v in r.items():
            log(f"{k:40s} " + "  ".join(f"{w} waves/SIMD: {g:7.1f} G/s" for w, g in v.items()))
        print(json.dumps({"valu_wave_instr_per_s_G": r, "model_line_G": VALU_PEAK_GIPS}), flush=True)
        return

    if args.counter_run:
        counter_run(args)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): there is no "
              f"multi-GPU path; pairs are independent, so several GPUs would each filter a contiguous "
              f"range of the batch with no exchange.", file=sys.stderr)
        sys.exit(2)

    import torch

    import pairgen
    import paper_1910_03936_amd as paf
    from paper_1910_03936_amd import costmodel

    if args.workload == "filters":
        filters_workload(args)
        return
    if args.workload in ("partitioned", "verify", "accuracy"):
        next_workloads(args)
        return
    if args.workload == "layouts":
        layouts_workload(args)
        return
    if args.workload != "fixed250":
        other_workload(args)
        return
    dev = torch.device("cuda", 0)
    ctx = paf.Context(0)
    w = pairgen.FIXED_250BP.with_E(args.E)
    n = args.pairs or w.n_pairs
    t = time.perf_counter()
    batch, first = build_batch(ctx, w, n, dev)
    log(f"generated and packed {n} pairs in {time.perf_counter() - t:.1f} s")
    W = paf.words_for(250)
    SS = paf.SNEAKYSNAKE

    # Plain batched filter.  The GPU's clocks ramp up under load: run the
    # filter untimed for a few hundred ms before the first timed region.
    out = ctx.alloc_out(n, SS, dev)
    ramp(lambda: ctx.filter(batch, SS, out=out))
    per, total_ms, _ = time_steps(lambda: ctx.filter(batch, SS, out=out), args.steps, args.warmup)
    ctx.check()
    plain_ms = total_ms / args.steps
    plain_kern_ms = sum(per) / len(per)
    plain_value = n / (plain_ms / 1e3)
    log(f"plain: {plain_ms:.3f} ms/step, {plain_value / 1e9:.2f} G pairs/s")
    plain_bytes_pair = 2 * W * 8 + 2 + 1 / 8
    valu_peak = valu_ceiling(mixes=[PROBE_MIX], waves_per_simd=(8,))[CALIB_MIXES[PROBE_MIX]][8]
    log(f"VALU issue ceiling (measured, {CALIB_MIXES[PROBE_MIX]}): {valu_peak:.1f} G wave-instr/s")

    def roof(kern_ms, bytes_pair, kernel, key):
        achieved = n * bytes_pair / (kern_ms / 1e3) / 1e9
        tr = traffic_record(key)
        r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(achieved / HBM_PEAK_GBS, 4),
             "traffic": None if tr is None else tr["bytes_per_launch"] * n / tr["n_pairs"],
             "kernel": kernel, "kernel_ms": round(kern_ms, 4), "alg_bytes_per_pair": round(bytes_pair, 3)}
        if tr is not None and "valu_insts_per_launch" in tr:
            # The filter is integer bit work: what it is bound by in fact is
            # the VALU issue rate.  Instructions per launch from the profiled
            # counters (same kernel source), over this run's time, against
            # the issue rate measured in this run on the probe's own pair of
            # instructions (the fastest VALU mix measured on the chip).
            ips = tr["valu_insts_per_launch"] * n / tr["n_pairs"] / (kern_ms / 1e3)
            r["valu_issue"] = {"achieved": round(ips / 1e9, 1), "peak": round(valu_peak, 1),
                               "unit": "G wave-instr/s", "frac": round(ips / 1e9 / valu_peak, 4),
                               "peak_kind": f"measured in this run: {CALIB_MIXES[PROBE_MIX]} at 8 waves per SIMD",
                               "model_line": VALU_PEAK_GIPS,
                               "lane_util": round(tr.get("valu_lane_util", 0.0), 3)}
        return r

    plain = {"value": plain_value, "ms_per_step": plain_ms,
             "roofline": roof(plain_kern_ms, plain_bytes_pair,
                              f"chunk_kernel<E={args.E}, uniform> (compacting SneakySnake, 6-tile chunks, 2-window passes)",
                              f"snake_chunk_plain_250bp_E{args.E}")}
    rec_value, rec_ms, roofline, learned = plain_value, plain_ms, plain["roofline"], None

    if not args.no_learned:
        # Cost model: trained outside the timed region on pairs drawn like the
        # workload (another seed), labelled by the filter itself at E = 31.
        t = time.perf_counter()
        losses = costmodel.train(ctx, w, n=args.train_pairs, epochs=4, batch=4096, lr=2e-3)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t
        log(f"trained the cost model on {args.train_pairs} pairs in {train_s:.1f} s, losses {losses}")
        # The learned pipeline: model levels, then the compacting filter with
        # each chunk ordered by them (one graph).
        out_l = ctx.alloc_out(n, SS, dev)
        # The same untimed ramp as the plain filter's (training leaves the
        # GPU idle for a while).
        ramp(lambda: ctx.filter_bucketed_local(batch, out=out_l))
        per_l, total_l, _ = time_steps(lambda: ctx.filter_bucketed_local(batch, out=out_l), args.steps,
                                       args.warmup)
        ctx.check()
        same = bool(torch.equal(out[SS][0], out_l[SS][0]) and torch.equal(out[SS][1], out_l[SS][1]))
        learned_ms = total_l / args.steps
        learned_value = n / (learned_ms / 1e3)
        # Its two stages, each launched and timed on its own.
        key = ctx.cost_levels(batch)
        ramp(lambda: ctx.cost_levels(batch))
        per_m, _, _ = time_steps(lambda: ctx.cost_levels(batch), args.steps, 1)
        out_k = ctx.alloc_out(n, SS, dev)
        ramp(lambda: ctx.filter_keyed(batch, key, out=out_k))
        per_k, _, _ = time_steps(lambda: ctx.filter_keyed(batch, key, out=out_k), args.steps, 1)
        model_ms, keyed_ms = sum(per_m) / len(per_m), sum(per_k) / len(per_k)
        hist = torch.bincount(key.to(torch.int64), minlength=16)
        # Ablations of the key (the keyed filter alone, same layout): a
        # constant key (the sort's own cost), the trivial length x E key
        # (constant on this uniform batch) and the true labels' levels (the
        # best any prediction could do).
        ablation = {}
        keys = (("constant", torch.full((n,), 15, dtype=torch.uint8, device=dev)),
                ("length x E", costmodel.length_e_key(batch)),
                ("true labels (bound)", costmodel.oracle_key(ctx, batch)),
                ("model", key))
        for _ in range(2):   # the best of two rounds (the first key timed runs slow)
            for kname, kk in keys:
                per_a, _, _ = time_steps(lambda: ctx.filter_keyed(batch, kk, out=out_k), args.steps, args.warmup)
                ablation[kname] = min(ablation.get(kname, 1e9), round(sum(per_a) / len(per_a), 4))
        ctx.check()
        # Where ordering pays: the per-tile engine (no compaction; each wave
        # keeps its 64 pairs until all are decided, so a wave lasts as long
        # as its costliest pair) in input order, in the model's 16-bucket
        # order and in the true labels' order.
        per_tile = {}
        ctx.set_layout({"lanes_per_pair": 1, "waves_per_block": 4, "blocks_per_cu": 0, "tiles_per_grab": 1,
                        "chunk_tiles": 0})
        try:
            pred = ctx.mlp_predict(batch)
            perm_model, _ = ctx.bucket(batch, pred)
            lab = costmodel.labels_for(ctx, batch).to(torch.int64)
            perm_true = torch.argsort(-lab, stable=True).to(torch.int32)
            out_o = ctx.alloc_out(n, SS, dev)
            for oname, fn in (("input order", lambda: ctx.filter(batch, SS, out=out_o)),
                              ("model's 16 buckets", lambda: ctx.filter_ordered(batch, perm_model, SS, out=out_o)),
                              ("true labels' order", lambda: ctx.filter_ordered(batch, perm_true, SS, out=out_o))):
                per_o, _, _ = time_steps(fn, args.steps, args.warmup)
                per_tile[oname] = round(sum(per_o) / len(per_o), 4)
            ctx.check()
        finally:
            ctx.set_layout(None)
        heldout = costmodel.evaluate(ctx, w)
        log(f"keyed filter by key: {ablation}; per-tile engine by order: {per_tile}; held-out MSE "
            f"{heldout['mse']:.3f} MAE {heldout['mae']:.3f} (predicting the mean: MSE {heldout['mse_of_mean']:.3f})")
        # For context: the same model with a global 16-bucket permutation.
        gsteps = max(3, args.steps // 4)
        out_g = ctx.alloc_out(n, SS, dev)
        _, total_g, _ = time_steps(lambda: ctx.filter_bucketed(batch, SS, out=out_g), gsteps, 1)
        torch.cuda.synchronize()
        log(f"learned: {learned_ms:.3f} ms/step, {learned_value / 1e9:.2f} G pairs/s "
            f"(x{plain_ms / learned_ms:.2f} vs plain), identical decisions: {same}; model {model_ms:.3f} ms, "
            f"keyed filter {keyed_ms:.3f} ms; global permutation {total_g / gsteps:.3f} ms")
        learned = {"value": learned_value, "ms_per_step": learned_ms,
                   "vs_plain": round(plain_ms / learned_ms, 3), "identical_decisions": same,
                   "stages_ms": {"features+model (levels)": round(model_ms, 4),
                                 "compacting filter, chunks ordered by level": round(keyed_ms, 4)},
                   # The levels stage on its own line: five words read per
                   # pair (three of the read, two of the reference) and one
                   # byte written.
                   "levels_roofline": roof(model_ms, 5 * 8 + 1,
                                           f"key_kernel<E={args.E}, two sets> (features, gate, bf16 MLP, level)",
                                           f"key_levels_250bp_E{args.E}"),
                   "level_sizes": hist.cpu().tolist(),
                   "keyed_filter_ms_by_key": ablation,
                   "per_tile_engine_ms_by_order": per_tile,
                   "heldout": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in heldout.items()},
                   "global_permutation_ms_per_step": round(total_g / gsteps, 4),
                   "train": {"pairs": args.train_pairs, "epochs": 4, "seconds": round(train_s, 2),
                             "epoch_mse": [round(float(x), 3) for x in losses]}}
        rec_value, rec_ms = learned_value, learned_ms
        if keyed_ms >= model_ms:
            roofline = roof(keyed_ms, plain_bytes_pair + 1,
                            f"chunk_kernel<E={args.E}, uniform> with chunks ordered by the model's levels",
                            f"snake_chunk_keyed_250bp_E{args.E}")
        else:
            flops = n * 2 * (64 * 128 + 128 * 128 + 128)
            a = flops / (model_ms / 1e3) / 1e12
            roofline = {"bound": "mfma", "achieved": round(a, 1), "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": round(a / 2500.0, 4), "traffic": None,
                        "kernel": "key_kernel (features + bf16 MLP + level)", "kernel_ms": round(model_ms, 4),
                        "alg_flops_per_pair": 2 * (64 * 128 + 128 * 128 + 128)}

    cpu = None
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        cpu = cpu_baseline(first, args.E)
        log(f"cpu baseline {cpu['value']:.3g} pairs/s ({time.perf_counter() - t:.1f} s)")

    rec = {
        "metric": "filtered pairs/sec at 250bp E=10, learned-bucketed vs plain; HBM GB/s %peak",
        "value": rec_value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{n} pairs, 250 bp, 2-bit packed, E={args.E}, 70% unrelated, "
                               f"k~U{{0..40}}; SneakySnake; "
                               + ("plain batched launch" if args.no_learned else
                                  "learned-bucketed (features, bf16 MLP, 16 cost levels ordering each "
                                  "compacting chunk, filter)"),
                   "pairs": n, "read_len": 250, "E": args.E, "filters": "sneakysnake",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain": plain,
        "learned": learned,
    }
    print(json.dumps(rec), flush=True)
    ctx.close()


def layouts_workload(args):
    """10M x 250 bp at E: the plain compacting filter under each forced layout,
    timed with HIP events after a clock ramp, outputs compared with the
    filter's own choice."""
    import torch

    import pairgen
    import paper_1910_03936_amd as paf

    dev = torch.device("cuda", 0)
    ctx = paf.Context(0)
    w = pairgen.FIXED_250BP.with_E(args.E)
    n = args.pairs or w.n_pairs
    batch, _ = build_batch(ctx, w, n, dev)
    SS = paf.SNEAKYSNAKE
    ref = ctx.filter(batch, SS)
    out = ctx.alloc_out(n, SS, dev)
    rows = []
    for lay in parse_layouts(args.layout or LAYOUT_SWEEP):
        ctx.set_layout(lay)
        step = lambda: ctx.filter(batch, SS, out=out)
        ramp(step)
        per, total, _ = time_steps(step, args.steps, args.warmup)
        same = all(torch.equal(out[SS][j], ref[SS][j]) for j in range(2))
        rows.append({"layout": layout_tuple(lay), "ms": round(total / args.steps, 4),
                     "ms_median": round(sorted(per)[len(per) // 2], 4), "identical": same})
        log(f"layout {layout_tuple(lay)} (waves per block, tiles per chunk, first / later pass windows): "
            f"{total / args.steps:.4f} ms, identical outputs: {same}")
    ctx.set_layout(None)
    ctx.check()
    best = min(rows, key=lambda r: r["ms"])
    emit(args, n / (rows[0]["ms"] / 1e3), rows[0]["ms"],
         f"{n} pairs, 250 bp, 2-bit packed, E={args.E}, 70% unrelated, k~U{{0..40}}; plain SneakySnake under "
         f"forced compacting layouts (value: the first)",
         {"pairs": n, "read_len": 250, "E": args.E}, None, None,
         {"layouts": rows, "fastest": best["layout"]})


def emit(args, metric_value, ms, workload_desc, cfg, roofline, cpu, extra):
    rec = {"metric": "filtered pairs/sec at 250bp E=10, learned-bucketed vs plain; HBM GB/s %peak",
           "value": metric_value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64", "data": "synthetic",
           "config": dict({"workload": workload_desc, "parallelism": "single GPU"}, **cfg),
           "roofline": roofline, "cpu_baseline": cpu}
    rec.update(extra)
    print(json.dumps(rec), flush=True)


def filters_workload(args):
    """10M x 250 bp pairs at E = 0, 5, 10, 25: each decision stage alone and all
    three on the same map (one plain launch each)."""
    import dataclasses

    import torch

    import pairgen
    import paper_1910_03936_amd as paf

    ctx = paf.Context(0)
    dev = torch.device("cuda", 0)
    w = pairgen.FIXED_250BP
    n = args.pairs or w.n_pairs
    base, _ = build_batch(ctx, w, n, dev)
    W = paf.words_for(250)
    SS, GK, SH = paf.SNEAKYSNAKE, paf.GATEKEEPER, paf.SHOUJI
    sets = {"sneakysnake": SS, "gatekeeper": GK, "shouji": SH, "all three": SS | GK | SH}
    by_E, steps = {}, max(3, args.steps // 2)
    for E in (0, 5, 10, 25):
        b = dataclasses.replace(base, uniform_E=E, max_E=E)
        row = {}
        for name, f in sets.items():
            out = ctx.alloc_out(n, f, dev)
            # Each stage gets its own clock ramp: the E = 0 stages are too short
            # to keep the clocks up, and a stage timed right after them runs slow.
            ramp(lambda: ctx.filter(b, f, out=out), 0.2)
            per, tot, _ = time_steps(lambda: ctx.filter(b, f, out=out), steps, args.warmup)
            ctx.check()
            ms = sum(per) / len(per)
            nf = bin(f).count("1")
            gbs = n * (2 * W * 8 + nf * (2 + 1 / 8)) / (ms / 1e3) / 1e9
            row[name] = {"ms": round(ms, 4), "pairs_per_s": n / (ms / 1e3), "hbm_GBps": round(gbs, 1)}
            del out
        out = ctx.alloc_out(n, SS, dev)
        ramp(lambda: ctx.filter_magnet(b, out=out), 0.2)
        per, _, _ = time_steps(lambda: ctx.filter_magnet(b, out=out), steps, args.warmup)
        ctx.check()
        ms = sum(per) / len(per)
        row["magnet"] = {"ms": round(ms, 4), "pairs_per_s": n / (ms / 1e3),
                         "hbm_GBps": round(n * (2 * W * 8 + 2 + 1 / 8) / (ms / 1e3) / 1e9, 1),
                         "accept_rate": round(float(paf.accept_bits_to_bool(out[SS][0], n).float().mean()), 5)}
        del out
        by_E[str(E)] = row
        log(f"E={E}: " + ", ".join(f"{k} {v['ms']:.3f} ms" for k, v in row.items()))
    r10 = by_E["10"]["all three"]
    gbs = r10["hbm_GBps"]
    emit(args, r10["pairs_per_s"], r10["ms"],
         f"{n} pairs, 250 bp, 2-bit packed, 70% unrelated, k~U{{0..40}}; SneakySnake, GateKeeper and Shouji in "
         f"one call (at E=10: SneakySnake on the compacting engine, GateKeeper and Shouji on one map); "
         f"value at E=10",
         {"pairs": n, "read_len": 250, "E": [0, 5, 10, 25], "filters": "each alone and all three"},
         {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
          "traffic": None, "kernel": "one call at E=10: chunk_kernel<10> (SneakySnake) + whole_kernel<10> (GateKeeper and Shouji)",
          "kernel_ms": r10["ms"], "alg_bytes_per_pair": round(2 * W * 8 + 3 * (2 + 1 / 8), 3)},
         None, {"by_E": by_E})
    ctx.close()


def other_workload(args):
    """The uneven-length, learned-uneven and streaming workloads."""
    import numpy as np
    import torch

    import pairgen
    import paper_1910_03936_amd as paf
    from paper_1910_03936_amd import costmodel
    from paper_1910_03936_amd.batches import device_batch

    ctx = paf.Context(0)
    SS = paf.SNEAKYSNAKE
    if args.workload in ("uneven", "learned-uneven"):
        w = pairgen.UNEVEN_MIX
        n = args.pairs or w.n_pairs
        t = time.perf_counter()
        b = device_batch(ctx, w, n)
        total_words = int(b.word_offset[-1].item()) + paf.words_for(int(b.len[-1].item()) & 0xFFFF)
        log(f"generated and packed {n} uneven pairs ({total_words} words per side) in {time.perf_counter() - t:.1f} s")
        # algorithmic bytes of the general filter: both sequences, offset, length, E in; count, bit out
        bytes_total = total_words * 16 + n * (8 + 2 + 1 + 2 + 1 / 8)
        out = ctx.alloc_out(n, SS, torch.device("cuda", 0))

        def timed(fn):
            ramp(fn)
            per, tot, _ = time_steps(fn, args.steps, args.warmup)
            ctx.check()
            return tot / args.steps, sum(per) / len(per)

        def roof(kern_ms, kernel):
            a = bytes_total / (kern_ms / 1e3) / 1e9
            return {"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(a / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kernel,
                    "kernel_ms": round(kern_ms, 4), "alg_bytes_per_pair": round(bytes_total / n, 3)}

        ctx.set_layout({"lanes_per_pair": 1, "waves_per_block": 4, "blocks_per_cu": 4, "tiles_per_grab": 2,
                        "chunk_tiles": 0})
        fixed_ms, fixed_k = timed(lambda: ctx.filter_persistent(b, SS, out=out))
        ctx.set_layout(None)
        tuned, best_ms, default_ms = ctx.autotune(b, SS)
        tuned_ms, tuned_k = timed(lambda: ctx.filter_persistent(b, SS, out=out))
        log(f"persistent fixed layout {fixed_ms:.3f} ms, autotuned {tuned} {tuned_ms:.3f} ms")
        cfg = {"pairs": n, "lengths": list(w.lens), "E": "floor(0.05 m)", "filters": "sneakysnake"}
        if args.workload == "uneven":
            emit(args, n / (tuned_ms / 1e3), tuned_ms,
                 f"{n} pairs, lengths {{64,100,150,250,300}}, E=floor(0.05 m), 70% unrelated; one persistent "
                 f"graph-captured launch, autotuned layout", cfg, roof(tuned_k, ("chunk_kernel<E<=15, general> (compacting)" if tuned.get("chunk_tiles")
                                   else "filter_kernel<Snake, E<=15, general>")),
                 None, {"fixed_layout": {"layout": {"waves_per_block": 4, "blocks_per_cu": 4, "tiles_per_grab": 2,
                                                    "chunk_tiles": 0},
                                         "ms_per_step": fixed_ms, "value": n / (fixed_ms / 1e3)},
                        "autotuned_layout": {"layout": tuned, "ms_per_step": tuned_ms,
                                             "value": n / (tuned_ms / 1e3)}})
            return
        t = time.perf_counter()
        losses = costmodel.train(ctx, pairgen.TRAIN_MIX, n=args.train_pairs, epochs=4, batch=4096, lr=2e-3)
        log(f"trained on {args.train_pairs} pairs in {time.perf_counter() - t:.1f} s: {losses}")
        out_l = ctx.alloc_out(n, SS, torch.device("cuda", 0))
        learned_ms, _ = timed(lambda: ctx.filter_bucketed_local(b, out=out_l))
        same = bool(torch.equal(out[SS][0], out_l[SS][0]) and torch.equal(out[SS][1], out_l[SS][1]))
        key = ctx.cost_levels(b)
        model_ms, model_k = timed(lambda: ctx.cost_levels(b))
        keyed_ms, keyed_k = timed(lambda: ctx.filter_keyed(b, key, out=out_l))
        hist = torch.bincount(key.to(torch.int64), minlength=16)
        ablation = {}
        for kname, kk in (("constant", torch.full((n,), 15, dtype=torch.uint8, device=b.reads.device)),
                          ("length x E", costmodel.length_e_key(b)),
                          ("true labels (bound)", costmodel.oracle_key(ctx, b)),
                          ("model", key)):
            ablation[kname] = round(timed(lambda: ctx.filter_keyed(b, kk, out=out_l))[1], 4)
        heldout = costmodel.evaluate(ctx, pairgen.TRAIN_MIX)
        log(f"keyed filter by key: {ablation}; held-out MSE {heldout['mse']:.3f} MAE {heldout['mae']:.3f}")
        log(f"learned {learned_ms:.3f} ms vs plain persistent {tuned_ms:.3f} ms, identical: {same}")
        emit(args, n / (learned_ms / 1e3), learned_ms,
             f"{n} pairs, lengths {{64,100,150,250,300}}, E=floor(0.05 m), 70% unrelated; learned-bucketed "
             f"(16 cost levels ordering each compacting chunk)",
             cfg, roof(keyed_k, "chunk_kernel<E<=15, general> with chunks ordered by the model's levels"), None,
             {"plain": {"value": n / (tuned_ms / 1e3), "ms_per_step": tuned_ms, "layout": tuned},
              "learned": {"value": n / (learned_ms / 1e3), "ms_per_step": learned_ms,
                          "vs_plain": round(tuned_ms / learned_ms, 3), "identical_decisions": same,
                          "stages_ms": {"features+model (levels)": round(model_k, 4),
                                        "compacting filter, chunks ordered by level": round(keyed_k, 4)},
                          "level_sizes": hist.cpu().tolist(),
                          "keyed_filter_ms_by_key": ablation,
                          "heldout": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in heldout.items()},
                          "train": {"pairs": args.train_pairs, "epoch_mse": [round(float(x), 3) for x in losses]}}})
        return
    # stream
    from paper_1910_03936_amd.hostbatch import host_batch
    w = pairgen.STREAM_MIX
    n = args.pairs or w.n_pairs
    t = time.perf_counter()
    hb = host_batch(w, n)
    log(f"generated and encoded {n} pairs into pinned host memory in {time.perf_counter() - t:.1f} s")
    costmodel.train(ctx, w, n=args.train_pairs, epochs=4, batch=4096, lr=2e-3)
    chunk = 8_000_000
    res = {}
    for learned in (False, True):
        paf.stream_filter(ctx, host_batch(w, min(n, 2 * chunk)), chunk, SS, learned)   # warm-up
        outs, st = paf.stream_filter(ctx, hb, chunk, SS, learned)
        ctx.check()
        res[learned] = (outs, st)
        log(f"stream learned={learned}: {st['seconds']:.3f} s, {n / st['seconds'] / 1e9:.3f} G pairs/s, "
            f"H2D {st['h2d_bytes'] / st['seconds'] / 1e9:.1f} GB/s")
    same = all(torch.equal(res[False][0][SS][i], res[True][0][SS][i]) for i in (0, 1))
    st = res[True][1]
    emit(args, n / st["seconds"], st["seconds"] * 1e3,
         f"{n} pairs, lengths {{100,150,250}} 1:1:1, E=m/10, 80% unrelated, streamed from pinned host memory "
         f"in 8M-pair chunks, learned bucketing on",
         {"pairs": n, "chunk_pairs": chunk, "filters": "sneakysnake"}, None, None,
         {"h2d_GBps": st["h2d_bytes"] / st["seconds"] / 1e9, "h2d_bytes": st["h2d_bytes"],
          "plain": {"value": n / res[False][1]["seconds"], "seconds": res[False][1]["seconds"],
                    "h2d_GBps": res[False][1]["h2d_bytes"] / res[False][1]["seconds"] / 1e9},
          "identical_decisions": same})


def next_workloads(args):
    """10M x 250 bp pairs: SneakySnake on partitioned mazes (sub-mazes of t
    columns), or the filter followed by verification of its survivors."""
    import dataclasses

    import torch

    import pairgen
    import paper_1910_03936_amd as paf

    ctx = paf.Context(0)
    dev = torch.device("cuda", 0)
    w = pairgen.FIXED_250BP
    n = args.pairs or w.n_pairs
    base, _ = build_batch(ctx, w, n, dev)
    W = paf.words_for(250)
    SS = paf.SNEAKYSNAKE
    steps = max(3, args.steps // 2)
    out = ctx.alloc_out(n, SS, dev)
    t = time.perf_counter()
    while time.perf_counter() - t < 0.3:
        ctx.filter(base, SS, out=out)
        torch.cuda.synchronize()

    def timed(fn):
        # A clock ramp before each timed call: a call timed right after the
        # short E = 0 launches would otherwise run at lower clocks.
        ramp(fn, 0.2)
        per, _, _ = time_steps(fn, steps, args.warmup)
        ctx.check()
        return sum(per) / len(per)

    if args.workload == "accuracy":
        # Sec. 3.1.2: a pair is a correct mapping when its edit distance is at
        # most E; paf_verify gives min(banded distance, E+1) of every pair,
        # which is the exact verdict.
        from paper_1910_03936_amd.accuracy import confusion
        GK, SH = paf.GATEKEEPER, paf.SHOUJI
        by_E = {}
        for E in (0, 5, 10, 25):
            b = dataclasses.replace(base, uniform_E=E, max_E=E)
            dist_t = torch.empty(n, dtype=torch.int16, device=dev)
            ver_ms = timed(lambda: ctx.verify(b, dist=dist_t))
            dist = paf.counts_u16(dist_t).cpu().numpy()
            runs = {"sneakysnake": (lambda o: ctx.filter(b, SS, out=o), SS, SS)}
            for t in (5, 10, 25, 50):
                runs[f"sneakysnake-{t}"] = ((lambda o, t=t: ctx.filter_partitioned(b, t, out=o)), SS, SS)
            runs["hardware t=8 y=3"] = (lambda o: ctx.filter_partitioned(b, 8, 3, out=o), SS, SS)
            runs["gatekeeper"] = (lambda o: ctx.filter(b, GK, out=o), GK, GK)
            runs["shouji"] = (lambda o: ctx.filter(b, SH, out=o), SH, SH)
            runs["magnet"] = (lambda o: ctx.filter_magnet(b, out=o), SS, SS)
            row = {"verify_every_pair_ms": round(ver_ms, 4)}
            for name, (fn, mask, slot) in runs.items():
                o = ctx.alloc_out(n, mask, dev)
                ms = timed(lambda: fn(o))
                acc = paf.accept_bits_to_bool(o[slot][0], n).cpu().numpy()
                c = confusion(acc, dist, E)
                row[name] = {"ms": round(ms, 4), "accept_rate": round(float(acc.mean()), 6),
                             "FAR": round(c["FAR"], 6), "FRR": round(c["FRR"], 6), "FA": c["FA"], "FR": c["FR"],
                             "correct": c["correct"], "incorrect": c["incorrect"]}
                del o
            if row["sneakysnake"]["FR"] != 0:
                raise AssertionError(f"E={E}: SneakySnake rejected {row['sneakysnake']['FR']} correct pairs")
            by_E[str(E)] = row
            log(f"E={E}: correct {row['sneakysnake']['correct']}, " + ", ".join(
                f"{k} FAR {v['FAR']:.4f} FRR {v['FRR']:.5f}" for k, v in row.items() if isinstance(v, dict)))
        r = by_E["10"]["sneakysnake"]
        emit(args, n / (r["ms"] / 1e3), r["ms"],
             f"{n} pairs, 250 bp, 2-bit packed, 70% unrelated, k~U{{0..40}}; false accept / false reject rates "
             f"of each filter against the exact banded edit distance (paf_verify); value: SneakySnake at E=10",
             {"pairs": n, "read_len": 250, "E": [0, 5, 10, 25]}, None, None, {"by_E": by_E})
        ctx.close()
        return
    if args.workload == "partitioned":
        by_E = {}
        for E in (0, 5, 10, 25):
            b = dataclasses.replace(base, uniform_E=E, max_E=E)
            row = {"whole maze": {"ms": round(timed(lambda: ctx.filter(b, SS, out=out)), 4)}}
            row["whole maze"]["accept_rate"] = float(paf.accept_bits_to_bool(out[SS][0], n).float().mean())
            for tp in (5, 10, 25, 50):
                ms = timed(lambda: ctx.filter_partitioned(b, tp, out=out))
                acc = float(paf.accept_bits_to_bool(out[SS][0], n).float().mean())
                row[f"t={tp}"] = {"ms": round(ms, 4), "accept_rate": round(acc, 5)}
            # The hardware form: sub-mazes of 8 columns, 3 replications each.
            ms = timed(lambda: ctx.filter_partitioned(b, 8, 3, out=out))
            acc = float(paf.accept_bits_to_bool(out[SS][0], n).float().mean())
            row["t=8, y=3"] = {"ms": round(ms, 4), "accept_rate": round(acc, 5)}
            by_E[str(E)] = row
            log(f"E={E}: " + ", ".join(f"{k} {v['ms']:.3f} ms (acc {v['accept_rate']:.4f})" for k, v in row.items()))
        r = by_E["10"]["t=5"]
        gbs = n * (2 * W * 8 + 2 + 1 / 8) / (r["ms"] / 1e3) / 1e9
        emit(args, n / (r["ms"] / 1e3), r["ms"],
             f"{n} pairs, 250 bp, 2-bit packed, 70% unrelated, k~U{{0..40}}; SneakySnake on sub-mazes of t "
             f"columns (compacting engine); value at E=10, t=5",
             {"pairs": n, "read_len": 250, "E": [0, 5, 10, 25], "t": [5, 10, 25, 50]},
             {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
              "kernel": "chunk_kernel<E=10, uniform, partitioned>", "kernel_ms": r["ms"],
              "alg_bytes_per_pair": round(2 * W * 8 + 2 + 1 / 8, 3)},
             None, {"by_E": by_E})
        ctx.close()
        return
    by_E = {}
    for E in (5, 10, 25):
        b = dataclasses.replace(base, uniform_E=E, max_E=E)
        dist = torch.empty(n, dtype=torch.int16, device=dev)
        filt_ms = timed(lambda: ctx.filter(b, SS, out=out))
        surv = int(paf.accept_bits_to_bool(out[SS][0], n).sum())
        ver_ms = timed(lambda: ctx.verify(b, out[SS][0], dist=dist))
        d_sel = dist.clone()
        all_ms = timed(lambda: ctx.verify(b, dist=dist))
        same = bool(torch.equal(d_sel, dist))
        within = int((paf.counts_u16(dist) <= E).sum())
        by_E[str(E)] = {"filter_ms": round(filt_ms, 4), "survivors": surv,
                        "verify_survivors_ms": round(ver_ms, 4), "filter_plus_verify_ms": round(filt_ms + ver_ms, 4),
                        "verify_every_pair_ms": round(all_ms, 4), "identical_distances": same,
                        "pairs_within_E": within}
        log(f"E={E}: filter {filt_ms:.3f} ms, {surv} survivors verified in {ver_ms:.3f} ms; every pair "
            f"{all_ms:.3f} ms; identical {same}; {within} pairs within E")
    r = by_E["10"]
    emit(args, n / (r["filter_plus_verify_ms"] / 1e3), r["filter_plus_verify_ms"],
         f"{n} pairs, 250 bp, 2-bit packed, 70% unrelated, k~U{{0..40}}; SneakySnake, then banded edit distance "
         f"of its survivors; value at E=10",
         {"pairs": n, "read_len": 250, "E": [5, 10, 25]}, None, None, {"by_E": by_E})
    ctx.close()


if __name__ == "__main__":
    main()
