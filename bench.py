#!/usr/bin/env python3
"""Benchmark: RS(10,4) encode at bandwidth scale on one MI355X.

Workload: Cauchy RS(10,4) over GF(2^8)/0x11D, 10 data blocks of 64 MiB of
seeded uniform random bytes (640 MiB in), 4 parity blocks (256 MiB out), each
block split into 8 contiguous strips.  One step = one ec_encode launch over
the whole stripe with inputs resident in HBM.  The headline value is the
compressed + fused + scheduled program; the plain bitmatrix program, a
4-erasure decode and a plain device copy run on the same data for comparison,
followed by the batched and the serving workloads and the oracle on the host.

Prints one JSON line (see the keys below).  ``--gpus`` above 1 is refused:
the executor runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "encode/decode GB/s (input bytes) and % HBM roofline, compressed SLP vs plain bitmatrix"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
PROFILES = os.path.join(HERE, "profiles")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # untimed launches of the timed kernel before each timed run (after the
    # copies of prewarm())
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--prewarm-ms", type=float, default=50.0,
                    help="ms of device copies before each timed run's warm-up launches (0 = none; counter runs)")
    ap.add_argument("--block-mib", type=int, default=64)
    ap.add_argument("--slots", type=int, default=0, help="slot budget of the compressed program (0 = default)")
    ap.add_argument("--plain-slots", type=int, default=0, help="slot budget of the plain program (0 = default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-block-mib", type=int, default=32, help="oracle sample: 10 blocks of this size")
    ap.add_argument("--only", choices=["all", "compressed", "plain", "decode", "copy", "batched", "serve",
                                       "decode_all", "codecs", "small", "schedulers", "batched_programs", "staged"],
                    default="all",
                    help="time one kernel only (for profiler runs)")
    ap.add_argument("--calib", action="store_true",
                    help="also run one device copy of 448 MiB (byte-counter calibration)")
    ap.add_argument("--batch-stripes", type=int, default=8192, help="stripes in the batched workload (0 = skip)")
    ap.add_argument("--batch-max-mib", type=int, default=4, help="largest block of the batched workload (MiB)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="seconds of Poisson arrivals (0 = skip)")
    ap.add_argument("--serve-runs", type=int, default=3,
                    help="serving runs of the same arrival stream, each with its own server; the latency and "
                         "drain figures are their medians (every run's in 'runs')")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--decode-all-slots", type=int, default=44, help="slot budget of the every-erasure-set decode")
    ap.add_argument("--exec", choices=["native", "interp"], default="native",
                    help="executor of the headline programs: their native kernels, or the record interpreter")
    ap.add_argument("--rotate-in", type=int, default=2,
                    help="input block sets the headline launches rotate over (1 = the same every launch)")
    ap.add_argument("--rotate-out", type=int, default=4,
                    help="output block sets the headline launches rotate over (1 = the same every launch)")
    ap.add_argument("--sweep", action="store_true",
                    help="time every (level, slot budget) pair on the workload and print one line each")
    ap.add_argument("--sweep-prefetch", action="store_true", help="with --sweep: also vary the prefetch distance")
    return ap.parse_args()


def log(msg):
    print("bench.py: %s" % msg, file=sys.stderr, flush=True)


# Device time spent on copy kernels right before each timed run's warm-up
# launches.  After 20 ms or more without work the GPU runs HBM-bound kernels
# up to 8% slower for the first ~15 ms of renewed load, whatever the kernel
# (the first launches after copies or matrix products that fill that window
# already run at full speed); the timed launches are meant to show the
# kernel, not that transition, which "cold_ms_per_step" reports separately.
PREWARM_MS = 50.0
_prewarm_bufs = []


def prewarm(stream, ms=PREWARM_MS):
    """Queue about `ms` of back-to-back device copies of 256 MiB on `stream`
    (no host synchronisation, so the launches that follow start with the
    device busy).  Returns the queued copies' estimated device time."""
    import torch
    import paper_2108_02692_amd as E
    if ms <= 0:
        return 0.0
    if not _prewarm_bufs:
        _prewarm_bufs.extend(torch.empty(256 << 20, dtype=torch.uint8, device="cuda") for _ in range(2))
    src, dst = _prewarm_bufs
    per_ms = 2 * src.numel() / 5.0e9  # at ~5 TB/s
    for _ in range(max(1, int(ms / per_ms))):
        E.ec_device_copy(dst, src, src.numel(), stream)
    return ms


def time_launches(fn, steps, warmup, stream, prewarm_ms=None):
    """Average ms per launch over `steps` back-to-back launches, bracketed by
    HIP events on the stream the kernels run on, after `prewarm_ms` of
    device copies and `warmup` untimed launches."""
    import torch
    prewarm(stream, PREWARM_MS if prewarm_ms is None else prewarm_ms)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def rotating(launch, ins_sets, outs_sets):
    """A launch function that takes the next (input set, output set) pair on
    every call: call i uses input set i % R_in and output set i % R_out, so
    that no launch writes the lines the launch before it wrote (a launch
    that rewrites them finds them in the memory-side cache, and stores that
    allocate there then look up to 13% faster than HBM allows)."""
    k = [0]

    def f():
        i = k[0]
        k[0] += 1
        launch(ins_sets[i % len(ins_sets)], outs_sets[i % len(outs_sets)])
    return f


def code_sha(*paths):
    """sha256 of C++/HIP sources with comments and blank lines removed, so
    that an edit of comments alone keeps a measurement valid."""
    out = []
    for path in paths:
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines()]
        out.append("\n".join(ln for ln in lines if ln.strip()))
    return hashlib.sha256("\n".join(out).encode()).hexdigest()


# The executor's kernels and everything their code depends on (the kernel
# arguments' layout, the record format).
EXECUTOR_SOURCES = ("exec.hip", "exec.hpp", "bytecode.hpp")


def executor_sha():
    import paper_2108_02692_amd
    csrc = os.path.join(os.path.dirname(paper_2108_02692_amd.__file__), "csrc")
    return code_sha(*[os.path.join(csrc, f) for f in EXECUTOR_SOURCES])


def program_sha(prog):
    import struct
    w = prog.bytecode()
    return hashlib.sha256(struct.pack("<%dI" % len(w), *w)).hexdigest()


def measured_traffic(prog, native=False):
    """HBM bytes per launch from the committed byte-counter profile of this
    workload, if it was taken on this executor and this program (else None).
    A native kernel is identified by its source, which holds both."""
    if native:
        exec_sha = "native"
        psha = hashlib.sha256(prog.native_source().encode()).hexdigest()
    else:
        exec_sha = executor_sha()
        psha = program_sha(prog)
    if not os.path.isdir(PROFILES):
        return None
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(PROFILES, name)) as f:
            for m in re.finditer(r"<!-- traffic (\{.*?\}) -->", f.read()):
                rec = json.loads(m.group(1))
                if rec.get("executor_code_sha256") == exec_sha and rec.get("program_sha256") == psha:
                    return rec["fetch_bytes"] + rec["write_bytes"]
    return None


def main():
    args = parse()
    global PREWARM_MS
    PREWARM_MS = args.prewarm_ms
    if args.gpus != 1:
        print("bench.py: the executor runs on one GPU; --gpus %d is not supported (stripes would be "
              "sharded across GPUs by the caller, one process per GPU)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2108_02692_amd as E
    from paper_2108_02692_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no ROCm GPU visible", file=sys.stderr)
        sys.exit(1)
    E.lib()  # fails loudly if the HIP library is missing
    stream = torch.cuda.current_stream()
    if args.only == "batched":
        print(json.dumps({"batched": bench_batched(args, stream)}), flush=True)
        return
    if args.only == "batched_programs":
        print(json.dumps({"batched_programs": bench_batched_programs(args, stream)}), flush=True)
        return
    if args.only == "decode_all":
        print(json.dumps({"decode_all": bench_decode_all(args, stream)}), flush=True)
        return
    if args.only in ("codecs", "small"):
        print(json.dumps({args.only: (bench_codecs if args.only == "codecs" else bench_small)(args, stream)}),
              flush=True)
        return
    if args.only == "serve":
        print(json.dumps({"serving": bench_serving(args)}), flush=True)
        return
    n, p = 10, 4
    S = args.block_mib << 20
    gen = E.ec_matrix_cauchy(n, p)
    # Launch i reads input set i % R_in and writes output set i % R_out, so
    # that no launch rewrites the output lines of the one before (the
    # memory-side cache could still hold them) or reads the inputs its
    # predecessor read.
    sets_in = [W.device_blocks(n, S, seed=2021 + r) for r in range(max(1, args.rotate_in))]
    sets_out = [W.empty_blocks(p, S) for _ in range(max(1, args.rotate_out))]
    data, parity = sets_in[0], sets_out[0]
    torch.cuda.synchronize()
    in_bytes = n * S
    moved = (n + p) * S  # algorithmic bytes per launch: read n blocks, write p blocks
    native = args.exec == "native"

    def measure(prog, ins_sets, outs_sets, decode=False, prewarm_ms=None):
        run = E.ec_decode if decode else E.ec_encode
        return time_launches(rotating(lambda i, o: run(prog, i, o, S, stream), ins_sets, outs_sets), args.steps,
                             args.warmup, stream, prewarm_ms=prewarm_ms)

    t0 = time.time()
    comp = E.ec_compile_slp(n, p, gen, level=E.LEVEL_CO_FU_SCHED, slot_budget=args.slots, native=native)
    compile_ms = (time.time() - t0) * 1e3
    plain = E.ec_compile_slp(n, p, gen, level=E.LEVEL_PLAIN, slot_budget=args.plain_slots, native=native)
    log("compiled (compressed %.0f ms, %d slots; plain %d slots; %s)" % (
        compile_ms, comp.info["slots"], plain.info["slots"], args.exec))
    if args.sweep:
        for level in (E.LEVEL_PLAIN, E.LEVEL_CO_FU_SCHED):
            for K in (32, 36, 38, 40, 44, 48):
                for dist in ((0, 4, 12) if args.sweep_prefetch else (0,)):
                    pr = E.ec_compile_slp(n, p, gen, level=level, slot_budget=K, prefetch=dist,
                                          native=native and dist == 0)
                    ms = measure(pr, sets_in, sets_out)
                    print(json.dumps({"sweep": True, "level": level, "slots": K, "prefetch": dist,
                                      "native": bool(pr.info["native"]), "ms": ms,
                                      "GB_s": in_bytes / ms / 1e6, "hbm_frac": moved / ms / 1e6 / HBM_PEAK_GBS,
                                      "n_xor2": pr.info["n_xor2"], "ops": pr.info["n_ops"],
                                      "records": pr.info["n_records"], "ring": pr.info["ring"],
                                      "open": pr.info["peak_open"]}), flush=True)
        return

    if args.only == "schedulers":
        print(json.dumps({"schedulers": bench_schedulers(args, stream, gen, data, parity)}), flush=True)
        return
    if args.only == "staged":
        print(json.dumps({"staged": bench_staged(args, stream, gen, data, parity)}), flush=True)
        return
    res = {}
    if args.only in ("all", "compressed"):
        res["compressed"] = measure(comp, sets_in, sets_out)
    if args.only in ("all", "plain"):
        res["plain"] = measure(plain, sets_in, sets_out)
    log("encode timed: %s" % res)
    cold = None
    if args.only == "all":
        # the same launches timed after 0.2 s idle with no copies before the
        # warm-up launches: what a run starting from an idle GPU sees
        time.sleep(0.2)
        cold = measure(comp, sets_in, sets_out, prewarm_ms=0)
    extra = {}
    if args.only == "all" and native:
        # the record interpreter on the same programs and buffers
        icomp = E.ec_compile_slp(n, p, gen, level=E.LEVEL_CO_FU_SCHED, slot_budget=args.slots)
        iplain = E.ec_compile_slp(n, p, gen, level=E.LEVEL_PLAIN, slot_budget=args.plain_slots)
        ic, ip = measure(icomp, sets_in, sets_out), measure(iplain, sets_in, sets_out)
        extra["interpreter"] = {
            "compressed": {"ms": ic, "hbm_frac": moved / ic / 1e6 / HBM_PEAK_GBS, "slots": icomp.info["slots"]},
            "plain": {"ms": ip, "hbm_frac": moved / ip / 1e6 / HBM_PEAK_GBS, "slots": iplain.info["slots"]},
            "kernel": "slp_exec_kernel_%d" % icomp.info["slots"]}
        log("interpreter: compressed %.4f ms, plain %.4f ms" % (ic, ip))
    if args.only in ("all", "decode"):
        # decode of 4 lost data blocks (the paper's decode example erases 4):
        # the survivors of input set r are its data blocks and their parity
        er = [2, 4, 5, 6]
        dprog = E.ec_compile_slp(n, p, gen, er, native=native)
        surv_sets = []
        for d in sets_in:
            par_d = W.empty_blocks(p, S)
            E.ec_encode(comp, d, par_d, S, stream)
            blocks = d + par_d
            surv_sets.append([blocks[i] for i in dprog.in_blocks])
        rec_sets = [W.empty_blocks(len(er), S) for _ in sets_out]
        ms_dec = measure(dprog, surv_sets, rec_sets, decode=True)
        torch.cuda.synchronize()
        for r, d in enumerate(sets_in):
            E.ec_decode(dprog, surv_sets[r], rec_sets[0], S, stream)
            torch.cuda.synchronize()
            for j, e in enumerate(er):
                if not torch.equal(rec_sets[0][j], d[e]):
                    raise SystemExit("bench.py: decode self-check failed for block %d" % e)
        dmoved = (n + len(er)) * S
        extra["decode"] = {"erased": er, "ms": ms_dec, "GB_s": in_bytes / ms_dec / 1e6,
                           "hbm_frac": dmoved / ms_dec / 1e6 / HBM_PEAK_GBS, "slots": dprog.info["slots"],
                           "n_xor2": dprog.info["n_xor2"], "plain_xor2": dprog.info["plain_xor2"],
                           "ops_per_tile": dprog.info["n_ops"], "executor": args.exec}
        del rec_sets, surv_sets
    if args.only in ("all", "copy") or args.calib:
        # plain device copy of the same number of bytes (read + write = moved)
        src = torch.empty(moved // 2, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        copy = (lambda: E.ec_device_copy(dst, src, src.numel(), stream))
        if args.only in ("all", "copy"):
            ms_copy = time_launches(copy, args.steps, args.warmup, stream)
            extra["copy_ceiling_GB_s"] = 2 * src.numel() / ms_copy / 1e6
        else:
            copy()
            torch.cuda.synchronize()
        del src, dst
    if args.only in ("all", "copy"):
        # the encode's own data movement (10 blocks read, 4 written, same
        # tile order) with no program: the ceiling for this access pattern
        ms_stream = time_launches(rotating(lambda i, o: E.ec_stripe_stream(i, o, S, stream), sets_in, sets_out),
                                  args.steps, args.warmup, stream)
        extra["stripe_ceiling"] = {"ms": ms_stream, "GB_s": moved / ms_stream / 1e6,
                                   "hbm_frac": moved / ms_stream / 1e6 / HBM_PEAK_GBS,
                                   "what": "ec_stripe_stream: 10 x %d MiB read, 4 x %d MiB written, executor tile "
                                           "order and cache policies, no program, same buffer rotation"
                                           % (args.block_mib, args.block_mib)}
    if args.only == "copy":
        print(json.dumps(extra), flush=True)
        return
    if args.only == "decode":
        print(json.dumps(extra), flush=True)
        return

    if args.only == "all":
        log("strip schedulers ...")
        extra["schedulers"] = bench_schedulers(args, stream, gen, data, parity)
        log("staged launches ...")
        extra["staged"] = bench_staged(args, stream, gen, data, parity)
    head = "compressed" if "compressed" in res else "plain"
    hprog = comp if head == "compressed" else plain
    ms = res[head]
    achieved = moved / ms / 1e6
    info = hprog.info
    out = {
        "metric": METRIC,
        "value": in_bytes / ms / 1e6,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": "RS(10,4) encode, Cauchy GF(2^8)/0x11D, 10 x %d MiB data -> 4 x %d MiB parity"
                        % (args.block_mib, args.block_mib),
            "program": "compressed+fused+scheduled" if head == "compressed" else "plain bitmatrix",
            "executor": "native kernel" if native else "record interpreter",
            "buffers": "%d input sets x %d output sets, rotating" % (len(sets_in), len(sets_out)),
            "block_bytes": S,
            "slots": info["slots"],
            "n_xor2": info["n_xor2"],
            "plain_xor2": info["plain_xor2"],
            "ops_per_tile": info["n_ops"],
            "records_per_tile": info["n_records"],
            "compile_ms": compile_ms,
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(hprog, native),
                     "kernel": "ec_native_kernel" if native else "slp_exec_kernel_%d" % info["slots"]},
    }
    out["prewarm"] = {"ms": PREWARM_MS, "kernel": "ec_device_copy, 256 MiB per launch",
                      "when": "before every timed run's warm-up launches"}
    if cold is not None:
        out["cold_ms_per_step"] = cold
        out["cold_hbm_frac"] = moved / cold / 1e6 / HBM_PEAK_GBS
    if "plain" in res and head == "compressed":
        pms = res["plain"]
        out["plain"] = {"ms": pms, "GB_s": in_bytes / pms / 1e6, "hbm_frac": moved / pms / 1e6 / HBM_PEAK_GBS,
                        "n_xor2": plain.info["n_xor2"], "ops_per_tile": plain.info["n_ops"],
                        "records_per_tile": plain.info["n_records"], "slots": plain.info["slots"]}
        out["compressed_vs_plain"] = pms / ms
    out.update(extra)
    if "copy_ceiling_GB_s" in out:
        out["roofline"]["frac_of_copy"] = achieved / out["copy_ceiling_GB_s"]
    if "stripe_ceiling" in out:
        out["roofline"]["frac_of_stripe_ceiling"] = achieved / out["stripe_ceiling"]["GB_s"]
    if args.only == "all":
        del data, parity, sets_in, sets_out
        torch.cuda.empty_cache()
        log("decode of every erasure set ...")
        out["decode_all"] = bench_decode_all(args, stream)
        log("decode all: %.3f ms" % out["decode_all"]["ms"])
        torch.cuda.empty_cache()
    if args.only == "all":
        log("codec sweep ...")
        out["codecs"] = bench_codecs(args, stream)
        out["small"] = bench_small(args, stream)
        torch.cuda.empty_cache()
    if args.only == "all" and args.batch_stripes > 0:
        log("batched ...")
        out["batched"] = bench_batched(args, stream)
        log("batched: %.3f ms" % out["batched"]["ms"])
        torch.cuda.empty_cache()
    if args.only == "all" and args.serve_seconds > 0:
        log("serving ...")
        out["serving"] = bench_serving(args, out.get("batched", {}).get("GB_s"))
        log("serving: p50 %.3f ms p99 %.3f ms" % (out["serving"]["p50_ms"], out["serving"]["p99_ms"]))
        torch.cuda.empty_cache()
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_block_mib)
    print(json.dumps(out), flush=True)


def bench_schedulers(args, stream, gen, data, parity):
    """The two strip orders (EC_SCHED_PUSH, EC_SCHED_GREEDY) at the
    compressed and the plain level, run by the interpreter and (with --exec
    native) as native kernels, on the RS(10,4) encode of 10 x 64 MiB (the
    data above), the decode of {2, 4, 5, 6} at that size, and the encode of
    10 x 1 MiB, through the single-stripe autotuner (every candidate timed,
    the fastest reported as its choice)."""
    import paper_2108_02692_amd as E
    from paper_2108_02692_amd import autotune
    from paper_2108_02692_amd import workloads as W
    n, p = 10, 4
    S = data[0].numel()
    timer = (lambda f: time_launches(f, args.steps, args.warmup, stream))
    name = {E.SCHED_PUSH: "push", E.SCHED_GREEDY: "greedy"}
    rows = []
    small = W.device_blocks(n, 1 << 20, seed=0)
    small_par = W.empty_blocks(p, 1 << 20)
    dec = E.ec_compile_slp(n, p, gen, [2, 4, 5, 6])
    E.ec_encode(E.ec_compile_slp(n, p, gen), data, parity, S, stream)
    blocks = data + parity
    rec = W.empty_blocks(4, S)
    cases = (("RS(10,4) encode 10 x 64 MiB", (), data, parity, S),
             ("RS(10,4) decode {2,4,5,6} 10 x 64 MiB", (2, 4, 5, 6), [blocks[i] for i in dec.in_blocks], rec, S),
             ("RS(10,4) encode 10 x 1 MiB", (), small, small_par, 1 << 20))
    cands = autotune.STRIPE_CANDIDATES_NATIVE if args.exec == "native" else autotune.STRIPE_CANDIDATES
    for what, er, ins, outs, bb in cases:
        best, table = autotune.tune_stripe(n, p, gen, er, ins, outs, bb, stream, candidates=cands, retune=True,
                                           time_fn=timer)
        moved = (n + len(outs)) * bb
        rows.append({"workload": what, "choice": {"level": best["level"], "scheduler": name[best["scheduler"]],
                                                  "slots": best["slots"], "native": best["native"]},
                     "candidates": [{"level": r["level"], "scheduler": name[r["scheduler"]], "slots": r["slots"],
                                     "native": r["native"], "ms": r["ms"],
                                     "hbm_frac": moved / r["ms"] / 1e6 / HBM_PEAK_GBS,
                                     "records": r["records"], "ops": r["ops"]} for r in table]})
        log("%s: %s" % (what, ", ".join("%s/%s%s %.4f ms" % (r["level"], name[r["scheduler"]],
                                                             "/native" if r["native"] else "", r["ms"])
                                         for r in table)))
    return rows


def bench_staged(args, stream, gen, data, parity):
    """The staged launch (each tile's input strips copied into LDS by one
    workgroup, its 4 waves on a quarter of the rows each) against the direct
    one (one wave per tile streaming strips into its registers), the same
    program level and defaults otherwise: RS(10,4) encode and the {2,4,5,6}
    decode of 10 x 64 MiB (the data above), and encodes of 10 x 8 MiB and
    10 x 1 MiB."""
    import paper_2108_02692_amd as E
    from paper_2108_02692_amd import workloads as W
    n, p = 10, 4
    S = data[0].numel()
    E.ec_encode(E.ec_compile_slp(n, p, gen), data, parity, S, stream)
    blocks = data + parity
    rec = W.empty_blocks(4, S)
    dec_in = [blocks[i] for i in E.ec_compile_slp(n, p, gen, [2, 4, 5, 6]).in_blocks]
    mid, mid_par = W.device_blocks(n, 8 << 20, seed=0), W.empty_blocks(p, 8 << 20)
    small, small_par = W.device_blocks(n, 1 << 20, seed=0), W.empty_blocks(p, 1 << 20)
    cases = (("RS(10,4) encode 10 x 64 MiB", (), data, parity, S),
             ("RS(10,4) decode {2,4,5,6} 10 x 64 MiB", [2, 4, 5, 6], dec_in, rec, S),
             ("RS(10,4) encode 10 x 8 MiB", (), mid, mid_par, 8 << 20),
             ("RS(10,4) encode 10 x 1 MiB", (), small, small_par, 1 << 20))
    rows = []
    for what, er, ins, outs, bb in cases:
        row = {"workload": what}
        for level, lname in ((E.LEVEL_CO_FU_SCHED, "compressed"), (E.LEVEL_PLAIN, "plain")):
            for split, sname in ((E.SPLIT_AUTO, "direct"), (E.SPLIT_STAGED, "staged")):
                prog = E.ec_compile_slp(n, p, gen, list(er), level=level, split=split)
                run = (E.ec_decode if er else E.ec_encode)
                ms = time_launches(lambda: run(prog, ins, outs, bb, stream), args.steps, args.warmup, stream)
                row["%s_%s" % (lname, sname)] = {"ms": ms, "hbm_frac": (n + len(outs)) * bb / ms / 1e6 / HBM_PEAK_GBS,
                                                 "slots": prog.info["slots"]}
        rows.append(row)
        log("%s: %s" % (what, ", ".join("%s %.4f ms" % (k, v["ms"]) for k, v in row.items() if k != "workload")))
    return rows


def worst_erasures(n, p, gen):
    """The set of p data blocks whose decode has the most plain XORs."""
    import itertools
    import paper_2108_02692_amd as E
    best = None
    for er in itertools.combinations(range(n), p):
        x = E.ec_compile_slp(n, p, gen, list(er), level=E.LEVEL_PLAIN).info["plain_xor2"]
        if best is None or x > best[0]:
            best = (x, list(er))
    return best[1]


def bench_codecs(args, stream):
    """RS(d,4), RS(d,3) and RS(d,2) for d = 8, 9, 10 (the codecs of the
    paper's throughput comparison, with Cauchy matrices): encode, and decode
    of the worst set of p lost data blocks, each compressed and plain, on
    d blocks of 64 MiB resident in HBM, with the headline's executor and
    buffer rotation (inputs over --rotate-in sets, outputs over
    --rotate-out sets; the programs are compiled on host threads first)."""
    from concurrent.futures import ThreadPoolExecutor
    import torch
    import paper_2108_02692_amd as E
    from paper_2108_02692_amd import workloads as W
    S = args.block_mib << 20
    native = args.exec == "native"
    codecs = [(n, p) for p in (4, 3, 2) for n in (8, 9, 10)]
    gens = {c: E.ec_matrix_cauchy(*c) for c in codecs}
    ers = {c: worst_erasures(c[0], c[1], gens[c]) for c in codecs}
    jobs = [(c, level, er) for c in codecs for level in (E.LEVEL_CO_FU_SCHED, E.LEVEL_PLAIN) for er in ((), tuple(ers[c]))]
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        progs = dict(zip(jobs, ex.map(lambda j: E.ec_compile_slp(j[0][0], j[0][1], gens[j[0]], list(j[2]),
                                                                 level=j[1], native=native), jobs)))
    rows = []
    for (n, p) in codecs:
        gen = gens[(n, p)]
        er = ers[(n, p)]
        data_sets = [W.device_blocks(n, S, seed=100 + 10 * n + p + 1000 * r) for r in range(max(1, args.rotate_in))]
        data = data_sets[0]
        par_sets = [W.empty_blocks(p, S) for _ in range(max(1, args.rotate_out))]
        parity = par_sets[0]
        rec_sets = [W.empty_blocks(p, S) for _ in range(max(1, args.rotate_out))]
        rec = rec_sets[0]
        row = {"codec": "RS(%d,%d)" % (n, p), "erased": er}
        ref = None
        for level, tag in ((E.LEVEL_CO_FU_SCHED, "comp"), (E.LEVEL_PLAIN, "plain")):
            enc = progs[((n, p), level, ())]
            ms = time_launches(rotating(lambda i, o: E.ec_encode(enc, i, o, S, stream), data_sets, par_sets),
                               args.steps, args.warmup, stream)
            E.ec_encode(enc, data, parity, S, stream)
            torch.cuda.synchronize()
            if ref is None:
                ref = [t.clone() for t in parity]
            elif not all(torch.equal(a, b) for a, b in zip(ref, parity)):
                raise SystemExit("bench.py: compressed and plain parity differ for %s" % row["codec"])
            row["enc_" + tag] = {"ms": ms, "GB_s": n * S / ms / 1e6,
                                 "hbm_frac": (n + p) * S / ms / 1e6 / HBM_PEAK_GBS,
                                 "n_xor2": enc.info["n_xor2"], "slots": enc.info["slots"]}
            dec = progs[((n, p), level, tuple(er))]
            blocks = data + ref
            surv = [blocks[i] for i in dec.in_blocks]
            if level == E.LEVEL_CO_FU_SCHED:  # the survivors of every input set (parity of each)
                surv_sets = [surv]
                for d in data_sets[1:]:
                    par_d = W.empty_blocks(p, S)
                    E.ec_encode(enc, d, par_d, S, stream)
                    surv_sets.append([(d + par_d)[i] for i in dec.in_blocks])
            ms = time_launches(rotating(lambda i, o: E.ec_decode(dec, i, o, S, stream), surv_sets, rec_sets),
                               args.steps, args.warmup, stream)
            E.ec_decode(dec, surv, rec, S, stream)
            torch.cuda.synchronize()
            for j, e in enumerate(dec.out_blocks):
                if not torch.equal(rec[j], blocks[e]):
                    raise SystemExit("bench.py: %s decode self-check failed" % row["codec"])
            row["dec_" + tag] = {"ms": ms, "GB_s": n * S / ms / 1e6,
                                 "hbm_frac": (n + len(er)) * S / ms / 1e6 / HBM_PEAK_GBS,
                                 "n_xor2": dec.info["n_xor2"], "slots": dec.info["slots"]}
        log("%s: enc %.1f GB/s dec %.1f GB/s" % (row["codec"], row["enc_comp"]["GB_s"],
                                                  row["dec_comp"]["GB_s"]))
        rows.append(row)
        del data, data_sets, parity, rec, ref, blocks, surv, surv_sets, par_sets, rec_sets
        torch.cuda.empty_cache()
    return rows


def bench_small(args, stream):
    """RS(10,4) encode of 10 x 1 MiB blocks: 14 MiB per launch, which the
    caches hold and the launch overhead dominates (not a roofline number);
    the interpreter, and with --exec native the programs' native kernels
    (the default split then runs the native block parts at this size)."""
    import paper_2108_02692_amd as E
    from paper_2108_02692_amd import workloads as W
    n, p, S = 10, 4, 1 << 20
    gen = E.ec_matrix_cauchy(n, p)
    data = W.device_blocks(n, S, seed=0)
    parity = W.empty_blocks(p, S)
    res = {"workload": "RS(10,4) encode, 10 x 1 MiB"}
    for level, tag in ((E.LEVEL_CO_FU_SCHED, "comp"), (E.LEVEL_PLAIN, "plain")):
        for native in ((0, E.NATIVE_WHOLE | E.NATIVE_PAIRS | E.NATIVE_BLOCKS) if args.exec == "native" else (0,)):
            prog = E.ec_compile_slp(n, p, gen, level=level, native=native)
            ms = time_launches(lambda: E.ec_encode(prog, data, parity, S, stream), max(args.steps, 100),
                               args.warmup, stream)
            res[tag + ("_native" if native else "")] = {"ms": ms, "GB_s": n * S / ms / 1e6}
    return res


def bench_serving(args, batched_GB_s=None):
    """The serving loop on 20k req/s Poisson arrivals, ``--serve-runs`` times
    (the host can interrupt the loop's thread, which moves p99 from run to
    run): medians of the latency and drain figures, every run's in 'runs';
    then a sweep of arrival rates (about 40,000 requests each) up to the
    drain, where every request is present at once."""
    import numpy as np
    import paper_2108_02692_amd as E
    from paper_2108_02692_amd import serve
    c0, _, _ = E.ec_program_pool_stats()
    t0 = time.perf_counter()
    native = args.exec == "native"
    server = serve.Server(native_encodes=native)
    setup_s = time.perf_counter() - t0
    c1, images, pool_bytes = E.ec_program_pool_stats()
    import torch

    def warm_up():  # the headline's copy warm-up, finished before the drain starts
        prewarm(torch.cuda.current_stream(), PREWARM_MS)
        torch.cuda.synchronize()
    runs = [serve.run(duration_s=args.serve_seconds, seed=7, server=server, warm_up=warm_up)
            for _ in range(max(1, args.serve_runs))]
    res = dict(runs[0])
    keys = ("p50_ms", "p99_ms", "mean_ms", "drain_GB_s", "drain_cold_GB_s", "requests_per_launch",
            "launch_size_p99", "requests_alone", "batched_same_GB_s", "drain_vs_batched_same")
    for k in keys:
        res[k] = float(np.median([r[k] for r in runs]))
    res["runs"] = [{k: r[k] for k in keys} for r in runs]
    sweep = []
    for rate in (20e3, 100e3, 500e3, 2e6, 8e6):
        r = serve.run(duration_s=40000.0 / rate, rate=rate, seed=8, server=server, drain=False)
        sweep.append({k: r[k] for k in ("rate_req_s", "requests", "GB_s", "p50_ms", "p99_ms", "mean_ms",
                                        "requests_per_launch", "launch_size_p50", "launch_size_p99",
                                        "launch_size_max", "requests_alone", "batches")})
        log("serving at %.0f req/s: %.1f GB/s, p50 %.3f ms, p99 %.3f ms, %.1f requests per launch "
            "(p50 %d, p99 %d, max %d; %.0f%% of requests alone)"
            % (rate, r["GB_s"], r["p50_ms"], r["p99_ms"], r["requests_per_launch"], r["launch_size_p50"],
               r["launch_size_p99"], r["launch_size_max"], 100 * r["requests_alone"]))
    res["sweep"] = sweep
    # compiling and uploading the server's programs (every erasure pattern
    # of its codecs): the device allocations the upload made, the distinct
    # records and their bytes
    res["setup"] = {"seconds": setup_s, "programs": len(server.cache), "pool_allocations": c1 - c0,
                    "pool_records": images, "pool_bytes": pool_bytes,
                    "native_kernels": "the codecs' encode programs" if native else "none"}
    if batched_GB_s:
        res["drain_vs_batched"] = res["drain_GB_s"] / batched_GB_s
    return res


def bench_batched(args, stream):
    """8192 stripes mixing RS(6,3), RS(10,4), RS(12,4), RS(14,4); block sizes
    log-uniform 4 KiB .. 4 MiB in 512 B steps; 70% encodes, 30% decodes with
    uniformly drawn erasure sets; one persistent graph launch per step.
    Every input block is its own range of one seeded random pool (no byte
    read twice in a launch); every output is its own buffer."""
    from paper_2108_02692_amd import autotune, batching

    specs, pool, inputs, outputs, out_buf = batching.mixed_workload(args.batch_stripes, hi=args.batch_max_mib << 20)
    out_total = out_buf.numel()
    in_bytes = sum(s.n_in * s.block_bytes for s in specs)
    key = "mix4-%d-%dMiB" % (args.batch_stripes, args.batch_max_mib)
    best, table = autotune.tune(key, specs, inputs, outputs, stream, retune=args.retune,
                                log=lambda r: log("autotune %s" % r))
    cache = batching.ProgramCache(level=best["level"], slots=best["slots"], scheduler=best.get("scheduler", 0))
    cache.warm({(s.n, s.p, s.erased) for s in specs})
    batch = batching.build_batch(specs, cache, inputs, outputs, tile_bytes=best["tile_bytes"], stream=stream)
    ms = autotune.time_batch(batch, stream, steps=max(3, args.steps // 2), warmup=1)
    res = {"stripes": len(specs), "work_items": batch.n_items, "in_bytes": in_bytes, "out_bytes": out_total,
           "ms": ms, "GB_s": in_bytes / ms / 1e6, "hbm_frac": (in_bytes + out_total) / ms / 1e6 / HBM_PEAK_GBS,
           "level": best["level"], "slots": best["slots"], "tile_bytes": best["tile_bytes"],
           "scheduler": "greedy" if best.get("scheduler", 0) else "push",
           "programs": len(cache), "graph": True}
    if table:
        res["autotune"] = table
    batch.free()
    del pool, out_buf, inputs, outputs
    return res


def bench_batched_programs(args, stream):
    """The batched workload's block sizes in four batches, to separate the
    cost of many programs in one launch and of strips that start off a
    128-byte line: the 8192-stripe mix itself (1713 programs), RS(10,4)
    encodes only (one program), RS(10,4) decodes of uniformly drawn erasure
    sets (up to 1470 programs), each of the same 8192 block sizes (multiples
    of 512 B, so a strip may start 64 B into a line), and the RS(10,4)
    encodes with the sizes rounded up to 1 KiB (every strip on a line
    boundary); the RS(10,4) batches' inputs are consecutive 4 KiB-aligned
    ranges of the mix's input pool (distinct bytes, wrapping to the start
    only past its end).  Each batch: the time per
    launch and its algorithmic bytes (a byte-counter run of this command
    gives the fetched bytes per dispatch, in this order, 1 + max(3, steps /
    2) dispatches each)."""
    import itertools
    import numpy as np
    import torch
    import paper_2108_02692_amd as E
    from paper_2108_02692_amd import autotune, batching
    specs, pool, inputs, outputs, _ = batching.mixed_workload(args.batch_stripes, hi=args.batch_max_mib << 20)
    # outputs of the RS(10,4) batches (at most 4 blocks per stripe, blocks
    # rounded up to 1 KiB at most)
    out_buf = torch.empty(sum(4 * (s.block_bytes + 512) for s in specs), dtype=torch.uint8, device="cuda")
    cache = batching.ProgramCache(level=E.LEVEL_CO_FU_SCHED, slots=44)
    rng = np.random.default_rng(9)
    pats = [c for r in range(1, 5) for c in itertools.combinations(range(14), r)]

    def rs10_4(decode, align=512):
        sp, ins, outs, off, cur = [], [], [], 0, 0
        for s0 in specs:
            bb = -(-s0.block_bytes // align) * align
            s = batching.StripeSpec(10, 4, bb, pats[int(rng.integers(len(pats)))] if decode else ())
            sp.append(s)
            span = -(-bb // 4096) * 4096
            blocks = []
            for _ in range(10):
                if cur + bb > pool.numel():
                    cur = 0
                blocks.append(pool[cur:cur + bb])
                cur += span
            ins.append(blocks)
            outs.append([out_buf[off + j * bb: off + (j + 1) * bb] for j in range(s.n_out)])
            off += s.n_out * bb
        assert off <= out_buf.numel()
        return sp, ins, outs

    rows = []
    for name, (sp, ins, outs) in (("mix", (specs, inputs, outputs)), ("rs10_4_encode", rs10_4(False)),
                                  ("rs10_4_decodes", rs10_4(True)), ("rs10_4_encode_1KiB", rs10_4(False, 1024))):
        cache.warm({(s.n, s.p, s.erased) for s in sp})
        batch = batching.build_batch(sp, cache, ins, outs, stream=stream)
        ms = autotune.time_batch(batch, stream, steps=max(3, args.steps // 2), warmup=1)
        rd = sum(s.n_in * s.block_bytes for s in sp)
        wr = sum(s.n_out * s.block_bytes for s in sp)
        rows.append({"batch": name, "stripes": len(sp), "programs": len({(s.n, s.p, s.erased) for s in sp}),
                     "work_items": batch.n_items, "read_bytes": rd, "write_bytes": wr, "ms": ms,
                     "hbm_frac": (rd + wr) / ms / 1e6 / HBM_PEAK_GBS, "launches": 1 + max(3, args.steps // 2)})
        log("%s: %.3f ms, %.3f of peak" % (name, ms, rows[-1]["hbm_frac"]))
        batch.free()
    return rows


def bench_decode_all(args, stream):
    """RS(10,4) decode of every erasure set of at most 4 blocks (1470 sets,
    1001 of them with 4 blocks lost): each set has its own 10 data blocks of
    1 MiB of seeded random bytes, encoded on the device; one batched launch
    reconstructs every erased block of every set, and every result is
    compared with the block it replaces."""
    import itertools
    import torch
    import paper_2108_02692_amd as E
    from paper_2108_02692_amd import batching

    n, p, S = 10, 4, 1 << 20
    pats = [c for r in range(1, p + 1) for c in itertools.combinations(range(n + p), r)]
    P = len(pats)
    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    data = torch.randint(0, 256, (P, n, S), dtype=torch.uint8, device="cuda", generator=g)
    parity = torch.empty((P, p, S), dtype=torch.uint8, device="cuda")
    K = args.decode_all_slots
    cache = batching.ProgramCache(level=E.LEVEL_CO_FU_SCHED, slots=K)
    enc = cache.get(n, p)
    encode = E.ec_batch_build([(enc, list(data[k]), list(parity[k]), S) for k in range(P)], stream=stream)
    encode.launch(stream)
    cache.warm([(n, p, er) for er in pats])
    n_out = sum(len(er) for er in pats)
    out = torch.empty((n_out, S), dtype=torch.uint8, device="cuda")
    stripes, want, o = [], [], 0
    for k, er in enumerate(pats):
        prog = cache.get(n, p, er)
        blocks = list(data[k]) + list(parity[k])
        stripes.append((prog, [blocks[i] for i in prog.in_blocks], list(out[o:o + len(er)]), S))
        want += [blocks[e] for e in er]
        o += len(er)
    batch = E.ec_batch_build(stripes, stream=stream)
    # five untimed launches (18 ms): past the first milliseconds of load, which run slower
    ms = time_launches(lambda: batch.launch(stream), max(3, args.steps // 2), 5, stream)
    ok = all(torch.equal(out[j], want[j]) for j in range(n_out))
    if not ok:
        raise SystemExit("bench.py: decode-all self-check failed")
    in_bytes = P * n * S
    res = {"patterns": P, "block_bytes": S, "ms": ms, "GB_s": in_bytes / ms / 1e6,
           "hbm_frac": (in_bytes + n_out * S) / ms / 1e6 / HBM_PEAK_GBS, "slots": K, "verified": ok}
    encode.free()
    batch.free()
    del data, parity, out
    return res


def cpu_baseline(block_mib: int):
    """The oracle, as is, on a bounded sample of the same workload."""
    import oracle
    from paper_2108_02692_amd import workloads as W
    S = block_mib << 20
    data = W.host_blocks(10, S, seed=2021)
    G = oracle.cauchy(10, 4)
    t = time.time()
    oracle.encode(G, 10, 4, data)
    dt = time.time() - t
    out = {"value": 10 * S / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": "RS(10,4) encode of 10 x %d MiB seeded random blocks, single-threaded C oracle, %.1f s"
                     % (block_mib, dt)}
    # The same oracle on T host threads at once, each encoding its own stripe
    # of 10 x 8 MiB (the C call releases the interpreter lock).
    from concurrent.futures import ThreadPoolExecutor
    T = max(1, min(16, len(os.sched_getaffinity(0))))
    Sp = 8 << 20
    stripes = [W.host_blocks(10, Sp, seed=3000 + i) for i in range(T)]
    with ThreadPoolExecutor(max_workers=T) as ex:
        t = time.time()
        list(ex.map(lambda d: oracle.encode(G, 10, 4, d), stripes))
        dt = time.time() - t
    out["parallel"] = {"value": T * 10 * Sp / dt / 1e9, "unit": "GB/s", "cores": T,
                       "sample": "%d threads, each an RS(10,4) encode of its own 10 x 8 MiB stripe, %.1f s"
                                 % (T, dt)}
    return out


if __name__ == "__main__":
    main()
