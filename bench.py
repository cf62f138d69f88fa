"""Benchmark of the ZSMILES codec hot path on one MI355X.

One step is one pass of the whole path over the bulk workload (10M synthetic SMILES
lines, log-normal length, median 45, clipped to 10..120 chars, about 0.52 GB):
  index   newline index of the raw buffer                 (zs_index_lines)
  compress ring-ID pre-processing + minimum-length parse  (zs_compress)
  decompress of the whole compressed buffer               (zs_decompress)
  random access of 100,000 uniformly random line ids      (zs_decompress_lines)
Inputs are resident in HBM before the timed region.  `value` is the codec's
round-trip throughput: raw bytes entering compression plus raw bytes leaving
decompression, per second of step time.  Per-kernel GB/s, the roofline of the
dominant kernel (compression), random-access p50/p99 latencies and the CPU oracle
timed on a bounded sample are reported beside it on the same JSON line.

    python bench.py [--steps K] [--warmup W] [--lines N] [--no-cpu]
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "compress & decompress GB/s on 1 MI355X (frac of HBM peak); p99 random-access latency"
HBM_PEAK_GBS = 8000.0
# wave64 VALU instructions issued per second: 256 CUs x 4 SIMDs, one wave-instruction per
# 4 cycles each (64 lanes on 16-wide SIMDs), at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
# the uneven workload's binned configuration: short lines in LDS, long lines in four
# bins with global-memory line buffers (more uniform tiles: 2.5% faster than one long
# bin, 0.7% faster than two, on the 20M lines of that workload)
UNEVEN_BINS = dict(edges=(128, 384, 640, 896), lines_per_tile=(256,) * 5, large_lds=(0, 2, 2, 2, 2))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lines", type=int, default=10_000_000)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--ra-batches", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-lines", type=int, default=800_000, help="one-thread oracle sample")
    ap.add_argument("--cpu-all-lines", type=int, default=3_200_000, help="all-cores oracle sample")
    ap.add_argument("--only", default="", help="comma list of ops to run (profiling runs)")
    ap.add_argument("--workload", default="bulk", choices=["bulk", "uneven", "serve", "random", "dicts"],
                    help="bulk: the headline step; uneven: plain vs length-binned / autotuned / graph "
                         "compression; serve: the request loop under Poisson arrivals; random: random-access "
                         "batches on a resident 40M-line shard; dicts: the L_max sweep on the bulk workload "
                         "and the Table I dictionary variants")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-gb", type=float, default=50.0, help="compressed shard bytes resident (GB)")
    ap.add_argument("--shard-lines", type=int, default=40_000_000)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--serve-plain", type=int, default=1000, help="requests replayed through the plain calls")
    ap.add_argument("--probe-copy", action="store_true",
                    help="after the timed steps, one plain 1 GiB device copy (scales the HBM byte counters)")
    ap.add_argument("--tune-lines", type=int, default=0,
                    help="sample the autotuner times (uneven, e.g. 1000000); 0: no autotuning, long lines in "
                         "global memory")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def compiler_version():
    try:
        return subprocess.run(["gcc", "--version"], stdout=subprocess.PIPE, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        return "unknown"


def cpu_baseline(buf, off, n_sample, n_all):
    """The oracle as it is on the host: one thread on the first n_sample lines of the same
    workload, and one process per usable core (at most 16) on the first n_all lines, each
    process on its own contiguous ranges of lines (timed from handing out the work to
    having every result back, the workers already started).  `value` is the all-cores
    figure."""
    import oracle
    from oracle import parallel
    path = os.path.join(ROOT, "paper_2404_19391_amd", "data", "default.zsd")
    d = oracle.Dict.load(path)
    n_sample = min(n_sample, off.size - 1)
    sb = buf[:int(off[n_sample])]
    so = off[:n_sample + 1]
    t0 = time.perf_counter()
    code, _, c, co = oracle.compress(d, sb, so)
    t1 = time.perf_counter()
    code2, _, back, bo = oracle.decompress(d, c, co)
    t2 = time.perf_counter()
    assert code == 0 and code2 == 0
    raw = float(sb.size)
    one = {"value": round((raw + float(back.size)) / (t2 - t0) / 1e9, 6),
           "compress_GBs": round(raw / (t1 - t0) / 1e9, 6),
           "decompress_GBs": round(float(back.size) / (t2 - t1) / 1e9, 6),
           "seconds": round(t2 - t0, 2),
           "sample": "first %d lines (%.1f MB)" % (n_sample, raw / 1e6)}
    # all cores: one worker process per core, disjoint line ranges; wall time includes
    # starting the workers
    n_all = min(n_all, off.size - 1)
    ab = buf[:int(off[n_all])]
    ao = off[:n_all + 1]
    procs = parallel.default_procs()
    with parallel.Pool(path, procs) as pool:
        cc, _, ac, aco, cw, _ = pool.compress(ab, ao)
        dc, _, aback, _, dw, _ = pool.decompress(ac, aco)
    assert cc == 0 and dc == 0
    araw, aout = float(ab.size), float(aback.size)
    return {
        "value": round((araw + aout) / (cw + dw) / 1e9, 6),
        "unit": "GB/s",
        "cores": procs,
        "kind": "oracle",
        "sample": "first %d lines of the bulk workload (%.1f MB): one compress and one decompress, "
                  "%d worker processes of one thread each on disjoint line ranges, in memory"
                  % (n_all, araw / 1e6, procs),
        "compress_GBs": round(araw / cw / 1e9, 6),
        "decompress_GBs": round(aout / dw / 1e9, 6),
        "seconds": round(cw + dw, 2),
        "one_core": one,
        "cpu": cpu_model(),
        "nproc": os.cpu_count(),
        "affinity_cores": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
        "compiler": compiler_version() + " -O2 (oracle/zs_oracle.c, no intrinsics, no threads)",
    }


KERNEL_SOURCES = ["paper_2404_19391_amd/csrc/zs_kernels.hip", "paper_2404_19391_amd/csrc/zs_common.hpp",
                  "paper_2404_19391_amd/csrc/zs_tables.hpp", "paper_2404_19391_amd/csrc/zs_dict.cpp"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(kernel):
    """The committed counter summary of `kernel` (HBM bytes, VALU instructions and LDS bank
    conflicts per launch), if it was taken from the kernel sources as they are now; else {}."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    e = t.get(kernel)
    if not e or e.get("source_sha256") != kernel_source_hash():
        return {}
    return e


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None."""
    return measured_counters(kernel).get("bytes_per_launch")


def copy_peak_gbs(dev, stream, reps=6):
    """Best device-to-device copy rate (GB/s, read + write bytes) of a 1 GiB buffer on this
    GPU: the measured HBM ceiling beside the published one."""
    import torch
    src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    t = time_ms(lambda: dst.copy_(src), stream, reps)
    del src, dst
    return 2.0 * (1 << 30) / (min(t) * 1e-3) / 1e9


def time_ms(fn, stream, reps):
    """Per-call times (ms) of fn on stream, HIP events around each call."""
    import torch
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


DATA = os.path.join(ROOT, "paper_2404_19391_amd", "data")
# L_max sweep (Sec. V-C): dictionary file, the L_max it was trained with
SWEEP = [("lmax5", 5), ("default", 8), ("lmax15", 15), ("long16", 16)]
# Table I (Sec. V-B): dictionary file, pre-processing, pre-population
TABLE1 = [("t1_prep_printable", True, "Printable"), ("t1_raw_printable", False, "Printable"),
          ("t1_prep_smiles", True, "SMILES alphabet"), ("t1_raw_smiles", False, "SMILES alphabet"),
          ("t1_prep_none", True, "None"), ("t1_raw_none", False, "None")]


def bench_dicts(args):
    """The paper's two dictionary experiments on synthetic data.  L_max sweep (Sec. V-C,
    Fig. 5): compression and decompression of the bulk workload with the dictionaries
    trained at L_max 5, 8 and 15, and the long-pattern dictionary (16-wide parse window);
    GB/s per kernel (median of --steps launches), ratio, and the first 200,000 lines of
    each output checked against the oracle.  Table I (Sec. V-B): the six pre-processing x
    pre-population dictionaries on their 50,000-line training set (train = test, as in
    the paper), every output line checked against the oracle."""
    import torch
    import oracle
    import paper_2404_19391_amd as zs
    import smilesgen
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    n = args.lines
    log("generating %d lines" % n)
    buf, off = smilesgen.generate("bulk", args.seed, n, threads=16)
    raw = int(buf.size)
    b = torch.from_numpy(buf).to(dev)
    o = torch.from_numpy(off.astype(np.int64)).to(dev)
    ws = zs.Workspaces(dev)
    res = zs.new_result(dev)
    ncheck = min(n, 200_000)
    sweep = []
    for name, lmax in SWEEP:
        path = os.path.join(DATA, name + ".zsd")
        d = zs.Dict.load(path)
        od = oracle.Dict.load(path)
        c_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
        zs.compress_into(d, b, o, None, c_off, ws.get(zs.OP_COMPRESS, n), res)
        ct = int(c_off[-1].item())
        c = torch.empty(ct, dtype=torch.uint8, device=dev)
        r = torch.empty(raw + 16, dtype=torch.uint8, device=dev)
        r_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
        wc, wd = ws.get(zs.OP_COMPRESS, n), ws.get(zs.OP_DECOMPRESS, n)
        fc = lambda: zs.compress_into(d, b, o, c, c_off, wc, res)  # noqa: E731
        fd = lambda: zs.decompress_into(d, c, c_off, r, r_off, wd, res)  # noqa: E731
        for _ in range(args.warmup):
            fc()
            fd()
        tc = float(np.median(time_ms(fc, stream, args.steps)))
        td = float(np.median(time_ms(fd, stream, args.steps)))
        code, fb = zs.read_result(res)
        assert code == 0, (name, code, fb)
        dec = int(r_off[-1].item())
        code, _, want, woff = oracle.compress(od, buf[:int(off[ncheck])], off[:ncheck + 1])
        got = c[:int(c_off[ncheck].item())].cpu().numpy()
        ok = code == 0 and got.tobytes() == want.tobytes() and \
            np.array_equal(c_off[:ncheck + 1].cpu().numpy().astype(np.uint64), woff)
        idx = 16 * (n + 1)
        sweep.append({"dict": name, "trained_lmax": lmax, "longest_pattern": od.lmax,
                      "parse_window": 8 if od.lmax <= 8 else 16, "ratio": round(ct / raw, 4),
                      "compress_ms": round(tc, 4), "compress_user_GBs": round(raw / tc / 1e6, 2),
                      "compress_hbm_alg_GBs": round((raw + ct + idx) / tc / 1e6, 2),
                      "decompress_ms": round(td, 4), "decompress_user_GBs": round(dec / td / 1e6, 2),
                      "decompress_hbm_alg_GBs": round((dec + ct + idx) / td / 1e6, 2),
                      "oracle_match_first_%d_lines" % ncheck: bool(ok)})
        log(json.dumps(sweep[-1]))
        del c, r, r_off, c_off
    del b, o
    torch.cuda.empty_cache()
    # Table I
    tb, to = smilesgen.generate("small", 1001, 50000)
    tbd = torch.from_numpy(tb).to(dev)
    tod = torch.from_numpy(to.astype(np.int64)).to(dev)
    table = []
    for name, prep, pop in TABLE1:
        path = os.path.join(DATA, name + ".zsd")
        d = zs.Dict.load(path)
        od = oracle.Dict.load(path)
        c, co = zs.compress(d, tbd, tod, preprocess=prep)
        code, _, want, woff = oracle.compress(od, tb, to, preprocess=prep)
        ok = code == 0 and c.cpu().numpy().tobytes() == want.tobytes() and \
            np.array_equal(co.cpu().numpy().astype(np.uint64), woff)
        table.append({"pre_processing": "Yes" if prep else "No", "pre_population": pop,
                      "ratio": round(c.numel() / tb.size, 4), "oracle_match_all_lines": bool(ok)})
        log(json.dumps(table[-1]))
    out = {
        "metric": METRIC, "value": None, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": True, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "dictionary variants: L_max sweep on %d bulk lines (%.3f GB raw); Table I "
                               "on 50,000 small-workload lines (train = test)" % (n, raw / 1e9)},
        "lmax_sweep": sweep, "table1": table,
    }
    print(json.dumps(out), flush=True)


def bench_uneven(args):
    """Uneven line lengths: 20M lines, 90% drug-like (10..120 chars) and 10% long chains
    (200..1,000 chars, deep branches, %nn ring labels), drawn independently per line.
    Compression by the plain call, by the length-binned call with a fixed configuration,
    with the autotuned configuration (--tune-lines 0: long lines in global memory instead),
    and as a replayed HIP graph of that call; all four must give the same bytes."""
    import torch
    import paper_2404_19391_amd as zs
    import smilesgen
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.lines if args.lines != 10_000_000 else 20_000_000
    log("generating %d uneven lines" % n)
    buf, off = smilesgen.generate("uneven", 3, n, threads=16)
    raw = int(buf.size)
    d = zs.Dict.load()
    b = torch.from_numpy(buf).to(dev)
    o = torch.from_numpy(off.astype(np.int64)).to(dev)
    del buf
    stream = torch.cuda.current_stream()
    res = zs.new_result(dev)
    oo = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ws_p = zs.Workspaces(dev).get(zs.OP_COMPRESS, n)
    zs.compress_into(d, b, o, None, oo, ws_p, res)
    total = int(oo[-1].item())
    out_p = torch.empty(total, dtype=torch.uint8, device=dev)
    zs.compress_into(d, b, o, out_p, oo, ws_p, res)
    torch.cuda.synchronize()
    ref_off = oo.clone()
    log("plain: %d -> %d bytes" % (raw, total))
    # autotune on a sample (the first tune-lines lines), or a fixed configuration
    k = min(args.tune_lines, n)
    if k > 0:
        t0 = time.perf_counter()
        cfg_t, tuned_ms, plain_sample_ms, tried = zs.autotune_binned(d, b, o[:k + 1])
        tune_s = time.perf_counter() - t0
        log("autotuned on %d lines in %.1f s over %d configs: %s" % (k, tune_s, tried, cfg_t.as_dict()))
        tname = "binned_autotuned"
    else:
        cfg_t = zs.BinConfig.make(**UNEVEN_BINS)
        tuned_ms = plain_sample_ms = tune_s = None
        tried = 0
        log("no autotuning: %s" % cfg_t.as_dict())
        tname = "binned_long_global"
    cfg_f = zs.BinConfig.make(edges=(128,), lines_per_tile=(256, 64), large_lds=(0, 1))
    ws_b = torch.empty(zs.binned_workspace_bytes(n, total), dtype=torch.uint8, device=dev)
    out_b = torch.empty(total, dtype=torch.uint8, device=dev)
    ob = torch.empty(n + 1, dtype=torch.int64, device=dev)
    runs = {
        "plain": lambda: zs.compress_into(d, b, o, out_p, oo, ws_p, res),
        "binned_fixed": lambda: zs.compress_binned_into(d, b, o, out_b, ob, cfg_f, ws_b, res),
        tname: lambda: zs.compress_binned_into(d, b, o, out_b, ob, cfg_t, ws_b, res),
    }
    identical = {}
    times = {}
    for name, fn in runs.items():
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        times[name] = time_ms(fn, stream, args.steps)
        code, fb = zs.read_result(res)
        identical[name] = bool(code == 0 and torch.equal(out_b if name != "plain" else out_p, out_p)
                               and torch.equal(ob if name != "plain" else oo, ref_off))
    # that call as a HIP graph on a side stream
    s = torch.cuda.Stream(device=dev)
    g = zs.Graph()
    out_b.fill_(0)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with g.capture(s):
            zs.compress_binned_into(d, b, o, out_b, ob, cfg_t, ws_b, res)
    for _ in range(args.warmup):
        g.replay(s)
    s.synchronize()
    times[tname + "_graph"] = time_ms(lambda: g.replay(s), s, args.steps)
    identical[tname + "_graph"] = bool(torch.equal(out_b, out_p) and torch.equal(ob, ref_off))
    med = {k: float(np.median(v)) for k, v in times.items()}
    best = min(med, key=med.get)
    per = {k: {"ms": round(v, 3), "user_GBs": round(raw / (v * 1e-3) / 1e9, 2),
               "speedup_vs_plain": round(med["plain"] / v, 3), "identical_to_plain": identical[k]}
           for k, v in med.items()}
    alg = raw + 2 * 8 * (n + 1) + total
    out = {
        "metric": METRIC,
        "value": round(raw / (med[best] * 1e-3) / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(med[best], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "uneven: %d synthetic SMILES lines, 90%% log-normal 10..120 chars, 10%% long "
                               "chains 200..1000 chars, %.3f GB raw, default dictionary; compression only"
                               % (n, raw / 1e9),
                   "lines": n, "raw_bytes": raw, "compressed_bytes": total, "best": best},
        "roofline": {"kernel": "compress (%s)" % best, "bound": "hbm", "achieved": round(alg / (med[best] * 1e-3) / 1e9, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / (med[best] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None},
        "compress": per,
        "autotune": ({"sample_lines": k, "configs_timed": tried, "seconds": round(tune_s, 2),
                      "chosen": cfg_t.as_dict(), "sample_best_ms": round(tuned_ms, 3),
                      "sample_plain_ms": round(plain_sample_ms, 3)} if k > 0 else None),
        "binned_config": cfg_t.as_dict(),
        "fixed_config": cfg_f.as_dict(),
    }
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Request loop: replicas of one compressed shard (the shard's lines from the bulk
    distribution) resident in HBM with their indexes and one dictionary; 70% random-access
    requests of log-uniform 1..100,000 ids over (replica x line), 30% compression requests of
    log-uniform 1..1,000,000 fresh lines (slices of a pool generated with another seed).
    First the closed-loop capacity (2 x slots clients), then Poisson arrivals at 0.7 x that
    rate; latency = completion - scheduled arrival."""
    import threading
    import torch
    import paper_2404_19391_amd as zs
    import smilesgen
    import oracle
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d = zs.Dict.load()
    n = args.shard_lines
    log("generating the %d-line shard" % n)
    buf, off = smilesgen.generate("bulk", 4, n, threads=16)
    b = torch.from_numpy(buf).to(dev)
    o = torch.from_numpy(off.astype(np.int64)).to(dev)
    del buf, off
    c, co = zs.compress(d, b, o)
    del b, o
    torch.cuda.synchronize()
    cbytes = int(c.numel())
    reps = max(1, int(np.ceil(args.serve_gb * 1e9 / cbytes)))
    log("shard: %d lines -> %.3f GB compressed; %d replicas resident" % (n, cbytes / 1e9, reps))
    srv = zs.Server(d, slots=args.slots, device_bytes=24 << 30, host_bytes=16 << 30)
    shards = [(c, co)] + [(c.clone(), co.clone()) for _ in range(reps - 1)]
    sids = [srv.add_shard(x, y) for x, y in shards]
    torch.cuda.synchronize()
    resident = sum(int(x.numel()) + 8 * int(y.numel()) for x, y in shards)
    log("pool of fresh lines")
    pbuf, poff = smilesgen.generate("bulk", 56, 2_000_000, threads=16)
    host_c = c.cpu().numpy()
    host_co = co.cpu().numpy().astype(np.uint64)

    def make(rng):
        if rng.random() < 0.7:
            k = int(np.exp(rng.uniform(0, np.log(100_000))))
            return ("d", int(rng.integers(0, reps)), rng.integers(0, n, k).astype(np.uint64))
        k = int(np.exp(rng.uniform(0, np.log(1_000_000))))
        s0 = int(rng.integers(0, poff.size - 1 - k))
        lines = pbuf[int(poff[s0]):int(poff[s0 + k])]
        return ("c", s0, k, lines, (poff[s0:s0 + k + 1] - poff[s0]).astype(np.uint64))

    def submit(r):
        if r[0] == "d":
            return srv.submit_decompress(sids[r[1]], r[2])
        return srv.submit_compress(r[3], r[4])

    # closed loop: capacity
    ncl = max(2, 2 * args.slots)
    per = max(20, args.serve_requests // (5 * ncl))
    done_bytes = [0] * ncl

    def client(i):
        rng = np.random.default_rng(1000 + i)
        for _ in range(per):
            r = make(rng)
            code, fb, data, offs, t = srv.wait(submit(r), copy=False)
            done_bytes[i] += t["bytes"] if r[0] == "d" else r[3].size

    log("closed loop: %d clients x %d requests" % (ncl, per))
    t0 = time.perf_counter()
    th = [threading.Thread(target=client, args=(i,)) for i in range(ncl)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    cap_s = time.perf_counter() - t0
    capacity = ncl * per / cap_s
    # open loop: Poisson arrivals at 0.7 x capacity
    rate = 0.7 * capacity
    nreq = args.serve_requests
    rng = np.random.default_rng(5)
    gaps = rng.exponential(1.0 / rate, nreq)
    rreq = np.random.default_rng(55)
    reqs = [make(rreq) for _ in range(nreq)]
    lat = np.zeros(nreq)
    sublag = np.zeros(nreq)  # scheduled arrival -> submission returned (the submitting thread)
    qlat = np.zeros(nreq)  # arrival -> admission (queueing)
    slat = np.zeros(nreq)  # admission -> completion (service: sizing, call, copies)
    kinds = np.array([r[0] == "d" for r in reqs])
    ubytes = np.zeros(nreq)
    replies = {}
    verify = set(int(x) for x in np.random.default_rng(7).choice(nreq, min(200, nreq), replace=False))
    tickets = [None] * nreq
    arrive = np.zeros(nreq)
    ready = threading.Semaphore(0)

    def waiter():
        while True:
            ready.acquire()
            i = next_wait[0]
            next_wait[0] += 1
            if i >= nreq:
                return
            keep = i in verify
            code, fb, data, offs, t = srv.wait(tickets[i], copy=keep)
            lat[i] = t["done"] - arrive[i]
            sublag[i] = t["submit"] - arrive[i]
            qlat[i] = t["admit"] - arrive[i]
            slat[i] = t["done"] - t["admit"]
            ubytes[i] = t["bytes"] if reqs[i][0] == "d" else reqs[i][3].size
            if keep or code != 0:
                replies[i] = (code, fb, data, offs)

    next_wait = [0]
    log("open loop: %d requests at %.1f req/s" % (nreq, rate))
    wt = threading.Thread(target=waiter)
    wt.start()
    base = time.monotonic()
    at = base
    for i in range(nreq):
        at += gaps[i]
        now = time.monotonic()
        if at > now:
            time.sleep(at - now)
        arrive[i] = at
        tickets[i] = submit(reqs[i])
        ready.release()
    ready.release()
    wt.join()
    span = max(time.monotonic() - base, 1e-9)
    st = srv.stats()
    srv.close()
    # the same requests through the plain per-launch calls, one at a time on one stream
    # (inputs to the device, size-only pass, the call, results to the host), no request loop
    nplain = min(nreq, args.serve_plain)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pbytes = 0
    for r in reqs[:nplain]:
        if r[0] == "d":
            sc, sco = shards[r[1]]
            data, offs = zs.decompress_lines(d, sc, sco, torch.from_numpy(r[2].astype(np.int64)).to(dev),
                                             check=False)
        else:
            data, offs = zs.compress(d, torch.from_numpy(r[3]).to(dev),
                                     torch.from_numpy(r[4].astype(np.int64)).to(dev), check=False)
        hd, ho = data.cpu().numpy(), offs.cpu().numpy()
        pbytes += hd.size if r[0] == "d" else r[3].size
    plain_s = time.perf_counter() - t0
    # verification of a sample against the oracle
    od = oracle.Dict.load(zs.default_dict_path())
    checked = bad = 0
    for i in sorted(verify):
        r = reqs[i]
        code, fb, data, offs = replies[i]
        if r[0] == "d":
            w = oracle.decompress_lines(od, host_c, host_co, r[2])
        else:
            if r[2] > 20000:
                continue
            w = oracle.compress(od, r[3], r[4])
        checked += 1
        bad += not (code == w[0] and data.tobytes() == w[2].tobytes() and np.array_equal(offs, w[3]))
    errors = sum(1 for i in replies if replies[i][0] != 0)
    p = lambda a, q: round(float(np.percentile(a, q)) * 1e3, 3) if a.size else None
    out = {
        "metric": METRIC,
        "value": round(float(ubytes.sum()) / span / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": nreq,
        "warmup": ncl * per,
        "ms_per_step": round(span / nreq * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "serving: %d replicas of a %d-line compressed shard (%.1f GB compressed + %.1f GB "
                               "indexes resident), 70%% random access of 1..100k ids, 30%% compression of 1..1M "
                               "new lines, Poisson arrivals at 0.7 x closed-loop capacity"
                               % (reps, n, reps * cbytes / 1e9, (resident - reps * cbytes) / 1e9),
                   "slots": args.slots, "requests": nreq},
        "serving": {"offered_req_s": round(rate, 2), "achieved_req_s": round(nreq / span, 2),
                    "closed_loop_capacity_req_s": round(capacity, 2),
                    "latency_ms": {"p50": p(lat, 50), "p99": p(lat, 99),
                                   "random_access_p50": p(lat[kinds], 50), "random_access_p99": p(lat[kinds], 99),
                                   "compress_p50": p(lat[~kinds], 50), "compress_p99": p(lat[~kinds], 99)},
                    "submit_lag_ms": {"p50": p(sublag, 50), "p99": p(sublag, 99)},
                    "queue_ms": {"p50": p(qlat, 50), "p99": p(qlat, 99)},
                    "service_ms": {"p50": p(slat, 50), "p99": p(slat, 99),
                                   "random_access_p50": p(slat[kinds], 50), "random_access_p99": p(slat[kinds], 99),
                                   "compress_p50": p(slat[~kinds], 50), "compress_p99": p(slat[~kinds], 99)},
                    "user_GBs": round(float(ubytes.sum()) / span / 1e9, 3),
                    "plain_calls": {"requests": nplain, "seconds": round(plain_s, 3),
                                    "req_s": round(nplain / plain_s, 2) if plain_s else None,
                                    "user_GBs": round(pbytes / plain_s / 1e9, 3) if plain_s else None,
                                    "served_capacity_vs_plain": round(capacity / (nplain / plain_s), 2)
                                    if plain_s else None,
                                    "what": "the first requests of the open-loop sequence through the plain calls "
                                            "(compress / decompress_lines with a size-only pass, results copied "
                                            "to the host), one at a time on one stream"},
                    "resident_GB": round(resident / 1e9, 2),
                    "verified": {"checked": checked, "mismatches": bad, "sample": "random requests, compression "
                                 "requests of at most 20,000 lines, against the oracle"},
                    "error_replies": errors, "server": st},
    }
    print(json.dumps(out), flush=True)


def bench_random(args):
    """Random access on a resident shard: 40M lines of the bulk distribution, compressed on
    the device and kept with its uint64 index; batches of 1k, 10k and 100k distinct uniform
    ids (10% of the 1k batches are one contiguous range instead), decompressed and packed in
    request order. Latency per batch is enqueue -> completion with the ids already on the
    device (all batches' ids are uploaded before the batches run), and again with the ids
    copied from pinned host memory inside the bracket. Every
    20th batch is compared with the same lines cut out of a bulk decompression of the shard."""
    import torch
    import paper_2404_19391_amd as zs
    import smilesgen
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.shard_lines
    nb = args.ra_batches if args.ra_batches != 200 else 1000
    log("generating the %d-line shard" % n)
    buf, off = smilesgen.generate("bulk", 4, n, threads=16)
    raw = int(buf.size)
    d = zs.Dict.load()
    b = torch.from_numpy(buf).to(dev)
    o = torch.from_numpy(off.astype(np.int64)).to(dev)
    del buf, off
    c, c_off = zs.compress(d, b, o)
    r, r_off = zs.decompress(d, c, c_off)
    del b, o
    torch.cuda.synchronize()
    cbytes = int(c.numel())
    c_len = (c_off[1:] - c_off[:-1]).cpu().numpy()
    r_len = (r_off[1:] - r_off[:-1]).cpu().numpy()
    log("shard: %d lines, %d raw -> %d compressed bytes" % (n, raw, cbytes))
    stream = torch.cuda.current_stream()
    kmax = 100_000
    ws = zs.Workspaces(dev).get(zs.OP_DECOMPRESS_LINES, kmax)
    res = zs.new_result(dev)
    out = torch.empty(kmax * 256, dtype=torch.uint8, device=dev)
    out_off = torch.empty(kmax + 1, dtype=torch.int64, device=dev)
    ids_pin = torch.empty(kmax, dtype=torch.int64, pin_memory=True)
    ids_dev = torch.empty(kmax, dtype=torch.int64, device=dev)
    rng = np.random.default_rng(44)
    per = {}
    checked = bad = 0
    for k in (1000, 10000, 100000):
        log("random access: %d batches of %d ids" % (nb, k))
        lat, lat_h2d, obytes, abytes, contiguous = [], [], [], [], 0
        # every batch's ids are drawn and put on the device before the batches run, so
        # that they run back to back (drawing 100k distinct ids takes the host ~6 ms,
        # long enough for the idle GPU to lower its clocks before the next batch)
        batches = []
        for it in range(nb + 3):
            if k == 1000 and rng.random() < 0.1:
                start = int(rng.integers(0, n - k))
                batches.append(np.arange(start, start + k, dtype=np.int64))
                contiguous += it >= 3
            else:
                batches.append(rng.choice(n, k, replace=False).astype(np.int64))
        ids_all = torch.from_numpy(np.concatenate(batches)).to(dev)
        for it in range(nb + 3):
            ids_h = batches[it]
            ids_pin[:k].copy_(torch.from_numpy(ids_h))
            ids = ids_all[it * k:(it + 1) * k]
            torch.cuda.synchronize()
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            zs.decompress_lines_into(d, c, c_off, ids, out, out_off[:k + 1], ws, res)
            e1.record(stream)
            e1.synchronize()
            # the same batch with the ids uploaded inside the bracket
            e2.record(stream)
            ids_dev[:k].copy_(ids_pin[:k], non_blocking=True)
            zs.decompress_lines_into(d, c, c_off, ids_dev[:k], out, out_off[:k + 1], ws, res)
            e3 = torch.cuda.Event(enable_timing=True)
            e3.record(stream)
            e3.synchronize()
            code, fb = zs.read_result(res)
            if code != 0:
                raise SystemExit("random access failed: code %d first_bad %d" % (code, fb))
            if it < 3:
                continue
            lat.append(e0.elapsed_time(e1) * 1e3)
            lat_h2d.append(e2.elapsed_time(e3) * 1e3)
            ob = int(r_len[ids_h].sum())
            obytes.append(ob)
            abytes.append(8 * k + 16 * k + int(c_len[ids_h].sum()) + ob + 8 * (k + 1))
            if it % 20 == 0:
                idt = torch.from_numpy(ids_h).to(dev)
                st = r_off[idt]
                ln = r_off[idt + 1] - st
                cum = torch.cumsum(ln, 0)
                pos = torch.repeat_interleave(st - (cum - ln), ln) + torch.arange(int(cum[-1]), device=dev)
                ok = bool(torch.equal(out[:int(cum[-1])], r[pos]) and int(out_off[0]) == 0
                          and torch.equal(out_off[1:k + 1], cum))
                checked += 1
                bad += not ok
        del ids_all
        lat = np.array(lat)
        lat_h2d = np.array(lat_h2d)
        med = float(np.median(lat))
        per[str(k)] = {"batches": len(lat), "contiguous_batches": contiguous,
                       "p50_us": round(float(np.percentile(lat, 50)), 2),
                       "p99_us": round(float(np.percentile(lat, 99)), 2),
                       "p50_us_with_id_upload": round(float(np.percentile(lat_h2d, 50)), 2),
                       "p99_us_with_id_upload": round(float(np.percentile(lat_h2d, 99)), 2),
                       "lines_per_s": round(k / (med * 1e-6), 1),
                       "output_GBs": round(float(np.median(np.array(obytes) / (lat * 1e-6))) / 1e9, 2),
                       "alg_GBs": round(float(np.median(np.array(abytes) / (lat * 1e-6))) / 1e9, 2)}
    big = per["100000"]
    res_line = {
        "metric": METRIC,
        "value": big["output_GBs"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": nb,
        "warmup": 3,
        "ms_per_step": round(big["p50_us"] * 1e-3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "random access: a %d-line shard of the bulk distribution (%.2f GB raw, %.2f GB "
                               "compressed + %.2f GB index resident), batches of 1k/10k/100k distinct uniform ids, "
                               "10%% of the 1k batches one contiguous range; value = output GB/s of the 100k "
                               "batches (median)" % (n, raw / 1e9, cbytes / 1e9, 8 * (n + 1) / 1e9),
                   "lines": n, "raw_bytes": raw, "compressed_bytes": cbytes},
        "roofline": {"kernel": "decompress_kernel (gather, 100k ids)", "bound": "hbm",
                     "achieved": big["alg_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(big["alg_GBs"] / HBM_PEAK_GBS, 4), "traffic": None},
        "random_access": per,
        "p99_random_access_us_100k": big["p99_us"],
        "verified": {"batches_checked": checked, "mismatches": bad,
                     "against": "the same lines cut from a bulk decompression of the shard"},
    }
    print(json.dumps(res_line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this codec's path runs on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2404_19391_amd as zs
    import smilesgen

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload == "uneven":
        return bench_uneven(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "random":
        return bench_random(args)
    if args.workload == "dicts":
        return bench_dicts(args)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    only = set(args.only.split(",")) if args.only else {"index", "compress", "decompress", "random"}

    log("generating %d lines" % args.lines)
    buf, off = smilesgen.generate("bulk", args.seed, args.lines, threads=16)
    raw_bytes = int(buf.size)
    n = args.lines
    d = zs.Dict.load()
    b = torch.from_numpy(buf).to(dev)
    o = torch.from_numpy(off.astype(np.int64)).to(dev)
    ws = zs.Workspaces(dev)
    res = zs.new_result(dev)

    # sizes (one untimed size-only pass), buffers allocated once
    c_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    zs.compress_into(d, b, o, None, c_off, ws.get(zs.OP_COMPRESS, n), res)
    c_total = int(c_off[-1].item())
    c = torch.empty(c_total, dtype=torch.uint8, device=dev)
    r = torch.empty(raw_bytes + 16, dtype=torch.uint8, device=dev)
    r_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    idx = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nl_out = torch.zeros(1, dtype=torch.int64, device=dev)
    ra_n = 100_000
    gen = torch.Generator(device="cpu").manual_seed(44)
    ra_ids = torch.randint(0, n, (ra_n,), generator=gen).to(dev)
    # random access output bound: longest decompressed line <= 120 chars + newline here
    ra_out = torch.empty(ra_n * 128, dtype=torch.uint8, device=dev)
    ra_off = torch.empty(ra_n + 1, dtype=torch.int64, device=dev)
    ws_c = ws.get(zs.OP_COMPRESS, n)
    ws_d = ws.get(zs.OP_DECOMPRESS, n)
    ws_r = ws.get(zs.OP_DECOMPRESS_LINES, ra_n)
    ws_i = ws.get(zs.OP_INDEX, raw_bytes)
    res_c, res_d, res_r, res_i = (zs.new_result(dev) for _ in range(4))

    ops = []
    if "index" in only:
        ops.append(("index", lambda: zs.index_into(b, idx, nl_out, ws_i, res_i)))
    ops.append(("compress", lambda: zs.compress_into(d, b, o, c, c_off, ws_c, res_c)))
    if "decompress" in only:
        ops.append(("decompress", lambda: zs.decompress_into(d, c, c_off, r, r_off, ws_d, res_d)))
    if "random" in only:
        ops.append(("random", lambda: zs.decompress_lines_into(d, c, c_off, ra_ids, ra_out, ra_off, ws_r, res_r)))

    stream = torch.cuda.current_stream()

    def step(events=None):
        for k, (name, fn) in enumerate(ops):
            if events is not None:
                events[k][0].record(stream)
            fn()
            if events is not None:
                events[k][1].record(stream)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for name, rr in (("compress", res_c), ("decompress", res_d), ("random", res_r), ("index", res_i)):
        if any(name == n_ for n_, _ in ops):
            code, fb = zs.read_result(rr)
            if code != 0:
                raise SystemExit("%s failed: code %d first_bad %d" % (name, code, fb))
    if "decompress" in only:
        assert int(r_off[-1].item()) <= r.numel()

    log("timing %d steps" % args.steps)
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in ops]
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_op = {name: [] for name, _ in ops}
    for s in range(args.steps):
        for k, (name, _) in enumerate(ops):
            per_op[name].append(evs[s][k][0].elapsed_time(evs[s][k][1]))
    ms_step = (t1 - t0) * 1e3 / args.steps
    med = {k: float(np.median(v)) for k, v in per_op.items()}
    mean = {k: float(np.mean(v)) for k, v in per_op.items()}

    dec_bytes = int(r_off[-1].item()) if "decompress" in only else raw_bytes
    # algorithmic bytes (per line: raw line + in_off entry + compressed line + out_off entry)
    idx_bytes = 8 * (n + 1)
    comp_alg = raw_bytes + idx_bytes + c_total + idx_bytes
    dec_alg = c_total + idx_bytes + dec_bytes + idx_bytes
    result = {}
    comp_gbs = raw_bytes / (med["compress"] * 1e-3) / 1e9
    comp_hbm = comp_alg / (mean["compress"] * 1e-3) / 1e9
    result["compress"] = {"ms": round(med["compress"], 4), "user_GBs": round(comp_gbs, 2),
                          "hbm_alg_GBs": round(comp_alg / (med["compress"] * 1e-3) / 1e9, 2),
                          "frac_hbm_peak": round(comp_alg / (med["compress"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "ratio": round(c_total / raw_bytes, 4)}
    if "decompress" in only:
        result["decompress"] = {"ms": round(med["decompress"], 4),
                                "user_GBs": round(dec_bytes / (med["decompress"] * 1e-3) / 1e9, 2),
                                "hbm_alg_GBs": round(dec_alg / (med["decompress"] * 1e-3) / 1e9, 2),
                                "frac_hbm_peak": round(dec_alg / (med["decompress"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if "index" in only:
        result["index"] = {"ms": round(med["index"], 4),
                           "hbm_alg_GBs": round((raw_bytes + idx_bytes) / (med["index"] * 1e-3) / 1e9, 2)}
    # the step's throughput: raw bytes into compression + raw bytes out of decompression
    step_raw = raw_bytes + (dec_bytes if "decompress" in only else 0)
    value = step_raw / (ms_step * 1e-3) / 1e9

    # random-access latency per batch size (enqueue -> completion, ids already on the device)
    ra = {}
    if "random" in only:
        rng = np.random.default_rng(45)
        for k in (1000, 10000, 100000):
            lat = []
            # all batches' ids on the device first, so that the batches run back to back
            batches = []
            for it in range(args.ra_batches + 3):
                if rng.random() < 0.1 and k == 1000:
                    start = int(rng.integers(0, n - k))
                    batches.append(np.arange(start, start + k, dtype=np.int64))
                else:
                    batches.append(rng.choice(n, k, replace=False).astype(np.int64) if k < n else np.arange(n))
            ids_all = torch.from_numpy(np.concatenate(batches)).to(dev)
            for it in range(args.ra_batches + 3):
                ids_d = ids_all[it * k:(it + 1) * k]
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                zs.decompress_lines_into(d, c, c_off, ids_d, ra_out, ra_off, ws_r, res_r)
                e1.record(stream)
                e1.synchronize()
                if it >= 3:
                    lat.append(e0.elapsed_time(e1) * 1e3)
            lat = np.array(lat)
            ra[str(k)] = {"p50_us": round(float(np.percentile(lat, 50)), 2),
                          "p99_us": round(float(np.percentile(lat, 99)), 2),
                          "lines_per_s": round(k / (np.median(lat) * 1e-6), 1)}
        result["random_access"] = ra

    roof = {"kernel": "compress_kernel", "bound": "hbm",
            "achieved": round(comp_hbm, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(comp_hbm / HBM_PEAK_GBS, 4), "traffic": measured_traffic("compress_kernel"),
            "alg_bytes_per_launch": comp_alg, "avg_launch_ms": round(mean["compress"], 4)}
    # the roof the kernel actually meets: VALU instruction issue (counters of the same sources,
    # divided by the live launch time), and the HBM fraction against a measured copy as well
    ctr = measured_counters("compress_kernel")
    if ctr.get("valu_insts_per_launch"):
        rate = ctr["valu_insts_per_launch"] / (mean["compress"] * 1e-3)
        roof["valu_issue"] = {"achieved_G_per_s": round(rate / 1e9, 1), "peak_G_per_s": VALU_ISSUE_PEAK / 1e9,
                              "frac": round(rate / VALU_ISSUE_PEAK, 4),
                              "lds_bank_conflict_frac": ctr.get("lds_bank_conflict_frac")}
    cp = copy_peak_gbs(dev, stream)
    roof["copy_peak_measured_GBs"] = round(cp, 1)
    roof["frac_of_measured_copy"] = round(comp_hbm / cp, 4)
    if args.probe_copy:
        # a plain copy of known size, for the counter scale factor of the HBM byte counters
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src.view(torch.int8))  # a dtype cast: an elementwise kernel (not a DMA copy), same bits
        torch.cuda.synchronize()
        del src, dst

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "bulk: %d synthetic SMILES lines, log-normal length (median 45, sigma 0.5, "
                               "clipped 10..120), %.3f GB raw, default dictionary" % (n, raw_bytes / 1e9),
                   "lines": n, "raw_bytes": raw_bytes, "compressed_bytes": c_total,
                   "step": "+".join(name for name, _ in ops)},
        "roofline": roof,
        "kernels": result,
        "p99_random_access_us_100k": ra.get("100000", {}).get("p99_us"),
    }
    if not args.no_cpu:
        log("cpu baseline on %d lines" % args.cpu_lines)
        out["cpu_baseline"] = cpu_baseline(buf, off, args.cpu_lines, args.cpu_all_lines)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
