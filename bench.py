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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lines", type=int, default=10_000_000)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--ra-batches", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-lines", type=int, default=120_000)
    ap.add_argument("--only", default="", help="comma list of ops to run (profiling runs)")
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


def cpu_baseline(buf, off, n_sample):
    """The oracle as it is, one thread, on the first n_sample lines of the same workload."""
    import oracle
    d = oracle.Dict.load(os.path.join(ROOT, "paper_2404_19391_amd", "data", "default.zsd"))
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
    return {
        "value": round((raw + float(back.size)) / (t2 - t0) / 1e9, 6),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "first %d lines of the bulk workload (%.1f MB): one compress and one decompress, "
                  "single thread, in memory" % (n_sample, raw / 1e6),
        "compress_GBs": round(raw / (t1 - t0) / 1e9, 6),
        "decompress_GBs": round(float(back.size) / (t2 - t1) / 1e9, 6),
        "seconds": round(t2 - t0, 2),
        "cpu": cpu_model(),
    }


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
            for it in range(args.ra_batches + 3):
                if rng.random() < 0.1 and k == 1000:
                    start = int(rng.integers(0, n - k))
                    ids_h = np.arange(start, start + k, dtype=np.int64)
                else:
                    ids_h = rng.choice(n, k, replace=False).astype(np.int64) if k < n else np.arange(n)
                ids_d = torch.from_numpy(ids_h).to(dev)
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
            "frac": round(comp_hbm / HBM_PEAK_GBS, 4), "traffic": None,
            "alg_bytes_per_launch": comp_alg, "avg_launch_ms": round(mean["compress"], 4)}

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
        out["cpu_baseline"] = cpu_baseline(buf, off, args.cpu_lines)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
