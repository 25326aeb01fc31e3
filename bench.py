#!/usr/bin/env python3
"""Benchmark of the radix-tree-forest sampling path on one MI355X.

One step = the whole hot path over one batch held in HBM:
    quantise f32 weights -> build guide table + radix tree forest -> sample
    2^26 uniforms to indices and continuous positions x.
Workload H24: n = 2^24 uniform(0,1] weights, S = 2^26; the number of guide
cells m is the autotuner's choice among m/n in {1/4, 1/2, 1, 2} (timed on the
same data before the measured steps; --cell-ratio fixes it instead).

Prints one JSON line (the last line of stdout).  ``value`` is samples per
second of the whole step; build Melem/s, sampling-only samples/s and the two
same-GPU baselines (binary search, Cutpoint + bisection) are extra fields.
Kernel times come from HIP events on the stream the library launches on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("samples/s + build Melem/s at n=2^24 (% HBM peak) vs binary search, bit-exact")
HBM_PEAK_GBS = 8000.0
NODE_B, CELL_B, U_B, IDX_B, X_B, W_B = 16, 64, 8, 4, 8, 4
# Bytes the memory system moves for one random load: a whole 128-byte line.
# Measured with the L2 request-size counters (TCC_EA0_RDREQ_{32B,64B,128B}):
# every read request k_sample makes is a 128-byte request.
LINE_B = 128
PROFILE_DIR = os.path.join(ROOT, "profiles")


def source_hash() -> str:
    """Hash of the library's HIP sources and header; a committed counter
    summary carries the hash it was taken with."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1901_05423_amd", "csrc", "*"))
                   + glob.glob(os.path.join(ROOT, "include", "*.h")))
    for fn in files:
        h.update(os.path.basename(fn).encode())
        with open(fn, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary
    (calibrated FETCH_SIZE + WRITE_SIZE), or None when there is none or the
    sources changed since the counters were taken."""
    path = os.path.join(PROFILE_DIR, f"{kernel}_{workload}.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    if f"source_hash: {source_hash()}" not in text:
        return None
    for line in text.splitlines():
        cols = [c.strip() for c in line.split("|")]
        if len(cols) > 9 and cols[1].startswith(f"`rtf::{kernel}"):
            return (float(cols[8]) + float(cols[9])) * 2 ** 20
    return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--log2n", type=int, default=24)
    p.add_argument("--log2s", type=int, default=26)
    p.add_argument("--kind", choices=["uniform", "zipf"], default="uniform")
    p.add_argument("--cell-ratio", type=float, default=None,
                   help="guide cells per weight m/n; default: the autotuner's choice for "
                        "this shape (tune.best_cell_ratio, timed on the same data)")
    p.add_argument("--tile", type=int, default=0, choices=[0, 1024, 2048],
                   help="build tile in elements (0: the tuner's choice on this data)")
    p.add_argument("--collapsed", action="store_true",
                   help="with --cell-ratio on a batched workload: descend collapsed 4-ary records")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--profile", action="store_true",
                   help="few steps, no baselines (for rocprofv3 runs)")
    p.add_argument("--config", choices=["h24", "c3", "c4", "c5", "table1", "grad1", "quality"],
                   default="h24",
                   help="h24: the benchmark line; c3/c4/c5: the 2D map, the uneven batch and "
                        "the differentiable workload; table1: load counts and speed on the "
                        "paper's high-dynamic-range densities; quality: the quadratic error of "
                        "Hammersley points mapped by the inverse and by the Alias Method on the "
                        "2D map (extra measurements)")
    return p.parse_args()


def replay_lookup(key, child, table, K, aux, m, u, wide=None):
    """Replay this library's lookup on the host (exported forest): the 64-byte
    cell record, and only when it does not resolve the sample, the descent
    from the cell tree's root, one 16-byte node per binary level, or with
    `wide` (the collapsed records as int64 [n, 8]) one 64-byte record per two
    levels.  The descent meets both keys of the sampled interval except when
    it ends at its cell's last leaf; then one more key is read for the
    position.  Returns per sample: whether it descended, the records the
    descent read, and whether the upper key was read after it."""
    g = ((u.astype(object) * m) >> 64).astype(np.int64)
    ref = table[g].astype(np.int64)
    ax = aux[g].astype(np.int64)
    deeper = (ref >= 0) & (ax >= 0) & (u >= K[g, K.shape[1] - 1])
    j = np.where(deeper, ax, -1).astype(np.int64)
    visits = np.zeros(u.size, np.int64)
    hi_seen = np.zeros(u.size, bool)
    if wide is not None:
        wk = wide[:, 0].view(np.uint64)
        wc = wide[:, 1:3].view(np.uint64)
        wr = wide[:, 3:5].copy().view(np.int32).reshape(-1, 4).astype(np.int64)
    active = j >= 0
    while active.any():
        ja, ua = j[active], u[active]
        visits[active] += 1
        if wide is None:
            right = ua >= key[ja]
            hs = ~right
            nj = np.where(right, child[ja, 1], child[ja, 0])
        else:
            right = ua >= wk[ja]
            g0 = np.where(right, wr[ja, 2], wr[ja, 0])
            g1 = np.where(right, wr[ja, 3], wr[ja, 1])
            kc = np.where(right, wc[ja, 1], wc[ja, 0])
            leaf = g0 == g1
            r2 = ua >= kc
            hs = ~right | (~leaf & ~r2)
            nj = np.where(leaf, g0, np.where(r2, g1, g0))
        hi_seen[active] |= hs
        j[active] = nj
        active = j >= 0
    late = deeper & ~hi_seen
    return deeper, visits, late


def sample_bytes_model(key, child, table, K, aux, m, u, wide=None):
    """Mean useful bytes a sample reads beyond its streams (the 64-byte cell
    record, the records of a descent and the late upper key), the mean number
    of dependent random reads per sample, the mean descent length and the
    fraction of samples the record resolves."""
    deeper, visits, late = replay_lookup(key, child, table, K, aux, m, u, wide)
    rec_b = NODE_B if wide is None else 64
    extra = CELL_B + deeper * (rec_b * visits + NODE_B * late)
    loads = 1 + deeper * (visits + late)
    return float(extra.mean()), float(loads.mean()), \
        float(visits[deeper].mean()) if deeper.any() else 0.0, float(1.0 - deeper.mean())


def loads_forest_alg2(key, child, table, m, u):
    """Alg. 2 load by load, as the paper counts it: the guide entry, then one
    node record per step until a leaf."""
    g = ((u.astype(object) * m) >> 64).astype(np.int64)
    j = table[g].astype(np.int64)
    loads = np.ones(u.size, np.int64)
    active = j >= 0
    while active.any():
        ja = j[active]
        loads[active] += 1
        j[active] = np.where(u[active] < key[ja], child[ja, 0], child[ja, 1])
        active = j >= 0
    return loads


def loads_forest_records(key, child, table, K, aux, m, u, wide=None):
    """Dependent reads per sample of this library's lookup (replay_lookup)."""
    deeper, visits, late = replay_lookup(key, child, table, K, aux, m, u, wide)
    return 1 + deeper * (visits + late)


def loads_bisection(key, lo, hi, u):
    """Key loads of the bisection the baselines run on [lo, hi]."""
    MAX = np.uint64(2 ** 64 - 1)
    a, b = lo.astype(np.int64).copy(), hi.astype(np.int64) + 1
    cnt = np.zeros(u.size, np.int64)
    act = b - a > 1
    while act.any():
        mid = a + (b - a) // 2
        k = key[np.minimum(mid, key.size - 1)]
        go = (k != MAX) & (k <= u)
        a = np.where(act & go, mid, a)
        b = np.where(act & ~go, mid, b)
        cnt += act
        act = b - a > 1
    return cnt


def loads_cutpoint(key, table, m, u):
    """The Cutpoint Method with bisection (Sec. 2.5): the guide entry, then a
    bisection between the cell's first overlapping interval and the next
    cell's."""
    n = key.size
    g = ((u.astype(object) * m) >> 64).astype(np.int64)
    r0 = table[g].astype(np.int64)
    r1 = np.where(g + 1 < m, table[np.minimum(g + 1, m - 1)].astype(np.int64), n - 1)
    covered = r0 < 0
    lo = np.where(covered, ~r0, np.maximum(r0 - 1, 0))
    hi = np.where(covered, ~r0, np.where(g + 1 < m, np.where(r1 < 0, ~r1, r1), n - 1))
    hi = np.maximum(hi, lo)
    return 1 + loads_bisection(key, lo, hi, u)


def load_stats(loads):
    """Maximum, average, and the average over groups of 32 and 64 consecutive
    samples of each group's maximum (a synchronised group waits for its
    slowest member)."""
    def group(G):
        k = (loads.size // G) * G
        return float(loads[:k].reshape(-1, G).max(axis=1).mean())
    return {"max": int(loads.max()), "avg": float(loads.mean()), "avg32": group(32),
            "avg64": group(64)}


def timed(fn, start, stop, reps, before=None):
    """Median and all times (ms) of fn() over reps runs, each bracketed by HIP
    events on the current stream (the stream the library launches on);
    before(), if given, runs ahead of each bracket (e.g. a cache flush).
    A short GPU spin (about 40 us) runs ahead of each bracket, so that the host
    has enqueued all of fn's kernels when the start event fires: the bracket
    then holds the kernels back to back, as in the timed steps, and not the
    host's launch latency."""
    import torch
    ts = []
    for _ in range(reps):
        if before is not None:
            before()
        torch.cuda._sleep(100000)
        start.record()
        fn()
        stop.record()
        stop.synchronize()
        ts.append(start.elapsed_time(stop))
    return float(np.median(ts)), ts


def probe_lib():
    """librtf_probe.so: the sampling step's memory pattern without a search."""
    import ctypes
    import importlib
    bmod = importlib.import_module("paper_1901_05423_amd.build")
    P = ctypes.CDLL(bmod.PROBE_LIB)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    P.rtf_probe_gather.argtypes = [vp, i64, vp, i64, vp, i64, i32, vp, vp, vp]
    P.rtf_probe_gather.restype = ctypes.c_int
    return P


def host_cpu():
    """Host CPU model and the cores this process may use."""
    model = ""
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, usable


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the forest of "
              "one distribution is built and sampled on a single device", file=sys.stderr)
        sys.exit(2)
    if args.config != "h24":
        {"c3": run_c3, "c4": run_c4, "c5": run_c5, "table1": run_table1,
         "grad1": run_grad1, "quality": run_quality}[args.config](args)
        return
    import ctypes
    import torch
    import paper_1901_05423_amd as rtf
    from paper_1901_05423_amd import workloads as wl

    dev = torch.device("cuda:0")
    n, S = 1 << args.log2n, 1 << args.log2s
    cid = wl.H24_UNIFORM if args.kind == "uniform" else wl.H24_ZIPF
    r = wl.rng(cid)
    v_h = wl.weights_uniform(r, n) if args.kind == "uniform" else wl.weights_zipf(r, n)
    u_h = wl.uniforms(r, S)
    v = torch.from_numpy(v_h).to(dev)
    u = torch.from_numpy(u_h).to(dev)
    q = torch.empty(n, dtype=torch.uint32, device=dev)
    scale = torch.empty(1, dtype=torch.float64, device=dev)
    tune_info = {"source": "fixed"}
    if args.cell_ratio is None:
        # the guide size m/n is the autotuner's choice, timed on this data
        from paper_1901_05423_amd import tune
        rtf.quantize(v, out=(q, scale))
        ratio, times = tune.best_cell_ratio(q, u, use_cache=False, with_times=True)
        tune_info = {"source": "tuner", "ms_build_plus_sample": times}
    else:
        ratio = args.cell_ratio
    m = max(1, int(round(ratio * n)))
    idx = torch.empty(S, dtype=torch.int32, device=dev)
    x = torch.empty(S, dtype=torch.float64, device=dev)
    holder = {}

    ws = torch.empty(rtf.lib().rtf_workspace_bytes(n, m), dtype=torch.uint8, device=dev)
    tile = args.tile
    if not tile:
        # the build tile is the tuner's choice too, at the chosen m
        from paper_1901_05423_amd import tune
        rtf.quantize(v, out=(q, scale))
        tile, tile_times = tune.best_tile(
            lambda tl: rtf.sample(rtf.build(q, m, ws=ws, tile=tl), u, out=(idx, x)))
        tune_info["ms_build_plus_sample_by_tile"] = tile_times

    def step():
        rtf.quantize(v, out=(q, scale))
        holder["f"] = rtf.build(q, m, ws=ws, tile=tile)
        rtf.sample(holder["f"], u, out=(idx, x))

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    # warmup
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    holder["f"].check()

    # timed whole steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for _ in range(args.steps):
        step()
    ev[1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev[0].elapsed_time(ev[1]) / args.steps

    # per-phase times: medians of separately bracketed launch sequences, HIP
    # events on the library's stream; warm (back to back) and cold (the
    # 256 MB Infinity Cache flushed by a 512 MiB write before each repetition)
    f = holder["f"]
    reps = 5 if args.profile else max(50, args.steps)
    t_quant, _ = timed(lambda: rtf.quantize(v, out=(q, scale)), ev[2], ev[3], reps)
    t_build, _ = timed(lambda: rtf.build(q, m, ws=ws), ev[2], ev[3], reps)
    t_sample, _ = timed(lambda: rtf.sample(f, u, out=(idx, x)), ev[2], ev[3], reps)
    out = {}
    if not args.profile:
        flush_buf = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        flush = lambda: flush_buf.fill_(7)  # noqa: E731
        t_build_cold, _ = timed(lambda: rtf.build(q, m, ws=ws), ev[2], ev[3], reps, flush)
        t_sample_cold, _ = timed(lambda: rtf.sample(f, u, out=(idx, x)), ev[2], ev[3], reps,
                                 flush)
        ref_idx = idx.clone()
        # the same-GPU baselines; their indices must equal the forest's
        idx_b = torch.empty_like(idx)
        x_b = torch.empty_like(x)
        t_bs, _ = timed(lambda: rtf.sample_bsearch(f, u, out=(idx_b, x_b)), ev[2], ev[3], 10)
        assert torch.equal(idx_b, ref_idx), "binary search and forest indices differ"
        t_cb, _ = timed(lambda: rtf.sample_cutpoint_bsearch(f, u, out=(idx_b, x_b)), ev[2], ev[3],
                        10)
        assert torch.equal(idx_b, ref_idx), "Cutpoint + bisection and forest indices differ"
        out["bsearch_samples_s"] = S / (t_bs * 1e-3)
        out["cutpoint_bsearch_samples_s"] = S / (t_cb * 1e-3)
        # coherent uniforms: the same uniforms sorted, so that neighbouring
        # lanes read neighbouring records (streaming instead of random lines)
        sign = torch.tensor(-(1 << 63), dtype=torch.int64, device=dev)
        u_sorted = (torch.sort(u.view(torch.int64) ^ sign).values ^ sign).view(u.dtype)
        t_sorted, _ = timed(lambda: rtf.sample(f, u_sorted, out=(idx_b, x_b)), ev[2], ev[3], reps)
        del u_sorted
        # the same memory pattern without the search: one random 64-byte
        # record per sample (and one more 16-byte node read for depth 2)
        P = probe_lib()
        pp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

        def gather(depth):
            rc = P.rtf_probe_gather(ctypes.c_void_p(f.desc.cells), m,
                                    ctypes.c_void_p(f.desc.nodes), n, pp(u), S, depth,
                                    pp(idx_b), pp(x_b), st)
            assert rc == 0, rc
        t_g1, _ = timed(lambda: gather(1), ev[2], ev[3], reps)
        t_g2, _ = timed(lambda: gather(2), ev[2], ev[3], reps)
        t_g1_cold, _ = timed(lambda: gather(1), ev[2], ev[3], reps, flush)
        del flush_buf
    if args.profile:
        # calibration for the HBM byte counters: a plain copy of known size
        src = torch.empty(1 << 28, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
    torch.cuda.synchronize()

    # algorithmic bytes per sample of the sampling kernel: stream u, idx, x;
    # one guide entry; the node records the descent reads; the two keys the
    # position reads (one record pair)
    key, child, table, W, (K, aux) = f.export(with_cells=True)
    sub = u_h[:: max(1, S // (1 << 20))]
    extra, loads, dbar, resolved = sample_bytes_model(key, child, table, K, aux, m, sub)
    streams = U_B + IDX_B + X_B
    per_sample = streams + LINE_B * loads  # what the memory system moves
    useful = streams + extra               # the bytes the search uses
    sample_bytes = per_sample * S
    # build bytes as the method defines them: read w (4 B), write the key (8 B)
    # and the two child references (8 B) per element, one 4-byte guide entry
    # per cell
    build_alg_bytes = (W_B + 8 + 8) * n + 4 * m
    # what this design reads and writes: the weights twice (tile sums, then
    # the tile kernel), 16-byte node records, 64-byte cell records
    build_design_bytes = (2 * W_B + NODE_B) * n + CELL_B * m
    achieved = sample_bytes / (t_sample * 1e-3) / 1e9
    build_gbs = build_alg_bytes / (t_build * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": S / (ms_step * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": f"H24-{args.kind}: one distribution of n=2^{args.log2n} "
                        f"{'uniform(0,1]' if args.kind == 'uniform' else 'Zipf(1.1) permuted'} "
                        f"f32 weights quantised to u32, m={ratio:g}n guide cells ({tune_info['source']}), "
                        f"S=2^{args.log2s} u64 uniforms -> int32 index + f64 position",
            "n": n, "m": m, "tile": tile, "samples": S, "cell_ratio": ratio,
            "cell_ratio_tuning": tune_info,
        },
        "phase_ms": {"quantize": t_quant, "build": t_build, "sample": t_sample,
                     "statistic": f"median of {reps}"},
        "build_melem_s": n / (t_build * 1e-3) / 1e6,
        "sample_only_samples_s": S / (t_sample * 1e-3),
        "descent_nodes_when_needed": dbar,
        "resolved_by_cell_record": resolved,
        "roofline": {
            "kernel": "k_sample (Alg. 2 descent + position)",
            "bound": "hbm",
            "counted_at": "L2 misses to the fabric: every random read moves a 128-byte line, and "
                          "reads the 256 MB Infinity Cache serves count too (no counter here "
                          "separates them from DRAM reads); cold-cache rate in sampling_cold",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": counted_traffic("k_sample", f"h24_{args.kind}")
            if m == n // 4 and S == 1 << 26 and n == 1 << 24 else None,
            "bytes_per_sample": per_sample,
            "random_loads_per_sample": loads,
            "line_bytes": LINE_B,
            "useful_bytes_per_sample": useful,
            "useful_frac": useful * S / (t_sample * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "build_roofline": {
            "kernels": "k_tile_sums + k_dist_params + k_build_tile + k_fixup",
            "bound": "hbm",
            "bytes_per_elem": build_alg_bytes / n,
            "bytes_definition": "read w 4 B + write key 8 B + child0/child1 8 B per element, "
                                "guide entry 4 B per cell",
            "achieved": build_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": build_gbs / HBM_PEAK_GBS,
            "design_bytes_per_elem": build_design_bytes / n,
            "design_frac": build_design_bytes / (t_build * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "design_bytes_definition": "w read twice, 16-byte node records, 64-byte cell records",
        },
        "wall_s_timed": wall,
    }
    if not args.profile:
        cold_gbs = sample_bytes / (t_sample_cold * 1e-3) / 1e9
        result["sampling_cold"] = {
            "ms": t_sample_cold, "samples_s": S / (t_sample_cold * 1e-3),
            "achieved_gbs": cold_gbs, "frac": cold_gbs / HBM_PEAK_GBS,
            "flush": "512 MiB written before each repetition", "statistic": f"median of {reps}"}
        result["build_cold"] = {
            "ms": t_build_cold, "melem_s": n / (t_build_cold * 1e-3) / 1e6,
            "frac": build_alg_bytes / (t_build_cold * 1e-3) / 1e9 / HBM_PEAK_GBS}
        result["sampling_sorted_u"] = {
            "ms": t_sorted, "samples_s": S / (t_sorted * 1e-3),
            "note": "the same uniforms in ascending order (coherent lanes)"}
        result["gather_ceiling"] = {
            "probe": "librtf_probe.so: stream u, read the 64-byte record floor(u m / 2^64) of the "
                     "same guide table, write idx and x; depth 2 adds one dependent 16-byte read "
                     "of the node array",
            "depth1_samples_s": S / (t_g1 * 1e-3), "depth2_samples_s": S / (t_g2 * 1e-3),
            "depth1_cold_samples_s": S / (t_g1_cold * 1e-3),
            "sample_vs_depth1": t_g1 / t_sample,
            "sample_cold_vs_depth1_cold": t_g1_cold / t_sample_cold,
        }
    result.update(out)

    if not args.no_cpu and not args.profile:
        result["cpu_baseline"] = cpu_baseline(v_h, u_h, n, m)
    print(json.dumps(result), flush=True)


def cpu_baseline(v_h, u_h, n, m):
    """The CPU oracle as it stands, timed on this host: quantise and prefix sum
    over all n weights (one thread, as the oracle is serial), then binary
    search with x on a bounded prefix of the uniforms, once on one thread and
    once split into disjoint slices over the usable cores (one thread per
    core, each calling the serial oracle; ctypes releases the GIL)."""
    import threading
    import oracle
    model, usable = host_cpu()
    threads = max(1, min(usable, 16))
    t0 = time.perf_counter()
    q, _ = oracle.quantize(v_h)
    C = oracle.prefix(q)
    t_setup = time.perf_counter() - t0
    S = u_h.size
    k1 = min(S, 1 << 22)
    t0 = time.perf_counter()
    oracle.search(q, u_h[:k1], C=C)
    t_one = time.perf_counter() - t0
    kN = min(S, k1 * threads)
    bounds = np.linspace(0, kN, threads + 1).astype(np.int64)
    work = [threading.Thread(target=oracle.search, args=(q, u_h[bounds[k]:bounds[k + 1]]),
                             kwargs={"C": C}) for k in range(threads)]
    t0 = time.perf_counter()
    for th in work:
        th.start()
    for th in work:
        th.join()
    t_all = time.perf_counter() - t0
    total_one = t_setup + t_one * (S / k1)
    total_all = t_setup + t_all * (S / kN)
    t0 = time.perf_counter()
    oracle.forest(q, m=m)
    t_forest = time.perf_counter() - t0
    return {
        "value": S / total_all,
        "unit": "samples/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"quantise + prefix over all n=2^{int(np.log2(n))} weights on one thread "
                  f"({t_setup:.2f} s), then binary search with x on the first {kN} of the "
                  f"2^{int(np.log2(S))} uniforms split over {threads} threads ({t_all:.2f} s), "
                  "scaled to the full step",
        "host_cpu": model,
        "usable_cores": usable,
        "single_thread_samples_s": S / total_one,
        "single_thread_sample": f"the same with the first {k1} uniforms on one thread "
                                f"({t_one:.2f} s)",
        "oracle_forest_melem_s": n / t_forest / 1e6,
    }


def event_time(fn, reps):
    """Mean milliseconds of fn() over reps runs, HIP events on the current stream."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def common(metric, unit, value, ms, args, dtype, workload, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": workload}}
    out.update(extra)
    return out


def run_table1(args):
    """The densities of the paper's load-count table (p ~ i^20,
    (i mod 32 + 1)^25, (i mod 64 + 1)^35) at n = 2^log2n with m = n (or
    --cell-ratio): loads per sample replayed on the host for Alg. 2 as
    printed, for this library's record lookup and for the Cutpoint Method
    with bisection (maximum, average, average over 32 and 64 synchronised
    lanes), and samples/s of the three on the GPU."""
    import torch
    import paper_1901_05423_amd as rtf
    from paper_1901_05423_amd import workloads as wl
    dev = torch.device("cuda:0")
    n = 1 << (args.log2n if args.log2n != 24 else 20)
    S = 1 << args.log2s
    ratio = args.cell_ratio if args.cell_ratio is not None else 1.0
    m = max(1, int(round(ratio * n)))
    r = wl.rng(wl.TABLE1)
    u_h = wl.uniforms(r, S)
    u = torch.from_numpy(u_h).to(dev)
    idx = torch.empty(S, dtype=torch.int32, device=dev)
    x = torch.empty(S, dtype=torch.float64, device=dev)
    sub = u_h[: 1 << 20]
    out = {}
    for fam in wl.TABLE1_FAMILIES:
        v = torch.from_numpy(wl.table1_weights(fam, n)).to(dev)
        q, _ = rtf.quantize(v)
        f = rtf.build(q, m)
        f.check()
        t_b = event_time(lambda: rtf.build(q, m, ws=f.ws), args.steps)
        t_s = event_time(lambda: rtf.sample(f, u, out=(idx, x)), args.steps)
        t_bs = event_time(lambda: rtf.sample_bsearch(f, u, out=(idx, x)), args.steps)
        t_cb = event_time(lambda: rtf.sample_cutpoint_bsearch(f, u, out=(idx, x)), args.steps)
        key, child, table, W, (K, aux) = f.export(with_cells=True)
        rtf.sample(f, u, out=(idx, x))
        ref_idx = idx.clone()
        # the same forest with collapsed 4-ary records for the descended cells
        t_w = event_time(lambda: f.widen(ws=getattr(f, "wide_ws", None)), args.steps)
        t_sw = event_time(lambda: rtf.sample(f, u, out=(idx, x)), args.steps)
        assert torch.equal(idx, ref_idx), "collapsed and binary descents differ"
        wide = f.wide_view().cpu().numpy()
        # the depth fallback (Sec. 3): degenerate cell trees rebuilt balanced
        rebuilt = f.balance()
        t_sb = event_time(lambda: rtf.sample(f, u, out=(idx, x)), args.steps)
        assert torch.equal(idx, ref_idx), "balanced and radix descents differ"
        keyb, childb, tableb, _, (Kb, auxb) = f.export(with_cells=True)
        out[fam] = {
            "loads_cutpoint_bisection": load_stats(loads_cutpoint(key, table, m, sub)),
            "loads_forest_alg2": load_stats(loads_forest_alg2(key, child, table, m, sub)),
            "loads_forest_records": load_stats(loads_forest_records(key, child, table, K, aux, m,
                                                                    sub)),
            "loads_forest_records_collapsed": load_stats(
                loads_forest_records(key, child, table, K, aux, m, sub, wide=wide)),
            "loads_forest_alg2_balanced": load_stats(loads_forest_alg2(keyb, childb, tableb, m,
                                                                       sub)),
            "loads_forest_records_balanced": load_stats(
                loads_forest_records(keyb, childb, tableb, Kb, auxb, m, sub)),
            "cells_rebuilt_by_fallback": rebuilt,
            "samples_s": {"forest": S / (t_s * 1e-3), "forest_collapsed": S / (t_sw * 1e-3),
                          "forest_balanced": S / (t_sb * 1e-3),
                          "cutpoint_bisection": S / (t_cb * 1e-3),
                          "binary_search": S / (t_bs * 1e-3)},
            "build_ms": t_b,
            "widen_ms": t_w,
        }
    res = common(METRIC, "samples/s", out[wl.TABLE1_FAMILIES[0]]["samples_s"]["forest"],
                 S / out[wl.TABLE1_FAMILIES[0]]["samples_s"]["forest"] * 1e3, args, "u64",
                 f"Table-1 densities p~i^20, (i mod 32+1)^25, (i mod 64+1)^35 at n=2^{int(np.log2(n))}, "
                 f"m={ratio:g}n, S=2^{args.log2s}; loads replayed on 2^20 of the uniforms",
                 families=out)
    print(json.dumps(res), flush=True)


def batch_choice(args, v, u, eo, so):
    """Guide cells per weight, descent form and build tile for a batched
    workload: --cell-ratio fixes the ratio (binary descent, --tile or 2048),
    else the autotuner times quantise + build (+ collapse) + sample over its
    candidates on this data."""
    if args.cell_ratio is not None:
        return args.cell_ratio, bool(args.collapsed), args.tile or 2048, {"source": "fixed"}
    from paper_1901_05423_amd import tune
    tiles = (args.tile,) if args.tile else tune.TILES
    r, c, tile, times = tune.best_batched(v, u, eo, so, use_cache=False, tiles=tiles)
    return r, c, tile, {"source": "tuner", "ms_by_ratio_collapsed_tile": times}


def run_c4(args):
    """10,000 uneven distributions: quantise + build + sample in one launch
    sequence, eagerly and as one replayed graph, against one library call
    sequence per distribution."""
    import torch
    import paper_1901_05423_amd as rtf
    from paper_1901_05423_amd import workloads as wl
    from paper_1901_05423_amd.plan import BatchedPlan
    r = wl.rng(wl.C4_BATCHED)
    v_h, eo_h, so_h = wl.batched_uneven(r)
    u_h = wl.uniforms(r, int(so_h[-1]))
    dev = torch.device("cuda:0")
    v, u = torch.from_numpy(v_h).to(dev), torch.from_numpy(u_h).to(dev)
    eo, so = torch.from_numpy(eo_h).to(dev), torch.from_numpy(so_h).to(dev)
    n, S, D = int(eo_h[-1]), int(so_h[-1]), eo_h.size - 1
    ratio, collapsed, tile, tuning = batch_choice(args, v, u, eo, so)
    co = rtf.cells_like(eo, ratio)
    mt = int(co[-1].item())
    plan = BatchedPlan(eo, co, so, n, mt, S, collapsed=collapsed, tile=tile)
    for _ in range(args.warmup):
        plan.run(v, u)
    plan.check()
    t_eager = event_time(lambda: plan.run(v, u), args.steps)
    g = plan.capture(v, u)
    t_graph = event_time(g.replay, args.steps)
    # per-distribution launches of the same library: one quantise, build and
    # sample call sequence per distribution, every buffer preallocated (one
    # workspace per distribution, slices of shared inputs and outputs), so
    # the loop times launches only
    import ctypes
    L = rtf.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n_d = np.diff(eo_h)
    m_d = np.maximum(1, np.round(ratio * n_d)).astype(np.int64)
    nb = np.array([L.rtf_workspace_bytes(int(a), int(b)) for a, b in zip(n_d, m_d)], np.int64)
    wo = np.concatenate([[0], np.cumsum(nb)])
    ws_all = torch.empty(int(wo[-1]), dtype=torch.uint8, device=dev)
    q_all = torch.empty(n, dtype=torch.uint32, device=dev)
    sc_all = torch.empty(D, dtype=torch.float64, device=dev)
    idx_all = torch.empty(S, dtype=torch.int32, device=dev)
    x_all = torch.empty(S, dtype=torch.float64, device=dev)
    descs = (rtf.rtf_forest * D)()
    P = ctypes.c_void_p
    calls = [(P(v.data_ptr() + 4 * int(eo_h[d])), int(n_d[d]), P(q_all.data_ptr() + 4 * int(eo_h[d])),
              P(sc_all.data_ptr() + 8 * d), int(m_d[d]), P(ws_all.data_ptr() + int(wo[d])),
              int(nb[d]), ctypes.byref(descs[d]), P(u.data_ptr() + 8 * int(so_h[d])),
              int(so_h[d + 1] - so_h[d]), P(idx_all.data_ptr() + 4 * int(so_h[d])),
              P(x_all.data_ptr() + 8 * int(so_h[d]))) for d in range(D)]
    quant, build1, samp = L.rtf_quantize_f32, L.rtf_build, L.rtf_sample

    def per_distribution():
        for (vp, nd, qp, sp, md, wp, wb, dp, up, sd, ip, xp) in calls:
            quant(vp, None, 1, nd, qp, sp, None, st)
            build1(qp, nd, md, wp, wb, st, dp)
            samp(dp, up, sd, ip, xp, st)

    per_distribution()
    torch.cuda.synchronize()
    assert torch.equal(idx_all, plan.idx), "per-distribution and batched indices differ"
    t0 = time.perf_counter()
    per_distribution()
    torch.cuda.synchronize()
    t_b3 = (time.perf_counter() - t0) * 1e3
    t_b3_gpu = event_time(per_distribution, 1)
    res = common(METRIC, "samples/s", S / (t_graph * 1e-3), t_graph, args, "u64",
                 f"C4: {D} distributions, sizes log-uniform in [16, 65536] (n_total={n}), "
                 f"uniform or Pareto(1.2) weights, m_d={ratio:g}n_d, {tile}-element build tiles "
                 f"({tuning['source']}), {'collapsed' if collapsed else 'binary'} descent, {S} "
                 "uniforms (64 per 1k weights), quantise + build + sample with x",
                 cell_ratio=ratio, collapsed=collapsed, tile=tile, tuning=tuning,
                 elements_per_s=n / (t_graph * 1e-3), ms_eager=t_eager, ms_graph=t_graph,
                 ms_per_distribution_launches=t_b3,
                 ms_per_distribution_launches_events=t_b3_gpu,
                 per_distribution_note="preallocated buffers, one quantise + build + sample "
                                       "call sequence per distribution on one stream",
                 speedup_vs_per_distribution=t_b3 / t_graph)
    print(json.dumps(res), flush=True)


def run_c3(args):
    """4096 x 4096 map: marginal + 4096 rows quantised and built as one batch,
    2^27 (row, column) pairs with sub-pixel positions.  The guide size and the
    descent form (binary nodes or collapsed 4-ary records) are tuned on this
    map: build (+ collapse) + 2D sampling timed per candidate."""
    import ctypes
    import torch
    import paper_1901_05423_amd as rtf
    from paper_1901_05423_amd import tune
    from paper_1901_05423_amd import workloads as wl
    r = wl.rng(wl.C3_MAP_2D)
    img, marg = wl.map_2d(r)
    R, C = img.shape
    v_h = np.concatenate([marg, img.ravel()])
    eo_h = np.concatenate([[0, R], R + C * np.arange(1, R + 1)]).astype(np.int64)
    pairs = 1 << 27
    u_h = wl.uniforms(r, 2 * pairs)
    dev = torch.device("cuda:0")
    v, u2 = torch.from_numpy(v_h).to(dev), torch.from_numpy(u_h).to(dev)
    eo = torch.from_numpy(eo_h).to(dev)
    n = int(eo_h[-1])
    q = torch.empty(n, dtype=torch.uint32, device=dev)
    scale = torch.empty(R + 1, dtype=torch.float64, device=dev)
    rc = torch.empty(2 * pairs, dtype=torch.int32, device=dev)
    xy = torch.empty(2 * pairs, dtype=torch.float64, device=dev)
    wide_ws = torch.empty(rtf.lib().rtf_wide_workspace_bytes(n), dtype=torch.uint8, device=dev)

    def setup(ratio, tile=2048):
        co = rtf.cells_like(eo, ratio)
        mt = int(co[-1].item())
        ws = torch.empty(rtf.lib().rtf_workspace_bytes_batched(R + 1, n, mt), dtype=torch.uint8,
                         device=dev)
        desc = rtf.rtf_forest()

        def build():
            rtf.quantize(v, eo, out=(q, scale))
            rtf._check(rtf.lib().rtf_build_batched_tiled(rtf._ptr(q), rtf._ptr(eo), rtf._ptr(co),
                                                         R + 1, n, mt, tile, rtf._ptr(ws),
                                                         ws.numel(), rtf._stream(),
                                                         ctypes.byref(desc)),
                       "rtf_build_batched_tiled")
        build()
        f = rtf.Forest(ws, desc, dev)
        return co, f, build

    def widen(f):
        f.widen(ws=wide_ws)

    def sample(f):
        rtf.sample_2d(f, u2, out=(rc, xy))

    if args.cell_ratio is not None:
        candidates, source = [(args.cell_ratio, bool(args.collapsed))], "fixed"
    else:
        candidates, source = [(0.125, False), (0.25, False), (0.5, False), (0.25, True),
                              (0.5, True), (1.0, True)], "tuner"
    times = {}

    def try_(ratio, coll, tile):
        _, f, build = setup(ratio, tile)

        def chain():
            build()
            if coll:
                widen(f)
            sample(f)
        times[f"{ratio}|{int(coll)}|{tile}"] = tune._time_ms(chain, 3)
        del f

    tiles = (args.tile,) if args.tile else tune.TILES
    for ratio, coll in candidates:
        try_(ratio, coll, tiles[0])
    best = min(times, key=times.get)
    for tile in tiles[1:]:  # the tile for the best ratio and descent form
        try_(float(best.split("|")[0]), bool(int(best.split("|")[1])), tile)
    best = min(times, key=times.get)
    ratio, collapsed, tile = float(best.split("|")[0]), bool(int(best.split("|")[1])), int(best.split("|")[2])
    co, f, build = setup(ratio, tile)
    torch.cuda.synchronize()
    f.check()
    t_build = event_time(build, args.steps)
    t_sample = event_time(lambda: sample(f), args.steps)
    rc_bin = rc.clone()
    # the same forest with collapsed 4-ary records for the descended row cells
    t_widen = event_time(lambda: widen(f), args.steps)
    t_sample_w = event_time(lambda: sample(f), args.steps)
    assert torch.equal(rc, rc_bin), "collapsed and binary descents differ"
    key, child, table, W, (K, aux) = f.export(with_cells=True)
    wide = f.wide_view().cpu().numpy()
    # row lookups replayed on the host for 2^20 pairs (rows from the GPU run)
    co_h = co.cpu().numpy()
    rows_h = rc_bin.view(-1, 2)[: 1 << 20, 0].cpu().numpy()
    uc = u_h[1::2][: 1 << 20]
    loads = {"binary": [], "collapsed": []}
    for r_ in np.unique(rows_h):
        sel = rows_h == r_
        d = 1 + int(r_)
        lo_e, hi_e = int(eo_h[d]), int(eo_h[d + 1])
        lo_c, m_d = int(co_h[d]), int(co_h[d + 1] - co_h[d])
        loc = lambda a: np.where(a >= 0, a - lo_e, ~(~a - lo_e))  # noqa: E731
        kd = key[lo_e:hi_e]
        cd = loc(child[lo_e:hi_e].astype(np.int64))
        td = loc(table[lo_c:lo_c + m_d].astype(np.int64))
        ad = aux[lo_c:lo_c + m_d].astype(np.int64)
        ad = np.where(ad >= 0, ad - lo_e, ad)
        wd = wide[lo_e:hi_e].copy()
        for col in (3, 4):
            pr = wd[:, col].copy().view(np.int32).astype(np.int64)
            wd[:, col] = loc(pr).astype(np.int32).view(np.int64)
        for mode, wv in (("binary", None), ("collapsed", wd)):
            loads[mode].append(loads_forest_records(kd, cd, td, K[lo_c:lo_c + m_d], ad, m_d,
                                                    uc[sel], wide=wv))
    row_loads = {k: load_stats(np.concatenate(v_)) for k, v_ in loads.items()}
    ms = t_build + (t_widen + t_sample_w if collapsed else t_sample)
    res = common(METRIC, "pairs/s", pairs / (ms * 1e-3), ms, args, "u64",
                 "C3: 4096x4096 log-normal(0,1.5) map + 8 hot spots (1e4, sigma 3 px); marginal + "
                 f"4096 rows quantised and built as one batch (m_d={ratio:g}n_d, {tile}-element "
                 f"tiles, {source}); "
                 f"{'collapsed' if collapsed else 'binary'} descent; 2^27 (row, col) pairs + "
                 "sub-pixel positions",
                 cell_ratio=ratio, collapsed=collapsed, tile=tile,
                 tuning={"source": source, "ms_build_plus_sample": times},
                 ms_build=t_build, ms_sample=t_sample, ms_widen=t_widen,
                 ms_sample_collapsed=t_sample_w,
                 build_melem_s=n / (t_build * 1e-3) / 1e6,
                 sample_only_pairs_s=pairs / (t_sample * 1e-3),
                 sample_only_pairs_s_collapsed=pairs / (t_sample_w * 1e-3),
                 row_lookup_loads=row_loads)
    print(json.dumps(res), flush=True)


def run_quality(args):
    """The quality study of Figs. 2d_zoom and convergence on the C3 map: the
    2D Hammersley set of N = 2^14 .. 2^26 points mapped to pixels by the
    inverse (marginal then row, through the forest) and by the Alias Method
    (marginal and row alias tables); e = sum over pixels (p - c / N)^2 with p
    the exact probability of the quantised map and c the pixel's count.  Also
    the sampling rate of both mappings at N = 2^26."""
    import torch
    import paper_1901_05423_amd as rtf
    from paper_1901_05423_amd import workloads as wl
    r = wl.rng(wl.C3_MAP_2D)
    img, marg = wl.map_2d(r)
    R, C = img.shape
    dev = torch.device("cuda:0")
    v = torch.from_numpy(np.concatenate([marg, img.ravel()])).to(dev)
    eo = torch.from_numpy(np.concatenate([[0, R], R + C * np.arange(1, R + 1)]).astype(np.int64)).to(dev)
    q, _ = rtf.quantize(v, eo)
    f = rtf.build_batched(q, eo, rtf.cells_like(eo, 0.25))
    t = rtf.alias_build(q, eo)
    f.check()
    t.export()  # raises on a recorded error
    qm = q[:R].to(torch.float64)
    rows = q[R:].to(torch.float64).view(R, C)
    p = ((qm / qm.sum())[:, None] * rows / rows.sum(dim=1, keepdim=True)).reshape(-1)
    curves = {"inverse": {}, "alias": {}}
    rates = {}
    for k in range(14, 27):
        N = 1 << k
        u2 = torch.from_numpy(wl.hammersley_u64(N)).to(dev)
        for name in ("inverse", "alias"):
            if name == "inverse":
                rc, _ = rtf.sample_2d(f, u2, want_xy=False)
            else:
                rc = rtf.alias_sample_2d(t, u2)
            rc = rc.view(-1, 2).to(torch.int64)
            cnt = torch.bincount(rc[:, 0] * C + rc[:, 1], minlength=R * C).to(torch.float64)
            curves[name][N] = float(((p - cnt / N) ** 2).sum().item())
            if k == 26:
                if name == "inverse":
                    ms = event_time(lambda: rtf.sample_2d(f, u2, want_xy=False), args.steps)
                else:
                    ms = event_time(lambda: rtf.alias_sample_2d(t, u2), args.steps)
                rates[name] = N / (ms * 1e-3)
        del u2
    inv, al = curves["inverse"], curves["alias"]
    Nmax = 1 << 26
    # the samples the inverse mapping needs to reach the alias mapping's error
    # at 2^26 (log-log interpolation between measured points), as Fig.
    # convergence reads its "3x as many samples"
    target = al[Nmax]
    Ns = sorted(inv)
    need = None
    for a_, b_ in zip(Ns, Ns[1:]):
        if inv[a_] >= target >= inv[b_]:
            fr = (np.log(inv[a_]) - np.log(target)) / (np.log(inv[a_]) - np.log(inv[b_]))
            need = float(np.exp(np.log(a_) + fr * (np.log(b_) - np.log(a_))))
    res = common("quadratic error e of Hammersley points mapped by the inverse vs the Alias "
                 "Method", "e ratio alias/inverse at N=2^26", al[Nmax] / inv[Nmax], 0.0, args,
                 "u64", "C3 map (4096x4096, marginal + rows, quantised): 2D Hammersley sets of "
                 "N = 2^14..2^26 points through the forest (inverse) and through alias tables",
                 curve_inverse={str(k_): v_ for k_, v_ in inv.items()},
                 curve_alias={str(k_): v_ for k_, v_ in al.items()},
                 inverse_samples_for_alias_error_at_2e26=need,
                 samples_ratio=(Nmax / need) if need else None,
                 pairs_s_at_2e26=rates)
    res["higher_is_better"] = False
    print(json.dumps(res), flush=True)


def run_c5(args):
    """256 distributions of 4096 softplus weights, 2^20 uniforms each: forward
    (quantise + build + sample) and the adjoint of L = sum sin(7x)."""
    import torch
    import paper_1901_05423_amd as rtf
    from paper_1901_05423_amd import workloads as wl
    D, nd, per = 256, 4096, 1 << 20
    r = wl.rng(wl.C5_DIFF)
    z_h = wl.logits(r, D, nd)
    u_h = wl.uniforms(r, D * per)
    dev = torch.device("cuda:0")
    z = torch.from_numpy(z_h).to(dev)
    u = torch.from_numpy(u_h).to(dev)
    eo = torch.arange(D + 1, dtype=torch.int64, device=dev) * nd
    so = torch.arange(D + 1, dtype=torch.int64, device=dev) * per
    v = torch.nn.functional.softplus(z).reshape(-1).contiguous()
    from paper_1901_05423_amd.plan import BatchedPlan
    ratio, collapsed, tile, tuning = batch_choice(args, v, u, eo, so)
    md = max(1, int(round(nd * ratio)))
    co = torch.arange(D + 1, dtype=torch.int64, device=dev) * md
    plan = BatchedPlan(eo, co, so, D * nd, D * md, D * per, collapsed=collapsed, tile=tile)
    plan.run(v, u)
    plan.check()
    f = plan
    gx = 7.0 * torch.cos(7.0 * plan.x)
    bws = torch.empty(rtf.lib().rtf_backward_workspace_bytes(D, D * nd), dtype=torch.uint8,
                      device=dev)
    forest = rtf.Forest(plan.ws, plan.desc, dev)

    def bwd():
        return rtf.backward(forest, u, plan.idx, gx, plan.scale, sample_off=so, ws=bws)

    t_fwd = event_time(lambda: plan.run(v, u), args.steps)
    t_bwd = event_time(bwd, args.steps)
    S = D * per
    res = common(METRIC, "samples/s", S / ((t_fwd + t_bwd) * 1e-3), t_fwd + t_bwd, args, "u64",
                 f"C5: 256 distributions x 4096 softplus(N(0,1)) weights, m_d={md} "
                 f"({tuning['source']}), {'collapsed' if collapsed else 'binary'} descent, 2^20 "
                 "uniforms each; forward quantise + build + sample with x, backward dL/dw of "
                 "L = sum sin(7x)",
                 cell_ratio=ratio, collapsed=collapsed, tile=tile, tuning=tuning,
                 ms_forward=t_fwd, ms_backward=t_bwd,
                 forward_samples_s=S / (t_fwd * 1e-3), backward_samples_s=S / (t_bwd * 1e-3))
    print(json.dumps(res), flush=True)


def run_grad1(args):
    """The adjoint of one large distribution: 2^22 uniform(0,1] weights,
    2^24 uniforms, L = sum sin(7x); forward (quantise + build + sample) and
    rtf_backward, whose combining pass spreads the distribution over all
    CUs."""
    import torch
    import paper_1901_05423_amd as rtf
    from paper_1901_05423_amd import workloads as wl
    n, S = 1 << 22, 1 << 24
    r = wl.rng(wl.H24_UNIFORM)
    dev = torch.device("cuda:0")
    v = torch.from_numpy(wl.weights_uniform(r, n)).to(dev)
    u = torch.from_numpy(wl.uniforms(r, S)).to(dev)
    q, scale = rtf.quantize(v)
    f = rtf.build(q, n // 4)
    idx, x = rtf.sample(f, u)
    gx = 7.0 * torch.cos(7.0 * x)
    bws = torch.empty(rtf.lib().rtf_backward_workspace_bytes(1, n), dtype=torch.uint8,
                      device=dev)
    t_bwd = event_time(lambda: rtf.backward(f, u, idx, gx, scale, ws=bws), args.steps)
    res = common(METRIC, "samples/s", S / (t_bwd * 1e-3), t_bwd, args, "u64",
                 "one distribution of 2^22 uniform(0,1] weights, m = n/4, 2^24 uniforms: "
                 "rtf_backward of L = sum sin(7x)",
                 ms_backward=t_bwd, backward_weights_s=n / (t_bwd * 1e-3))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
