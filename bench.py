"""Benchmark: a batch of 4096 exact circular convolutions of N = 2^16 modulo
m = 13631489 (root 2^8 = 256 of exact order 2^16), one GPU.

A step is one conv_batched call over the whole batch (forward transforms of f
and g, pointwise product, inverse, N^-1, canonical store): a single fused
persistent kernel launch.  Operands are seeded synthetic uint32 words uniform
in [0, m), resident in HBM before timing.

Prints one JSON line (see the README for the fields); diagnostic lines go to
stderr.
"""
import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact convolutions/s and HBM GB/s (% roofline), batched N=2^16; p50/p99 latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# fp64 vector lanes: 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 FMA-or-add per second
# (the published 78.6 TFLOP/s fp64 vector counts an FMA as two flops)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
N_LOG2 = 16
COUNT = 4096


def alg_ops_per_conv(n_log2: int) -> int:
    """fp64 lane operations of the exact arithmetic per convolution: three
    transforms of (N/2) log2 N butterflies at 5 ops (3-FMA modular product + two
    adds), plus N pointwise products at 7 ops (N^-1 folded in)."""
    N = 1 << n_log2
    return 5 * 3 * (N // 2) * n_log2 + 7 * N


def kernel_source_sha() -> str:
    """Hash of the device sources; a stored traffic measurement is used only
    while the kernels are unchanged since the counters were taken."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1005_1497_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (each scaled by its reading for a plain
    1 GiB copy), or None when the kernels changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_k_conv_fused_w32_n65536_b4096.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t["hbm_bytes_per_launch"]


def write_traffic(prof_dir):
    """Reduces the four rocprofv3 counter runs under prof_dir (FETCH_SIZE and
    WRITE_SIZE of the headline bench, and of --calibrate-copy: directories
    FETCH_SIZE, WRITE_SIZE, copy_FETCH_SIZE, copy_WRITE_SIZE) to HBM bytes per
    launch of the fused kernel, each counter scaled by its reading for the
    1 GiB copy, and writes the summary that measured_traffic() reads."""
    import collections
    import csv
    import glob

    def per_dispatch(sub, counter, kernel):
        files = glob.glob(os.path.join(prof_dir, sub, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit("no counter_collection.csv under %s" % os.path.join(prof_dir, sub))
        vals = collections.defaultdict(float)
        with open(files[0]) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and kernel in r["Kernel_Name"]:
                    vals[r.get("Dispatch_Id") or r.get("Correlation_Id")] += float(r["Counter_Value"])
        if not vals:
            raise SystemExit("no %s dispatches of %s in %s" % (counter, kernel, sub))
        return sum(vals.values()) / len(vals)

    fe = per_dispatch("FETCH_SIZE", "FETCH_SIZE", "k_conv_fused")
    wr = per_dispatch("WRITE_SIZE", "WRITE_SIZE", "k_conv_fused")
    cf = per_dispatch("copy_FETCH_SIZE", "FETCH_SIZE", "copy")
    cw = per_dispatch("copy_WRITE_SIZE", "WRITE_SIZE", "copy")
    copy_bytes = 1 << 30
    ff, wf = copy_bytes / 1024 / cf, copy_bytes / 1024 / cw
    out = {"kernel": "k_conv_fused<W32,16>", "workload": "batch4096_n65536_m13631489",
           "source_sha": kernel_source_sha(),
           "fetch_kb_per_launch": round(fe, 1), "write_kb_per_launch": round(wr, 1),
           "copy_calibration": {"bytes": copy_bytes, "fetch_kb": round(cf, 1), "write_kb": round(cw, 1),
                                "fetch_factor": ff, "write_factor": wf},
           "hbm_bytes_per_launch": fe * 1024 * ff + wr * 1024 * wf}
    path = os.path.join(ROOT, "profiles", "traffic_k_conv_fused_w32_n65536_b4096.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def copy_bandwidth(nbytes=1 << 31, reps=10):
    """Device-to-device copy bandwidth measured in the same run (torch's copy
    kernel over nbytes, read + write counted): GB/s."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for _ in range(3):
        b.copy_(a)
    per = _time_ms(lambda: b.copy_(a), reps, st)
    del a, b
    return 2 * nbytes / (float(np.median(per)) / 1e3) / 1e9


def valu_peaks():
    """Sustained vector-ALU rates on the device (libnttbench.so), in lane
    operations per second (an FMA or multiply-add counts one): fp64 FMA, fp64
    add, int32 add, 24-bit integer multiply-add."""
    import ctypes
    path = os.path.join(ROOT, "paper_1005_1497_amd", "libnttbench.so")
    L = ctypes.CDLL(path)
    L.ntt_bench_valu.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_float),
                                 ctypes.POINTER(ctypes.c_double)]
    L.ntt_bench_valu.restype = ctypes.c_int
    out = {}
    for kind, name in enumerate(("fp64_fma", "fp64_add", "int32_add", "int32_mad_u24")):
        ms, ops = ctypes.c_float(0), ctypes.c_double(0)
        # 256 CUs x 8 workgroups of 256 threads, 256 x 16 x 8 operations per thread
        rc = L.ntt_bench_valu(kind, 256 * 8, 256, ctypes.byref(ms), ctypes.byref(ops))
        if rc:
            raise RuntimeError("ntt_bench_valu(%d) failed: %d" % (kind, rc))
        out[name] = ops.value / (ms.value / 1e3)
    return out


def cpu_baseline(f, g, m, N, gpu_out=None, budget_s=12.0):
    """The oracle (direct O(N^2) sum of Eq. 1, plain C, all host threads) on a
    bounded sample of items of the same workload.  Returns the baseline and,
    when the GPU's output of the batch is given, whether it equals the
    oracle's on every item of the sample (None otherwise)."""
    import oracle
    threads = oracle.threads()
    t0 = time.perf_counter()
    done, refs = 0, []
    while True:
        o = done * N
        refs.append(oracle.conv_direct(f[o:o + N], g[o:o + N], m))
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s or done >= 64 or el / done * (done + 1) > 2.5 * budget_s:
            break
    same = None
    if gpu_out is not None:
        same = all(np.array_equal(gpu_out[i * N:(i + 1) * N], r.astype(gpu_out.dtype)) for i, r in enumerate(refs))
    base = {"value": done / el, "unit": "conv/s", "cores": threads, "kind": "oracle",
            "sample": "%d of the %d items (N=%d), direct O(N^2) sum, %.1f s" % (done, COUNT, N, el)}
    # the same oracle on one core: a slice of one item's outputs (each the
    # O(N) direct sum), scaled to whole convolutions
    oracle.set_threads(1)
    try:
        k = N // 32
        idx = np.arange(k, dtype=np.uint64) * 32
        t1 = time.perf_counter()
        part = oracle.conv_entries(f[:N], g[:N], m, idx)
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    if gpu_out is not None:
        same = bool(same) and bool(np.array_equal(gpu_out[idx.astype(int)], part.astype(gpu_out.dtype)))
    base["single_thread"] = {"value": (k / N) / el1, "unit": "conv/s", "cores": 1,
                             "sample": "%d of the %d outputs of item 0, direct O(N) sums, %.1f s" % (k, N, el1)}
    return base, same


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the GPU clock ramps over the first launches: 3 warm-up steps left the
    # 2^16 batch at 1.98 ms per launch, 50 bring it to its steady 1.88 ms
    ap.add_argument("--warmup", type=int, default=50, help="untimed steps before the timed ones")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the per-item comparison form")
    ap.add_argument("--workload", choices=["batch", "serve", "uneven", "single", "deconv", "euler", "crt", "conv2d", "u64",
                                           "lengths", "peak", "serve-sweep"], default="batch",
                    help="batch: 4096 x N=2^16 (default); serve: Poisson-arrival serving, 64-bit words; "
                         "uneven: 10000 items, n uniform in [6,19]; single: one N=1024 and one N=2^19 convolution")
    ap.add_argument("--requests", type=int, default=4000, help="serve: timed requests")
    ap.add_argument("--lengths", default="8,10,11,12,13,14,15,16,17,18,19",
                    help="lengths: the log2 N of the uniform 2^26-element batches")
    ap.add_argument("--rho", type=float, default=0.7, help="serve: offered load / saturated throughput")
    ap.add_argument("--rhos", default="0.3,0.5,0.7,0.9", help="serve-sweep: the offered loads")
    ap.add_argument("--streams", type=int, default=8, help="serve-sweep: streams of the native scheduler")
    ap.add_argument("--inflight", type=int, default=8, help="serve-sweep: batches in flight (native scheduler)")
    ap.add_argument("--arenas", choices=("host", "device"), default="host",
                    help="serve, serve-sweep: the native scheduler's arenas: pinned host memory that the kernels read "
                         "and write directly (ntt_server_create_host), or device memory with copies each way "
                         "(ntt_server_create)")
    ap.add_argument("--clients", type=int, default=4,
                    help="serve-sweep: client thread pairs submitting to the native scheduler")
    ap.add_argument("--solo", type=int, default=16,
                    help="serve-sweep: requests of 2^SOLO words and more run as batches of their own (0: never)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB device buffer 4 times (reference kernel for the HBM byte counters)")
    ap.add_argument("--traffic-from", metavar="DIR",
                    help="only reduce the rocprofv3 FETCH_SIZE / WRITE_SIZE runs under DIR to the HBM-bytes summary "
                         "in profiles/ (no GPU)")
    args = ap.parse_args()
    if args.traffic_from:
        return write_traffic(args.traffic_from)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(a batch would shard by items, one process per GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        import torch
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 1 << 30, "copies": 4}))
        return
    if args.workload == "serve":
        return serve_bench(args)
    if args.workload == "serve-sweep":
        return serve_sweep(args)
    if args.workload == "uneven":
        return uneven_bench(args)
    if args.workload == "lengths":
        return lengths_bench(args)
    if args.workload == "single":
        return single_bench(args)
    if args.workload in ("deconv", "euler", "crt", "conv2d", "u64"):
        return variant_bench(args)
    if args.workload == "peak":
        import torch
        torch.cuda.init()
        print(json.dumps({"metric": "device peaks measured on this GPU", "copy_gbs": copy_bandwidth(),
                          "valu_lane_ops_per_s": valu_peaks(),
                          "nominal": {"hbm_gbs": HBM_PEAK_GBS, "valu_lane_ops_per_s": ALU_PEAK_TOPS * 1e12}}),
              flush=True)
        return

    import torch
    import paper_1005_1497_amd as nt
    import seeded_inputs as si

    w = si.batch_n65536(COUNT)
    m, N = w.m, 1 << N_LOG2
    t0 = time.perf_counter()
    f_h, g_h = si.operands(w)
    log("inputs drawn in %.1f s" % (time.perf_counter() - t0))
    dev = torch.device("cuda", 0)
    f = torch.from_numpy(f_h.view(np.int32)).to(dev)
    g = torch.from_numpy(g_h.view(np.int32)).to(dev)
    h = torch.empty_like(f)
    desc = nt.BatchDesc([N_LOG2] * COUNT, si.offsets([N_LOG2] * COUNT))
    stream = torch.cuda.current_stream()

    def step(flags=0):
        nt.conv_batched(f, g, desc, m, out=h, flags=flags, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done (%d steps)" % args.warmup)

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) for a, b in evs])   # ms, one fused launch each
    log("timed %d steps: wall %.3f s, launch mean %.3f ms" % (args.steps, wall, per.mean()))

    hh = h.cpu().numpy().view(np.uint32)

    forms = {}
    if not args.no_forms:
        # the plain one-launch-sequence-per-convolution form on the same GPU
        step(nt.FLAG_PER_ITEM)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        step(nt.FLAG_PER_ITEM)
        torch.cuda.synchronize()
        forms["per_item_ms_per_step"] = (time.perf_counter() - t1) * 1e3
        forms["per_item_conv_per_s"] = COUNT / (forms["per_item_ms_per_step"] / 1e3)
        # the same fused launch captured once in a HIP graph and replayed
        gs = torch.cuda.Stream()
        nt.conv_batched(f, g, desc, m, out=h, stream=gs)     # plans and workspaces of the capture stream
        gs.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gs):
            nt.conv_batched(f, g, desc, m, out=h, stream=gs)
        torch.cuda.synchronize()
        greps = max(args.steps, 5)
        gevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(greps)]
        eevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(greps)]
        with torch.cuda.stream(gs):                          # replay() launches on the current stream
            # warm-up replays (the first replay uploads the graph) and eager
            # launches on the same stream, so that both are timed after the
            # per-item form's small launches at the same clock
            for _ in range(max(args.warmup // 5, 5)):
                graph.replay()
                nt.conv_batched(f, g, desc, m, out=h, stream=gs)
            for (a, b), (c, d) in zip(gevs, eevs):
                a.record(gs)
                graph.replay()
                b.record(gs)
                c.record(gs)
                nt.conv_batched(f, g, desc, m, out=h, stream=gs)
                d.record(gs)
        torch.cuda.synchronize()
        gper = np.array([a.elapsed_time(b) for a, b in gevs])
        eper = np.array([a.elapsed_time(b) for a, b in eevs])
        forms["graph_replay_ms_per_step"] = float(gper.mean())
        forms["graph_replay_conv_per_s"] = COUNT / (gper.mean() / 1e3)
        forms["eager_interleaved_ms_per_step"] = float(eper.mean())
        with torch.cuda.stream(gs):                          # the replay alone writes h
            h.zero_()
            graph.replay()
        torch.cuda.synchronize()
        gok = bool(np.array_equal(h.cpu().numpy().view(np.uint32), hh))
        forms["graph_replay_matches_eager"] = gok
        if not gok:
            log("graph replay output differs from the eager output")
        del graph

    # the same GPU's copy bandwidth and vector-ALU rates, measured after the
    # timed region
    copy_gbs = copy_bandwidth()
    peaks = valu_peaks()
    log("copy %.0f GB/s; fp64 FMA %.1f T lane-ops/s" % (copy_gbs, peaks["fp64_fma"] / 1e12))

    value = COUNT * args.steps / wall
    ms = wall / args.steps * 1e3
    alg_bytes = 12 * N * COUNT                     # read f, read g, write h (4-byte words)
    launch_s = per.mean() / 1e3
    alg_ops = alg_ops_per_conv(N_LOG2) * COUNT
    achieved_tops = alg_ops / launch_s / 1e12
    hbm_gbs = alg_bytes / launch_s / 1e9
    traffic = measured_traffic()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "conv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "count": COUNT, "n": N, "m": m, "root": 256,
                   "words": "u32", "parallelism": "batch (one workgroup per convolution)"},
        "elements_per_s": value * N,
        "hbm_gbs_algorithmic": hbm_gbs,
        "hbm_frac_of_8tbs": hbm_gbs / HBM_PEAK_GBS,
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
        "roofline": {"bound": "alu", "achieved": achieved_tops, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
                     "frac": achieved_tops / ALU_PEAK_TOPS, "traffic": traffic,
                     "kernel": "k_conv_fused<16>", "alg_ops_per_launch": alg_ops,
                     "launch_ms": per.mean()},
        "hbm_roofline": {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": hbm_gbs / HBM_PEAK_GBS, "alg_bytes_per_launch": alg_bytes},
        # bytes the kernel actually moves (counter-measured for these device
        # sources, scratch round trips included) over the same launch time
        "hbm_measured": (None if traffic is None else
                         {"bytes_per_launch": traffic, "gbs": traffic / launch_s / 1e9,
                          "frac_of_8tbs": traffic / launch_s / 1e9 / HBM_PEAK_GBS}),
        "measured_peaks": {"copy_gbs": copy_gbs, "hbm_frac_of_copy": hbm_gbs / copy_gbs,
                           "valu_lane_ops_per_s": peaks,
                           "alu_frac_of_measured_fp64_fma": achieved_tops * 1e12 / peaks["fp64_fma"]},
        "forms": forms,
        "parity_sampled": None,
    }
    if not args.no_cpu:
        # the baseline leg: the oracle on the first items, which the timed
        # output must equal element for element
        out["cpu_baseline"], ok = cpu_baseline(f_h, g_h, m, N, gpu_out=hh)
        out["parity_sampled"] = ok
        if not ok:
            log("PARITY FAILURE in the timed output")
    print(json.dumps(out), flush=True)


def _time_ms(fn, reps, stream):
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in evs])


def uneven_bench(args):
    """10000 convolutions of lengths 2^n, n uniform in [6, 19], m = 13631489,
    packed back to back: one conv_batched call as a single persistent launch,
    against one launch per length class and one launch sequence per item."""
    import torch
    import paper_1005_1497_amd as nt
    import seeded_inputs as si
    w = si.uneven_batch(10000)
    f_h, g_h = si.operands(w)
    dev = torch.device("cuda", 0)
    f = torch.from_numpy(f_h.view(np.int32)).to(dev)
    g = torch.from_numpy(g_h.view(np.int32)).to(dev)
    h = torch.empty_like(f)
    desc = nt.BatchDesc(w.log2n, si.offsets(w.log2n))
    st = torch.cuda.current_stream()
    run = lambda flags=0: nt.conv_batched(f, g, desc, w.m, out=h, flags=flags, stream=st)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    per = _time_ms(run, args.steps, st)
    ref = h.cpu()
    run(nt.FLAG_PER_CLASS)
    torch.cuda.synchronize()
    per_class = _time_ms(lambda: run(nt.FLAG_PER_CLASS), args.steps, st)
    same_class = bool(torch.equal(h.cpu(), ref))
    run(nt.FLAG_PER_ITEM)
    torch.cuda.synchronize()
    per_item = _time_ms(lambda: run(nt.FLAG_PER_ITEM), 2, st)
    same_item = bool(torch.equal(h.cpu(), ref))
    run(nt.FLAG_AUTOTUNE)                 # tunes this batch shape once, then cached
    torch.cuda.synchronize()
    tuned = _time_ms(run, args.steps, st)
    same_tuned = bool(torch.equal(h.cpu(), ref))
    total = w.total_elems
    out = {"metric": "exact convolutions/s, uneven batch", "value": 10000 / (per.mean() / 1e3), "unit": "conv/s",
           "ms_per_step": float(per.mean()), "elements_per_s": total / (per.mean() / 1e3),
           "hbm_gbs_algorithmic": 12 * total / (per.mean() / 1e3) / 1e9,
           "config": {"workload": w.name, "total_elements": total},
           "forms": {"single_launch_ms": float(per.mean()),
                     "per_class_ms": float(per_class.mean()), "per_class_matches": same_class,
                     "autotuned_ms": float(tuned.mean()), "autotuned_matches": same_tuned,
                     "per_item_ms": float(per_item.mean()), "per_item_matches": same_item,
                     "per_item_conv_per_s": 10000 / (per_item.mean() / 1e3)}}
    print(json.dumps(out), flush=True)


def lengths_bench(args):
    """Per-length throughput of the default batch form: for each n, a batch of
    2^26 elements (2^(26-n) convolutions of length 2^n, m = 13631489, items
    back to back), one conv_batched call per step, in element-stages
    (elements x log2 N) per second."""
    import torch
    import paper_1005_1497_amd as nt
    import seeded_inputs as si
    m = si.M_13631489
    st = torch.cuda.current_stream()
    res = {}
    for n in [int(x) for x in args.lengths.split(",")]:
        count = (1 << 26) >> n
        tot = count << n
        f = torch.from_numpy(si.uniform(100 + n, tot, m).view(np.int32)).cuda()
        g = torch.from_numpy(si.uniform(200 + n, tot, m).view(np.int32)).cuda()
        h = torch.empty_like(f)
        desc = nt.BatchDesc([n] * count, si.offsets([n] * count))
        run = lambda: nt.conv_batched(f, g, desc, m, out=h, stream=st)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        per = _time_ms(run, args.steps, st)
        ms = float(per.mean())
        res["n%d" % n] = {"items": count, "ms_per_batch": ms, "element_stages_per_s": tot * n / (ms / 1e3),
                          "conv_per_s": count / (ms / 1e3)}
        log("n=%d: %d items, %.3f ms" % (n, count, ms))
        del f, g, h
    print(json.dumps({"metric": "per-length batch throughput, 2^26 elements per batch", "unit": "element-stages/s",
                      "config": {"workload": "lengths_2^26_elements_m13631489", "m": m}, "results": res}), flush=True)


def single_bench(args):
    """Latency of one convolution: N = 1024 (root 2^512) and N = 2^19 (root 2,
    operands in {0..3}), p50/p99 over repeated launches."""
    import torch
    import paper_1005_1497_amd as nt
    import seeded_inputs as si
    st = torch.cuda.current_stream()
    res = {}
    for w in (si.single_n1024(), si.single_n524288_small()):
        f_h, g_h = si.operands(w)
        f = torch.from_numpy(f_h.view(np.int32)).cuda()
        g = torch.from_numpy(g_h.view(np.int32)).cuda()
        h = torch.empty_like(f)
        n = w.log2n[0]
        run = lambda: nt.conv_circular(f, g, w.m, out=h, stream=st)
        for _ in range(20):
            run()
        torch.cuda.synchronize()
        per = _time_ms(run, 1000 if n <= 12 else 200, st)
        res[w.name] = {"p50_us": float(np.percentile(per, 50) * 1e3), "p99_us": float(np.percentile(per, 99) * 1e3),
                       "conv_per_s": 1e3 / float(per.mean())}
    print(json.dumps({"metric": "single convolution latency", "results": res}), flush=True)


def variant_bench(args):
    """The adjacent transforms on the headline shape, 4096 x N = 2^16:
    deconv  exact deconvolution g = inverse(forward(h) / forward(f)),
            m = 13631489 (rows in 1 GiB scratch chunks, four-step launches,
            Fermat inverses), against conv_circular-style convolution of the
            same rows through the same launches (flag FLAG_PER_CLASS form);
    euler   the batch convolution with the Euler-form prime 7340033 = 7*2^20+1
            and a root of order 2^16 that is not a power of two;
    u64     the batch convolution with 64-bit words and the 45-bit Rader prime
            31065037602817 (root 2^(2^18 / N))."""
    import torch
    import paper_1005_1497_amd as nt
    import seeded_inputs as si
    count, n = 4096, 16
    N = 1 << n
    st = torch.cuda.current_stream()
    if args.workload == "deconv":
        m = si.M_13631489
        rng = np.random.default_rng(7)
        f = torch.from_numpy(rng.integers(0, m, (count, N), dtype=np.uint32).view(np.int32)).cuda()
        h = torch.from_numpy(rng.integers(0, m, (count, N), dtype=np.uint32).view(np.int32)).cuda()
        g = torch.empty_like(f)

        def run():
            try:
                nt.deconvolve(f, h, m, out=g, stream=st)
            except nt.NttError as e:          # a singular draw still times the full path
                if e.name != "NTT_E_SINGULAR":
                    raise
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        out = {"metric": "exact deconvolutions/s, 4096 x N=2^16", "value": count / (ms / 1e3), "unit": "deconv/s",
               "ms_per_step": ms, "config": {"workload": "deconv4096_n65536_m13631489", "count": count, "n": N},
               "note": "includes the singular-coefficient readback and stream synchronisation of every call"}
    elif args.workload == "conv2d":
        m, R, C = si.M_13631489, 4096, 4096
        rng = np.random.default_rng(10)
        f = torch.from_numpy(rng.integers(0, m, (R, C), dtype=np.uint32).view(np.int32)).cuda()
        g = torch.from_numpy(rng.integers(0, m, (R, C), dtype=np.uint32).view(np.int32)).cuda()
        h = torch.empty_like(f)
        run = lambda: nt.conv2d(f, g, m, out=h, stream=st)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        per = _time_ms(run, args.steps, st)
        ms = float(per.mean())
        out = {"metric": "2-D circular convolutions/s, 4096 x 4096, m = 13631489", "value": 1e3 / ms,
               "unit": "conv2d/s", "ms_per_step": ms, "elements_per_s": R * C / (ms / 1e3),
               "config": {"workload": "conv2d_4096x4096_m13631489", "rows": R, "cols": C}}
    elif args.workload == "crt":
        rng = np.random.default_rng(9)
        f = torch.from_numpy(rng.integers(0, 1 << 15, (count, N), dtype=np.uint32).view(np.int32)).cuda()
        g = torch.from_numpy(rng.integers(0, 1 << 15, (count, N), dtype=np.uint32).view(np.int32)).cuda()
        h = torch.empty((count, N), dtype=torch.int64, device="cuda")
        run = lambda: nt.conv_crt(f, g, out=h, stream=st)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        per = _time_ms(run, args.steps, st)
        ms = float(per.mean())
        out = {"metric": "exact integer convolutions/s (two primes + CRT), 4096 x N=2^16, 15-bit operands",
               "value": count / (ms / 1e3), "unit": "conv/s", "ms_per_step": ms,
               "config": {"workload": "crt4096_n65536_15bit", "count": count, "n": N, "primes": [13631489, 7340033]}}
    elif args.workload == "u64":
        m = si.M_U64
        rng = np.random.default_rng(12)
        f = torch.from_numpy(rng.integers(0, m, count * N, dtype=np.uint64).view(np.int64)).cuda()
        g = torch.from_numpy(rng.integers(0, m, count * N, dtype=np.uint64).view(np.int64)).cuda()
        h = torch.empty_like(f)
        desc = nt.BatchDesc([n] * count, si.offsets([n] * count))
        run = lambda: nt.conv_batched(f, g, desc, m, out=h, stream=st)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        per = _time_ms(run, args.steps, st)
        ms = float(per.mean())
        out = {"metric": "exact convolutions/s, 64-bit words, 4096 x N=2^16", "value": count / (ms / 1e3),
               "unit": "conv/s", "ms_per_step": ms,
               "achieved_gbs_algorithmic": 24 * count * N / (ms / 1e3) / 1e9,
               "config": {"workload": "u64_4096_n65536_m31065037602817", "count": count, "n": N}}
    else:
        m = 7340033
        root = nt.euler_root(m, 20)
        rng = np.random.default_rng(8)
        f = torch.from_numpy(rng.integers(0, m, count * N, dtype=np.uint32).view(np.int32)).cuda()
        g = torch.from_numpy(rng.integers(0, m, count * N, dtype=np.uint32).view(np.int32)).cuda()
        h = torch.empty_like(f)
        desc = nt.BatchDesc([n] * count, si.offsets([n] * count))
        run = lambda: nt.conv_batched(f, g, desc, m, root=root, root_log2order=20, out=h, flags=nt.FLAG_EULER,
                                      stream=st)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        per = _time_ms(run, args.steps, st)
        ms = float(per.mean())
        out = {"metric": "exact convolutions/s, Euler-form prime, 4096 x N=2^16", "value": count / (ms / 1e3),
               "unit": "conv/s", "ms_per_step": ms,
               "config": {"workload": "euler4096_n65536_m7340033", "count": count, "n": N, "root": root}}
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """Serving: Poisson arrivals of convolution requests, lengths 2^n with n
    uniform in [8, 18], m = 31065037602817 (64-bit words), continuous batching
    over four streams, at most a quarter of the arena per batch; p50/p99
    latency and throughput at offered load rho * (saturated throughput).  The
    headline runs the library's native
    scheduler (ntt_server_*); beside it, the same at one request per batch, and
    the Python scheduler with operands copied in at submission and with
    zero-copy submission, against one launch sequence per request."""
    import threading

    import paper_1005_1497_amd.serve as sv
    import seeded_inputs as si

    m = si.M_U64
    warm, n = 200, args.requests
    lens = si.served_lengths(warm + n, seed=5)
    rng = np.random.default_rng(5)
    t0 = time.perf_counter()
    reqs = [(rng.integers(0, m, 1 << int(k), dtype=np.uint64), rng.integers(0, m, 1 << int(k), dtype=np.uint64))
            for k in lens]
    log("drew %d requests (%.1f M elements) in %.1f s" % (len(reqs), sum(1 << int(k) for k in lens) / 1e6,
                                                         time.perf_counter() - t0))
    cap = 24   # 2^24 elements per arena (3 arenas x 128 MiB)

    # zero-copy form: each request's operands already sit in a pinned staging
    # block of the server (written there by the client before submission)
    stager = sv.GpuExecutor(m, capacity_log2=0, elem_bits=64, streams=1)
    t0 = time.perf_counter()
    staged = []
    for f, g in reqs:
        blk = stager.staging(f.size)
        bf, bg = stager.operand_views(blk)
        bf[...] = f
        bg[...] = g
        staged.append((blk, int(f.size).bit_length() - 1))
    log("staged %d requests in pinned blocks in %.1f s" % (len(staged), time.perf_counter() - t0))

    def run(reqs_, rate, max_batch, zero_copy=False):
        ex = sv.GpuExecutor(m, capacity_log2=cap, elem_bits=64, streams=4)
        srv = sv.ConvServer(ex, capacity_log2=cap, max_batch=max_batch, max_inflight=4,
                            max_batch_elems=1 << (cap - 2)).start()

        def submit(i):
            if zero_copy:
                return srv.submit_staged(sv.StagedToken(*staged[i]))
            return srv.submit(*reqs_[i])

        for i in range(warm):
            submit(i)
        srv.drain()
        srv.stats = sv.ServeStats()
        body = range(warm, len(reqs_))
        gaps = np.random.default_rng(11).exponential(1.0 / rate, len(body)) if rate else np.zeros(len(body))
        # the set-up objects (drawn requests, staging blocks) are long-lived:
        # keep the cyclic collector from walking them during the timed run
        gc.collect()
        gc.freeze()
        t_start = time.perf_counter()

        def client():
            nxt = time.perf_counter()
            for i, gap in zip(body, gaps):
                nxt += gap
                d = nxt - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                submit(i)

        th = threading.Thread(target=client)
        th.start()
        th.join()
        srv.drain()
        el = time.perf_counter() - t_start
        srv.stop()
        st = srv.stats
        return {"throughput_conv_per_s": len(body) / el, "p50_ms": st.percentile(50) * 1e3,
                "p99_ms": st.percentile(99) * 1e3, "mean_batch": float(np.mean(st.batch_sizes)),
                "peak_inflight_batches": st.peak_inflight, "elapsed_s": el}

    def run_native(rate, max_batch=512):
        """The library's scheduler thread (ntt_server_*; --arenas): a producer
        thread submits with Poisson gaps (the copy into the request's pinned
        slot or staging block runs inside the library), a consumer thread collects the results in order into a reused
        buffer; latency is measured inside the library from submission to
        completion."""
        srv = sv.NativeConvServer(m, capacity_log2=cap, elem_bits=64, streams=4, max_batch=max_batch,
                                  max_batch_elems=1 << (cap - 2), max_inflight=4,
                                  host_arenas=args.arenas == "host")
        for t in [srv.submit(f, g) for f, g in reqs[:warm]]:
            srv.result(t)
        srv.stats(reset=True)
        body = reqs[warm:]
        gaps = np.random.default_rng(11).exponential(1.0 / rate, len(body)) if rate else np.zeros(len(body))
        tickets = [None] * len(body)
        ready = threading.Semaphore(0)
        gc.collect()
        gc.freeze()
        t_start = time.perf_counter()

        def producer():
            nxt = time.perf_counter()
            for i, ((f, g), gap) in enumerate(zip(body, gaps)):
                nxt += gap
                d = nxt - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(f, g)
                ready.release()

        sink = np.empty(1 << 18, dtype=np.uint64)     # the client's reused result buffer
        sink.fill(0)                                   # (its pages faulted in before timing)

        def consumer():
            for i in range(len(body)):
                ready.acquire()
                srv.result(tickets[i], out=sink[:tickets[i][1]])

        ths = [threading.Thread(target=producer), threading.Thread(target=consumer)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        el = time.perf_counter() - t_start
        st = srv.stats()
        srv.close()
        return {"throughput_conv_per_s": len(body) / el, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                "mean_batch": st["mean_batch"], "elapsed_s": el}

    sat = run(reqs, None, 512)
    log("python closed loop: %.0f conv/s" % sat["throughput_conv_per_s"])
    rate = args.rho * sat["throughput_conv_per_s"]
    served = run(reqs, rate, 512)
    log("python served at %.0f/s: p50 %.3f ms p99 %.3f ms" % (rate, served["p50_ms"], served["p99_ms"]))
    nat_sat = run_native(None)
    log("native closed loop: %.0f conv/s" % nat_sat["throughput_conv_per_s"])
    nat_rate = args.rho * nat_sat["throughput_conv_per_s"]
    nat = run_native(nat_rate)
    log("native served at %.0f/s: p50 %.3f ms p99 %.3f ms" % (nat_rate, nat["p50_ms"], nat["p99_ms"]))
    nat_same = run_native(rate)
    log("native served at %.0f/s: p50 %.3f ms p99 %.3f ms" % (rate, nat_same["p50_ms"], nat_same["p99_ms"]))
    nat_single = run_native(rate, max_batch=1)
    zc_sat = run(reqs, None, 512, zero_copy=True)
    log("zero-copy closed loop: %.0f conv/s" % zc_sat["throughput_conv_per_s"])
    zc_rate = args.rho * zc_sat["throughput_conv_per_s"]
    zc = run(reqs, zc_rate, 512, zero_copy=True)
    log("zero-copy served at %.0f/s: p50 %.3f ms p99 %.3f ms" % (zc_rate, zc["p50_ms"], zc["p99_ms"]))
    zc_same = run(reqs, rate, 512, zero_copy=True)
    single_sat = run(reqs, None, 1)
    single = run(reqs, args.rho * single_sat["throughput_conv_per_s"], 1)
    single_at_rate = run(reqs, rate, 1) if rate <= single_sat["throughput_conv_per_s"] else None
    out = {
        "metric": "served exact convolutions: throughput and p50/p99 latency",
        "value": nat["throughput_conv_per_s"], "unit": "conv/s", "n_gpus": 1, "steps": n, "warmup": warm,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "latency_ms": {"p50": nat["p50_ms"], "p99": nat["p99_ms"]},
        "config": {"workload": "serve_poisson_n2^8to2^18_m31065037602817", "rho": args.rho,
                   "offered_per_s": nat_rate,
                   "scheduler": "native (ntt_server_*), %s arenas" % args.arenas,
                   "words": "u64", "streams": 4,
                   "max_batch_elems": 1 << (cap - 2)},
        "saturated": nat_sat, "served": nat,
        "forms": {"native_at_python_rate": nat_same, "native_one_request_per_batch_at_python_rate": nat_single,
                  "python_saturated": sat, "python_at_rho": served,
                  "zero_copy_saturated": zc_sat, "zero_copy_at_rho": zc, "zero_copy_at_same_rate": zc_same,
                  "one_launch_per_request_saturated": single_sat, "one_launch_per_request_at_rho": single,
                  "one_launch_per_request_at_same_rate": single_at_rate},
    }
    print(json.dumps(out), flush=True)


def serve_sweep(args):
    """The served workload at several offered loads: --requests timed requests
    (20000 by default here) after 1000 warm-up ones, lengths 2^n with n uniform
    in [8, 18], m = 31065037602817 (64-bit words), Poisson arrivals at rho times
    the saturated throughput of the library's native scheduler (--arenas: host
    arenas by default; --clients submitting/waiting thread pairs, 4 by default;
    --streams and --inflight, 8 each by default); beside each,
    the same arrivals served one launch sequence per request (Python
    scheduler, one request per batch) where that form keeps up, and that form
    at rho times its own saturated throughput.  Every request has operands of
    its own: slices at seeded random offsets of one 2^23-word random buffer per
    operand (distinct contents without 16 GB of host payloads; the servers
    copy every request's operands)."""
    import threading

    import paper_1005_1497_amd.serve as sv
    import seeded_inputs as si

    m = si.M_U64
    warm = 1000
    n = args.requests if args.requests != 4000 else 20000
    lens = si.served_lengths(warm + n, seed=5)
    rng = np.random.default_rng(5)
    big = 1 << 23
    fbuf = rng.integers(0, m, big, dtype=np.uint64)
    gbuf = rng.integers(0, m, big, dtype=np.uint64)
    reqs = []
    for k in lens:
        nk = 1 << int(k)
        a, b = rng.integers(0, big - nk + 1, 2)
        reqs.append((fbuf[a:a + nk], gbuf[b:b + nk]))
    cap = 24
    rhos = [float(x) for x in args.rhos.split(",")]

    def native(rate, max_batch=512):
        srv = sv.NativeConvServer(m, capacity_log2=cap, elem_bits=64, streams=args.streams, max_batch=max_batch,
                                  max_batch_elems=1 << (cap - 2), max_inflight=args.inflight,
                                  solo_log2n=args.solo, host_arenas=args.arenas == "host")
        for t in [srv.submit(f, g) for f, g in reqs[:warm]]:
            srv.result(t)
        srv.stats(reset=True)
        body = reqs[warm:]
        # --clients client pairs (a submitting and a waiting thread each) take
        # every k-th request, each with Poisson gaps at rate / clients, so that
        # the merged arrivals are Poisson at the rate; several clients keep one
        # client's submission loop from capping the saturated throughput
        k_cl = max(1, args.clients)
        gc.collect()
        gc.freeze()
        t_start = time.perf_counter()

        def client(k):
            part = body[k::k_cl]
            gaps = (np.random.default_rng(11 + k).exponential(k_cl / rate, len(part)) if rate
                    else np.zeros(len(part)))
            tickets = [None] * len(part)
            ready = threading.Semaphore(0)
            sink = np.zeros(1 << 18, dtype=np.uint64)

            def producer():
                nxt = time.perf_counter()
                for i, ((f, g), gap) in enumerate(zip(part, gaps)):
                    nxt += gap
                    d = nxt - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                    tickets[i] = srv.submit(f, g)
                    ready.release()

            def consumer():
                for i in range(len(part)):
                    ready.acquire()
                    srv.result(tickets[i], out=sink[:tickets[i][1]])

            ths = [threading.Thread(target=producer), threading.Thread(target=consumer)]
            for t in ths:
                t.start()
            for t in ths:
                t.join()

        cls = [threading.Thread(target=client, args=(k,)) for k in range(k_cl)]
        for t in cls:
            t.start()
        for t in cls:
            t.join()
        el = time.perf_counter() - t_start
        st = srv.stats()
        srv.close()
        return {"throughput_conv_per_s": len(body) / el, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                "mean_batch": st["mean_batch"], "elapsed_s": el}

    def per_request(rate):
        ex = sv.GpuExecutor(m, capacity_log2=cap, elem_bits=64, streams=4)
        srv = sv.ConvServer(ex, capacity_log2=cap, max_batch=1, max_inflight=4,
                            max_batch_elems=1 << (cap - 2)).start()
        for i in range(warm):
            srv.submit(*reqs[i])
        srv.drain()
        srv.stats = sv.ServeStats()
        body = range(warm, len(reqs))
        gaps = np.random.default_rng(11).exponential(1.0 / rate, len(body)) if rate else np.zeros(len(body))
        gc.collect()
        gc.freeze()
        t_start = time.perf_counter()
        nxt = time.perf_counter()
        for i, gap in zip(body, gaps):
            nxt += gap
            d = nxt - time.perf_counter()
            if d > 0:
                time.sleep(d)
            srv.submit(*reqs[i])
        srv.drain()
        el = time.perf_counter() - t_start
        srv.stop()
        st = srv.stats
        return {"throughput_conv_per_s": len(body) / el, "p50_ms": st.percentile(50) * 1e3,
                "p99_ms": st.percentile(99) * 1e3, "elapsed_s": el}

    sat = native(None)
    log("native saturated: %.0f conv/s" % sat["throughput_conv_per_s"])
    single_sat = per_request(None)
    log("one launch per request, saturated: %.0f conv/s" % single_sat["throughput_conv_per_s"])
    rows = []
    for rho in rhos:
        rate = rho * sat["throughput_conv_per_s"]
        r = native(rate)
        row = {"rho": rho, "offered_per_s": rate, "served": r}
        if rate < 0.95 * single_sat["throughput_conv_per_s"]:
            row["one_launch_per_request"] = per_request(rate)
        else:
            row["one_launch_per_request"] = "offered rate above its saturated throughput (%.0f/s)" % \
                single_sat["throughput_conv_per_s"]
        own = rho * single_sat["throughput_conv_per_s"]
        row["one_launch_per_request_at_own_rho"] = {"offered_per_s": own, "served": per_request(own)}
        log("rho %.1f: %.0f/s offered, p50 %.3f ms, p99 %.3f ms" % (rho, rate, r["p50_ms"], r["p99_ms"]))
        rows.append(row)
    print(json.dumps({"metric": "served exact convolutions: p50/p99 latency across offered loads",
                      "unit": "ms", "n_gpus": 1, "requests": n, "warmup": warm, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "serve_poisson_n2^8to2^18_m31065037602817", "words": "u64",
                                 "scheduler": "native (ntt_server_*), %s arenas" % args.arenas,
                                 "clients": args.clients,
                                 "streams": args.streams,
                                 "max_inflight": args.inflight, "solo_log2n": args.solo,
                                 "max_batch_elems": 1 << (cap - 2)},
                      "saturated": sat, "one_launch_per_request_saturated": single_sat, "sweep": rows}), flush=True)


if __name__ == "__main__":
    main()
