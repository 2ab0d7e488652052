#!/usr/bin/env python3
"""Box-histogram query throughput of the Mixture Graph on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2]

Workload (default): 512^3 uint32 Voronoi volume, 353 cells (one Lloyd step),
100,000 boxes with per-axis edge length log-uniform in [1, 512]; dense fp32
[n, 353] histograms. One step = one batch of all boxes through
mg_query_boxes (footprint, node-ID gather, scatter, reverse push, readout),
inputs already resident in HBM. Prints one JSON line.

Also measured on the same inputs: the plain per-box kernel and the naive
level-0 range scan (GPU competitors), the dominant kernel's HIP-event time for
the roofline, and the CPU oracle (brute-force scan) on a bounded sample of the
boxes (all host cores and one thread), whose results also give the maximum
relative error of the GPU output.

Further legs, each on its own workload and graph (--legs):
  aniso   2048x2048x300 Voronoi volume, 1,182 cells (z stretched by 7): its
          50,000 boxes and frames of 8 random RGBA8 transfer functions
  capsule 614x961x600 volume of 15,917 capsules: 10^6 boxes (0.1% the whole
          volume, 1% single voxels) in one sparse-output launch
  stream  1178x1125x789 Voronoi volume, 353 cells: Poisson arrivals at 5k,
          20k, 50k, 100k and 200k requests/s through the continuous-batching
          server, 10% of requests with one transfer function; per-request
          p50/p99 latency (completion - arrival)
"""
import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "box-histogram queries/s + p99 latency at ≤1e-5 rel err vs naive GPU range scan"


def kernel_source_sha() -> str:
    with open(os.path.join(ROOT, "paper_2009_02702_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(kernel: str, workload: str, bytes_per_launch_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it matches this kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        e = rec[kernel][workload]
    except (KeyError, ValueError):
        return None
    if e.get("kernel_sha") != kernel_source_sha():
        return None
    return float(e["hbm_bytes_per_launch"])


def measure_tf(g, w, T, steps, warmup):
    """Frames of T transfer functions propagated leaf -> node; HIP-event time of the step kernels."""
    import numpy as np
    import torch
    from paper_2009_02702_amd import synth
    inf = g.info()
    S, N, D = inf["nseg"], inf["n_nodes"], inf["depth"]
    tf = torch.from_numpy(synth.make_tfs(w, S, T)).cuda()
    pal = torch.empty((T, N, 4), dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        g.propagate_tf(tf, out=pal)
    torch.cuda.synchronize()
    g.timing_read()
    g.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        g.propagate_tf(tf, out=pal)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, k = g.timing_read()
    g.timing(False)
    kern_ms = ms / max(k, 1)
    internal = N - S
    # the method's bytes per frame: per internal node its (a, b, w) triple (12 B), its T colours
    # written (16 B each) and read once by a successor (16 B each); per source its T RGBA8 colours
    alg = internal * (12.0 + 32.0 * T) + S * 4.0 * T
    achieved = alg / (kern_ms * 1e-3) / 1e9
    traffic = read_traffic("tf_step_kernel", w.name, alg)
    return {"frames_per_s": steps / el, "ms_per_frame": 1e3 * el / steps, "tfs_per_frame": T,
            "nodes": N, "depth": D, "order": "ranks" if g.launch_config()["tf_schedule"] == 0 else "deferred steps",
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                         "kernel": "tf_step_kernel per rank (the first also writes the sources' colours and, "
                                   "in rank order, takes rank 2 too) and tf_tail_kernel for the small last ranks "
                                   "(one frame, timed together)",
                         "kernel_ms": kern_ms, "alg_bytes_per_launch": alg,
                         "alg_bytes_formula": "internal nodes x (12 + 32 T) + sources x 4 T",
                         # the first launch rebuilds rank-1 colours for rank-2 nodes instead of reading
                         # them, so the kernels move fewer bytes than the formula counts
                         "frac_measured_bytes": (traffic / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                                 if traffic else None)}}


def measure_serve(g, w, qps_list, seconds, trace_dir=None):
    """Poisson arrivals through the continuous-batching server; per-request p50/p99 latency and
    achieved rate per offered rate. trace_dir: also write each rate's per-batch trace there."""
    import numpy as np
    from paper_2009_02702_amd import synth
    from paper_2009_02702_amd.serve import TRACE_FIELDS, Server
    S = g.info()["nseg"]
    srv = Server(g, slots=4, max_batch=4096, max_tf=64)
    out = []
    for qps in qps_list:
        n = max(1000, int(qps * seconds))
        boxes = synth.make_boxes(w, n)
        arr = synth.poisson_arrivals(w, n, qps)
        tf_index = np.full(n, -1, dtype=np.int64)
        rows = np.arange(0, n, 10)                     # 10% of the requests carry a TF
        tf_index[rows] = np.arange(len(rows))
        tfs = synth.make_tfs(w, S, len(rows))
        st = srv.serve(boxes, arr, tf_index, tfs)
        r = st.summary()
        r["offered_qps"] = qps
        out.append(r)
        if trace_dir:
            os.makedirs(trace_dir, exist_ok=True)
            np.savetxt(os.path.join(trace_dir, "serve_trace_%s_%d.txt" % (w.name, int(qps))), st.trace,
                       header=" ".join(TRACE_FIELDS), fmt="%.6f")
        print("[bench] serve %s" % r, file=sys.stderr, flush=True)
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(vol, boxes, seconds, threads, chunk):
    """The CPU oracle (O1) on consecutive chunks of the box list until about `seconds` have
    passed: (boxes/s, boxes done, elapsed, fractions of the boxes done)."""
    import numpy as np
    from oracle import scan
    ids, vol_c = scan.compact(vol)
    m, el, refs = 0, 0.0, []
    while m < len(boxes) and el < seconds:
        t0 = time.perf_counter()
        _, r = scan.box_counts(vol_c, len(ids), boxes[m:m + chunk], threads=threads)
        el += time.perf_counter() - t0
        refs.append(r)
        m += len(r)
    return m / el, m, el, np.concatenate(refs)


def _timed(fn, steps, warmup, g=None):
    """Run fn() warmup + steps times; (wall seconds of the timed steps, library kernel ms per
    step from the HIP events the library records around its launches, or None)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if g is not None:
        g.timing_read()
        g.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern = None
    if g is not None:
        ms, k = g.timing_read()
        g.timing(False)
        kern = ms / max(k, 1)
    return el, kern


def leg_aniso(args):
    """2048x2048x300 Voronoi volume: its 50,000 boxes (batched) and frames of 8 TFs."""
    import numpy as np
    import torch
    from paper_2009_02702_amd import Graph, synth
    w = synth.workload(3)
    vol = synth.make_volume(w)
    boxes = synth.make_boxes(w)
    t0 = time.perf_counter()
    g = Graph.build(vol)
    t_build = time.perf_counter() - t0
    g.upload(0)
    del vol
    inf = g.info()
    S, n = inf["nseg"], len(boxes)
    db = torch.from_numpy(boxes.view(np.int32)).cuda()
    out = torch.empty((n, S), dtype=torch.float32, device="cuda")
    ws = g.workspace(n)
    el, kern = _timed(lambda: g.query(db, out=out, workspace=ws), max(3, args.steps // 2), 1, g)
    steps = max(3, args.steps // 2)
    r = {"workload": w.name, "boxes": n, "segments": S, "nodes": inf["n_nodes"], "depth": inf["depth"],
         "levels": inf["n_levels"], "build_s": t_build, "device_bytes": inf["device_bytes"],
         "query": {"value": steps * n / el, "unit": "queries/s", "ms_per_step": 1e3 * el / steps,
                   "kernel_ms": kern}}
    del out, ws
    r["tf_propagation"] = measure_tf(g, w, 8, max(5, args.steps), 2)
    print("[bench] aniso: %.3f ms per batch of %d boxes; %.3f ms per frame of 8 TFs (frac %.2f)"
          % (r["query"]["ms_per_step"], n, r["tf_propagation"]["ms_per_frame"],
             r["tf_propagation"]["roofline"]["frac"]), file=sys.stderr, flush=True)
    g.close()
    return r


def leg_capsule(args):
    """614x961x600 capsule volume: 10^6 boxes in one sparse-output launch."""
    import numpy as np
    import torch
    from paper_2009_02702_amd import Graph, synth
    w = synth.workload(4)
    vol = synth.make_volume(w)
    boxes = synth.make_boxes(w)
    t0 = time.perf_counter()
    g = Graph.build(vol)
    t_build = time.perf_counter() - t0
    g.upload(0)
    del vol
    inf = g.info()
    n = len(boxes)
    db = torch.from_numpy(boxes.view(np.int32)).cuda()
    ws = g.workspace(n)
    cap = 300_000_000
    bufs = (torch.empty((n, 2), dtype=torch.int32, device="cuda"), torch.empty(cap, dtype=torch.int32, device="cuda"),
            torch.empty(cap, dtype=torch.float32, device="cuda"), torch.empty(1, dtype=torch.int32, device="cuda"))
    steps = 3
    el, kern = _timed(lambda: g.query_sparse(db, capacity=cap, workspace=ws, bufs=bufs), steps, 1, g)
    nnz = int(bufs[3].item())
    r = {"workload": w.name, "boxes": n, "segments": inf["nseg"], "nodes": inf["n_nodes"], "depth": inf["depth"],
         "build_s": t_build, "entries": nnz, "output": "sparse (segment, fraction) entries",
         "value": steps * n / el, "unit": "queries/s", "ms_per_step": 1e3 * el / steps, "kernel_ms": kern}
    print("[bench] capsule: %.2f ms per launch of %d boxes (%d entries)" % (r["ms_per_step"], n, nnz),
          file=sys.stderr, flush=True)
    del bufs, ws
    g.close()
    return r


def leg_stream(args):
    """1178x1125x789 Voronoi volume served at 5k-200k requests/s."""
    from paper_2009_02702_amd import Graph, synth
    w = synth.workload(5)
    vol = synth.make_volume(w)
    t0 = time.perf_counter()
    g = Graph.build(vol)
    t_build = time.perf_counter() - t0
    g.upload(0)
    del vol
    inf = g.info()
    qps = [float(x) for x in args.qps.split(",") if x]
    levels = measure_serve(g, w, qps, args.serve_seconds, args.trace_dir)
    g.close()
    return {"workload": w.name, "segments": inf["nseg"], "nodes": inf["n_nodes"], "depth": inf["depth"],
            "build_s": t_build,
            "what": "per-request latency (completion seen by the server - arrival) of Poisson arrivals "
                    "through the continuous-batching server (4 HIP-stream slots, captured graphs), 10% of "
                    "requests with one TF (propagated, and the box coloured with it)",
            "levels": levels}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--competitor-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu1-seconds", type=float, default=6.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=("full", "query", "copy", "tf", "serve"), default="full",
                    help="full: the JSON line; query: only the timed batched launches (for profilers); "
                         "copy: one device copy of --copy-mib MiB (calibrates HBM byte counters); "
                         "tf: transfer-function propagation frames (8 TFs) on --config; "
                         "serve: Poisson-arrival stream through the continuous-batching server on --config")
    ap.add_argument("--variant", default="batched", help="query mode: batched, plain, naive or lut")
    ap.add_argument("--tf-count", type=int, default=8)
    ap.add_argument("--qps", type=str, default="5000,20000,50000,100000,200000")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--autotune", action="store_true", help="serve mode: autotune the launch on the workload's boxes first")
    ap.add_argument("--legs", type=str, default="aniso,capsule,stream",
                    help="full mode: further workloads (aniso, capsule, stream; empty for none)")
    ap.add_argument("--trace-dir", type=str, default=None, help="write the serving legs' per-batch traces here")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(queries shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2009_02702_amd import Graph, synth

    dev = torch.device("cuda:0")
    if args.mode == "copy":
        n_el = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n_el, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read": n_el * 4, "bytes_written": n_el * 4}), flush=True)
        return
    w = synth.workload(args.config)
    t0 = time.perf_counter()
    vol = synth.make_volume(w)
    boxes = synth.make_boxes(w)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = Graph.build(vol)
    t_build = time.perf_counter() - t0
    g.upload(0)
    inf = g.info()
    S, n = inf["nseg"], len(boxes)
    print("[bench] workload %s: dims %s, %d segments, %d boxes; graph %d nodes, depth %d, built in %.2f s"
          % (w.name, w.dims, S, n, inf["n_nodes"], inf["depth"], t_build), file=sys.stderr, flush=True)

    dboxes = torch.from_numpy(boxes.view(np.int32)).to(dev)
    out = torch.empty((n, S), dtype=torch.float32, device=dev) if args.mode != "tf" else None
    ws = g.workspace(n) if args.mode != "tf" else None
    torch.cuda.synchronize()

    if args.mode == "tf":
        r = measure_tf(g, w, args.tf_count, args.steps, args.warmup)
        r.update({"mode": "tf", "workload": w.name})
        print(json.dumps(r), flush=True)
        return
    if args.mode == "serve":
        if args.autotune:
            print("[bench] autotuned %s" % (g.autotune(dboxes, out=out, reps=3, workspace=ws),), file=sys.stderr,
                  flush=True)
        qps = [float(x) for x in args.qps.split(",") if x]
        r = {"mode": "serve", "workload": w.name, "levels": measure_serve(g, w, qps, args.serve_seconds,
                                                                         args.trace_dir)}
        print(json.dumps(r), flush=True)
        return
    if args.mode == "query":
        # same launch selection as the full run (untimed), so profilers see the same kernels
        tuned = g.autotune(dboxes, out=out, reps=5, workspace=ws)
        print("[bench] autotuned %s" % (tuned,), file=sys.stderr, flush=True)
        if args.variant == "lut":
            g.lut_build()
        el, _ = _timed(lambda: g.query(dboxes, out=out, variant=args.variant, workspace=ws), args.steps,
                       args.warmup)
        print(json.dumps({"mode": "query", "variant": args.variant, "workload": w.name, "steps": args.steps,
                          "ms_per_step": 1e3 * el / args.steps}), flush=True)
        return

    # launch configuration picked by the autotuner on this batch (not timed)
    t0 = time.perf_counter()
    tuned = g.autotune(dboxes, out=out, reps=5, workspace=ws)
    t_tune = time.perf_counter() - t0
    print("[bench] autotuned %s in %.2f s" % (tuned, t_tune), file=sys.stderr, flush=True)

    # accounting pass: per-box cubes and graph nodes touched (not timed)
    _, stats = g.query_stats(dboxes, out=out, workspace=ws)
    torch.cuda.synchronize()
    st = stats.cpu().numpy().view(np.uint32)
    cubes = st[:, 0].astype(np.float64)
    touched = (st[:, 1] & 0x3FFFFFFF).astype(np.float64)
    fallback = (st[:, 1] >> 31).astype(bool)
    retried = ((st[:, 1] >> 30) & 1).astype(bool)
    lvl_counts, _ = g.footprint(dboxes)
    cubes0 = lvl_counts.cpu().numpy()[:, 0].astype(np.float64)
    # the method's algorithmic bytes per box: the box, a 32-bit node ID per cube, one (a, b, w)
    # triple per graph node touched, the dense fp32 row
    alg_bytes = float(np.sum(24.0 + 4.0 * cubes + 12.0 * touched + 4.0 * S))
    # the same with level-0 IDs at the 2 bytes the 16-bit copy stores (S < 65535)
    id0 = 2.0 if S < 65535 else 4.0
    alg_bytes_stored = float(np.sum(24.0 + id0 * cubes0 + 4.0 * (cubes - cubes0) + 12.0 * touched + 4.0 * S))

    def run(variant, steps, warmup, timing, g=g, ws=ws):
        el, kern = _timed(lambda: g.query(dboxes, out=out, variant=variant, workspace=ws), steps, warmup,
                          g if timing else None)
        return el, kern

    el, kern_ms = run("batched", args.steps, args.warmup, True)
    value = args.steps * n / el
    # completion time of one whole batch, from events around each call (not a per-request latency)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    for a, b in evs:
        a.record()
        g.query(dboxes, out=out, workspace=ws)
        b.record()
    torch.cuda.synchronize()
    batch_ms = np.array([a.elapsed_time(b) for a, b in evs])
    res_main = out.cpu().numpy()

    comp = {}
    t0 = time.perf_counter()
    lut_nnz = g.lut_build()
    t_lut = time.perf_counter() - t0
    print("[bench] mixture lookup table: %d entries, built in %.2f s" % (lut_nnz, t_lut), file=sys.stderr,
          flush=True)
    for v in ("plain", "naive", "lut"):
        e2, k2 = run(v, args.competitor_steps, 1, True)
        comp[v] = {"value": args.competitor_steps * n / e2, "ms_per_step": 1e3 * e2 / args.competitor_steps,
                   "kernel_ms": k2}
        # HBM bytes per batch from the committed counter summaries, where they match this kernel source
        hbm = read_traffic({"naive": "naive_kernel", "lut": "query_lut"}.get(v, ""), w.name, 0.0)
        if hbm is not None:
            comp[v]["hbm_bytes_per_batch"] = hbm
            comp[v]["hbm_gbs"] = hbm / (k2 * 1e-3) / 1e9
        if v == "lut":
            comp[v]["max_abs_diff_vs_push"] = float((out - torch.from_numpy(res_main).to(out.device)).abs().max())
            comp[v]["lut_entries"] = lut_nnz
            comp[v]["lut_build_s"] = t_lut
        print("[bench] %s: %.3f ms/step" % (v, comp[v]["ms_per_step"]), file=sys.stderr, flush=True)

    # the same boxes on a graph from the paper's greedy factorizer (max-reduction, tau = 3)
    t0 = time.perf_counter()
    gg = Graph.build(vol, factorizer="reduction", tau=3)
    t_gb = time.perf_counter() - t0
    gg.upload(0)
    gg.set_launch_config(**{k: v for k, v in tuned.items()})
    wsg = gg.workspace(n)
    e2, k2 = run("batched", args.competitor_steps, 1, True, g=gg, ws=wsg)
    gi = gg.info()
    comp["greedy_push"] = {"value": args.competitor_steps * n / e2, "ms_per_step": 1e3 * e2 / args.competitor_steps,
                           "kernel_ms": k2, "nodes": gi["n_nodes"], "depth": gi["depth"], "build_s": t_gb,
                           "max_abs_diff_vs_push": float((out - torch.from_numpy(res_main).to(out.device)).abs().max())}
    print("[bench] greedy_push: %.3f ms/step (graph %d nodes, depth %d, built in %.2f s)"
          % (comp["greedy_push"]["ms_per_step"], gi["n_nodes"], gi["depth"], t_gb), file=sys.stderr, flush=True)
    gg.close()
    del gg, wsg

    tf_meas = measure_tf(g, w, args.tf_count, max(3, args.steps // 2), 1)
    print("[bench] tf: %.3f ms per frame of %d TFs" % (tf_meas["ms_per_frame"], args.tf_count), file=sys.stderr,
          flush=True)

    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    traffic = read_traffic("query_tier_kernel", w.name, alg_bytes)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "query_tier_kernel big + small tiers, with query_retry_kernel and query_fallback_kernel (timed together)",
                "kernel_ms": kern_ms,
                "alg_bytes_per_launch": alg_bytes,
                "alg_bytes_formula": "sum over boxes of 24 + 4*cubes + 12*graph nodes touched + 4*S (dense output)",
                # level-0 node IDs counted at the 2 bytes of the 16-bit copy the kernels read
                "frac_level0_as_stored": alg_bytes_stored / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                # the node triples (12 B x nodes touched) may be served from L2 / MALL rather than HBM
                "frac_excl_node_triples": (alg_bytes - 12.0 * float(touched.sum())) / (kern_ms * 1e-3) / 1e9
                / HBM_PEAK_GBS}

    cpu = None
    max_rel = None
    m = 0
    if not args.no_cpu_baseline:
        from oracle import scan
        threads = scan.max_threads()
        rate, m, el_cpu, ref = oracle_rate(vol, boxes, args.cpu_seconds, threads, 2000)
        rate1, m1, el1, _ = oracle_rate(vol, boxes, args.cpu1_seconds, 1, 200)
        cpu = {"value": rate, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": "first %d of the %d boxes (%.1f s, %d OpenMP threads)" % (m, n, el_cpu, threads),
               "value_1_thread": rate1, "sample_1_thread": "first %d boxes (%.1f s, 1 thread)" % (m1, el1),
               "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count()}
        got = res_main[:m].astype(np.float64)
        nz = ref > 0
        support_ok = bool(np.array_equal(got == 0, ref == 0))
        max_rel = float((np.abs(got[nz] - ref[nz]) / ref[nz]).max()) if nz.any() else 0.0
        if not support_ok:
            max_rel = float("inf")
    g.close()
    del vol, out, ws, dboxes
    gc.collect()
    torch.cuda.empty_cache()

    legs = {}
    for leg in [x for x in args.legs.split(",") if x]:
        fn = {"aniso": leg_aniso, "capsule": leg_capsule, "stream": leg_stream}[leg]
        legs[leg] = fn(args)
        gc.collect()
        torch.cuda.empty_cache()

    line = {
        "metric": METRIC, "value": value, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "dims": list(w.dims), "segments": S, "boxes": n,
                   "box_edges": "log-uniform per axis" if w.box_mode != "corners" else "two uniform corners",
                   "output": "dense fp32 [n, S]", "parallelism": "single GPU"},
        "batch_completion_ms": {"median": float(np.median(batch_ms)), "max": float(batch_ms.max()),
                                "what": "device time from before to after one call answering all boxes "
                                        "(a batch figure, not a per-request latency: see serving)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": max_rel,
        "oracle_checked_boxes": m,
        "serving": legs.get("stream"),
        "competitors": comp,
        "tf_propagation": tf_meas,
        "aniso": legs.get("aniso"),
        "capsule": legs.get("capsule"),
        "speedup_vs_naive": value / comp["naive"]["value"],
        "speedup_vs_plain": value / comp["plain"]["value"],
        "launch": tuned,
        "graph": {"nodes": inf["n_nodes"], "depth": inf["depth"], "levels": inf["n_levels"],
                  "build_s": t_build, "volume_gen_s": t_gen, "device_bytes": inf["device_bytes"]},
        "work": {"cubes_mean": float(cubes.mean()), "level0_cubes_mean": float(cubes0.mean()),
                 "nodes_touched_mean": float(touched.mean()),
                 "nodes_touched_max": int(touched.max()), "boxes_via_fallback": int(fallback.sum()),
                 "boxes_via_retry": int(retried.sum()),
                 "cubes_share_via_fallback": float(cubes[fallback].sum() / max(cubes.sum(), 1.0)),
                 "touched_max_big_tier": int(touched[cubes >= 16384].max(initial=0)),
                 "touched_max_small_tier": int(touched[cubes < 16384].max(initial=0))},
        "paper_context": "178.95x footprint assembly vs 10-core naive CPU range query (Polymer 256^3, "
                         "i9-9820X; Table 'query'); other hardware and data, not a target",
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
