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
boxes, whose results also give the maximum relative error of the GPU output.
"""
import argparse
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
    # per internal node: its 16-B schedule entry, T pairs of 16-B gathers and one 16-B store
    alg = internal * (16.0 + 48.0 * T)
    achieved = alg / (kern_ms * 1e-3) / 1e9
    return {"frames_per_s": steps / el, "ms_per_frame": 1e3 * el / steps, "tfs_per_frame": T,
            "nodes": N, "depth": D, "steps_launched": D,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "tf_step_kernel x depth",
                         "kernel_ms": kern_ms, "alg_bytes_per_launch": alg,
                         "alg_bytes_formula": "internal nodes x (16 + 48 T)"}}


def measure_serve(g, w, qps_list, seconds):
    """Poisson arrivals through the continuous-batching server; p50/p99 latency and achieved rate."""
    import numpy as np
    from paper_2009_02702_amd import synth
    from paper_2009_02702_amd.serve import Server
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
        print("[bench] serve %s" % r, file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--competitor-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=("full", "query", "copy", "tf", "serve"), default="full",
                    help="full: the JSON line; query: only the timed batched launches (for profilers); "
                         "copy: one device copy of --copy-mib MiB (calibrates HBM byte counters); "
                         "tf: transfer-function propagation frames (8 TFs) on --config; "
                         "serve: Poisson-arrival stream through the continuous-batching server on --config")
    ap.add_argument("--tf-count", type=int, default=8)
    ap.add_argument("--qps", type=str, default="5000,20000,50000,100000,200000")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--autotune", action="store_true", help="serve mode: autotune the launch on the workload's boxes first")
    ap.add_argument("--serve-qps", type=float, default=100000.0,
                    help="full mode: offered rate of the short serving leg (per-request p50/p99); 0 skips it")
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
    out = torch.empty((n, S), dtype=torch.float32, device=dev)
    ws = g.workspace(n)
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
        r = {"mode": "serve", "workload": w.name, "levels": measure_serve(g, w, qps, args.serve_seconds)}
        print(json.dumps(r), flush=True)
        return
    if args.mode == "query":
        # same launch selection as the full run (untimed), so profilers see the same kernels
        tuned = g.autotune(dboxes, out=out, reps=5, workspace=ws)
        print("[bench] autotuned %s" % (tuned,), file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            g.query(dboxes, out=out, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.query(dboxes, out=out, workspace=ws)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"mode": "query", "workload": w.name, "steps": args.steps,
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
        for _ in range(warmup):
            g.query(dboxes, out=out, variant=variant, workspace=ws)
        torch.cuda.synchronize()
        if timing:
            g.timing_read()
            g.timing(True)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in evs:
            a.record()
            g.query(dboxes, out=out, variant=variant, workspace=ws)
            b.record()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kern = None
        if timing:
            ms, k = g.timing_read()
            g.timing(False)
            kern = ms / max(k, 1)
        lat = np.array([a.elapsed_time(b) for a, b in evs])
        return el, lat, kern

    el, lat, kern_ms = run("batched", args.steps, args.warmup, True)
    value = args.steps * n / el
    res_main = out.cpu().numpy()

    comp = {}
    t0 = time.perf_counter()
    lut_nnz = g.lut_build()
    t_lut = time.perf_counter() - t0
    print("[bench] mixture lookup table: %d entries, built in %.2f s" % (lut_nnz, t_lut), file=sys.stderr,
          flush=True)
    for v in ("plain", "naive", "lut"):
        e2, l2, k2 = run(v, args.competitor_steps, 1, True)
        comp[v] = {"value": args.competitor_steps * n / e2, "ms_per_step": 1e3 * e2 / args.competitor_steps,
                   "kernel_ms": k2}
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
    e2, l2, k2 = run("batched", args.competitor_steps, 1, True, g=gg, ws=wsg)
    gi = gg.info()
    comp["greedy_push"] = {"value": args.competitor_steps * n / e2, "ms_per_step": 1e3 * e2 / args.competitor_steps,
                           "kernel_ms": k2, "nodes": gi["n_nodes"], "depth": gi["depth"], "build_s": t_gb,
                           "max_abs_diff_vs_push": float((out - torch.from_numpy(res_main).to(out.device)).abs().max())}
    print("[bench] greedy_push: %.3f ms/step (graph %d nodes, depth %d, built in %.2f s)"
          % (comp["greedy_push"]["ms_per_step"], gi["n_nodes"], gi["depth"], t_gb), file=sys.stderr, flush=True)
    del gg, wsg

    tf_meas = measure_tf(g, w, args.tf_count, max(3, args.steps // 2), 1)
    print("[bench] tf: %.3f ms per frame of %d TFs" % (tf_meas["ms_per_frame"], args.tf_count), file=sys.stderr,
          flush=True)

    serving = None
    if args.serve_qps > 0:
        serving = measure_serve(g, w, [args.serve_qps], args.serve_seconds)[0]
        serving["what"] = ("per-request latency (completion - arrival) of Poisson arrivals through the "
                           "continuous-batching server, 10% of requests with one TF")

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
    if not args.no_cpu_baseline:
        from oracle import scan
        ids, vol_c = scan.compact(vol)
        threads = scan.max_threads()
        # time consecutive chunks of the box list until about --cpu-seconds have passed
        chunk, m, el_cpu, refs = 2000, 0, 0.0, []
        while m < n and el_cpu < args.cpu_seconds:
            t0 = time.perf_counter()
            _, r = scan.box_counts(vol_c, len(ids), boxes[m:m + chunk], threads=threads)
            el_cpu += time.perf_counter() - t0
            refs.append(r)
            m += len(r)
        ref = np.concatenate(refs)
        cpu = {"value": m / el_cpu, "unit": "queries/s", "cores": threads, "kind": "oracle",
               "sample": "first %d of the %d boxes (%.1f s, %d OpenMP threads)" % (m, n, el_cpu, threads)}
        got = res_main[:m].astype(np.float64)
        nz = ref > 0
        support_ok = bool(np.array_equal(got == 0, ref == 0))
        max_rel = float((np.abs(got[nz] - ref[nz]) / ref[nz]).max()) if nz.any() else 0.0
        if not support_ok:
            max_rel = float("inf")

    line = {
        "metric": METRIC, "value": value, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "dims": list(w.dims), "segments": S, "boxes": n,
                   "box_edges": "log-uniform per axis" if w.box_mode != "corners" else "two uniform corners",
                   "output": "dense fp32 [n, S]", "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "completion latency of one batch of all boxes"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "max_rel_err_vs_oracle": max_rel,
        "oracle_checked_boxes": (m if not args.no_cpu_baseline else 0),
        "serving": serving,
        "competitors": comp,
        "tf_propagation": tf_meas,
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
