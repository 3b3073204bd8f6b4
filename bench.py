"""Benchmark of the BFS-kNN hot path on one MI355X.

The headline step is the whole hot path over the Barabasi-Albert workload
(n = 100,000, 4 edges per new vertex, m = 399,990; seeded synthetic input
standing in for the paper's scale-free graphs):
  1. CSR ingest: canonicalise the input CSR (its rows arrive unsorted);
  2. all-source BFS hop distances from 4,096 seeded sample sources, written as
     a uint8 hop matrix (409.6 MB), and the (hop, id) kNN of those rows, k = 15;
  3. truncated partial BFS kNN from all 100,000 vertices, k = 15;
  4. UMAP membership weights of those 100,000 rows.
value = Graph500-convention GTEPS of the step: 4,096 sources x m undirected
edges (the graph is connected) divided by the whole step's time.

The default run (--workload all) adds the rest of the metric under
"workloads": the 32 x 32 grid and the dense Erdos-Renyi graph (GTEPS of the
all-source path), the batch of 2,048 uneven graphs (graphs/s batched against
the plain per-graph loop) and the served stream of 4,096 distinct jobs (p50 /
p99 latency and graphs/s against the plain loop), each with its parity check,
roofline and CPU-oracle baseline.

Prints one JSON line (progress goes to stderr).  --gpus > 1 is refused
(one-GPU build).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GTEPS + kNN graphs/sec vs plain; p50/p99 served latency, bit-exact"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--workload", default="all", choices=["all", "ba100k", "grid", "er", "batch", "serve", "stress",
                                                          "neighborhood", "layout", "sparsify"])
    p.add_argument("--layout-iters", type=int, default=200)
    p.add_argument("--batch-graphs", type=int, default=2048)
    p.add_argument("--serve-jobs", type=int, default=4096)
    p.add_argument("--serve-warmup", type=int, default=256)
    p.add_argument("--serve-budget-gb", type=float, default=64.0)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--k", type=int, default=15)
    p.add_argument("--sources", type=int, default=4096)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-parity", action="store_true")
    p.add_argument("--no-tune", action="store_true",
                   help="skip the all-source autotuner (gumap_knn_build_tune) before the warm-up")
    p.add_argument("--cpu-one-thread-fraction", type=int, default=8,
                   help="the one-thread oracle time is measured on 1/N of each workload and scaled")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    p.add_argument("--traffic-from", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                   help="turn four rocprofv3 --pmc runs (FETCH_SIZE / WRITE_SIZE of this bench and of "
                        "--calibrate-copy) into the traffic file and exit")
    p.add_argument("--traffic-kernel", default="msbfs_level_kernel")
    p.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_ba100k.json"),
                   help="HBM bytes per launch of the dominant kernel measured with rocprofv3 counters")
    return p.parse_args()


def main():
    args = parse()
    if args.traffic_from:
        write_traffic(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(one GPU's share of the work is what it runs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        return calibrate_copy()
    single = {"batch": run_batch, "serve": run_serve, "grid": lambda a: run_allsource(a, "grid"),
              "er": lambda a: run_allsource(a, "er"), "ba100k": run_ba}
    if args.workload in single:
        out = single[args.workload](args)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "stress":
        return bench_stress(args)
    if args.workload == "neighborhood":
        return bench_neighborhood(args)
    if args.workload == "layout":
        return bench_layout(args)
    if args.workload == "sparsify":
        return bench_sparsify(args)
    # all: the headline BA step, then the other workloads of the metric
    t_all = time.perf_counter()
    _progress("ba100k")
    out = run_ba(args)
    subs = {}
    for name, fn in (("grid32", lambda: run_allsource(args, "grid")), ("er16k", lambda: run_allsource(args, "er")),
                     ("batch2048", lambda: run_batch(args)), ("stream%d" % args.serve_jobs, lambda: run_serve(args))):
        _progress(name)
        subs[name] = _sub(fn())
    out["workloads"] = subs
    b = subs["batch2048"]
    v = subs["stream%d" % args.serve_jobs]
    out["knn_graphs_per_s_batched"] = b["value"]
    out["knn_graphs_per_s_plain_loop"] = b["graphs_per_s_plain_loop"]
    out["batched_vs_plain"] = b["speedup_vs_plain"]
    out["served_graphs_per_s"] = v["value"]
    out["served_saturation_graphs_per_s"] = v["saturation_graphs_per_s"]
    out["served_vs_plain"] = v["speedup_vs_plain"]
    out["served_p50_ms"] = v["p50_ms"]
    out["served_p99_ms"] = v["p99_ms"]
    out["parity_all_workloads"] = bool(out.get("parity_sampled_bit_exact", True) and all(
        w.get("parity_sampled_bit_exact", True) for w in subs.values()))
    out["bench_wall_s"] = time.perf_counter() - t_all
    print(json.dumps(out), flush=True)


def _progress(name):
    print("bench: %s" % name, file=sys.stderr, flush=True)


def _sub(d):
    """A workload's record inside the headline line (the top-level keys that
    only describe the line itself are dropped)."""
    return {key: val for key, val in d.items() if key not in ("metric", "n_gpus", "higher_is_better", "scaling",
                                                              "vs_baseline", "data")}


def calibrate_copy():
    """A plain 1 GiB device copy, the reference for the HBM byte counters."""
    import torch
    n_bytes = 1 << 30
    a = torch.empty(n_bytes // 4, dtype=torch.int32, device="cuda")
    b_ = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b_.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": n_bytes,
                      "bytes_written_per_copy": n_bytes, "copies": 3}), flush=True)


def cpu_model() -> str | None:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _timed(fn):
    t0 = time.perf_counter()
    fn()
    return time.perf_counter() - t0


def cpu_block(work, unit, t_all, threads, t_one, sample):
    """cpu_baseline record: `work` units of the workload took t_all seconds on
    `threads` threads and t_one (estimated) on one thread."""
    return {"value": work / t_all, "unit": unit, "cores": threads, "kind": "oracle", "sample": sample,
            "seconds_all_cores": t_all, "value_one_thread": work / t_one, "seconds_one_thread": t_one,
            "cpu_model": cpu_model()}


def run_ba(args):
    """The headline step on the BA graph (canonicalise, all-source BFS from
    4,096 sources with the hop matrix and kNN, partial BFS from every vertex,
    membership)."""
    import numpy as np
    import torch

    import graphgen as G
    import paper_2509_19703_amd as gm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    k = args.k
    g = G.config_ba()                                  # canonical reference graph
    shuffled = G.dirty(g, G.BASE_SEED + 5, dup_frac=0.0, loop_frac=0.0)   # same edges, rows unsorted
    src = G.config_ba_sources(args.sources)
    n, m = g.n, g.m

    rp_in = torch.from_numpy(shuffled.row_ptr).to(dev)
    ci_in = torch.from_numpy(shuffled.col_idx).to(dev)
    src_d = torch.from_numpy(src).to(dev)
    rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    ci = torch.empty(shuffled.nnz, dtype=torch.int32, device=dev)
    b_ids = torch.empty((len(src), k), dtype=torch.int32, device=dev)
    b_hops = torch.empty((len(src), k), dtype=torch.uint8, device=dev)
    hop_matrix = torch.empty((len(src), n), dtype=torch.uint8, device=dev)
    p_ids = torch.empty((n, k), dtype=torch.int32, device=dev)
    p_hops = torch.empty((n, k), dtype=torch.uint8, device=dev)
    w = torch.empty((n, k), dtype=torch.float32, device=dev)
    rho = torch.empty(n, dtype=torch.float32, device=dev)
    sigma = torch.empty(n, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    g_in = gm.make_graph(rp_in, ci_in, flags=0)

    def step():
        nnz = gm.gumap_csr_canonicalize(g_in, rp, ci, stream)
        gc = gm.gumap_graph(n, nnz, gm._ptr(rp), gm._ptr(ci), gm.CSR_SORTED)
        gm.gumap_knn_build(gc, k, src_d, len(src), b_ids, b_hops, hop_matrix, stream)
        gm.gumap_knn_partial(gc, k, p_ids, p_hops, stream)
        gm.gumap_membership(n, k, p_hops, w, rho, sigma, stream)

    tune = None
    if not args.no_tune:
        # the autotuner times its candidates on this graph and sources (outside
        # the timed region); the timed calls then run with its pick
        nnz0 = gm.gumap_csr_canonicalize(g_in, rp, ci, stream)
        gc0 = gm.gumap_graph(n, nnz0, gm._ptr(rp), gm._ptr(ci), gm.CSR_SORTED)
        tune = gm.gumap_knn_build_tune(gc0, k, src_d, len(src), b_ids, b_hops, hop_matrix, stream)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: the K steps, with HIP events on the dominant kernel's launches
    dt, prof, dom, prof_all = _profiled(gm, step, args.steps, want_breakdown=True)
    # the same K steps without events, for the event overhead
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt_plain = (time.perf_counter() - t1) / args.steps
    teps = len(src) * m / dt
    d = prof[dom]
    traffic = None
    if os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            tj = json.load(f)
        if tj.get("kernel") == dom and tj.get("source_sha") == kernel_source_sha():
            traffic = tj.get("hbm_bytes_per_launch")
    out = {
        "metric": METRIC,
        "value": teps / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "ba100k: Barabasi-Albert n=100000 m_attach=4 (m=%d), seed %d; "
                               "canonicalise + all-source BFS from %d sampled sources with uint8 hop "
                               "matrix + (hop,id) kNN k=%d + partial BFS kNN from all vertices + "
                               "FP32 membership" % (m, G.BASE_SEED + 1, len(src), k),
                   "n": n, "m": m, "sources": len(src), "k": k},
        "roofline": _hbm_roofline(d, dom, traffic, prof_all.get(dom)),
        "kernels_ms_per_step": {kname: v["total_ms"] / args.steps for kname, v in prof.items()},
        "ms_per_step_without_events": dt_plain * 1e3,
        "steps_per_s": 1.0 / dt,
        "autotune": tune,
    }
    if not args.no_parity:
        import oracle as O
        pick = np.arange(0, len(src), 97)
        oi, oh, ohm = O.knn_build(g, k, sources=src[pick], hop_matrix=True)
        ok = (np.array_equal(b_ids[torch.from_numpy(pick).to(dev)].cpu().numpy(), oi)
              and np.array_equal(b_hops[torch.from_numpy(pick).to(dev)].cpu().numpy(), oh)
              and np.array_equal(hop_matrix[torch.from_numpy(pick).to(dev)].cpu().numpy(), ohm))
        vs = np.arange(0, n, 499)
        pi, ph = O.knn_partial(g, k, sources=vs)
        ok = ok and np.array_equal(p_ids[torch.from_numpy(vs).to(dev)].cpu().numpy(), pi) \
            and np.array_equal(p_hops[torch.from_numpy(vs).to(dev)].cpu().numpy(), ph)
        out["parity_sampled_bit_exact"] = bool(ok)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_ba(g, src, k, m, args.cpu_one_thread_fraction)
    return out


def _profiled(gm, fn, steps, want_breakdown=False):
    """Runs fn() `steps` times with events on every kernel launch (the
    per-kernel breakdown, which names the dominant kernel), then `steps`
    timed times with events on the dominant kernel's launches only.
    Returns (s per step of the timed pass, entries, dominant kernel): the
    dominant kernel's entry is the timed pass's, the others the breakdown's
    (and, with want_breakdown, the breakdown pass's entries unchanged)."""
    import torch
    gm.profile_reset()
    gm.profile_only(None)
    gm.profile_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    gm.profile_enable(False)
    prof = gm.profile_entries()
    breakdown = dict(prof)
    dom = max(prof, key=lambda kname: prof[kname]["total_ms"])
    # timed region: HIP events around the dominant kernel's launches only
    gm.profile_reset()
    gm.profile_only([dom])
    gm.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    gm.profile_enable(False)
    gm.profile_only(None)
    prof[dom] = gm.profile_entries()[dom]
    if want_breakdown:
        return dt, prof, dom, breakdown
    return dt, prof, dom


def _hbm_roofline(d, dom, traffic, breakdown=None):
    """HBM roofline record of the dominant kernel: its algorithmic bytes per
    launch (the per-level count of the traversal) over its average launch
    time, and beside it the same with the bytes it moves beyond that (for the
    BFS level kernel: the lazy commit of the previous level)."""
    avg_s = d["total_ms"] / 1e3 / d["launches"]
    alg = d["alg_bytes"] / d["launches"]
    extra = d.get("extra_bytes", 0.0) / d["launches"]
    achieved = alg / avg_s / 1e9
    out = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "launches": d["launches"],
           "avg_launch_us": avg_s * 1e6, "alg_bytes_per_launch": alg}
    if extra > 0:
        with_extra = (alg + extra) / avg_s / 1e9
        out.update({"extra_bytes_per_launch": extra, "achieved_with_extra": with_extra,
                    "frac_with_extra": with_extra / HBM_PEAK_GBS,
                    "extra_note": "bytes beyond the per-level count: the lazy commit of the previous level "
                                  "(the visited word written back, plus bit-plane read-modify-writes for hops "
                                  "above the frontier history)"})
    return out


FP64_PEAK_TFLOPS = 78.6


def _roofline(prof, steps, dom):
    d = prof[dom]
    if dom in ("neighborhood", "msbfs_stress"):
        # FP64 distance arithmetic against the vector FP64 peak; the counter
        # holds FP64 operations, not bytes
        achieved = d["alg_bytes"] / (d["total_ms"] / 1e3) / 1e12
        return {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "launches": d["launches"],
                "avg_launch_us": d["total_ms"] * 1e3 / d["launches"],
                "alg_flops_per_launch": d["alg_bytes"] / d["launches"]}, \
            {kname: v["total_ms"] / steps for kname, v in prof.items()}
    return _hbm_roofline(d, dom, None), {kname: v["total_ms"] / steps for kname, v in prof.items()}


def run_allsource(args, which):
    """Plain GUMAP C0 + C1 on one graph: all-source BFS with the uint8 hop
    matrix, (hop, id) kNN and membership (the 32 x 32 grid, or the dense ER
    graph the paper flags as costly)."""
    import numpy as np
    import torch

    import graphgen as G
    import paper_2509_19703_amd as gm
    k = args.k
    g = G.config_grid() if which == "grid" else G.config_er()
    n, m = g.n, g.m
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    ids = torch.empty((n, k), dtype=torch.int32, device="cuda")
    hops = torch.empty((n, k), dtype=torch.uint8, device="cuda")
    hm = torch.empty((n, n), dtype=torch.uint8, device="cuda")
    w = torch.empty((n, k), dtype=torch.float32, device="cuda")
    rho = torch.empty(n, dtype=torch.float32, device="cuda")
    sigma = torch.empty(n, dtype=torch.float32, device="cuda")
    gg = gm.make_graph(rp, ci, flags=gm.CSR_SORTED)
    stream = torch.cuda.current_stream()

    def step():
        gm.gumap_knn_build(gg, k, None, 0, ids, hops, hm, stream)
        gm.gumap_membership(n, k, hops, w, rho, sigma, stream)

    tune = None if args.no_tune else gm.gumap_knn_build_tune(gg, k, None, 0, ids, hops, hm, stream)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    dt, prof, dom = _profiled(gm, step, args.steps)
    roof, kms = _roofline(prof, args.steps, dom)
    out = {"metric": METRIC, "value": n * m / dt / 1e9, "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "%s: all-source BFS from all %d vertices with uint8 hop matrix, (hop,id) kNN "
                                  "k=%d, FP32 membership" % (g.name or which, n, k), "n": n, "m": m, "k": k},
           "roofline": roof, "kernels_ms_per_step": kms, "autotune": tune}
    if not args.no_parity:
        import oracle as O
        if which == "grid":
            oi, oh, ohm = O.knn_build(g, k, hop_matrix=True)
            ok = (np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(hops.cpu().numpy(), oh)
                  and np.array_equal(hm.cpu().numpy(), ohm))
            out["parity_sample"] = "every row against the oracle (ids, hops, hop matrix)"
        else:
            pick = np.arange(0, n, max(1, n // 64))
            oi, oh, ohm = O.knn_build(g, k, sources=pick, hop_matrix=True)
            pt = torch.from_numpy(pick).cuda()
            ok = (np.array_equal(ids[pt].cpu().numpy(), oi) and np.array_equal(hops[pt].cpu().numpy(), oh)
                  and np.array_equal(hm[pt].cpu().numpy(), ohm))
            # every row against the diameter-2 closed form: 0 on the diagonal,
            # 1 for an edge, 2 otherwise (the oracle's BFS certifies diameter 2
            # on the sampled rows)
            exp = torch.full((n, n), 2, dtype=torch.uint8, device="cuda")
            rows = torch.repeat_interleave(torch.arange(n, device="cuda"), rp[1:] - rp[:-1])
            exp[rows, ci.long()] = 1
            exp.fill_diagonal_(0)
            ok = ok and bool(torch.equal(exp, hm)) and int(ohm.max()) <= 2
            del exp
            out["parity_sample"] = ("%d rows against the oracle; every row against the closed form (1 if adjacent, "
                                    "else 2)" % len(pick))
        out["parity_sampled_bit_exact"] = bool(ok)
    if not args.no_cpu_baseline:
        import oracle as O
        threads = O.default_threads()
        if which == "grid":
            t_all = _timed(lambda: O.knn_build(g, k, hop_matrix=True, threads=threads))
            t_one = _timed(lambda: O.knn_build(g, k, hop_matrix=True, threads=1))
            sample = "oracle: all %d sources on all %d host threads, and on one thread" % (n, threads)
        else:
            sub = np.arange(0, n, 16, dtype=np.int32)
            one = np.arange(0, n, 256, dtype=np.int32)
            t_all = _timed(lambda: O.knn_build(g, k, sources=sub, hop_matrix=True, threads=threads)) * n / len(sub)
            t_one = _timed(lambda: O.knn_build(g, k, sources=one, hop_matrix=True, threads=1)) * n / len(one)
            sample = ("oracle: %d of the %d sources on all %d host threads, %d on one thread, each scaled to all "
                      "sources" % (len(sub), n, threads, len(one)))
        out["cpu_baseline"] = cpu_block(n * m / 1e9, "GTEPS", t_all, threads, t_one, sample)
    return out


def bench_stress(args):
    """Aggregated stress (Sec. 4.1.3) of a seeded random drawing of the BA graph
    over all ordered vertex pairs: the all-source BFS from every vertex with
    the stress terms folded into its hop-row pass."""
    import numpy as np
    import torch

    import graphgen as G
    import paper_2509_19703_amd as gm
    g = G.config_ba()
    n, m = g.n, g.m
    xy = (G.uniform(G.BASE_SEED + 300, 2 * n).reshape(n, 2) * 100.0).astype(np.float32)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    dxy = torch.from_numpy(xy).cuda()
    gg = gm.make_graph(rp, ci, flags=gm.CSR_SORTED)
    stream = torch.cuda.current_stream()
    res = {}

    def step():
        res["v"] = gm.gumap_stress(gg, dxy, None, 0, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 10))
    dt, prof, dom = _profiled(gm, step, steps)
    roof, kms = _roofline(prof, steps, dom)
    total, pairs = res["v"]
    out = {"metric": METRIC, "value": n * m / dt / 1e9, "unit": "GTEPS", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8+f64", "data": "synthetic",
           "config": {"workload": "stress: BA n=%d m=%d, seeded uniform drawing in [0, 100)^2; aggregated stress "
                                  "over all ordered pairs (all-source BFS, terms in FP64)" % (n, m),
                      "n": n, "m": m},
           "stress": total / pairs, "pairs": pairs, "pairs_per_s": pairs / dt,
           "roofline": roof, "kernels_ms_per_step": kms}
    if not args.no_parity:
        import oracle as O
        pick = G.sample_sources(n, 64, G.BASE_SEED + 301)
        gs, gp = gm.gumap_stress(gg, dxy, torch.from_numpy(pick).cuda(), len(pick), stream)
        os_, op = O.stress(g, xy, sources=pick)
        out["parity_sampled_pairs_exact"] = bool(gp == op)
        out["parity_sampled_sum_rel_diff"] = abs(gs - os_) / abs(os_)
    if not args.no_cpu_baseline:
        import oracle as O
        threads = O.default_threads()
        sub = G.sample_sources(n, 256, G.BASE_SEED + 302)
        t0 = time.perf_counter()
        O.stress(g, xy, sources=sub, threads=threads)
        t = (time.perf_counter() - t0) * n / len(sub)
        out["cpu_baseline"] = {"value": n * m / t / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
                               "sample": "oracle stress rows of 256 of the %d sources, scaled" % n}
    print(json.dumps(out), flush=True)


def bench_neighborhood(args):
    """Neighbourhood preservation (Sec. 4.1.3, r = 2) of a seeded random drawing
    of the BA graph, scored for its 4,096 sampled vertices."""
    import numpy as np
    import torch

    import graphgen as G
    import paper_2509_19703_amd as gm
    g = G.config_ba()
    n, m = g.n, g.m
    verts = G.config_ba_sources()
    xy = (G.uniform(G.BASE_SEED + 300, 2 * n).reshape(n, 2) * 100.0).astype(np.float32)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    dxy = torch.from_numpy(xy).cuda()
    dv = torch.from_numpy(verts).cuda()
    gg = gm.make_graph(rp, ci, flags=gm.CSR_SORTED)
    score = torch.empty(len(verts), dtype=torch.float64, device="cuda")
    ball = torch.empty(len(verts), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        gm.gumap_neighborhood(gg, dxy, 2, dv, len(verts), score, ball, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 10))
    dt, prof, dom = _profiled(gm, step, steps)
    roof, kms = _roofline(prof, steps, dom)
    sc = score.cpu().numpy()
    ok = ~np.isnan(sc)
    out = {"metric": METRIC, "value": len(verts) / dt, "unit": "scored vertices/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "neighborhood: BA n=%d m=%d, seeded uniform drawing in [0, 100)^2; "
                                  "neighbourhood preservation r=2 of the %d sampled vertices" % (n, m, len(verts)),
                      "n": n, "m": m, "vertices": len(verts), "r": 2},
           "np_mean": float(sc[ok].mean()), "np_sum": float(sc[ok].sum()), "mean_ball": float(ball.float().mean()),
           "roofline": roof, "kernels_ms_per_step": kms}
    if not args.no_parity:
        import oracle as O
        pick = np.arange(0, len(verts), 64)
        osc, oball = O.neighborhood_scores(g, xy, 2, vertices=verts[pick])
        out["parity_sampled_bit_exact"] = bool(np.array_equal(sc[pick], osc, equal_nan=True)
                                               and np.array_equal(ball.cpu().numpy()[pick], oball))
    if not args.no_cpu_baseline:
        import oracle as O
        threads = O.default_threads()
        sub = verts[:256]
        t0 = time.perf_counter()
        O.neighborhood_scores(g, xy, 2, vertices=sub, threads=threads)
        t = (time.perf_counter() - t0) * len(verts) / len(sub)
        out["cpu_baseline"] = {"value": len(verts) / t, "unit": "scored vertices/s", "cores": threads,
                               "kind": "oracle", "sample": "oracle scores of 256 of the %d vertices, scaled"
                               % len(verts)}
    print(json.dumps(out), flush=True)


def bench_layout(args):
    """SL-GUMAP's layout run on the BA graph (Alg. 3): partial BFS kNN and
    membership (k = 15), fuzzy union, the spectral initial drawing, shuffle
    of E_k and t GradSample iterations (Alg. 5, window floor(|E_k|^0.9),
    5 negative samples per edge).  GradSample's parity is checked from a
    seeded uniform drawing (the oracle takes no input from the device), the
    spectral drawing by its eigen-residual."""
    import numpy as np
    import torch

    import graphgen as G
    import paper_2509_19703_amd as gm
    g = G.config_ba()
    n, m_g, k, t = g.n, g.m, args.k, args.layout_iters
    xy0 = ((G.uniform(G.BASE_SEED + 400, 2 * n).reshape(n, 2) - 0.5) * 20.0).astype(np.float32)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    gg = gm.make_graph(rp, ci, flags=gm.CSR_SORTED)
    stream = torch.cuda.current_stream()
    ids = torch.empty((n, k), dtype=torch.int32, device="cuda")
    hops = torch.empty((n, k), dtype=torch.uint8, device="cuda")
    w = torch.empty((n, k), dtype=torch.float32, device="cuda")
    urp = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    ucol = torch.empty(2 * n * k, dtype=torch.int32, device="cuda")
    uval = torch.empty(2 * n * k, dtype=torch.float32, device="cuda")
    head = torch.empty(2 * n * k, dtype=torch.int32, device="cuda")
    tail = torch.empty(2 * n * k, dtype=torch.int32, device="cuda")
    ew = torch.empty(2 * n * k, dtype=torch.float32, device="cuda")
    xy0_d = torch.from_numpy(xy0).cuda()
    xy = torch.empty_like(xy0_d)
    xy_init = torch.empty_like(xy0_d)
    seed_shuffle, seed_neg = G.BASE_SEED + 401, G.BASE_SEED + 402
    res = {}

    sp_params = gm.gumap_spectral_params(0, 0, 0.0, G.BASE_SEED + 403)

    def step():
        gm.gumap_knn_partial(gg, k, ids, hops, stream)
        gm.gumap_membership(n, k, hops, w, None, None, stream)
        mm = gm.gumap_fuzzy_union(n, k, ids, w, urp, ucol, uval, 2 * n * k, stream)
        res["ev"], res["sp_steps"] = gm.gumap_spectral_layout(n, urp, ucol, uval, sp_params, xy, stream)
        xy_init.copy_(xy)
        gm.gumap_edge_shuffle(n, urp, ucol, uval, mm, seed_shuffle, head, tail, ew, stream)
        p = gm.layout_params(t=t, neg=5, samp=0.9, seed=seed_neg)
        gm.gumap_grad_sample(n, xy, mm, head, tail, ew, p, 0, t, stream)
        res["m"] = mm

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 10))
    dt, prof, dom = _profiled(gm, step, steps)
    roof, kms = _roofline(prof, steps, dom)
    mm = res["m"]
    s_win = int(np.floor(mm ** 0.9))
    samples = t * s_win
    out = {"metric": METRIC, "value": samples / dt, "unit": "edge samples/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64 (2^-32 fixed-point positions)", "data": "synthetic",
           "config": {"workload": "layout: BA n=%d m=%d; partial BFS kNN k=%d + membership + fuzzy union + "
                                  "spectral initial drawing + shuffle + %d GradSample iterations (window "
                                  "floor(|E_k|^0.9), 5 negative samples)" % (n, m_g, k, t),
                      "n": n, "m": m_g, "k": k, "edges_Ek": mm, "window": s_win, "iterations": t},
           "window_ms": kms.get("grad_window", 0.0) / t, "roofline": roof, "kernels_ms_per_step": kms}
    out["spectral_eigenvalues"] = list(res["ev"])
    out["spectral_lanczos_steps"] = res["sp_steps"]
    # quality (neighbourhood preservation, r = 2, the 4,096 sampled vertices):
    # a random drawing, the spectral drawing and the final layout
    verts = torch.from_numpy(G.config_ba_sources()).cuda()
    for name, d in (("random", xy0_d), ("spectral", xy_init), ("layout", xy)):
        sc, _ = gm.neighborhood(rp, ci, d, 2, verts, flags=gm.CSR_SORTED)
        out["np_mean_" + name] = float(torch.nanmean(sc))
    if not args.no_parity:
        # the spectral drawing: eigen-residual of each coordinate vector (host sparse products)
        import scipy.sparse as sp
        mm = res["m"]
        Wm = sp.csr_matrix((uval[:mm].cpu().numpy().astype(float), ucol[:mm].cpu().numpy(), urp.cpu().numpy()),
                           shape=(n, n))
        dg = np.asarray(Wm.sum(axis=1)).ravel()
        sm = sp.diags(1 / np.sqrt(dg))
        Lm = sp.identity(n) - sm @ Wm @ sm
        p0 = xy_init.cpu().numpy().astype(float)
        out["spectral_residuals"] = [float(np.linalg.norm(Lm @ (p0[:, c] / np.linalg.norm(p0[:, c]))
                                                          - res["ev"][c] * p0[:, c] / np.linalg.norm(p0[:, c])))
                                     for c in range(2)]
    if not args.no_parity or not args.no_cpu_baseline:
        import oracle as O
        threads = O.default_threads()
        t0 = time.perf_counter()
        oi, oh = O.knn_partial(g, k, threads=threads)
        ow, _, _ = O.membership(oh, threads=threads)
        orp, ocol, oval = O.fuzzy_union(oi, ow)
        eh, et, ew_ = O.edge_shuffle(orp, ocol, oval, seed_shuffle)
        t_prep = time.perf_counter() - t0
        few = 5
        t0 = time.perf_counter()
        oxy = O.grad_sample(n, eh, et, ew_, xy0, a=gm.UMAP_A, b=gm.UMAP_B, window=s_win, neg=5, t=t,
                            seed=seed_neg, it_begin=0, it_end=few)
        t_win = (time.perf_counter() - t0) / few
        if not args.no_parity:
            chk = xy0_d.clone()
            p = gm.layout_params(t=t, neg=5, samp=0.9, seed=seed_neg)
            gm.gumap_grad_sample(n, chk, mm, head, tail, ew, p, 0, few, stream)
            wxy = O.grad_sample_window(n, eh, et, ew_, xy0, a=gm.UMAP_A, b=gm.UMAP_B, window=s_win, neg=5, t=t,
                                       seed=seed_neg, it_begin=0, it_end=few, parts=gm.LAYOUT_DEFAULT_PARTS)
            out["parity_sampled_bit_exact"] = bool(
                len(ocol) == mm and np.array_equal(head[:mm].cpu().numpy(), eh)
                and np.array_equal(tail[:mm].cpu().numpy(), et) and np.array_equal(chk.cpu().numpy(), wxy))
            out["parity_sample"] = ("union + shuffled E_k, and the drawing after the first %d iterations from a "
                                    "seeded uniform drawing against the oracle of the device's synchronous "
                                    "parts (the serial order of Alg. 5 is checked by the tests)" % few)
        if not args.no_cpu_baseline:
            est = t_prep + t * t_win
            out["cpu_baseline"] = {"value": samples / est, "unit": "edge samples/s", "cores": threads,
                                   "kind": "oracle",
                                   "sample": "oracle kNN/membership/union/shuffle in full (%d threads) and %d of %d "
                                             "GradSample iterations in the serial order (one thread), scaled; the spectral drawing is "
                                             "left out (the oracle's dense eigendecomposition does not scale to "
                                             "n = 100,000); run estimate %.1f s" % (threads, few, t, est)}
    print(json.dumps(out), flush=True)


def bench_sparsify(args):
    """SS-GUMAP's front end on the dense ER graph G(16,384, 1/16) (the case
    the paper sparsifies for, Sec. 3.2): effective resistances (32 random
    projections, CG to 1e-8), the sparsified graph of ceil(n ln n) edges,
    and GUMAP's all-source BFS kNN (hop matrix, k = 15) and membership on it,
    against the same kNN on the whole graph."""
    import numpy as np
    import torch

    import graphgen as G
    import paper_2509_19703_amd as gm
    k = args.k
    g = G.config_er()
    n, m = g.n, g.m
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    gg = gm.make_graph(rp, ci, flags=gm.CSR_SORTED)
    stream = torch.cuda.current_stream()
    R = torch.empty(g.nnz // 2, dtype=torch.float64, device="cuda")
    srp = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    scol = torch.empty(g.nnz, dtype=torch.int32, device="cuda")
    ids = torch.empty((n, k), dtype=torch.int32, device="cuda")
    hops = torch.empty((n, k), dtype=torch.uint8, device="cuda")
    hm = torch.empty((n, n), dtype=torch.uint8, device="cuda")
    w = torch.empty((n, k), dtype=torch.float32, device="cuda")
    res = {}

    def sparsify():
        res["m"], res["its"] = gm.gumap_effective_resistance(gg, 32, G.BASE_SEED + 500, 1e-8, 1000, R, stream)
        res["snnz"] = gm.gumap_sparsify_select(gg, R, 0, srp, scol, stream)

    def knn(graph):
        gm.gumap_knn_build(graph, k, None, 0, ids, hops, hm, stream)
        gm.gumap_membership(n, k, hops, w, None, None, stream)

    def step():
        sparsify()
        knn(gm.gumap_graph(n, res["snnz"], gm._ptr(srp), gm._ptr(scol), gm.CSR_SORTED))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 10))
    dt, prof, dom = _profiled(gm, step, steps)
    roof, kms = _roofline(prof, steps, dom)
    t0 = time.perf_counter()
    for _ in range(steps):
        knn(gg)
    torch.cuda.synchronize()
    t_full = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        sparsify()
    torch.cuda.synchronize()
    t_sp = (time.perf_counter() - t0) / steps
    out = {"metric": METRIC, "value": m / t_sp / 1e9, "unit": "G input edges/s (sparsifier)", "n_gpus": 1,
           "steps": steps, "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64 (resistances), u8 (hops)", "data": "synthetic",
           "config": {"workload": "sparsify: ER G(%d, 1/16), m=%d; effective resistances (32 projections, CG to "
                                  "1e-8) + spectral sparsification to ceil(n ln n) edges + all-source BFS kNN "
                                  "k=%d with hop matrix + membership on the sparsified graph" % (n, m, k),
                      "n": n, "m": m, "k": k},
           "sparsified_edges": res["snnz"] // 2, "cg_iterations": res["its"], "sparsify_ms": t_sp * 1e3,
           "ss_gumap_ms": dt * 1e3, "gumap_full_graph_ms": t_full * 1e3,
           "roofline": roof, "kernels_ms_per_step": kms}
    if not args.no_parity:
        # Foster's theorem for the estimate, and the sparsified graph connected
        import scipy.sparse as sp
        from scipy.sparse.csgraph import connected_components
        Rn = R[:res["m"]].cpu().numpy()
        A = sp.csr_matrix((np.ones(res["snnz"]), scol[:res["snnz"]].cpu().numpy(), srp.cpu().numpy()), shape=(n, n))
        out["resistance_sum_over_n_minus_1"] = float(Rn.sum() / (n - 1))
        out["sparsified_connected"] = bool(connected_components(A)[0] == 1)
    if not args.no_cpu_baseline:
        import oracle as O
        q = 1
        t0 = time.perf_counter()
        O.effective_resistance(n, g.row_ptr, g.col_idx, q=q, seed=G.BASE_SEED + 500, tol=1e-8, max_iters=1000)
        t1 = (time.perf_counter() - t0) * 32 / q
        out["cpu_baseline"] = {"value": m / t1 / 1e9, "unit": "G input edges/s (sparsifier)", "cores": 1,
                               "kind": "oracle", "sample": "oracle resistances with 1 of the 32 projections "
                               "(numpy, one thread), scaled to 32; selection not included"}
    print(json.dumps(out), flush=True)


def run_batch(args):
    """Many uneven graphs: partial BFS kNN + membership for every vertex of
    every graph, as one persistent launch (captured plan) against the plain
    per-graph loop (two synchronous calls per graph)."""
    import ctypes

    import numpy as np
    import torch

    import graphgen as G
    import paper_2509_19703_amd as gm
    k = args.k
    t0 = time.perf_counter()
    graphs = G.config_batch_graphs(args.batch_graphs)
    t_gen = time.perf_counter() - t0
    pb = gm.PackedBatch(graphs)
    rows = pb.total_vertices
    voff, eoff = pb.vtx_offset_host, pb.edge_offset_host
    ids = torch.empty((rows, k), dtype=torch.int32, device="cuda")
    hops = torch.empty((rows, k), dtype=torch.uint8, device="cuda")
    w = torch.empty((rows, k), dtype=torch.float32, device="cuda")
    rho = torch.empty(rows, dtype=torch.float32, device="cuda")
    sigma = torch.empty(rows, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    # plain per-graph loop, arguments prepared up front
    plain_args = []
    for i, g in enumerate(graphs):
        gg = gm.gumap_graph(g.n, g.nnz, ctypes.c_void_p(pb.row_ptr.data_ptr() + 4 * int(voff[i] + i)),
                            ctypes.c_void_p(pb.col_idx.data_ptr() + 4 * int(eoff[i])) if g.nnz else None,
                            gm.CSR_SORTED)
        r0 = int(voff[i])
        plain_args.append((gg, g.n, ctypes.c_void_p(ids.data_ptr() + 4 * r0 * k),
                           ctypes.c_void_p(hops.data_ptr() + r0 * k), ctypes.c_void_p(w.data_ptr() + 4 * r0 * k),
                           ctypes.c_void_p(rho.data_ptr() + 4 * r0), ctypes.c_void_p(sigma.data_ptr() + 4 * r0)))
    lib = gm.lib

    def plain():
        for gg, n, pi, ph, pw, pr, ps in plain_args:
            st = lib.gumap_knn_partial(ctypes.byref(gg), k, pi, ph, sp)
            st |= lib.gumap_membership(n, k, ph, pw, pr, ps, sp)
            if st:
                raise gm.GumapError(st, gm.last_error())

    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ref = [t.cpu().numpy() for t in (ids, hops, w, rho, sigma)]
    for t in (ids, hops, w, rho, sigma):
        t.zero_()
    b = pb.struct()

    def batched():
        gm.gumap_knn_partial_batch(b, k, ids, hops, w, rho, sigma, stream)

    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    dt_batch, prof, dom = _profiled(gm, batched, args.steps)
    roof, kms = _roofline(prof, args.steps, dom)
    same_plain = all(np.array_equal(a, t.cpu().numpy()) for a, t in zip(ref, (ids, hops, w, rho, sigma)))
    plan = gm.BatchPlan(pb, k)
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    dt_plan = (time.perf_counter() - t0) / args.steps
    same_plan = all(np.array_equal(a, t.cpu().numpy()) for a, t in
                    zip(ref, (plan.ids, plan.hops, plan.weights, plan.rho, plan.sigma)))
    ng = len(graphs)
    best = min(dt_batch, dt_plan)
    out = {"metric": METRIC, "value": ng / best, "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": best * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u8+f64", "data": "synthetic",
           "config": {"workload": "batch%d: %d graphs, n log-uniform [256, 16384], mean degree U[4, 32], "
                                  "BA/RGG/SBM thirds; partial BFS kNN k=%d + FP32 membership for all %d rows"
                                  % (ng, ng, k, rows), "graphs": ng, "rows": rows, "nnz": pb.total_nnz, "k": k},
           "graphs_per_s_plain_loop": ng / t_plain, "speedup_vs_plain": t_plain / best,
           "ms_batched_call": dt_batch * 1e3, "ms_plan_replay": dt_plan * 1e3, "ms_plain_loop": t_plain * 1e3,
           "plan_autotune": plan.tuning(),
           "rows_per_s": rows / best, "roofline": roof, "kernels_ms_per_step": kms,
           "batched_equals_plain": bool(same_plain), "plan_equals_plain": bool(same_plan),
           "host_generation_s": t_gen}
    if not args.no_parity:
        import oracle as O
        ok = same_plain and same_plan
        wmax = 0.0
        for i in range(0, ng, max(1, ng // 32)):
            oi, oh = O.knn_partial(graphs[i], k)
            ow, orho, _ = O.membership(oh, k)
            r0, r1 = int(voff[i]), int(voff[i + 1])
            ok = ok and np.array_equal(ref[0][r0:r1], oi) and np.array_equal(ref[1][r0:r1], oh) \
                and np.array_equal(ref[3][r0:r1], orho)
            err = np.abs(ref[2][r0:r1].astype(np.float64) - ow) - (1e-5 * np.abs(ow) + 2.0**-126)
            wmax = max(wmax, float(err.max()) if err.size else 0.0)
        out["parity_sampled_bit_exact"] = bool(ok and wmax <= 0.0)
        out["parity_sample"] = ("ids, hops and rho bit-exact, weights within 1e-5 relative, on every row of %d of "
                                "the %d graphs; the batched call and the plan replay equal to the plain loop on "
                                "every row" % (len(range(0, ng, max(1, ng // 32))), ng))
    if not args.no_cpu_baseline:
        import oracle as O
        threads = O.default_threads()
        frac = args.cpu_one_thread_fraction

        def run(sel, th):
            for i in sel:
                _, oh = O.knn_partial(graphs[i], k, threads=th)
                O.membership(oh, k, threads=th)

        t_all = _timed(lambda: run(range(ng), threads))
        one = range(0, ng, frac)
        scale = sum(g.nnz + g.n for g in graphs) / max(1, sum(graphs[i].nnz + graphs[i].n for i in one))
        t_one = _timed(lambda: run(one, 1)) * scale
        out["cpu_baseline"] = cpu_block(ng, "graphs/s", t_all, threads, t_one,
                                        "oracle partial BFS + membership: all %d graphs on all %d host threads; every "
                                        "%dth graph on one thread, scaled by vertices + entries (x%.1f)"
                                        % (ng, threads, frac, scale))
    return out


def run_serve(args):
    """Served request stream: jobs (graph + k) arrive by a Poisson process at
    0.8 x the measured saturation rate; latency submit -> done per job.  Every
    job is a distinct graph of the stream's generator mix."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import graphgen as G
    import paper_2509_19703_amd as gm
    jobs = G.config_stream_jobs(args.serve_jobs)
    nj = len(jobs)
    warm = min(args.serve_warmup, nj // 2)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:   # the generators run in C, off the GIL
        graphs = list(ex.map(G.stream_job_graph, jobs))
    t_gen = time.perf_counter() - t0
    ks = [j["k"] for j in jobs]
    budget = int(args.serve_budget_gb * (1 << 30))
    server = gm.Server(budget)
    # warm-up burst (first launches load code objects), then a saturation
    # burst of distinct jobs submitted at once; rate from the server's clock
    for t in [server.submit(graphs[i].row_ptr, graphs[i].col_idx, ks[i]) for i in range(warm)]:
        server.wait(t, copy_results=False)
        server.release(t)
    sat_jobs = list(range(warm, min(nj, warm + 1024)))
    tk = [server.submit(graphs[i].row_ptr, graphs[i].col_idx, ks[i]) for i in sat_jobs]
    t_first = t_last = None
    for t in tk:
        r = server.wait(t, copy_results=False)
        server.release(t)
        t_first = r["t_submit_ns"] if t_first is None else min(t_first, r["t_submit_ns"])
        t_last = r["t_done_ns"] if t_last is None else max(t_last, r["t_done_ns"])
    sat_rate = len(tk) / ((t_last - t_first) / 1e9)
    rate = 0.8 * sat_rate
    # Poisson arrivals at `rate` over the whole stream (its first `warm` jobs
    # are left out of the statistics)
    gaps = -np.log1p(-G.uniform(G.BASE_SEED + 200, nj)) / rate
    arrivals = np.cumsum(gaps)
    tickets = [None] * nj
    check = set(np.linspace(warm, nj - 1, 8).astype(int).tolist()) if not args.no_parity else set()

    def submitter():
        start = time.perf_counter()
        for i in range(nj):
            delay = arrivals[i] - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            tickets[i] = server.submit(graphs[i].row_ptr, graphs[i].col_idx, ks[i])

    th = threading.Thread(target=submitter)
    t_start = time.perf_counter()
    th.start()
    lat = []
    first_sub = last_done = None
    kept = {}
    for i in range(nj):
        while tickets[i] is None:
            time.sleep(0.0002)
        r = server.wait(tickets[i], copy_results=(i in check))
        if r["status"] != gm.OK:
            raise RuntimeError("job %d failed: %d" % (i, r["status"]))
        if i >= warm:
            lat.append((r["t_done_ns"] - r["t_submit_ns"]) / 1e6)
            first_sub = r["t_submit_ns"] if first_sub is None else min(first_sub, r["t_submit_ns"])
            last_done = r["t_done_ns"] if last_done is None else max(last_done, r["t_done_ns"])
        if i in check:
            kept[i] = r
        server.release(tickets[i])
    th.join()
    t_total = time.perf_counter() - t_start
    stats = server.stats()
    server.close()
    lat = np.array(lat)
    measured = nj - warm
    out = {"metric": METRIC, "value": measured / ((last_done - first_sub) / 1e9), "unit": "graphs/s",
           "n_gpus": 1, "steps": nj, "warmup": warm, "ms_per_step": float(np.mean(lat)),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8+f64",
           "data": "synthetic",
           "config": {"workload": "stream: %d distinct jobs (first %d left out of the statistics), Poisson arrivals "
                                  "at 0.8x saturation (%.1f jobs/s), graphs BA/RGG/SBM n log-uniform [1e3, 2e5], "
                                  "degree U[4, 64], k in {10, 15, 30}; partial BFS kNN + FP32 membership per job; "
                                  "budget %.0f GB" % (nj, warm, rate, args.serve_budget_gb),
                      "jobs": nj, "rate_jobs_per_s": rate, "budget_bytes": budget,
                      "vertices": int(sum(g.n for g in graphs)), "nnz": int(sum(g.nnz for g in graphs))},
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "saturation_graphs_per_s": sat_rate, "saturation_jobs": len(sat_jobs), "iterations": stats["iterations"],
           "peak_resident_bytes": stats["peak_resident_bytes"], "wall_s": t_total, "host_generation_s": t_gen,
           "roofline": None,
           "roofline_note": "bound by host-device transfers (each job's CSR in, its rows out), not by a kernel"}
    # plain loop on the same GPU: copy in, two synchronous calls, copy out, per job
    plain = list(range(warm, min(nj, warm + 256)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in plain:
        drp = torch.from_numpy(graphs[i].row_ptr).cuda()
        dci = torch.from_numpy(graphs[i].col_idx).cuda()
        i_, h_ = gm.knn_partial(drp, dci, ks[i], flags=gm.CSR_SORTED)
        w_, r_, s_ = gm.membership(h_)
        i_.cpu(), h_.cpu(), w_.cpu(), r_.cpu(), s_.cpu()
    t_plain = (time.perf_counter() - t0) / len(plain)
    # the same plain calls with the graphs already resident and the results
    # left on the device: what the per-graph launches cost without transfers
    resident = [(torch.from_numpy(graphs[i].row_ptr).cuda(), torch.from_numpy(graphs[i].col_idx).cuda(), ks[i])
                for i in plain]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for drp, dci, k in resident:
        i_, h_ = gm.knn_partial(drp, dci, k, flags=gm.CSR_SORTED)
        gm.membership(h_)
    torch.cuda.synchronize()
    del resident
    out["graphs_per_s_plain_loop_resident"] = len(plain) / (time.perf_counter() - t0)
    out["graphs_per_s_plain_loop"] = 1.0 / t_plain
    out["speedup_vs_plain"] = out["saturation_graphs_per_s"] * t_plain
    out["speedup_vs_plain_at_rate"] = out["value"] * t_plain
    if not args.no_parity:
        import oracle as O
        ok = True
        for i, r in kept.items():
            oi, oh = O.knn_partial(graphs[i], ks[i])
            ow, orho, _ = O.membership(oh, ks[i])
            ok = ok and np.array_equal(r["ids"], oi) and np.array_equal(r["hops"], oh) \
                and np.array_equal(r["rho"], orho) \
                and bool(np.all(np.abs(r["weights"].astype(np.float64) - ow) <= 1e-5 * np.abs(ow) + 2.0**-126))
        out["parity_sampled_bit_exact"] = bool(ok)
        out["parity_sample"] = ("%d jobs spread over the stream, every row: ids, hops, rho bit-exact, weights "
                                "within 1e-5 relative" % len(kept))
    if not args.no_cpu_baseline:
        import oracle as O
        threads = O.default_threads()
        frac = args.cpu_one_thread_fraction
        sel = list(range(warm, min(nj, warm + 64)))

        def run(sel_, th):
            for i in sel_:
                _, oh = O.knn_partial(graphs[i], ks[i], threads=th)
                O.membership(oh, ks[i], threads=th)

        t_all = _timed(lambda: run(sel, threads))
        one = sel[::frac]
        scale = sum(graphs[i].nnz + graphs[i].n for i in sel) / max(1, sum(graphs[i].nnz + graphs[i].n for i in one))
        t_one = _timed(lambda: run(one, 1)) * scale
        out["cpu_baseline"] = cpu_block(len(sel), "graphs/s", t_all, threads, t_one,
                                        "oracle partial BFS + membership: %d jobs of the stream on all %d host "
                                        "threads; %d of them on one thread, scaled by vertices + entries (x%.1f)"
                                        % (len(sel), threads, len(one), scale))
    del graphs
    return out


def _counter_avg_kib(run_dir: str, kernel_substr: str):
    """Average counter value (KiB) per dispatch of the kernels whose name contains kernel_substr."""
    import csv
    import glob
    import sqlite3
    csvs = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if csvs:
        # one or more rows per dispatch: summed per dispatch, averaged over dispatches
        per = {}
        with open(csvs[0]) as f:
            for r in csv.DictReader(f):
                if kernel_substr in r["Kernel_Name"]:
                    per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        vals = list(per.values())
        return (sum(vals) / len(vals) if vals else None), len(vals)
    dbs = glob.glob(os.path.join(run_dir, "**", "*.db"), recursive=True)
    if not dbs:
        raise FileNotFoundError("no rocprofv3 output under %s" % run_dir)
    con = sqlite3.connect(dbs[0])
    rows = con.execute("select kernel_name, value from counters_collection").fetchall()
    vals = [v for name, v in rows if kernel_substr in name]
    return (sum(vals) / len(vals) if vals else None), len(vals)


def write_traffic(args):
    """HBM bytes per launch of the dominant kernel from FETCH_SIZE / WRITE_SIZE,
    each scaled by the reading of the same counter for a plain 1 GiB copy."""
    fetch, nf = _counter_avg_kib(args.traffic_from[0], args.traffic_kernel)
    write, nw = _counter_avg_kib(args.traffic_from[1], args.traffic_kernel)
    cf, _ = _counter_avg_kib(args.traffic_from[2], "copyBuffer")
    cw, _ = _counter_avg_kib(args.traffic_from[3], "copyBuffer")
    gib_kib = float(1 << 20)
    f_fetch = cf / gib_kib          # counter KiB per KiB the copy must read
    f_write = cw / gib_kib
    read_b = fetch * 1024.0 / f_fetch
    write_b = write * 1024.0 / f_write
    name = {"msbfs_level_kernel": "msbfs_level"}.get(args.traffic_kernel, args.traffic_kernel)
    out = {"kernel": name, "counter_kernel": args.traffic_kernel, "source_sha": kernel_source_sha(),
           "fetch_kib_per_launch": fetch, "write_kib_per_launch": write, "launches": [nf, nw],
           "copy_fetch_factor": f_fetch, "copy_write_factor": f_write,
           "hbm_read_bytes_per_launch": read_b, "hbm_write_bytes_per_launch": write_b,
           "hbm_bytes_per_launch": read_b + write_b}
    with open(args.traffic_json, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def kernel_source_sha() -> str:
    """Hash of the sources of the BFS level kernel and of the host code that
    picks its launch configuration (the stored counter readings are for that
    kernel), so they go stale when either changes."""
    import hashlib
    h = hashlib.sha256()
    for name in ("msbfs.hip", "kernels.h", "device.h", "api.hip"):
        with open(os.path.join(ROOT, "paper_2509_19703_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline_ba(g, src, k, m, frac):
    """The oracle (as it stands) on the whole headline step with all host
    cores (all-source BFS with the hop matrix and kNN from the 4,096 sources,
    partial BFS and membership on all rows), and on one thread over 1/frac of
    the sources and rows, scaled."""
    import numpy as np
    import oracle as O
    threads = O.default_threads()

    def step(sources, rows, th):
        O.knn_build(g, k, sources=sources, hop_matrix=True, threads=th)
        _, ph = O.knn_partial(g, k, sources=rows, threads=th)
        O.membership(ph, k, threads=th)

    t_all = _timed(lambda: step(src, None, threads))
    sub = src[:max(1, len(src) // frac)]
    rows = np.arange(0, g.n, frac, dtype=np.int32)
    t_one = _timed(lambda: step(sub, rows, 1)) * frac
    return cpu_block(len(src) * m / 1e9, "GTEPS", t_all, threads, t_one,
                     "oracle: the whole step on all %d host threads; one thread on %d of the %d sources and every "
                     "%dth row, scaled x%d" % (threads, len(sub), len(src), frac, frac))


if __name__ == "__main__":
    main()
