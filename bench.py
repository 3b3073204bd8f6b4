"""Benchmark of the BFS-kNN hot path on one MI355X.

One step = the whole hot path over the Barabasi-Albert workload (n = 100,000,
4 edges per new vertex, m = 399,990; seeded synthetic input standing in for
the paper's scale-free graphs):
  1. CSR ingest: canonicalise the input CSR (its rows arrive unsorted);
  2. all-source BFS hop distances from 4,096 seeded sample sources, written as
     a uint8 hop matrix (409.6 MB), and the (hop, id) kNN of those rows, k = 15;
  3. truncated partial BFS kNN from all 100,000 vertices, k = 15;
  4. UMAP membership weights of those 100,000 rows.
value = Graph500-convention GTEPS of the step: 4,096 sources x m undirected
edges (the graph is connected) divided by the whole step's time.

Prints one JSON line.  --gpus > 1 is refused (one-GPU build).
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
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--k", type=int, default=15)
    p.add_argument("--sources", type=int, default=4096)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-parity", action="store_true")
    p.add_argument("--cpu-sample-sources", type=int, default=1024)
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
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import graphgen as G
    import paper_2509_19703_amd as gm

    if args.calibrate_copy:
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
        return

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

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: the K steps, with the library's per-launch HIP events on
    gm.profile_reset()
    gm.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    gm.profile_enable(False)
    prof = gm.profile_entries()
    # the same K steps without events, for the event overhead
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt_plain = (time.perf_counter() - t1) / args.steps
    teps = len(src) * m / dt
    dom = max(prof, key=lambda kname: prof[kname]["total_ms"])
    d = prof[dom]
    achieved = d["alg_bytes"] / (d["total_ms"] / 1e3) / 1e9
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
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "launches": d["launches"], "avg_launch_us": d["total_ms"] * 1e3 / d["launches"],
                     "alg_bytes_per_launch": d["alg_bytes"] / d["launches"]},
        "kernels_ms_per_step": {kname: v["total_ms"] / args.steps for kname, v in prof.items()},
        "ms_per_step_without_events": dt_plain * 1e3,
        "knn_graphs_per_s": 1.0 / dt,
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
        out["cpu_baseline"] = cpu_baseline(g, src, k, m, args.cpu_sample_sources)
    print(json.dumps(out), flush=True)


def _counter_avg_kib(run_dir: str, kernel_substr: str):
    """Average counter value (KiB) per dispatch of the kernels whose name contains kernel_substr."""
    import glob
    import sqlite3
    dbs = glob.glob(os.path.join(run_dir, "**", "*.db"), recursive=True)
    if not dbs:
        raise FileNotFoundError("no rocprofv3 database under %s" % run_dir)
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
    """Hash of the HIP sources, so stored counter readings go stale when a kernel changes."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2509_19703_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(g, src, k, m, sample_sources):
    """The oracle (as it stands) on a bounded sample of the same step, scaled
    to the whole step: all-source BFS + kNN from `sample_sources` of the
    sampled sources (time x len(src)/sample), partial BFS + membership on all
    rows."""
    import oracle as O
    threads = O.default_threads()
    sub = src[:sample_sources]
    t0 = time.perf_counter()
    O.knn_build(g, k, sources=sub, hop_matrix=True, threads=threads)
    t_build = (time.perf_counter() - t0) * len(src) / len(sub)
    t0 = time.perf_counter()
    _, ph = O.knn_partial(g, k, threads=threads)
    t_partial = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.membership(ph, k, threads=threads)
    t_memb = time.perf_counter() - t0
    t = t_build + t_partial + t_memb
    return {"value": len(src) * m / t / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": "oracle all-source BFS + kNN from %d of the %d sources (scaled x%.0f), partial BFS "
                      "+ membership on all %d rows; step estimate %.2f s" % (
                          len(sub), len(src), len(src) / len(sub), g.n, t),
            "seconds_per_step_est": t}


if __name__ == "__main__":
    main()
