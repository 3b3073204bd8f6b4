"""GPU parity of the batched persistent launch, its captured plan, and the
request server (alone vs in a mix), all against the CPU oracle."""
import os
import sys

import numpy as np
import pytest

import graphgen as G
import oracle as O

sys.path.insert(0, os.path.dirname(__file__))
from gpu_util import assert_weights_close, first_mismatch  # noqa: E402

pytestmark = pytest.mark.gpu


def _mix(count, n_hi=3000, seed=G.BASE_SEED + 3):
    return [G._family_graph(kd, n, d, s)
            for (kd, n, d, s) in G.config_batch_params(count, seed=seed, n_lo=20, n_hi=n_hi)]


def _oracle_rows(graphs, k):
    ids, hops = [], []
    for g in graphs:
        i, h = O.knn_partial(g, k)
        ids.append(i)
        hops.append(h)
    ids = np.concatenate(ids) if ids else np.zeros((0, k), np.int32)
    hops = np.concatenate(hops) if hops else np.zeros((0, k), np.uint8)
    w, rho, sigma = O.membership(hops, k)
    return ids, hops, w, rho, sigma


@pytest.mark.parametrize("k", [10, 15, 30, 40, 100])
def test_batch_matches_oracle(gumap, k):
    graphs = _mix(60)
    graphs += [G.empty(1), G.empty(3), G.path(2), G.star(5)]      # tiny graphs share chunks
    print("batch k=%d graphs=%d rows=%d" % (k, len(graphs), sum(g.n for g in graphs)), flush=True)
    pb = gumap.PackedBatch(graphs)
    ids, hops, w, rho, sigma = gumap.knn_partial_batch(pb, k)
    oi, oh, ow, orho, osig = _oracle_rows(graphs, k)
    assert np.array_equal(ids.cpu().numpy(), oi), first_mismatch(ids.cpu().numpy(), oi)
    assert np.array_equal(hops.cpu().numpy(), oh)
    assert_weights_close(w.cpu().numpy(), ow, rho.cpu().numpy(), orho, sigma.cpu().numpy(), osig)


def test_batch_unsorted_and_validated(gumap):
    graphs = _mix(30, n_hi=1500, seed=G.BASE_SEED + 33)
    dirty = [G.dirty(g, 100 + i) for i, g in enumerate(graphs)]
    pb = gumap.PackedBatch(dirty, flags=gumap.VALIDATE)
    ids, hops, w, rho, sigma = gumap.knn_partial_batch(pb, 15)
    oi, oh, ow, orho, osig = _oracle_rows(graphs, 15)
    assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(hops.cpu().numpy(), oh)
    assert_weights_close(w.cpu().numpy(), ow, rho.cpu().numpy(), orho, sigma.cpu().numpy(), osig)
    # a sorted batch that is validated takes the check-only path
    pb = gumap.PackedBatch(graphs, flags=gumap.VALIDATE | gumap.CSR_SORTED)
    ids2, hops2, *_ = gumap.knn_partial_batch(pb, 15)
    assert np.array_equal(ids2.cpu().numpy(), oi)


def test_batch_rejects_malformed(gumap):
    g = G.grid_2d(4, 4)
    bad = G.CSR(g.n, g.row_ptr.copy(), g.col_idx.copy())
    bad.col_idx[3] = 99                       # id outside its graph
    pb = gumap.PackedBatch([G.path(5), bad], flags=gumap.VALIDATE | gumap.CSR_SORTED)
    with pytest.raises(gumap.GumapError) as e:
        gumap.knn_partial_batch(pb, 5)
    assert e.value.status == gumap.EGRAPH


def test_batch_without_weights(gumap):
    graphs = _mix(20, n_hi=800, seed=G.BASE_SEED + 44)
    pb = gumap.PackedBatch(graphs)
    ids, hops, w, rho, sigma = gumap.knn_partial_batch(pb, 15, weights=False)
    oi, oh, *_ = _oracle_rows(graphs, 15)
    assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(hops.cpu().numpy(), oh)


def test_plan_replays_match_plain(gumap):
    import torch
    graphs = _mix(40, n_hi=2500, seed=G.BASE_SEED + 55)
    pb = gumap.PackedBatch(graphs)
    ref = gumap.knn_partial_batch(pb, 15)
    ref = [t.cpu().numpy() for t in ref]
    plan = gumap.BatchPlan(pb, 15)
    for rep in range(4):
        out = plan.launch()
        got = [t.cpu().numpy() for t in out]
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3])
        assert np.array_equal(got[4], ref[4])
        # eager work and a synchronisation between replays
        for t in out:
            t.zero_()
        gumap.knn_partial_batch(pb, 10)
        torch.cuda.synchronize()
    plan.close()


@pytest.mark.parametrize("k", [15, 40])
def test_plan_autotuner_pick_is_valid(gumap, k):
    """The tuner times every candidate on the batch; its pick is a valid
    configuration, no slower than the defaults, and the plan built with it
    gives the oracle's rows."""
    graphs = _mix(30, n_hi=3000, seed=G.BASE_SEED + 57 + k)
    pb = gumap.PackedBatch(graphs)
    plan = gumap.BatchPlan(pb, k)
    t = plan.tuning()
    valid_lanes = [l for l in (16, 32, 64) if k + 1 <= l] + [-1, 0]
    assert t["lanes"] in valid_lanes
    assert t["candidates"] >= 2 * len(valid_lanes) - 2
    assert 0 < t["best_ms"] <= t["default_ms"]
    ids, hops, w, rho, sigma = [x.cpu().numpy() for x in plan.launch()]
    plan.close()
    off = 0
    for g in graphs:
        oi, oh = O.knn_partial(g, k)
        assert np.array_equal(ids[off:off + g.n], oi) and np.array_equal(hops[off:off + g.n], oh)
        ow, orho, osig = O.membership(oh)
        assert_weights_close(w[off:off + g.n], ow, rho[off:off + g.n], orho, sigma[off:off + g.n], osig)
        off += g.n


@pytest.mark.parametrize("lanes,chunk", [("16", "16"), ("32", "64"), ("64", "32"), ("0", "8")])
def test_batch_launch_shape_invariance(gumap, monkeypatch, lanes, chunk):
    """Lanes per source and rows per grab change only the speed."""
    graphs = _mix(24, n_hi=2000, seed=G.BASE_SEED + 59)
    pb = gumap.PackedBatch(graphs)
    ref = [t.cpu().numpy() for t in gumap.knn_partial_batch(pb, 15)]
    monkeypatch.setenv("GUMAP_PARTIAL_LANES", lanes)
    monkeypatch.setenv("GUMAP_BATCH_CHUNK", chunk)
    got = [t.cpu().numpy() for t in gumap.knn_partial_batch(pb, 15)]
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_server_results_match_oracle_and_alone(gumap):
    jobs = G.config_stream_jobs(24, n_lo=200, n_hi=6000, d_lo=4, d_hi=40)
    graphs = [G.stream_job_graph(j) for j in jobs]
    with gumap.Server(4 << 30) as s:
        tickets = [s.submit(g.row_ptr, g.col_idx, j["k"]) for g, j in zip(graphs, jobs)]
        results = [s.wait(t, 60000) for t in tickets]
        st = s.stats()
    assert st["completed"] == len(jobs)
    for g, j, r in zip(graphs, jobs, results):
        assert r is not None and r["status"] == gumap.OK
        oi, oh = O.knn_partial(g, j["k"])
        ow, orho, osig = O.membership(oh)
        assert np.array_equal(r["ids"], oi) and np.array_equal(r["hops"], oh)
        assert_weights_close(r["weights"], ow, r["rho"], orho, r["sigma"], osig)
    # the same jobs one at a time on a fresh server: bit-identical
    with gumap.Server(4 << 30) as s:
        for g, j, r in list(zip(graphs, jobs, results))[:6]:
            t = s.submit(g.row_ptr, g.col_idx, j["k"])
            a = s.wait(t, 60000)
            assert np.array_equal(a["ids"], r["ids"]) and np.array_equal(a["hops"], r["hops"])
            assert np.array_equal(a["weights"], r["weights"])
            assert np.array_equal(a["rho"], r["rho"]) and np.array_equal(a["sigma"], r["sigma"])


def test_server_bad_job_fails_alone(gumap):
    good = [G.ba(3000, 4, 7), G.rgg(2000, 8, 8)]
    rp = np.array([0, 1, 1], dtype=np.int32)        # 0 -> 1 without 1 -> 0
    ci = np.array([1], dtype=np.int32)
    with gumap.Server(1 << 30) as s:
        t0 = s.submit(good[0].row_ptr, good[0].col_idx, 15)
        tb = s.submit(rp, ci, 3, flags=gumap.VALIDATE)
        t1 = s.submit(good[1].row_ptr, good[1].col_idx, 15)
        r0, rb, r1 = s.wait(t0, 60000), s.wait(tb, 60000), s.wait(t1, 60000)
    assert rb["status"] == gumap.EGRAPH
    assert r0["status"] == gumap.OK and r1["status"] == gumap.OK
    oi, oh = O.knn_partial(good[1], 15)
    assert np.array_equal(r1["ids"], oi)


def test_server_unsorted_jobs(gumap):
    g = G.sbm(4000, 12, 9)
    d = G.dirty(g, 10)
    with gumap.Server(1 << 30) as s:
        t = s.submit(d.row_ptr, d.col_idx, 15, flags=0)
        r = s.wait(t, 60000)
    oi, oh = O.knn_partial(g, 15)
    assert r["status"] == gumap.OK and np.array_equal(r["ids"], oi) and np.array_equal(r["hops"], oh)


def _sampled_rows(g, per_graph, seed):
    """First, last and seeded rows of a graph (sorted, unique)."""
    if g.n == 0:
        return np.zeros(0, np.int32)
    rng = np.random.default_rng(seed)
    pick = np.concatenate([[0, g.n - 1], rng.integers(0, g.n, per_graph)])
    return np.unique(pick).astype(np.int32)


def test_batch2048_full_size_sampled(gumap):
    """The batch workload at its full size (2,048 graphs, n log-uniform in
    [256, 16,384], mean degree U[4, 32], BA / RGG / SBM; 7.9 M rows, int64
    offsets): the batched call and the captured plan against the oracle on
    sampled rows of EVERY graph (ids, hops, rho bit-exact; weights to 1e-5)
    and against each other on every row."""
    k = 15
    graphs = G.config_batch_graphs(2048)
    pb = gumap.PackedBatch(graphs)
    print("batch2048 rows=%d nnz=%d" % (pb.total_vertices, pb.total_nnz), flush=True)
    got = [t.cpu().numpy() for t in gumap.knn_partial_batch(pb, k)]
    plan = gumap.BatchPlan(pb, k)
    rep = [t.cpu().numpy() for t in plan.launch()]
    plan.close()
    for a, b in zip(got, rep):
        assert np.array_equal(a, b)
    voff = pb.vtx_offset_host
    for i, g in enumerate(graphs):
        rows = _sampled_rows(g, 3, i)
        oi, oh = O.knn_partial(g, k, sources=rows)
        ow, orho, osig = O.membership(oh, k)
        r = int(voff[i]) + rows
        assert np.array_equal(got[0][r], oi) and np.array_equal(got[1][r], oh), "graph %d" % i
        assert_weights_close(got[2][r], ow, got[3][r], orho, got[4][r], osig)


def _stream_pick():
    """Jobs of the served stream's own generator: for each k in {10, 15, 30}
    the two largest graphs of its first 4,096 jobs, plus 18 seeded others."""
    jobs = G.config_stream_jobs(4096)
    pick = []
    for k in (10, 15, 30):
        with_k = sorted((j for j in jobs if j["k"] == k), key=lambda j: -j["n"])
        pick += with_k[:2]
    rng = np.random.default_rng(G.BASE_SEED + 205)
    for i in rng.choice(len(jobs), 18, replace=False):
        if jobs[i] not in pick:
            pick.append(jobs[i])
    return pick


def test_served_stream_full_size_mix_and_alone(gumap):
    """Jobs of the served workload at full size (n up to 2e5, degree up to
    64, k in {10, 15, 30}) submitted in waves while earlier ones run: every
    job equals the oracle (ids, hops, rho bit-exact, weights to 1e-5) and,
    for the largest of each k, the same job run alone on a fresh server."""
    jobs = _stream_pick()
    graphs = [G.stream_job_graph(j) for j in jobs]
    print("stream jobs: n max %d, total nnz %d" % (max(g.n for g in graphs), sum(g.nnz for g in graphs)),
          flush=True)
    assert max(g.n for g in graphs) > 150000
    results = {}
    with gumap.Server(64 << 30) as s:
        pending = []
        for w0 in range(0, len(jobs), 5):
            for i in range(w0, min(len(jobs), w0 + 5)):
                pending.append((i, s.submit(graphs[i].row_ptr, graphs[i].col_idx, jobs[i]["k"])))
            # collect the oldest half while the newer ones run
            while len(pending) > 4:
                i, t = pending.pop(0)
                results[i] = s.wait(t, 120000)
                s.release(t)
        for i, t in pending:
            results[i] = s.wait(t, 120000)
            s.release(t)
    for i, (g, j) in enumerate(zip(graphs, jobs)):
        r = results[i]
        assert r["status"] == gumap.OK
        oi, oh = O.knn_partial(g, j["k"])
        ow, orho, osig = O.membership(oh, j["k"])
        assert np.array_equal(r["ids"], oi) and np.array_equal(r["hops"], oh), "job %d" % i
        assert_weights_close(r["weights"], ow, r["rho"], orho, r["sigma"], osig)
    with gumap.Server(64 << 30) as s:
        for i in range(6):
            t = s.submit(graphs[i].row_ptr, graphs[i].col_idx, jobs[i]["k"])
            a = s.wait(t, 120000)
            for key in ("ids", "hops", "weights", "rho", "sigma"):
                assert np.array_equal(a[key], results[i][key]), (i, key)
            s.release(t)
