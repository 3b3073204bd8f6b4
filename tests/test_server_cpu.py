"""Scheduler and admission logic of the request server, on the CPU
(GUMAP_SERVER_NO_DEVICE: no device work, results are zeros)."""
import time

import numpy as np
import pytest

import graphgen as G


def _server(gumap, budget, slots=0):
    return gumap.Server(budget, slots, gumap.SERVER_NO_DEVICE)


def test_submit_poll_release_roundtrip(gumap):
    g = G.grid_2d(6, 7)
    with _server(gumap, 1 << 30) as s:
        t = s.submit(g.row_ptr, g.col_idx, 5)
        r = s.wait(t, 5000)
        assert r is not None and r["status"] == gumap.OK
        assert r["ids"].shape == (42, 5) and r["weights"].shape == (42, 5)
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_start_ns"] <= r["t_done_ns"]
        assert s.release(t) == gumap.OK
        with pytest.raises(gumap.GumapError) as e:
            s.release(t)
        assert e.value.status == gumap.ENOTFOUND
        r = gumap.gumap_result()
        assert gumap.lib.gumap_poll(s._h, 12345, r) == gumap.ENOTFOUND


def test_job_larger_than_budget_is_rejected(gumap):
    g = G.ba(20000, 8, 3)
    with _server(gumap, 1 << 20) as s:
        with pytest.raises(gumap.GumapError) as e:
            s.submit(g.row_ptr, g.col_idx, 15)
        assert e.value.status == gumap.E2BIG
        small = G.path(10)
        t = s.submit(small.row_ptr, small.col_idx, 3)
        assert s.wait(t, 5000)["status"] == gumap.OK


def test_bad_job_arguments(gumap):
    g = G.path(10)
    with _server(gumap, 1 << 30) as s:
        for k in (0, 255):
            with pytest.raises(gumap.GumapError) as e:
                s.submit(g.row_ptr, g.col_idx, k)
            assert e.value.status == gumap.EINVAL
        with pytest.raises(gumap.GumapError):
            s.submit(g.row_ptr, g.col_idx, 3, flags=0x40)


def test_budget_forces_fifo_admission(gumap):
    """With room for about one job at a time, jobs are admitted in arrival order
    and never more bytes than the budget are resident."""
    gs = [G.ba(3000 + 100 * i, 4, 10 + i) for i in range(8)]
    with _server(gumap, 3 << 20, slots=0) as s:
        tickets = [s.submit(g.row_ptr, g.col_idx, 15) for g in gs]
        res = [s.wait(t, 10000) for t in tickets]
        assert all(r["status"] == gumap.OK for r in res)
        admits = [r["t_admit_ns"] for r in res]
        assert admits == sorted(admits)
        st = s.stats()
        assert st["peak_resident_bytes"] <= st["budget_bytes"]
        assert st["completed"] == 8 and st["submitted"] == 8


def test_slot_limit(gumap):
    gs = [G.path(50) for _ in range(6)]
    with _server(gumap, 1 << 30, slots=2) as s:
        tickets = [s.submit(g.row_ptr, g.col_idx, 4) for g in gs]
        for t in tickets:
            assert s.wait(t, 10000)["status"] == gumap.OK
        assert s.stats()["completed"] == 6


def test_empty_graph_job(gumap):
    with _server(gumap, 1 << 20) as s:
        t = s.submit(np.zeros(1, np.int32), np.zeros(0, np.int32), 4)
        r = s.wait(t, 5000)
        assert r["status"] == gumap.OK and r["n"] == 0


def test_destroy_with_jobs_in_flight(gumap):
    g = G.grid_2d(30, 30)
    s = _server(gumap, 1 << 30)
    for _ in range(50):
        s.submit(g.row_ptr, g.col_idx, 15)
    s.close()   # must return without waiting for a device
    s.close()


def test_executor_device_error_fails_only_its_jobs(gumap, monkeypatch):
    """The executor reports an iteration as failed (as a device error would):
    the jobs with rows in it end with EDEVICE, jobs of other iterations
    finish normally, and the server keeps serving."""
    monkeypatch.setenv("GUMAP_SERVE_NODEV_FAIL_ITER", "0")
    first = G.ba(2000, 4, 31)
    with _server(gumap, 1 << 30) as s:
        t0 = s.submit(first.row_ptr, first.col_idx, 15)
        r0 = s.wait(t0, 10000)
        assert r0["status"] == gumap.EDEVICE
        later = [G.ba(1500 + 10 * i, 4, 40 + i) for i in range(4)]
        ts = [s.submit(g.row_ptr, g.col_idx, 15) for g in later]
        rs = [s.wait(t, 10000) for t in ts]
        assert all(r["status"] == gumap.OK for r in rs)
        st = s.stats()
        assert st["failed"] == 1 and st["completed"] == 4
        for t in [t0] + ts:
            s.release(t)
