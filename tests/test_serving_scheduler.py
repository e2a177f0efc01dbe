"""Scheduler logic of the serving loop, with a fake device backend (no GPU):
admission by footprint under a memory budget, slot limit, arrival order,
rejection of jobs that can never fit, failure isolation and latency
bookkeeping."""
import threading
import time

import numpy as np
import pytest

from paper_2406_01342_amd.serving import ImagingRequest, Server, latency_summary, run_plain


class FakeBackend:
    """Each job takes `steps` steps of `dt` seconds; the footprint comes from
    the request's params.  Tracks the bytes and jobs in use."""

    def __init__(self, dt=0.002):
        self.dt = dt
        self.lock = threading.Lock()
        self.used = 0
        self.peak_used = 0
        self.running = 0
        self.peak_running = 0
        self.started = []

    def footprint(self, req):
        return int(req.params["fp"])

    def open(self, req):
        if req.params.get("fail_open"):
            raise RuntimeError("cannot open")
        with self.lock:
            self.used += req.params["fp"]
            self.running += 1
            self.peak_used = max(self.peak_used, self.used)
            self.peak_running = max(self.peak_running, self.running)
            self.started.append(req.rid)
        return {"req": req, "left": int(req.params.get("steps", 3))}

    def step(self, h):
        time.sleep(self.dt)
        if h["req"].params.get("fail_step"):
            raise RuntimeError("step failed")
        h["left"] -= 1
        return h["left"] <= 0

    def close(self, h):
        with self.lock:
            self.used -= h["req"].params["fp"]
            self.running -= 1
        return {"rid": h["req"].rid}

    def solve_plain(self, req):
        time.sleep(self.dt * int(req.params.get("steps", 3)))
        return {"rid": req.rid}


def req(rid, t, fp, steps=3, **kw):
    p = {"fp": fp, "steps": steps}
    p.update(kw)
    return ImagingRequest(rid, t, np.zeros((1, 2)), 16, 0.01, np.zeros(1, np.complex64), p)


def test_all_complete_and_results_match_requests():
    be = FakeBackend()
    srv = Server(be, slots=3)
    rs = [req(i, 0.0, 10) for i in range(10)]
    out = srv.run(rs)
    assert out["completed"] == 10 and out["rejected"] == 0 and out["failed"] == 0
    for rec in srv.records:
        assert rec.result == {"rid": rec.rid}
    assert out["peak_running"] <= 3 and be.peak_running <= 3
    assert out["peak_running"] == 3  # the slots were actually used together


def test_budget_bounds_device_bytes():
    be = FakeBackend()
    srv = Server(be, slots=8, hbm_budget=100)
    rs = [req(i, 0.0, fp) for i, fp in enumerate([60, 30, 50, 20, 70, 10, 40, 90])]
    out = srv.run(rs)
    assert out["completed"] == 8
    assert be.peak_used <= 100 and srv.peak_used <= 100


def test_oversized_job_rejected_others_served():
    be = FakeBackend()
    srv = Server(be, slots=2, hbm_budget=100)
    out = srv.run([req(0, 0.0, 50), req(1, 0.0, 101), req(2, 0.0, 50)])
    st = {r.rid: r.status for r in srv.records}
    assert st == {0: "done", 1: "rejected", 2: "done"}
    assert out["rejected"] == 1
    assert "exceeds the budget" in srv.records[1].error


def test_arrival_order_and_no_starvation():
    """A job that needs the whole budget is admitted before small jobs that
    arrive after it, although they would fit earlier."""
    be = FakeBackend(dt=0.003)
    srv = Server(be, slots=4, hbm_budget=100)
    rs = [req(0, 0.0, 40, steps=5), req(1, 0.0, 40, steps=5), req(2, 0.001, 100, steps=2)]
    rs += [req(3 + i, 0.002 + 0.0005 * i, 10) for i in range(6)]
    srv.run(rs)
    adm = {r.rid: r.admitted_s for r in srv.records}
    big = adm[2]
    assert all(adm[k] >= big for k in range(3, 9))
    # admission follows arrival order
    order = sorted(srv.records, key=lambda r: (r.arrival_s, r.rid))
    times = [r.admitted_s for r in order if r.status == "done"]
    assert times == sorted(times)


def test_arrivals_respected_and_latency_bookkeeping():
    be = FakeBackend(dt=0.002)
    srv = Server(be, slots=2)
    arr = [0.0, 0.01, 0.02, 0.05]
    rs = [req(i, t, 1, steps=2) for i, t in enumerate(arr)]
    out = srv.run(rs)
    for r in srv.records:
        assert r.admitted_s >= r.arrival_s - 1e-9
        assert r.finished_s >= r.admitted_s + 2 * 0.002 * 0.9
        assert r.latency_s == pytest.approx(r.finished_s - r.arrival_s)
    lat = np.array([r.latency_s for r in srv.records])
    assert out["p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert out["p99_s"] == pytest.approx(np.percentile(lat, 99))
    assert out["wall_s"] >= 0.05


def test_failed_job_does_not_stop_the_server():
    be = FakeBackend()
    srv = Server(be, slots=2, hbm_budget=50)
    out = srv.run([req(0, 0.0, 20), req(1, 0.0, 20, fail_step=True), req(2, 0.0, 20,
                                                                          fail_open=True),
                   req(3, 0.0, 50)])
    st = {r.rid: r.status for r in srv.records}
    assert st == {0: "done", 1: "failed", 2: "failed", 3: "done"}
    assert out["completed"] == 2 and out["failed"] == 2
    assert be.used == 0  # the failed step's job was closed


def test_plain_path_runs_one_at_a_time():
    be = FakeBackend(dt=0.002)
    summary, recs = run_plain(be, [req(i, 0.0, 1, steps=2) for i in range(4)])
    assert summary["completed"] == 4
    for a, b in zip(recs, recs[1:]):
        assert b.admitted_s >= a.finished_s
    assert latency_summary(recs, summary["wall_s"])["p99_s"] == summary["p99_s"]


def test_slots_validation():
    with pytest.raises(ValueError):
        Server(FakeBackend(), slots=0)
