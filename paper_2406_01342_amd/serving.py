"""Continuous-batching server for imaging solves of different sizes.

A request carries its geometry (uv, grid, field of view), its visibilities
and its solve parameters.  The server keeps up to `slots` solves in flight,
each on a worker thread with a stream of its own; their per-iteration work
(candidate search, restricted APGD solve, residual) overlaps on the device,
and their full-grid adjoints go through one batcher, which merges the ones
that meet into shared launches.  A request is admitted, in arrival order,
once it has arrived, a slot is free and its device footprint (plan workspace
plus resident solver state) fits in the memory budget; one that can never fit
is rejected at once.  Head-of-line order means a large job is never passed by
later small ones (no starvation).  Each job's latency runs from its arrival
to its result.

The backend is pluggable: `DeviceBackend` drives the HIP library, and tests
substitute a fake one to check admission and bookkeeping without a device.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


def _n_scales(req) -> int:
    """Images per certificate: the dictionary's scale count, else one."""
    sc = req.params.get("scales")
    return len(sc[0]) if sc is not None else 1


@dataclass
class ImagingRequest:
    rid: int
    arrival_s: float            # offset from the start of the run
    uv: np.ndarray              # (L, 2) float64 wavelengths, caller order
    npix: int
    fov_rad: float
    vis: np.ndarray             # (L,) complex64, caller order
    params: Dict[str, float] = field(default_factory=dict)
    want_certificate: bool = False  # return the dual certificate image


@dataclass
class JobRecord:
    rid: int
    arrival_s: float
    admitted_s: float = float("nan")
    finished_s: float = float("nan")
    footprint: int = 0
    status: str = "pending"     # done | rejected | failed
    result: Optional[dict] = None
    error: str = ""

    @property
    def latency_s(self) -> float:
        return self.finished_s - self.arrival_s

    @property
    def wait_s(self) -> float:
        return self.admitted_s - self.arrival_s


def latency_summary(records: List[JobRecord], wall_s: float) -> dict:
    """p50 / p99 / mean latency and solves/s over the completed jobs."""
    lat = np.array([r.latency_s for r in records if r.status == "done"])
    wait = np.array([r.wait_s for r in records if r.status == "done"])
    done = int(lat.size)
    out = {"completed": done, "rejected": sum(r.status == "rejected" for r in records),
           "failed": sum(r.status == "failed" for r in records),
           "wall_s": wall_s, "solves_per_s": done / wall_s if wall_s > 0 else None}
    if done:
        out.update(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                   mean_s=float(lat.mean()), max_s=float(lat.max()),
                   mean_wait_s=float(wait.mean()))
    return out


class DeviceBackend:
    """Runs jobs through the HIP library on one device."""

    #: solver state resident per job beyond the plan: sorted visibilities and
    #: residual (2 x 8 L), dirty-residual image (4 n^2), with a dictionary the
    #: dense synthesis image (4 n^2) and the per-scale analysis (4 S n^2),
    #: caller-order upload (8 L) and a fixed allowance for candidate lists and
    #: atom tables
    FIXED_BYTES = 4 << 20

    def __init__(self, device: int = 0, batched: bool = True):
        import torch

        from . import api
        self.torch = torch
        self.api = api
        self.device = torch.device("cuda", device)
        self.batcher = api.Batcher(device) if batched else None

    def footprint(self, req: ImagingRequest) -> int:
        L = int(req.uv.shape[0])
        plan = self.api.pc_plan_footprint(req.uv, req.npix, req.fov_rad)
        S = _n_scales(req)
        cert = 4 * S * req.npix * req.npix if req.want_certificate else 0
        # the dirty residual, plus the synthesis image and the per-scale
        # analysis with a dictionary
        img = 4 * req.npix * req.npix * ((2 + S) if "scales" in req.params else 1)
        # solver arrays come in the device pool's size classes (<= 25 % more)
        return int(plan) + (5 * (24 * L + img)) // 4 + cert + self.FIXED_BYTES

    def _params(self, req: ImagingRequest) -> dict:
        prm = dict(req.params)
        if req.want_certificate:
            prm["want_certificate"] = 1
        return prm

    def open(self, req: ImagingRequest):
        torch = self.torch
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            plan = self.api.pc_plan_create(req.uv, req.npix, req.fov_rad, stream=stream)
            vis = torch.from_numpy(np.ascontiguousarray(req.vis, dtype=np.complex64)).to(
                self.device, non_blocking=False)
            solver = self.api.Solver(plan, vis, stream=stream, batcher=self.batcher,
                                     **self._params(req))
            del vis
        return {"plan": plan, "solver": solver, "stream": stream, "req": req}

    def step(self, h) -> bool:
        return h["solver"].step()

    def close(self, h) -> dict:
        req = h["req"]
        cert = None
        if req.want_certificate:
            with self.torch.cuda.stream(h["stream"]):
                cert = self.torch.empty((_n_scales(req), req.npix, req.npix),
                                        dtype=self.torch.float32,
                                        device=self.device)
        res = h["solver"].result(cert=cert)
        h["solver"].close()
        h["stream"].synchronize()
        h["plan"].close()
        if cert is not None:
            res["certificate"] = cert  # device image, mu = Phi*(V - Phi x) / lambda
        return res

    def solve_plain(self, req: ImagingRequest) -> dict:
        """The one-job-at-a-time path: plan, upload, pc_polyclean_solve."""
        torch = self.torch
        plan = self.api.pc_plan_create(req.uv, req.npix, req.fov_rad)
        vis = torch.from_numpy(np.ascontiguousarray(req.vis, dtype=np.complex64)).to(self.device)
        cert = None
        if req.want_certificate:
            cert = torch.empty((_n_scales(req), req.npix, req.npix), dtype=torch.float32,
                               device=self.device)
        res = self.api.pc_polyclean_solve(plan, vis, cert=cert, **self._params(req))
        if cert is not None:
            res["certificate"] = cert
        plan.close()
        return res

    def stats(self) -> dict:
        return self.batcher.stats() if self.batcher is not None else {}

    def close_backend(self):
        if self.batcher is not None:
            self.batcher.close()
            self.batcher = None


class Server:
    """Admission, worker slots and latency bookkeeping (see module doc)."""

    def __init__(self, backend, slots: int = 8, hbm_budget: Optional[int] = None,
                 clock: Callable[[], float] = time.perf_counter):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.backend = backend
        self.slots = slots
        self.budget = hbm_budget
        self.clock = clock
        self._cv = threading.Condition()
        self._queue: List[JobRecord] = []
        self._req: Dict[int, ImagingRequest] = {}
        self._used = 0
        self.peak_used = 0
        self.peak_running = 0
        self._running = 0
        self._closed = False
        self.records: List[JobRecord] = []
        self._t0 = 0.0

    def _now(self) -> float:
        return self.clock() - self._t0

    def _next(self) -> Optional[JobRecord]:
        with self._cv:
            while True:
                if not self._queue:
                    if self._closed:
                        return None
                    self._cv.wait()
                    continue
                rec = self._queue[0]
                if self.budget is not None and rec.footprint > self.budget:
                    self._queue.pop(0)
                    rec.status = "rejected"
                    rec.error = f"footprint {rec.footprint} B exceeds the budget {self.budget} B"
                    rec.admitted_s = rec.finished_s = self._now()
                    continue
                t = self._now()
                if rec.arrival_s > t:
                    self._cv.wait(timeout=rec.arrival_s - t)
                    continue
                if self.budget is not None and self._used + rec.footprint > self.budget:
                    self._cv.wait()
                    continue
                self._queue.pop(0)
                self._used += rec.footprint
                self._running += 1
                self.peak_used = max(self.peak_used, self._used)
                self.peak_running = max(self.peak_running, self._running)
                rec.admitted_s = t
                return rec

    def _release(self, rec: JobRecord):
        with self._cv:
            self._used -= rec.footprint
            self._running -= 1
            self._cv.notify_all()

    def _worker(self):
        while True:
            rec = self._next()
            if rec is None:
                return
            req = self._req.pop(rec.rid)
            h = None
            try:
                h = self.backend.open(req)
                while not self.backend.step(h):
                    pass
                rec.result = self.backend.close(h)
                h = None
                rec.status = "done"
            except Exception as e:  # the job fails, the server goes on
                rec.status = "failed"
                rec.error = repr(e)
                if h is not None:
                    try:
                        self.backend.close(h)
                    except Exception:
                        pass
            rec.finished_s = self._now()
            self._release(rec)

    def run(self, requests: List[ImagingRequest]) -> dict:
        """Replays `requests` in real time (arrival offsets from now) and
        returns the latency summary; per-job records are in `records`."""
        reqs = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        self.records = [JobRecord(r.rid, r.arrival_s, footprint=self.backend.footprint(r))
                        for r in reqs]
        self._req = {r.rid: r for r in reqs}
        self._queue = list(self.records)
        self._closed = True
        self._used = self._running = self.peak_used = self.peak_running = 0
        self._t0 = self.clock()
        threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(self.slots)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        wall = self._now()
        out = latency_summary(self.records, wall)
        out.update(slots=self.slots, peak_running=self.peak_running, peak_bytes=self.peak_used)
        return out


def run_plain(backend, requests: List[ImagingRequest],
              clock: Callable[[], float] = time.perf_counter) -> (dict, List[JobRecord]):
    """One job at a time in arrival order on the calling thread (the plain
    path), replayed in real time like Server.run."""
    reqs = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
    recs = []
    t0 = clock()
    for r in reqs:
        wait = r.arrival_s - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        rec = JobRecord(r.rid, r.arrival_s)
        rec.admitted_s = clock() - t0
        try:
            rec.result = backend.solve_plain(r)
            rec.status = "done"
        except Exception as e:
            rec.status = "failed"
            rec.error = repr(e)
        rec.finished_s = clock() - t0
        recs.append(rec)
    wall = clock() - t0
    return latency_summary(recs, wall), recs
