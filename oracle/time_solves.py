"""Wall-clock time of the FP64 oracle's PolyCLEAN solves on the host cores
(a reported baseline, not a target): the plain workload (3,968 visibilities
of 32 antennas, 128^2, 50 Frank-Wolfe iterations) and the LOFAR-like
workload (424,800 visibilities, 1024^2, stop at relative duality gap 1e-4),
both in full.  Inputs come from the seeded generator and the oracle's own
forward operator.  Prints one JSON line; run as `python -m oracle.time_solves`
from the repository root.  Test infrastructure: nothing in the product path
runs it."""
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import sim  # noqa: E402
from oracle import operator, solver  # noqa: E402


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        return os.cpu_count() or 1


def time_solve(p, **kw):
    vclean = operator.forward(p.uv, p.npix, p.fov_rad, p.sky_pix, p.sky_amp)
    vis = sim.add_noise(vclean, p.noise, p.psnr_db).astype(np.complex64).astype(np.complex128)
    t = time.perf_counter()
    r = solver.pfw_solve(p.uv, p.npix, p.fov_rad, vis, **kw)
    dt = time.perf_counter() - t
    return {"workload": p.name, "nvis": p.nvis, "npix": p.npix, "seconds": dt, "iters": r.iters,
            "natoms": int(r.pix.size), "objective": r.objective, "rel_gap": r.rel_gap,
            "converged": bool(r.converged)}


def main():
    which = sys.argv[1:] or ["c1", "c2"]
    out = {"cpu": cpu_model(), "threads": threads(), "solves": []}
    if "c1" in which:
        p = sim.config_c1()
        out["solves"].append(time_solve(p, alpha=p.alpha, delta=p.delta, max_iter=p.max_iter))
        print(json.dumps(out["solves"][-1]), file=sys.stderr, flush=True)
    if "c2" in which:
        p = sim.config_c2()
        out["solves"].append(time_solve(p, alpha=p.alpha, delta=p.delta, max_iter=p.max_iter,
                                        rel_gap_tol=p.rel_gap_tol))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
