#!/usr/bin/env python3
"""Benchmark: PolyCLEAN on the memory-pressure large job (one MI355X).

A step is one full PolyCLEAN solve (Alg. 2: dirty image, polyatomic
exploration, restricted APGD, pruning, full-grid residual adjoint each
iteration, stopping test, dual certificate returned) of the largest
single-GPU workload: 512 stations (SKA-low-like core and arms, 40 km), 16
snapshots x 4 channels (120-180 MHz) stacked -> 8,372,224 complex64
visibilities, 8192^2 image (16384^2 fine grid), FOV 3 deg, 200 log-normal
point sources at 20 dB, lambda = 0.05 lambda_max, stop at relative objective
change 1e-4.  Inputs are synthesised from the seeded generator and resident
in HBM before timing; the plan is built once, outside the timed region, and
its build time is reported separately.

value = adjoint throughput in Mvis/s: visibilities gridded per second of
device time of the gridded adjoint (spread, fold, two FFT passes, correction
and maximum), measured with HIP events by the library around every
full-grid adjoint of the timed solves.  The line also carries the adjoint's
dominant kernel against the HBM roofline, the other workloads (LOFAR-like
solves in Gram and operator form, the precision workload's adjoint), the
direct-DFT pair rates (M2), the serving legs and the FP64 oracle timed on the
host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "adjoint Mvis/s (%HBM roofline); solves/s + p50/p99 latency vs plain @1e-4"
HBM_PEAK_GBS = 8000.0
# Direct-DFT pair-rate ceiling of the vector ALUs: 256 CUs x 2.4 GHz x 128
# FP32 lanes = 78.6e12 FP32 lane-slots/s; one visibility-atom pair costs about
# 19 slots (FP64 multiply and FMA for the phase at half rate, FP64 round and
# subtract, FP64->FP32 convert, sin and cos at quarter rate, two FP32 FMA).
DFT_PEAK_GPAIRS = 78.6e3 / 19.0
# The one-pass forward + restricted adjoint uses each pair's sin/cos twice: the
# same 19 slots plus two FP32 FMAs for the adjoint's accumulation.
FUSED_PEAK_GPAIRS = 78.6e3 / 21.0
# The point-spread sums (unit visibilities) need only the cosine and one FMA:
# 19 - 4 (sin) - 1 (FMA) = 14 slots per pair.
PSF_PEAK_GPAIRS = 78.6e3 / 14.0
# Source files each kernel is compiled from (with the shared headers): a
# stored HBM-traffic figure is used only while these are unchanged.
CSRC = os.path.join(ROOT, "paper_2406_01342_amd", "csrc")
KERNEL_FILES = {
    "adjoint_sparse": ["kernels_dft.hip"], "adjoint_sparse_reduce": ["kernels_dft.hip"],
    "forward_sparse": ["kernels_dft.hip"], "forward_adjoint_sparse": ["kernels_dft.hip"],
    "adjoint_sparse_acc64": ["kernels_dft.hip"], "psf_sums_acc64": ["kernels_dft.hip"],
    "spread": ["kernels_grid.hip", "fft_lds.h"], "fold": ["kernels_grid.hip", "fft_lds.h"],
    "passA_adj": ["kernels_grid.hip", "fft_lds.h"], "passB_adj": ["kernels_grid.hip", "fft_lds.h"],
    "dict_analysis": ["kernels_dict.hip"],
}
# kernel name in the library's statistics -> substring of its symbol
KERNEL_SYMBOLS = {
    "adjoint_sparse": "adjoint_sparse_kernel<float, float, false, false>",
    "forward_sparse": "forward_sparse_kernel<float, false>",
    "adjoint_sparse_reduce": "adjoint_sparse_reduce_kernel<float, float>",
    "forward_adjoint_sparse": "forward_adjoint_kernel<",
    "adjoint_sparse_acc64": "adjoint_sparse_kernel<float, double, false, false>",
    "psf_sums_acc64": "adjoint_sparse_kernel<float, double, true, false>",
    "spread": "spread_quad_kernel<", "fold": "fold_kernel<float>",
    "passA_adj": "passA_adj_kernel<float", "passB_adj": "passB_adj_kernel<float",
    "dict_analysis": "dict_tile_h_kernel<16>",  # the widest of the paper's scales (sigma 8)
}
PROFILES = os.path.join(ROOT, "profiles")
COPY_PROBE_BYTES = 512 << 20


def kernel_source_hash(name):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_FILES.get(name, []) + ["common.h"]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(name):
    """HBM bytes per launch of `name` from the committed counter summary, or
    None when there is none or the kernel's sources changed since."""
    path = os.path.join(PROFILES, f"traffic_{name}.json")
    if name not in KERNEL_FILES or not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_sha256") != kernel_source_hash(name):
        return None
    return d["traffic_bytes_per_launch"]


def copy_probe(torch):
    """One plain device copy of COPY_PROBE_BYTES, the reference dispatch for
    scaling the FETCH_SIZE / WRITE_SIZE counters to bytes.  The destination
    is filled after the source, so that none of the source is still in the
    L2 caches when the copy reads it."""
    a = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def summarize_pmc(kernel, fetch_dir, write_dir, command):
    """Writes profiles/traffic_<kernel>.json from a FETCH_SIZE run and a
    WRITE_SIZE run of the same command (KiB per dispatch, scaled by the copy
    probe's reading of the same counter)."""
    sym = KERNEL_SYMBOLS[kernel]
    out = {"kernel": kernel, "symbol": sym, "command": command,
           "copy_probe_bytes": COPY_PROBE_BYTES}
    for ctr, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r["Counter_Name"] == ctr]
        kv = [float(r["Counter_Value"]) for r in rows if sym in r["Kernel_Name"]]
        cp = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
              or "copy" in r["Kernel_Name"].lower()]
        if not kv or not cp:
            raise SystemExit(f"{ctr}: no dispatches of {sym} or of the copy probe in {d}")
        probe = max(cp)
        factor = COPY_PROBE_BYTES / (probe * 1024.0)
        out[ctr.lower() + "_kib_per_dispatch"] = sum(kv) / len(kv)
        out[ctr.lower() + "_dispatches"] = len(kv)
        out[ctr.lower() + "_copy_probe_kib"] = probe
        out[ctr.lower() + "_scale"] = factor
    out["traffic_bytes_per_launch"] = 1024.0 * (
        out["fetch_size_kib_per_dispatch"] * out["fetch_size_scale"] +
        out["write_size_kib_per_dispatch"] * out["write_size_scale"])
    out["source_sha256"] = kernel_source_hash(kernel)
    os.makedirs(PROFILES, exist_ok=True)
    with open(os.path.join(PROFILES, f"traffic_{kernel}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def summarize_counters(pmc_dirs, out_name, command, top=8):
    """Writes a short text table of per-dispatch means of every counter found
    in rocprofv3 --pmc runs (several directories: one per counter pass) for
    the kernels with the most dispatch time."""
    import collections
    sums = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in pmc_dirs:
        for r in _counter_rows(d):
            sums[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted(sums, key=lambda k: -sum(len(v) for v in sums[k].values()))
    ctrs = sorted({c for k in sums for c in sums[k]})
    lines = ["# rocprofv3 counters, mean per dispatch", f"# command: {command}", ""]
    keep = [k for k in names if any(s_ in k for s_ in KERNEL_SYMBOLS.values())][:top]
    for k in keep:
        short = k if len(k) <= 90 else k[:87] + "..."
        lines.append(short)
        for c in ctrs:
            v = sums[k].get(c)
            if v:
                lines.append(f"    {c:28s} {sum(v) / len(v):16.1f}   ({len(v)} dispatches)")
    os.makedirs(PROFILES, exist_ok=True)
    with open(os.path.join(PROFILES, out_name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_trace(trace_dir, out_name, command, top=14):
    """Writes a short text summary of a rocprofv3 --kernel-trace --stats run."""
    import csv
    import glob
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no kernel_stats.csv under {trace_dir}")
    with open(f[0]) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics", f"# command: {command}", "",
             f"{'kernel':64s} {'calls':>7s} {'total_us':>11s} {'avg_us':>9s} {'pct':>6s}"]
    for r in rows[:top]:
        name = r["Name"]
        name = name if len(name) <= 64 else name[:61] + "..."
        lines.append(f"{name:64s} {int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e3:11.1f} "
                     f"{float(r['AverageNs']) / 1e3:9.2f} {float(r['Percentage']):6.2f}")
    os.makedirs(PROFILES, exist_ok=True)
    with open(os.path.join(PROFILES, out_name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--adjoint-reps", type=int, default=50)
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests of the serving trace (0 skips the serving leg)")
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the adjoint measurements at the 4096^2 and 8192^2 workloads")
    ap.add_argument("--dictionary-only", action="store_true",
                    help="run only the synthesis-dictionary adjoint at 4096^2 and print its JSON")
    ap.add_argument("--w-only", action="store_true",
                    help="only the non-coplanar LOFAR-like leg (w-stacked adjoint, solve)")
    ap.add_argument("--adjoint-only", choices=("c2", "c3", "c5l"),
                    help="run only the gridded adjoint (caller-order input) at one workload, "
                         "--adjoint-reps times after 3 warm-up calls, and print its JSON "
                         "(for profiler runs)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("KERNEL", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic_KERNEL.json from two rocprofv3 --pmc runs")
    ap.add_argument("--summarize-counters", nargs="+", metavar="ARG",
                    help="OUT_NAME PMC_DIR...: write profiles/OUT_NAME from rocprofv3 --pmc runs")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DIR", "OUT_NAME"),
                    help="write profiles/OUT_NAME from a rocprofv3 --kernel-trace --stats run")
    ap.add_argument("--command", default="", help="the profiled command, recorded in summaries")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def synth_inputs(api, torch, p):
    """Noisy visibilities of the sky: forward of the sky atoms on the GPU plus
    the generator's noise draw scaled to the PSNR (input synthesis only)."""
    import numpy as np
    import sim
    plan = api.pc_plan_create(p.uv[:, :2], p.npix, p.fov_rad,
                              w=p.uv[:, 2] if p.uv.shape[1] > 2 else None)
    pix = torch.from_numpy(p.sky_pix.astype(np.int32)).cuda()
    amp = torch.from_numpy(p.sky_amp.astype(np.float32)).cuda()
    vclean = api.pc_forward_sparse(plan, pix, amp).cpu().numpy().astype(np.complex128)
    vis = sim.add_noise(vclean, p.noise, p.psnr_db).astype(np.complex64)
    return plan, vis


def dominant_roofline(stats, plan_info):
    """Roofline object for the kernel with the largest device time."""
    top = max(stats, key=lambda s: s["ms"])
    avg_ms = top["ms"] / top["launches"]
    name = top["name"]
    if name in ("forward_sparse", "adjoint_sparse", "forward_adjoint_sparse",
                "adjoint_sparse_acc64", "psf_sums_acc64"):
        pairs = top["work"] / top["launches"]
        achieved = pairs / (avg_ms * 1e-3) / 1e9
        peak = {"forward_adjoint_sparse": FUSED_PEAK_GPAIRS,
                "psf_sums_acc64": PSF_PEAK_GPAIRS}.get(name, DFT_PEAK_GPAIRS)
        return {"kernel": name, "bound": "alu", "achieved": achieved,
                "peak": peak, "unit": "Gpair/s",
                "frac": achieved / peak,
                "traffic": stored_traffic(name), "avg_ms": avg_ms, "launches": top["launches"],
                "work_per_launch": pairs}
    b = top["bytes"] / top["launches"]
    achieved = b / (avg_ms * 1e-3) / 1e9
    # single-workgroup solver steps are bound by latency, not by a unit's peak
    bound = "latency" if name in ("gram_fista", "gram_lanczos", "lanczos_step") else "hbm"
    return {"kernel": name, "bound": bound, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(name),
            "avg_ms": avg_ms, "launches": top["launches"], "bytes_per_launch": b}


def adjoint_at(api, torch, p, reps, label):
    """Gridded adjoint throughput on another workload (caller-order input):
    device time per adjoint (sum of its kernels, library events), Mvis/s and
    the fraction of HBM peak for the implemented dataflow and for the
    unpruned 16 L + 100 N byte model."""
    t = time.perf_counter()
    plan, vis = synth_inputs(api, torch, p)
    torch.cuda.synchronize()
    synth_s = time.perf_counter() - t
    dv = torch.from_numpy(vis).cuda()
    img = torch.empty((p.npix, p.npix), dtype=torch.float32, device="cuda")
    for _ in range(3):
        api.pc_adjoint_grid(plan, dv, img, want_max=False)
    api.pc_plan_profile(plan, True)
    for _ in range(reps):
        api.pc_adjoint_grid(plan, dv, img, want_max=False)
    st = api.pc_plan_kernel_stats(plan)
    api.pc_plan_profile(plan, False)
    ms = sum(x["ms"] for x in st) / reps
    b = sum(x["bytes"] for x in st) / reps
    n = p.npix
    f1 = 16 * p.nvis + 100 * n * n
    out = {"workload": label, "nvis": p.nvis, "npix": n, "fine_grid": plan.info["fine"],
           "band": [plan.info["band_nu"], plan.info["band_nv"]], "wraps": plan.info["wraps"],
           "device_ms": ms, "mvis_per_s": p.nvis / ms / 1e3,
           "algorithmic_bytes": b, "hbm_frac_implemented": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "bytes_model_f1": f1, "hbm_frac_f1": f1 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "kernels_us": {x["name"]: round(1e3 * x["ms"] / x["launches"], 2) for x in st},
           "setup_s": synth_s}
    log(label, {k: out[k] for k in ("device_ms", "mvis_per_s", "hbm_frac_implemented")})
    plan.close()
    return out


def w_leg(api, torch, reps):
    """The LOFAR-like workload with its baselines' w kept (non-coplanar):
    the w-stacked adjoint per kernel and a full solve (direct sums with the w
    phase inside APGD, w-stacked exploration)."""
    import sim
    p = sim.config_c2(keep_w=True)
    t = time.perf_counter()
    plan, vis = synth_inputs(api, torch, p)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    dv = torch.from_numpy(vis).cuda()
    img = torch.empty((p.npix, p.npix), dtype=torch.float32, device="cuda")
    for _ in range(2):
        api.pc_adjoint_grid(plan, dv, img, want_max=False)
    api.pc_plan_profile(plan, True)
    for _ in range(reps):
        api.pc_adjoint_grid(plan, dv, img, want_max=False)
    st = api.pc_plan_kernel_stats(plan)
    api.pc_plan_profile(plan, False)
    ms = sum(x["ms"] for x in st) / reps
    info = plan.info
    out = {"workload": "LOFAR-like with w: 424,800 visibilities, 1024^2, FOV 4 deg, w from the "
                       "Earth-rotation formulas (|w| <= 3,713 wavelengths)",
           "w_planes": info["w_planes"], "w_step": info["w_step"], "setup_s": setup_s,
           "adjoint_device_ms": ms, "adjoint_mvis_per_s": p.nvis / ms / 1e3,
           "adjoint_ms_per_plane": ms / max(1, info["w_planes"]),
           "kernels_us_per_launch": {x["name"]: round(1e3 * x["ms"] / x["launches"], 2)
                                     for x in st},
           "kernels_ms_per_adjoint": {x["name"]: round(x["ms"] / reps, 4) for x in st}}
    prm = dict(alpha=p.alpha, delta=p.delta, max_iter=p.max_iter, rel_gap_tol=p.rel_gap_tol)
    out["solve"] = solve_leg(api, torch, p, plan, dv, prm, 3, 1, "C2 with w", False)
    log("C2 with w", {k: out[k] for k in ("w_planes", "adjoint_device_ms", "adjoint_mvis_per_s")})
    plan.close()
    return out


def dictionary_leg(api, torch, reps, with_solve=True):
    """Synthesis-dictionary path (the paper's four Gaussian scales, sigma 0,
    2, 5, 8, gamma 1.2^s): Psi* Phi* on the precision workload's 4096^2 image
    with the stencil kernels' HBM rates, and a synthesis-form solve on the
    64^2 diffuse workload."""
    import numpy as np
    import sim
    sig, gam = [0.0, 2.0, 5.0, 8.0], [1.2 ** s for s in range(4)]
    p = sim.config_c3()
    plan, vis = synth_inputs(api, torch, p)
    dv = torch.from_numpy(vis).cuda()
    n = p.npix
    imgs = torch.empty((4, n, n), dtype=torch.float32, device="cuda")
    for _ in range(2):
        api.pc_adjoint_grid_ms(plan, dv, sig, gam, imgs, want_max=True)
    api.pc_plan_profile(plan, True)
    for _ in range(reps):
        api.pc_adjoint_grid_ms(plan, dv, sig, gam, imgs, want_max=True)
    st = api.pc_plan_kernel_stats(plan)
    api.pc_plan_profile(plan, False)
    kern = {}
    for x in st:
        if x["name"].startswith("dict_"):
            avg = x["ms"] / x["launches"]
            gbs = x["bytes"] / x["launches"] / (avg * 1e-3) / 1e9
            kern[x["name"]] = {"avg_us": round(1e3 * avg, 2), "GB/s": round(gbs, 1),
                               "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                               "bytes_per_launch": x["bytes"] / x["launches"]}
    total_ms = sum(x["ms"] for x in st) / reps
    out = {"adjoint_ms": {"workload": "precision workload (2,088,960 visibilities, 4096^2), "
                                      "4 scales",
                          "device_ms": total_ms, "mvis_per_s": p.nvis / total_ms / 1e3,
                          "kernels": kern,
                          "traffic_sigma8_bytes_per_launch": stored_traffic("dict_analysis")}}
    log("dictionary adjoint", out["adjoint_ms"])
    plan.close()
    del dv, imgs
    if not with_solve:
        return out
    p = sim.config_diffuse(npix=64)
    plan, vis = synth_inputs(api, torch, p)
    dv = torch.from_numpy(vis).cuda()
    prm = dict(alpha=0.05, delta=p.delta, max_iter=300, rel_gap_tol=1e-4, scales=(sig, gam))
    api.pc_polyclean_solve(plan, dv, **prm)  # warm
    r = api.pc_polyclean_solve(plan, dv, **prm)
    out["solve"] = {"workload": f"diffuse workload: {p.nvis} visibilities, 64^2, 3 blobs + 4 "
                                "points, 20 dB, lambda = 0.05 lambda_max, stop at relative "
                                "duality gap 1e-4",
                    "seconds": r["seconds"], "iters": r["iters"], "natoms": r["natoms"],
                    "atoms_per_scale": np.bincount(r["pix"] // (64 * 64), minlength=4).tolist(),
                    "rel_gap": r["rel_gap"], "converged": r["converged"]}
    log("dictionary solve", out["solve"])
    plan.close()
    return out


def serving_leg(api, torch, n_req, slots):
    """Serving mix: n_req requests (grids 256^2..2048^2, 1e4-5e5 visibilities,
    32-128 antennas, 5-200 sources, 20 dB, lambda = 0.05 lambda_max, stop at
    relative objective change 1e-4 or 100 iterations).  Runs the plain path
    (one pc_polyclean_solve at a time) and the batched server with every
    request present at t = 0 (saturation), then both on Poisson arrival
    traces at 0.5x and 1.0x the plain path's solves/s."""
    import numpy as np
    import sim
    from paper_2406_01342_amd import serving
    t = time.perf_counter()
    reqs = []
    for k in range(n_req):
        p = sim.config_c4_request(k)
        plan0, vis = synth_inputs(api, torch, p)
        plan0.close()
        prm = dict(alpha=p.alpha, delta=p.delta, max_iter=p.max_iter,
                   rel_obj_tol=p.rel_obj_tol, rel_gap_tol=p.rel_gap_tol)
        reqs.append(serving.ImagingRequest(k, 0.0, p.uv, p.npix, p.fov_rad, vis, prm))
    log(f"serving: {n_req} requests synthesised in {time.perf_counter() - t:.1f} s, "
        f"{sum(r.uv.shape[0] for r in reqs)} visibilities")
    be = serving.DeviceBackend(batched=True)
    # warm the code paths (kernels of every grid size) outside the timed runs
    for n in (256, 512, 1024, 2048):
        r0 = next((r for r in reqs if r.npix == n), None)
        if r0 is not None:
            be.solve_plain(r0)
    plain, precs = serving.run_plain(be, reqs)
    log("serving plain", plain)
    srv = serving.Server(be, slots=slots)
    sat = srv.run(reqs)
    log("serving batched", sat)
    plain_by = {r.rid: r for r in precs}
    dobj = max(abs(r.result["objective"] - plain_by[r.rid].result["objective"]) /
               max(abs(plain_by[r.rid].result["objective"]), 1e-300)
               for r in srv.records if r.status == "done")
    out = {"workload": "serving mix: grids 256^2-2048^2, 1e4-5e5 visibilities "
                       "(log-uniform), 32-128 antennas, 5-200 sources, 20 dB, "
                       "lambda = 0.05 lambda_max, stop at relative objective change 1e-4",
           "requests": n_req, "slots": slots,
           "saturation": {"plain": plain, "batched": sat,
                          "solves_per_s_ratio": sat["solves_per_s"] / plain["solves_per_s"]},
           "max_rel_objective_diff_batched_vs_plain": dobj}
    for mult in (0.5, 1.0):
        rate = mult * plain["solves_per_s"]
        arr = sim.poisson_arrivals(n_req, rate)
        for r, a in zip(reqs, arr):
            r.arrival_s = float(a)
        srv = serving.Server(be, slots=slots)
        bat = srv.run(reqs)
        # the plain path replayed on the same arrival trace (measured, one job
        # at a time in arrival order)
        pl, _ = serving.run_plain(be, reqs)
        out[f"poisson_{mult}x"] = {"rate_per_s": rate, "batched": bat, "plain": pl}
        log(f"serving poisson {mult}x", bat, pl)
    out["batcher"] = be.stats()
    be.close_backend()
    return out


ADJ_KERNELS = ("spread", "fold", "passA_adj", "passB_adj")


def cpu_model():
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def solve_leg(api, torch, p, plan, dv, prm, steps, warmup, label, with_cert=True):
    """Warm-up and timed solves of one problem: wall time per solve and the
    in-solve full-grid adjoint throughput (library events)."""
    cert = (torch.empty((p.npix, p.npix), dtype=torch.float32, device="cuda")
            if with_cert else None)
    kw = dict(prm)
    if with_cert:
        kw.update(cert=cert, want_certificate=1)
    for w in range(warmup):
        r = api.pc_polyclean_solve(plan, dv, **kw)
        log(label, "warmup", w, {k: r[k] for k in ("iters", "natoms", "objective", "rel_gap",
                                                      "seconds")})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(steps):
        r = api.pc_polyclean_solve(plan, dv, **kw)
        results.append(r)
        log(label, "step", k, {kk: r[kk] for kk in ("iters", "inner_iters", "natoms",
                                                     "objective", "rel_gap", "seconds",
                                                     "adjoint_calls")})
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    calls = sum(r["adjoint_calls"] for r in results)
    adj_s = sum(r["adjoint_seconds"] for r in results)
    last = results[-1]
    return {"ms_per_solve": wall / steps * 1e3, "solves_per_s": steps / wall,
            "adjoint_mvis_per_s": p.nvis * calls / adj_s / 1e6,
            "adjoint_ms": adj_s / calls * 1e3, "adjoint_calls_per_solve": calls / steps,
            "iters": last["iters"], "inner_iters": last["inner_iters"],
            "natoms": last["natoms"], "objective": last["objective"],
            "rel_gap": last["rel_gap"], "converged": last["converged"],
            "cert_max": last["cert_max"], "wall_s": wall}


def profiled(api, plan, fn):
    """Per-kernel statistics (library events) of fn()."""
    api.pc_plan_profile(plan, True)
    fn()
    st = api.pc_plan_kernel_stats(plan)
    api.pc_plan_profile(plan, False)
    return st


def adjoint_roofline(stats):
    """Roofline object of the gridded adjoint's dominant kernel: the one with
    the longest launch in a full adjoint (the spread and fold also serve the
    APGD's row-restricted adjoints, whose passes carry names of their own)."""
    adj = [x for x in stats if x["name"] in ADJ_KERNELS]
    top = max(adj, key=lambda x: x["ms"] / x["launches"])
    return dominant_roofline([top], None)


def m2_sweep(api, torch):
    """M2: direct-DFT pair rates of the forward (a7) and the restricted
    adjoint (a8) at nS in {100, 1000, 10000} atoms for the visibility counts of
    the LOFAR-like and precision workloads (their own uv coverage), device
    time from library events, against the derived vector-ALU ceiling."""
    import numpy as np
    import sim
    out = []
    for p in (sim.config_c2(), sim.config_c3()):
        plan = api.pc_plan_create(p.uv, p.npix, p.fov_rad)
        dv = torch.from_numpy(p.noise.astype(np.complex64)).cuda()
        rng = np.random.default_rng(11)
        for ns in (100, 1000, 10000):
            pix = torch.from_numpy(rng.choice(p.npix * p.npix, ns, replace=False).astype(np.int32)).cuda()
            w = torch.from_numpy(rng.lognormal(size=ns).astype(np.float32)).cuda()
            reps = max(2, int(2e10 // (p.nvis * ns)))
            for _ in range(2):
                api.pc_forward_sparse(plan, pix, w)
                api.pc_adjoint_sparse(plan, dv, pix)
            st = profiled(api, plan, lambda: [(api.pc_forward_sparse(plan, pix, w),
                                               api.pc_adjoint_sparse(plan, dv, pix))
                                              for _ in range(reps)])
            by = {x["name"]: x for x in st}
            row = {"nvis": p.nvis, "natoms": ns}
            for key, names in (("forward", ("forward_sparse",)),
                               ("restricted_adjoint", ("adjoint_sparse", "adjoint_sparse_reduce"))):
                ms = sum(by[n]["ms"] for n in names if n in by) / reps
                gp = p.nvis * ns / (ms * 1e-3) / 1e9
                row[key] = {"us": round(ms * 1e3, 1), "Gpair_per_s": round(gp, 1),
                            "alu_frac": round(gp / DFT_PEAK_GPAIRS, 3)}
            out.append(row)
            log("M2", row)
        plan.close()
    return out


def c5_mix_leg(api, torch, n_large, n_small):
    """Memory-pressure mix, scaled down to n_large large jobs (8192^2,
    8,372,224 visibilities) and n_small small ones (512^2, 50,400), each
    returning its dual-certificate image, under an HBM budget that holds two
    large jobs at once (admission by footprint): batched server against the
    plain one-at-a-time path, all requests present at t = 0."""
    import sim
    from paper_2406_01342_amd import serving
    reqs = []
    for k in range(n_large + n_small):
        p = sim.config_c5_large(job_id=k) if k < n_large else sim.config_c5_small(job_id=k)
        plan0, vis = synth_inputs(api, torch, p)
        plan0.close()
        prm = dict(alpha=p.alpha, delta=p.delta, max_iter=p.max_iter,
                   rel_obj_tol=p.rel_obj_tol, rel_gap_tol=p.rel_gap_tol)
        reqs.append(serving.ImagingRequest(k, 0.0, p.uv, p.npix, p.fov_rad, vis, prm,
                                           want_certificate=True))
    torch.cuda.empty_cache()
    be = serving.DeviceBackend(batched=True)
    big = be.footprint(reqs[0])
    budget = 2 * big + 8 * be.footprint(reqs[-1])
    be.solve_plain(reqs[-1])  # warm the small grid's kernels
    plain, precs = serving.run_plain(be, reqs)
    log("C5 mix plain", plain)
    srv = serving.Server(be, slots=8, hbm_budget=budget)
    bat = srv.run(reqs)
    log("C5 mix batched", bat)
    by = {r.rid: r for r in precs}
    dobj = max(abs(r.result["objective"] - by[r.rid].result["objective"]) /
               abs(by[r.rid].result["objective"]) for r in srv.records if r.status == "done")
    be.close_backend()
    return {"workload": f"memory-pressure mix scaled to {n_large} large jobs (8192^2, 8,372,224 "
                        f"visibilities) + {n_small} small jobs (512^2, 50,400 visibilities), "
                        "certificate per job, all at t = 0",
            "hbm_budget_bytes": budget, "large_job_footprint_bytes": big,
            "plain": plain, "batched": bat,
            "solves_per_s_ratio": bat["solves_per_s"] / plain["solves_per_s"],
            "max_rel_objective_diff_batched_vs_plain": dobj}


def cpu_baseline_c5(p, vis, seconds):
    """FP64 oracle adjoint of a visibility sample onto the full 8192^2 image
    of the memory-pressure large job, on the host cores, in Mvis/s."""
    import numpy as np
    from oracle import operator
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    v = vis.astype(np.complex128)
    # calibrate the sample size on growing trial sizes (the first call also
    # pays for thread start-up), then time one call of about `seconds`
    m, dt = 64, 0.0
    while dt < 0.1 * seconds and m < len(v):
        t = time.perf_counter()
        operator.adjoint(p.uv[:m], p.npix, p.fov_rad, v[:m])
        dt = time.perf_counter() - t
        if dt < 0.1 * seconds:
            m *= 2
    m = int(min(len(v), max(m, m * seconds / max(dt, 1e-3))))
    t = time.perf_counter()
    operator.adjoint(p.uv[:m], p.npix, p.fov_rad, v[:m])
    dt = time.perf_counter() - t
    return {"value": m / dt / 1e6, "unit": "Mvis/s", "cores": int(cores), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"FP64 exact adjoint (direct sum as chunked complex GEMM) of the first {m} "
                      f"of {len(v)} visibilities of the memory-pressure large job onto its full "
                      f"{p.npix}^2 image, {dt:.1f} s"}


def main():
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.command)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[1:], args.summarize_counters[0], args.command)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, args.command)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import sim
    from paper_2406_01342_amd import api

    torch.cuda.set_device(0)
    copy_probe(torch)
    if args.adjoint_only:
        cfg = {"c2": (sim.config_c2, "LOFAR-like workload: 424,800 visibilities, 1024^2"),
               "c3": (sim.config_c3, "precision workload: 256 stations, 2,088,960 "
                                     "visibilities, 4096^2, FOV 3 deg"),
               "c5l": (sim.config_c5_large, "memory-pressure large job: 512 stations x 16 "
                                            "snapshots x 4 channels, 8,372,224 visibilities, "
                                            "8192^2 (16384^2 fine grid), FOV 3 deg")}
        make, label = cfg[args.adjoint_only]
        print(json.dumps({"adjoint": adjoint_at(api, torch, make(), args.adjoint_reps, label)}),
              flush=True)
        return
    if args.w_only:
        print(json.dumps({"lofar_like_w": w_leg(api, torch, max(3, args.adjoint_reps // 5))}),
              flush=True)
        return
    if args.dictionary_only:
        print(json.dumps({"dictionary": dictionary_leg(api, torch, max(5, args.adjoint_reps // 4),
                                                       with_solve=False)}), flush=True)
        return

    # ---- headline: the memory-pressure large job, full solves ----------------
    p = sim.config_c5_large()
    log("workload C5-large", p.nvis, "visibilities", p.npix, "pixels")
    plan0, vis = synth_inputs(api, torch, p)
    plan0.close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan = api.pc_plan_create(p.uv, p.npix, p.fov_rad)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t) * 1e3
    log("plan", f"{plan_ms:.1f} ms", plan.info)
    dv = torch.from_numpy(vis).cuda()
    prm = dict(alpha=p.alpha, delta=p.delta, max_iter=p.max_iter, rel_obj_tol=p.rel_obj_tol,
               rel_gap_tol=p.rel_gap_tol)
    head = solve_leg(api, torch, p, plan, dv, prm, args.steps, args.warmup, "C5-large")
    value = head["adjoint_mvis_per_s"]
    cert = torch.empty((p.npix, p.npix), dtype=torch.float32, device="cuda")
    stats = profiled(api, plan, lambda: api.pc_polyclean_solve(plan, dv, cert=cert,
                                                               want_certificate=1, **prm))
    roof = adjoint_roofline(stats)
    # per full adjoint: each kernel's own average (the restricted adjoints
    # inside APGD share the spread and fold, their passes have names of
    # their own)
    adj_bytes = sum(x["bytes"] / x["launches"] for x in stats if x["name"] in ADJ_KERNELS)
    adj_ms = sum(x["ms"] / x["launches"] for x in stats if x["name"] in ADJ_KERNELS)
    n = p.npix
    out = {
        "metric": METRIC, "value": value, "unit": "Mvis/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "memory-pressure large job, full PolyCLEAN solve with dual "
                               "certificate: 512 stations (SKA-low-like core and arms, 40 km), 16 "
                               "snapshots x 4 channels 120-180 MHz stacked, 8,372,224 complex64 "
                               "visibilities, 8192^2 image (16384^2 fine grid), FOV 3 deg, 200 "
                               "log-normal sources, 20 dB, lambda = 0.05 lambda_max, stop at "
                               "relative objective change 1e-4",
                   "nvis": p.nvis, "npix": n, "fine_grid": plan.info["fine"],
                   "band": [plan.info["band_nu"], plan.info["band_nv"]],
                   "kernel_width": plan.info["kernel_width"]},
        "roofline": roof,
        "solve": head,
        "plan_ms": plan_ms,
        "adjoint": {"per_launch_ms_sum_of_kernels": adj_ms,
                    "algorithmic_bytes_per_adjoint": adj_bytes,
                    "hbm_frac_implemented": adj_bytes / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "bytes_model_f1": 16 * p.nvis + 100 * n * n,
                    "kernels_us": {x["name"]: round(1e3 * x["ms"] / x["launches"], 2)
                                   for x in stats if x["name"] in ADJ_KERNELS}},
        "kernels": sorted(({"name": x["name"], "launches": x["launches"],
                            "ms": round(x["ms"], 3)} for x in stats),
                          key=lambda d: -d["ms"])[:10],
        "alu_ceiling": {"Gpair_per_s": DFT_PEAK_GPAIRS,
                        "derivation": "256 CUs x 2.4 GHz x 128 FP32 lane-slots per clock = "
                                      "78.6e12 lane-slots/s (the published 157.3 TFLOP/s FP32 "
                                      "vector peak counts an FMA as two flops); one "
                                      "visibility-atom pair of the direct DFT costs about 19 "
                                      "slots (FP64 phase FMA pair and range reduction at the "
                                      "78.6 TFLOP/s FP64 rate, FP32 sin and cos at quarter "
                                      "rate, two FP32 FMAs)"},
    }
    # standalone adjoint of caller-order visibilities (the dirty image)
    img = torch.empty((n, n), dtype=torch.float32, device="cuda")
    for _ in range(2):
        api.pc_adjoint_grid(plan, dv, img, want_max=False)
    s_ = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(3, args.adjoint_reps // 5)
    e0.record(s_)
    for _ in range(reps):
        api.pc_adjoint_grid(plan, dv, img, want_max=False)
    e1.record(s_)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out["adjoint"]["standalone_caller_order_ms"] = ms
    out["adjoint"]["standalone_mvis_per_s"] = p.nvis / ms / 1e3
    log("C5-large adjoint", out["adjoint"])
    # operator-form solve of the same job (gram_atoms < 0: a7/a8 inside APGD)
    op = solve_leg(api, torch, p, plan, dv, dict(prm, gram_atoms=-1), max(1, args.steps // 5), 1,
                   "C5-large operator form")
    out["solve_operator_form"] = op
    del dv, img, cert
    plan.close()
    torch.cuda.empty_cache()

    # ---- LOFAR-like solves: Gram form (default), operator form, positivity ----
    p2 = sim.config_c2()
    plan2, vis2 = synth_inputs(api, torch, p2)
    dv2 = torch.from_numpy(vis2).cuda()
    prm2 = dict(alpha=p2.alpha, delta=p2.delta, max_iter=p2.max_iter,
                rel_gap_tol=p2.rel_gap_tol)
    c2 = {"workload": "LOFAR-like: 60 stations (48-station 300 m Gaussian core + 12 in a 1-10 km "
                      "ring), 240 snapshots over 4 h, 424,800 visibilities, 1024^2, FOV 4 deg, 150 "
                      "sources, 20 dB, lambda = 0.05 lambda_max, stop at relative duality gap 1e-4"}
    c2["gram_form"] = solve_leg(api, torch, p2, plan2, dv2, prm2, 10, 2, "C2 gram", False)
    c2["operator_form"] = solve_leg(api, torch, p2, plan2, dv2, dict(prm2, gram_atoms=-1), 5, 1,
                                    "C2 operator", False)
    st2 = profiled(api, plan2, lambda: api.pc_polyclean_solve(plan2, dv2, gram_atoms=-1, **prm2))
    c2["operator_form"]["dominant_kernel"] = dominant_roofline(st2, None)
    c2["positive"] = solve_leg(api, torch, p2, plan2, dv2, dict(prm2, positivity=1), 5, 1,
                               "C2 positive", False)
    c2["adjoint_standalone"] = adjoint_at(api, torch, p2, args.adjoint_reps,
                                          "LOFAR-like workload: 424,800 visibilities, 1024^2")
    out["lofar_like"] = c2
    plan2.close()
    del dv2
    out["lofar_like_w"] = w_leg(api, torch, max(3, args.adjoint_reps // 5))

    if not args.no_other_workloads:
        out["adjoint_precision_workload"] = adjoint_at(
            api, torch, sim.config_c3(), args.adjoint_reps,
            "precision workload: 256 stations, 2,088,960 visibilities, 4096^2, FOV 3 deg")
        out["m2_direct_dft"] = m2_sweep(api, torch)
        out["dictionary"] = dictionary_leg(api, torch, max(5, args.adjoint_reps // 4))
    if args.serving_requests > 0:
        torch.cuda.empty_cache()
        out["serving"] = serving_leg(api, torch, args.serving_requests, args.serving_slots)
        out["serving_memory_pressure"] = c5_mix_leg(api, torch, 2, 16)
    # last: the oracle's thread pool on the host cores would otherwise still
    # compete with the host side of the latency-bound legs above
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline_c5(p, vis, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
