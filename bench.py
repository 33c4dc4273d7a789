"""Benchmark of the RMRT-LB collide-and-stream hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--only LIST] [--no-cpu-baseline]

Headline (value): rD3Q19 NSE 3D Taylor-Green, 256 x 256 x 128 nodes with
dz = 2 dx (a physical 256^3 cube), U0 = 0.02, nu = 0.005, FP32 deviation
storage with FP32 collision arithmetic, AA pattern: whole-job MLUPS of K timed
steps (one fused launch per step, replayed from a HIP graph).  The same JSON
line carries the roofline of that kernel, the FP64 oracle timed on the host
cores, the HBM copy ceiling, and per-lattice MLUPS / % HBM of the other
workloads (rD2Q9 NCDE 2048 x 1024, rD3Q19 FP16, rD3Q27, the 64-domain batched
rD3Q27 channel launch, rD2Q9 Taylor-Green 64 x 32 FP64).  Inputs are seeded
and synthetic and are resident in HBM before the timed region starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
CONFIG_KEYS = ("threads", "tile_nodes", "blocks_per_cu", "persistent", "nodes_per_thread")

# HBM bytes per launch of the headline step kernel from the rocprofv3 FETCH_SIZE
# and WRITE_SIZE passes (profiles/k_step_q19_f32dev_256x256x128_pmc.md), scaled
# by the counters of a plain copy of known size.  Keyed by the hash of the
# kernel code the counters were taken on: any later code change reports null.
MEASURED_TRAFFIC = {"691cb16803d1e347": 1275195792}
KERNEL_SOURCES = ["lbm_device.hpp", "lbm_kernels.hpp", "lbm_params.hpp", "lbm_launch.hpp", "lbm_q19_f32.hip"]


def kernel_source_hash():
    """Hash of the step kernel's code: the sources with their // comments,
    indentation and blank lines dropped, so that an edit of a comment keeps it."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2206_00366_amd", "csrc", f)) as fh:
            lines = (re.sub(r"//.*", "", ln).strip() for ln in fh.read().splitlines())
        h.update(f.encode() + b"\0")
        h.update("\n".join(ln for ln in lines if ln).encode() + b"\0")
    return h.hexdigest()[:16]
METRIC = "MLUPS and % HBM peak per lattice; steps/time-to-1e-6 residual plain vs warm-start"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sizeof(storage):
    return {"f64": 8, "f32dev": 4, "f16dev": 2}[storage]


def timed_steps(torch, step_fn, steps, warmup, prepare=None):
    """Warm up, then time exactly `steps` steps: wall clock between two
    synchronisations and HIP events on the current stream (where the kernels run).
    prepare(steps), when given, captures the HIP graphs of the timed call before
    the clock starts (graph capture is set-up, not part of a step)."""
    step_fn(warmup)
    if prepare is not None:
        prepare(steps)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    step_fn(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    return wall, ev_ms


def settle(torch, R, seconds=0.3, nbytes=64 << 20):
    """Keep the GPU busy with plain copies for `seconds`, so that a leg's warm-up
    starts at the GPU's working clocks.  Measured on MI355X: after 2 s idle the
    first 50 rD3Q19 256 x 256 x 128 steps take 208-216 us each and the rate
    reaches 201 us only after about 100 steps; right after a 1 s busy period
    it is 201 us from the first step (20-step graph: 211.8 against 199.0 us).
    The copies stay in the memory-side cache (64 MiB source and destination):
    on a box without that ramp, 0.3 s of 1 GiB copies left the next 20 steps
    1.2% slower than after 2 s idle (202.5 against 200.0 us), 64 MiB copies
    did not (199.6 us)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            R.stream_copy(dst, src)
        torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


def tg3d_fields(n, dx, U0, cs2):
    from inputs import taylor_green_3d
    rho, u, _ = taylor_green_3d(n, dx, U0, cs2)
    return rho, u


def run_single(torch, R, prm, rho, u, steps, warmup, solid=None, launch=None, settle_s=0.3):
    """One domain: W warm-up steps, then exactly `steps` timed steps; with
    settle_s > 0 the GPU is kept busy for that long first (settle())."""
    dom = R.Domain(R.make_params(**prm), rho, u, solid=solid)
    torch.cuda.synchronize()
    if settle_s > 0:
        settle(torch, R, settle_s)
    wall, ev_ms = timed_steps(torch, dom.step, steps, warmup, prepare=dom.prepare)
    red = dom.reduce()
    finite = all(math.isfinite(v) for v in red)
    if launch is not None:
        launch.update(dict(zip(("blocks_per_cu_cap", "flags"), dom.get_launch())))
    dom.close()
    del dom
    torch.cuda.empty_cache()
    return wall, ev_ms, finite


def lattice_entry(name, q, storage, N, steps, wall, ev_ms, note=None, extra_bytes=0):
    """extra_bytes: algorithmic bytes per update beyond the 2 q populations
    (the rD2Q5 / rD3Q7 history field: one read and one write)."""
    mlups = N * steps / wall / 1e6
    bpu = 2 * q * sizeof(storage) + extra_bytes
    gbs_ev = N * bpu / (ev_ms / steps * 1e-3) / 1e9
    e = {"workload": name, "MLUPS": round(mlups, 1), "bytes_per_update": bpu,
         "kernel_GBps": round(gbs_ev, 1), "pct_hbm_peak": round(100 * gbs_ev / HBM_PEAK_GBS, 1),
         "ms_per_step": round(wall / steps * 1e3, 4)}
    if note:
        e["note"] = note
    return e


def copy_ceiling(torch, R, nbytes=2 << 30, reps=20):
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        R.stream_copy(dst, src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        R.stream_copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_per_launch": 2 * nbytes, "GBps": round(2 * nbytes / (ms * 1e-3) / 1e9, 1),
            "pct_hbm_peak": round(100 * 2 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 1)}


def cpu_baseline():
    """The FP64 oracle as it stands, on a bounded sample of the headline workload.
    The primary figure runs numpy's BLAS on one thread (cores = 1, the threads
    the oracle keeps busy: its dense products are small and most of its time is
    single-threaded numpy work); a second, shorter figure lets BLAS use its
    whole pool, for comparison.  Returns the baseline record and the oracle's
    final state for the accuracy check."""
    import numpy as np
    from oracle import rmrt_oracle as O
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        pool = max([1] + [int(i.get("num_threads", 1)) for i in threadpool_info()])
    except ImportError:
        threadpool_limits, pool = None, 1
    n, dx = (32, 32, 32), (1.0, 1.0, 2.0)
    prm = dict(lattice="Q19", n=n, dx=dx, nu=0.005, cs2=1.0 / 3.0)
    m = O.Model(prm)
    rho, u = tg3d_fields(n, dx, 0.02, m.cs2)

    def run(seconds, min_steps):
        f = m.init(rho, u)
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds or steps < min_steps:
            f = m.step(f, 5)
            steps += 5
        return f, steps, time.perf_counter() - t0

    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            f, steps, dt = run(12.0, 10)
        cores = 1
    else:
        f, steps, dt = run(12.0, 10)
        cores = pool
    assert np.isfinite(f).all()
    rec = {"value": round(m.N * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"rD3Q19 NSE Taylor-Green 32x32x32 (dz = 2 dx, nu = 0.005), {steps} steps of the dense "
                     f"FP64 numpy oracle ({dt:.1f} s), numpy BLAS limited to {cores} thread(s)"}
    if threadpool_limits is not None and pool > 1:
        _, s2, d2 = run(5.0, 5)
        rec["blas_pool"] = {"value": round(m.N * s2 / d2 / 1e6, 4), "unit": "MLUPS", "blas_threads": pool,
                            "sample": f"the same case, {s2} steps ({d2:.1f} s) with BLAS free to use {pool} "
                                      f"threads; the oracle's small products keep few of them busy"}
    rec["host_cpu"] = host_cpu()
    r_o, u_o = m.macroscopic(f)
    return rec, dict(prm=prm, rho=rho, u=u, steps=steps, rho_o=r_o, u_o=u_o)


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "cores_available": avail}


def accuracy_vs_oracle(torch, R, ref):
    """Error of each storage mode against the oracle state of the CPU-baseline sample."""
    import numpy as np
    out = {}
    for storage in ("f64", "f32dev", "f16dev"):
        dom = R.Domain(R.make_params(**ref["prm"], storage=storage, pattern="AA"), ref["rho"], ref["u"])
        dom.step(ref["steps"])
        r, u = dom.moments()
        r, u = r.cpu().numpy(), u.cpu().numpy()
        dom.close()
        out[storage] = {"max_abs_rho_err": float(np.abs(r - ref["rho_o"]).max()),
                        "max_u_err_over_U0": float(np.abs(u - ref["u_o"]).max() / 0.02)}
    out["sample"] = f"rD3Q19 TG 32^3, {ref['steps']} steps against the FP64 oracle"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--only", default="all",
                    help="comma list of: q19,q19f16,q19f64,q19local,q9ncde,q5ncde,q7ncde,q27,q27batch,q9tg,bases,copy "
                         "(the q19 headline always runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--warmstart", action="store_true",
                    help="run the warm-start study (solver-generated training set, training, held-out evaluation)")
    ap.add_argument("--ws-train", type=int, default=512)
    ap.add_argument("--ws-test", type=int, default=100)
    ap.add_argument("--ws-epochs", type=int, default=40)
    ap.add_argument("--ws-train-tol", type=float, default=1e-5)
    ap.add_argument("--ws-max-steps", type=int, default=300_000)
    ap.add_argument("--ws-log", default=None, help="file receiving one JSON line per finished stage")
    ap.add_argument("--no-warmstart", action="store_true",
                    help="skip the reduced warm-start study of the default run")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    from paper_2206_00366_amd import rmrt as R

    if args.warmstart:
        print(json.dumps(warmstart_study(torch, args)))
        return

    only = set(args.only.split(",")) if args.only != "all" else {"q19f16", "q19f64", "q9ncde", "q27", "q27batch", "q9tg",
                                                                 "q5ncde", "q7ncde", "q19local", "bases", "copy"}
    K, W = args.steps, args.warmup

    # ---------------- headline: rD3Q19 FP32-dev 256 x 256 x 128 ----------------
    n_h, dx_h = (256, 256, 128), (1.0, 1.0, 2.0)
    N_h = n_h[0] * n_h[1] * n_h[2]
    prm_h = dict(lattice="Q19", equation="NSE", n=n_h, dx=dx_h, nu=0.005, cs2=1.0 / 3.0, rho0=1.0,
                storage="f32dev", pattern="AA")
    log("[bench] headline rD3Q19 256x256x128 f32dev AA, on the GPU as it comes")
    rho_h, u_h = tg3d_fields(n_h, dx_h, 0.02, 1.0 / 3.0)
    wall_c, ev_c, _ = run_single(torch, R, prm_h, rho_h, u_h, K, W, settle_s=0.0)
    log("[bench] HBM copy ceiling")
    ceiling = copy_ceiling(torch, R)
    mall_ceiling = copy_ceiling(torch, R, nbytes=96 << 20, reps=400)
    log("[bench] headline rD3Q19 256x256x128 f32dev AA")
    launch = {}
    wall, ev_ms, finite = run_single(torch, R, prm_h, rho_h, u_h, K, W, launch=launch)
    head = lattice_entry("rD3Q19 NSE TG 256x256x128 dz=2dx FP32-dev AA", 19, "f32dev", N_h, K, wall, ev_ms)
    head["finite"] = finite
    bytes_per_launch = 2 * 19 * 4 * N_h
    avg_launch_s = ev_ms / K * 1e-3
    achieved = bytes_per_launch / avg_launch_s / 1e9
    src_hash = kernel_source_hash()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": MEASURED_TRAFFIC.get(src_hash),
                "kernel_source_hash": src_hash,
                "kernel": "k_step<Q19, F32, NSE, no force, periodic, AA even/odd>",
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "avg_launch_us": round(avg_launch_s * 1e6, 2),
                "launch": dict(launch, workgroup=256, tile_nodes=256)}

    head["cold_gpu"] = {"MLUPS": round(N_h * K / wall_c / 1e6, 1), "ms_per_step": round(wall_c / K * 1e3, 4),
                        "avg_launch_us": round(ev_c / K * 1e3, 2),
                        "note": "the same K steps after the same W warm-up steps, timed first on a GPU idle "
                                "before (its clocks rise during the first ~100 steps); value and every other "
                                "leg are timed after 0.3 s of plain copies that bring the clocks up"}
    per = {"rD3Q19_f32dev": head}
    if "q19local" in only:
        log("[bench] rD3Q19 strain-rate output")
        per["rD3Q19_strain_rate_output"] = bench_local(torch, R, prm_h, rho_h, u_h, N_h)
        fused = bench_step_local(torch, R, prm_h, rho_h, u_h, N_h)
        sep = per["rD3Q19_strain_rate_output"]["us_per_call"] + 1e3 * head["ms_per_step"]
        fused["speedup_vs_step_plus_on_demand"] = round(sep / fused["us_per_step"], 3)
        per["rD3Q19_step_fused_strain"] = fused
    if "q19f16" in only:
        log("[bench] rD3Q19 f16dev")
        prm = dict(prm_h, storage="f16dev")
        w2, e2, fin = run_single(torch, R, prm, rho_h, u_h, K, W)
        per["rD3Q19_f16dev"] = lattice_entry("rD3Q19 NSE TG 256x256x128 FP16-dev AA", 19, "f16dev", N_h, K, w2, e2)
        per["rD3Q19_f16dev"]["finite"] = fin
        per["rD3Q19_f16dev"]["speedup_vs_f32dev"] = round(per["rD3Q19_f16dev"]["MLUPS"] / head["MLUPS"], 3)
    if "q19f64" in only:
        log("[bench] rD3Q19 f64")
        prm = dict(prm_h, storage="f64")
        w2, e2, fin = run_single(torch, R, prm, rho_h, u_h, max(K // 2, 10), W)
        per["rD3Q19_f64"] = lattice_entry("rD3Q19 NSE TG 256x256x128 FP64 AA", 19, "f64", N_h, max(K // 2, 10), w2, e2)
    del rho_h, u_h
    if "q27" in only:
        log("[bench] rD3Q27 f32dev 256x256x128")
        prm = dict(prm_h, lattice="Q27")
        rho, u = tg3d_fields(n_h, dx_h, 0.02, 1.0 / 3.0)
        w2, e2, fin = run_single(torch, R, prm, rho, u, K, W)
        per["rD3Q27_f32dev"] = lattice_entry("rD3Q27 NSE TG 256x256x128 dz=2dx FP32-dev AA", 27, "f32dev", N_h, K, w2, e2)
        per["rD3Q27_f32dev"]["finite"] = fin
        del rho, u
    if "q9ncde" in only:
        log("[bench] rD2Q9 NCDE 2048x1024 f32dev")
        from inputs import gaussian_hill_field
        n2 = (2048, 1024, 1)
        prm = dict(lattice="Q9", equation="NCDE", n=n2, dx=(1.0, 0.5, 1.0), D0=0.01, D2=1.0, adv=(0.05, 0.02, 0.0),
                   rho0=0.0, storage="f32dev", pattern="AA")
        phi = gaussian_hill_field(2048, 1024, 1.0, 0.5, 40.0, 1024.0, 256.0)
        w2, e2, fin = run_single(torch, R, prm, phi, None, 4 * K, W)
        per["rD2Q9_ncde_f32dev"] = lattice_entry(
            "rD2Q9 NCDE Gaussian hill 2048x1024 dy=0.5 FP32-dev AA", 9, "f32dev", 2048 * 1024, 4 * K, w2, e2,
            note="75.5 MB working set fits the 256 MB MALL: % HBM may be cache-inflated")
        per["rD2Q9_ncde_f32dev"]["finite"] = fin
    if "q5ncde" in only:
        log("[bench] rD2Q5 NCDE 2048x1024 f32dev")
        from inputs import gaussian_hill_field
        n2 = (2048, 1024, 1)
        prm = dict(lattice="Q5", equation="NCDE", n=n2, dx=(1.0, 0.5, 1.0), D0=0.01, D2=1.0, adv=(0.05, 0.02, 0.0),
                   rho0=0.0, storage="f32dev", pattern="AA")
        phi = gaussian_hill_field(2048, 1024, 1.0, 0.5, 40.0, 1024.0, 256.0)
        w2, e2, fin = run_single(torch, R, prm, phi, None, 4 * K, W)
        per["rD2Q5_ncde_f32dev"] = lattice_entry(
            "rD2Q5 NCDE Gaussian hill 2048x1024 dy=0.5 FP32-dev AA, linear equilibrium + dB/dt history",
            5, "f32dev", 2048 * 1024, 4 * K, w2, e2, extra_bytes=8,
            note="50 MB working set fits the 256 MB MALL: % HBM may be cache-inflated")
        per["rD2Q5_ncde_f32dev"]["finite"] = fin
    if "q7ncde" in only:
        import numpy as np
        n3 = (256, 256, 128)
        x = np.arange(n3[0]) * 1.0
        Z, Y, X = np.meshgrid(np.arange(n3[2]) * 2.0, np.arange(n3[1]) * 1.0, x, indexing="ij")
        phi = np.exp(-((X - 128) ** 2 + (Y - 128) ** 2 + (Z - 128) ** 2) / (2 * 24.0**2)).reshape(-1)
        del X, Y, Z
        for st in ("f32dev", "f16dev"):
            log(f"[bench] rD3Q7 NCDE 256x256x128 {st}")
            prm = dict(lattice="Q7", equation="NCDE", n=n3, dx=(1.0, 1.0, 2.0), D0=0.01, D2=1.0,
                       adv=(0.05, 0.02, 0.01), rho0=0.0, storage=st, pattern="AA")
            w2, e2, fin = run_single(torch, R, prm, phi, None, K, W)
            key = f"rD3Q7_ncde_{st}"
            per[key] = lattice_entry(f"rD3Q7 NCDE 3D Gaussian 256x256x128 dz=2dx {st} AA, linear equilibrium + "
                                     f"dB/dt history", 7, st, N_h, K, w2, e2, extra_bytes=8)
            per[key]["finite"] = fin
        del phi
    if "q9tg" in only:
        log("[bench] rD2Q9 TG 64x32 f64")
        from inputs import taylor_green_2d
        prm = dict(lattice="Q9", n=(64, 32, 1), dx=(1.0, 0.5, 1.0), nu=0.02, nu_b=0.05, storage="f64", pattern="AA")
        rho, u, _ = taylor_green_2d(64, 32, 1.0, 0.5, 0.01, 0.25 / 3.0, noise=1e-4, seed=1)
        w2, e2, fin = run_single(torch, R, prm, rho, u, 2000, W)
        per["rD2Q9_tg_f64"] = lattice_entry("rD2Q9 NSE TG 64x32 dy=0.5 FP64 (launch-bound, MLUPS only)", 9, "f64",
                                            2048, 2000, w2, e2)
        per["rD2Q9_tg_f64"].pop("pct_hbm_peak")
    if "bases" in only:
        per["moment_bases"] = bench_bases(torch, R, K, W, prm_h, head)
    if "q27batch" in only:
        log("[bench] rD3Q27 batch of 64 channels f32dev")
        per["rD3Q27_batch64_f32dev"] = bench_batch(torch, R, max(K // 10, 20), W)
        log("[bench] rD3Q27 batch of 512 small channels f32dev")
        per["rD3Q27_batch512_small_f32dev"] = bench_batch(torch, R, K, W, nd=512, nmin=16, nmax=48)

    out = {"metric": METRIC, "value": head["MLUPS"], "unit": "MLUPS", "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "rD3Q19 NSE 3D Taylor-Green, periodic 256x256x128 nodes, dz = 2 dx, U0 = 0.02, "
                                  "nu = 0.005, FP32 deviation storage, FP32 collision, AA pattern",
                      "lattice": "rD3Q19", "nodes": N_h, "storage": "f32dev", "pattern": "AA"},
           "roofline": roofline}
    if ceiling:
        out["hbm_copy_ceiling"] = ceiling
        mall_ceiling["note"] = ("the same copy over 96 MiB source and destination, which stay in the 256 MB "
                                "memory-side cache (MALL) from pass to pass: the most any reuse of data across "
                                "steps through that cache could reach")
        out["mall_copy_ceiling"] = mall_ceiling
        roofline["frac_of_copy_ceiling"] = round(achieved / ceiling["GBps"], 4)
        roofline["note"] = ("achieved = algorithmic bytes / kernel time; with the alternating tile order each step "
                            "starts on data the 256 MB MALL still holds from the previous step, so achieved can "
                            "exceed the copy ceiling, which streams 4 GiB with no reuse")
    out["per_lattice"] = per
    if args.only == "all" and not args.no_warmstart:
        # reduced live study (the full one: --warmstart --ws-train 2000 --ws-test 100 --ws-epochs 120)
        log("[bench] warm-start study (reduced)")
        ws_args = argparse.Namespace(ws_train=384, ws_test=50, ws_epochs=100, ws_train_tol=1e-5,
                                     ws_max_steps=300_000, ws_log=None)
        ws = warmstart_study(torch, ws_args)
        for m in ws["results"].values():
            m.pop("steps_per_domain", None)
        ws.pop("stages", None)
        out["warm_start"] = ws
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"], ref = cpu_baseline()
        out["accuracy_vs_fp64_oracle"] = accuracy_vs_oracle(torch, R, ref)
    print(json.dumps(out), flush=True)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def bench_bases(torch, R, K, W, prm_h, head):
    """The collision in the central, Hermite, central-Hermite and BHLL moments
    (eq. 5-1-1 / 5-1-2) at full size, FP32-dev AA, next to the raw-moment
    collision of the same lattice and workload: the basis transforms add
    arithmetic per node, the bytes per update stay 2 q sizeof."""
    from inputs import taylor_green_2d
    n3, dx3 = prm_h["n"], prm_h["dx"]
    N3 = n3[0] * n3[1] * n3[2]
    out = {}
    rho, u = tg3d_fields(n3, dx3, 0.02, 1.0 / 3.0)
    cases3 = [("rD3Q19_hermite", "Q19", dict(hermite=True)),
              ("rD3Q27_raw", "Q27", {}),
              ("rD3Q27_central", "Q27", dict(central=True)),
              ("rD3Q27_hermite", "Q27", dict(hermite=True)),
              ("rD3Q27_central_hermite", "Q27", dict(central=True, hermite=True))]
    for key, lat, extra in cases3:
        log(f"[bench] moment bases: {key}")
        prm = dict(prm_h, lattice=lat, **extra)
        w2, e2, fin = run_single(torch, R, prm, rho, u, K, W)
        q = 19 if lat == "Q19" else 27
        out[key] = lattice_entry(f"{lat} NSE TG 256x256x128 dz=2dx FP32-dev AA, basis {extra or 'raw'}", q,
                                 "f32dev", N3, K, w2, e2)
        out[key]["finite"] = fin
    out["rD3Q19_hermite"]["vs_raw"] = round(out["rD3Q19_hermite"]["MLUPS"] / head["MLUPS"], 3)
    for key in ("rD3Q27_central", "rD3Q27_hermite", "rD3Q27_central_hermite"):
        out[key]["vs_raw"] = round(out[key]["MLUPS"] / out["rD3Q27_raw"]["MLUPS"], 3)
    del rho, u
    nx, ny = 4096, 2048
    rho2, u2, _ = taylor_green_2d(nx, ny, 1.0, 0.5, 0.02, 0.25 / 3.0)
    base2 = dict(lattice="Q9", n=(nx, ny, 1), dx=(1.0, 0.5, 1.0), nu=0.01, nu_b=0.03, s_hi=1.2,
                 storage="f32dev", pattern="AA")
    for key, extra in (("rD2Q9_raw", {}), ("rD2Q9_bhll", dict(bhll=True)), ("rD2Q9_hermite", dict(hermite=True)),
                       ("rD2Q9_central", dict(central=True))):
        log(f"[bench] moment bases: {key}")
        w2, e2, fin = run_single(torch, R, dict(base2, **extra), rho2, u2, K, W)
        out[key] = lattice_entry(f"rD2Q9 NSE TG {nx}x{ny} dy=0.5 FP32-dev AA, basis {extra or 'raw'}", 9,
                                 "f32dev", nx * ny, K, w2, e2)
        out[key]["finite"] = fin
    for key in ("rD2Q9_bhll", "rD2Q9_hermite", "rD2Q9_central"):
        out[key]["vs_raw"] = round(out[key]["MLUPS"] / out["rD2Q9_raw"]["MLUPS"], 3)
    return out


def bench_local(torch, R, prm, rho, u, N, reps=50):
    """On-demand strain-rate output of the headline domain (FP32 state, FP32
    output): HIP-event time per call and its bytes (q populations read, six
    components written)."""
    dom = R.Domain(R.make_params(**prm), rho, u)
    dom.step(3)
    out = torch.empty(6 * N, dtype=torch.float32, device="cuda")
    lib = R.lib()
    def call(n):
        for _ in range(n):
            R._check(lib.rmrt_local_gradients(dom._ctx, R.GRAD_STRAIN, R._ptr(out), R.OUT_F32, R._stream()),
                     "rmrt_local_gradients")
    settle(torch, R)
    wall, ev_ms = timed_steps(torch, call, reps, 3)
    dom.close()
    del out
    torch.cuda.empty_cache()
    bpn = 19 * 4 + 6 * 4
    us = ev_ms / reps * 1e3
    return {"workload": "rmrt_local_gradients(GRAD_STRAIN) on the rD3Q19 256x256x128 FP32-dev state, FP32 output",
            "us_per_call": round(us, 1), "bytes_per_node": bpn,
            "kernel_GBps": round(bpn * N / (us * 1e-6) / 1e9, 1),
            "pct_hbm_peak": round(100 * bpn * N / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 1)}


def bench_step_local(torch, R, prm, rho, u, N, reps=50):
    """rmrt_step_local on the headline domain: one step fused with the FP32
    strain-rate output of the state it starts from (HIP-event time per call;
    bytes: q populations read and written, six components written)."""
    dom = R.Domain(R.make_params(**prm), rho, u)
    dom.step(2)
    out = torch.empty(6 * N, dtype=torch.float32, device="cuda")
    lib = R.lib()
    def call(n):
        for _ in range(n):
            R._check(lib.rmrt_step_local(dom._ctx, R.GRAD_STRAIN, R._ptr(out), R.OUT_F32, R._stream()),
                     "rmrt_step_local")
    settle(torch, R)
    wall, ev_ms = timed_steps(torch, call, reps, 4)
    dom.close()
    del out
    torch.cuda.empty_cache()
    bpn = 2 * 19 * 4 + 6 * 4
    us = ev_ms / reps * 1e3
    return {"workload": "rmrt_step_local(GRAD_STRAIN): one rD3Q19 256x256x128 FP32-dev AA step fused with its "
                        "FP32 strain-rate output",
            "us_per_step": round(us, 1), "MLUPS": round(N / (us * 1e-6) / 1e6, 1), "bytes_per_node": bpn,
            "kernel_GBps": round(bpn * N / (us * 1e-6) / 1e9, 1),
            "pct_hbm_peak": round(100 * bpn * N / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 1)}


def bench_batch(torch, R, steps, warmup, nd=64, nmin=32, nmax=256, seq_steps=20):
    """One graph-captured persistent launch per step over nd force-driven rD3Q27
    channels (sizes U{nmin..nmax} per axis, seed 4), autotuned; then the same
    domains as nd separate contexts stepped one after the other (each with its
    default launch and graph replay), the plain path the batch replaces."""
    import numpy as np
    from inputs import channel_batch
    doms = channel_batch(seed=4, nd=nd, nmin=nmin, nmax=nmax)
    params = []
    total = 0
    for d in doms:
        params.append(R.make_params(lattice="Q27", n=d["n"], dx=d["dx"], nu=d["nu"], nu_b=d["nu_b"],
                                    force=d["force"], wall_faces=R.WALL_YM | R.WALL_YP | R.WALL_ZM | R.WALL_ZP,
                                    storage="f32dev", pattern="AA", rho0=1.0))
        total += d["n"][0] * d["n"][1] * d["n"][2]
    b = R.Batch(params)
    torch.cuda.synchronize()
    cfg = b.autotune(steps=4)
    settle(torch, R)
    wall, ev_ms = timed_steps(torch, b.step, steps, warmup, prepare=b.prepare)
    red = b.domains[0].reduce()
    fin = all(math.isfinite(v) for v in red)
    e = lattice_entry(f"rD3Q27 batch of {nd} force-driven channels (seed 4, {nmin}..{nmax} nodes per axis), "
                      f"{total} nodes, FP32-dev AA, graph-captured launches over a tile list (one per step, or "
                      f"one per domain group and step)", 27, "f32dev", total, steps, wall, ev_ms)
    e["autotuned_config"] = dict(zip(CONFIG_KEYS, R.Batch.configs()[cfg]))
    gbytes, ngroups = b.group_bytes()
    e["autotuned_groups"] = {"group_bytes": gbytes, "groups": ngroups}
    mode, nchunked = b.xcd_chunks()
    e["autotuned_xcd_chunks"] = {"mode": mode, "groups_with_straddling_rows": nchunked}
    e["finite"] = fin
    # the single persistent launch per step (one group): its best tile shape
    b.set_group_bytes(0)
    best = None
    for k, shape in enumerate(R.Batch.configs()):
        if not shape[3]:
            continue
        b.set_config(k)
        w_k, ev_k = timed_steps(torch, b.step, min(steps, 20), 4, prepare=b.prepare)
        if best is None or ev_k < best[1]:
            best = (k, ev_k, min(steps, 20))
    k, ev_k, n_k = best
    e["persistent_single_launch"] = {
        "MLUPS": round(total * n_k / (ev_k * 1e-3) / 1e6, 1),
        "kernel_GBps": round(total * 2 * 27 * sizeof("f32dev") / (ev_k / n_k * 1e-3) / 1e9, 1),
        "config": dict(zip(CONFIG_KEYS, R.Batch.configs()[k])), "steps": n_k,
        "note": "best persistent tile shape with every domain in one launch per step (HIP events)"}
    b.close()
    del b
    torch.cuda.empty_cache()
    ctxs = []
    for prm, d in zip(params, doms):
        N = d["n"][0] * d["n"][1] * d["n"][2]
        ctxs.append(R.Domain(prm, np.ones(N), np.zeros((3, N))))
    def seq(n):
        for c in ctxs:
            c.step(n)

    def seq_prepare(n):
        for c in ctxs:
            c.prepare(n)
    settle(torch, R)
    seq_wall, _ = timed_steps(torch, seq, seq_steps, 2, prepare=seq_prepare)
    for c in ctxs:
        c.close()
    del ctxs
    torch.cuda.empty_cache()
    seq_mlups = total * seq_steps / seq_wall / 1e6
    e["sequential_contexts"] = {"MLUPS": round(seq_mlups, 1), "steps": seq_steps,
                                "note": f"the {nd} domains as separate contexts, stepped one after the other"}
    e["speedup_vs_sequential"] = round(e["MLUPS"] / seq_mlups, 3)
    return e


def warmstart_study(torch, args):
    """Steps and time to a 1e-6 steady residual for cold, Poiseuille-prior and
    surrogate warm starts on held-out rD2Q9 obstacle channels (512 x 256,
    dy = 0.5, walls at the y faces, force-driven, Re 10..100)."""
    import numpy as np
    from inputs import obstacle_channel
    from paper_2206_00366_amd import surrogate as S

    stages = []

    def record(name, **kw):
        kw["stage"] = name
        stages.append(kw)
        log(json.dumps(kw))
        if args.ws_log:
            with open(args.ws_log, "a") as fh:
                fh.write(json.dumps(kw) + "\n")

    nb = 64
    t_start = time.perf_counter()
    # ---- training set: steady fields from the solver (Poiseuille-prior start) ----
    X, T, Wt = [], [], []
    gen_steps = 0
    cfg = None
    for s0 in range(0, args.ws_train, nb):
        geoms = [obstacle_channel(seed) for seed in range(s0, min(s0 + nb, args.ws_train))]
        b = S.make_batch(geoms)
        if cfg is None:
            cfg = b.autotune(steps=20)
            group_bytes = b.group_bytes()[0]
            record("autotune", config=dict(zip(CONFIG_KEYS, b.configs()[cfg])), group_bytes=group_bytes)
        else:
            b.set_config(cfg)
            b.set_group_bytes(group_bytes)
        rho, u = S.initial_fields(geoms)
        S.apply_initial(b, rho, u)
        steps, conv, wall, n, _ = S.run_to_steady(b, tol=args.ws_train_tol, max_steps=args.ws_max_steps, log=log,
                                               label=f"train batch {s0 // nb}")
        tgt, wgt = S.steady_targets(b, geoms)
        x0, _ = S.features(geoms)
        X.append(x0)
        T.append(tgt)
        Wt.append(wgt)
        gen_steps += n
        record("train_batch", first_seed=s0, domains=len(geoms), steps=int(n), converged=int(conv.sum()),
               wall_s=round(wall, 1))
        b.close()
        del b
    X, T, Wt = torch.cat(X), torch.cat(T), torch.cat(Wt)
    t_gen = time.perf_counter() - t_start
    # ---- training ----
    net = S.Surrogate(seed=0, B=16, H=X.shape[1], W=X.shape[2])
    t0 = time.perf_counter()
    hist = S.train(net, X, T, Wt, epochs=args.ws_epochs, batch_size=16, lr=2e-3, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    record("train", samples=int(X.shape[0]), epochs=args.ws_epochs, loss_first=hist[0], loss_last=hist[-1],
           wall_s=round(t_train, 1))
    # ---- evaluation on held-out geometries ----
    test = [obstacle_channel(seed) for seed in range(2000, 2000 + args.ws_test)]
    results = {}
    for mode in ("cold", "prior", "warm"):
        all_steps, all_conv, all_time, wall_tot, inf_tot = [], [], [], 0.0, 0.0
        restarts = 0
        for s0 in range(0, len(test), 50):
            geoms = test[s0:s0 + 50]
            b = S.make_batch(geoms)
            b.set_config(cfg)
            b.set_group_bytes(group_bytes)
            t_inf = 0.0
            if mode != "cold":
                torch.cuda.synchronize()
                ti = time.perf_counter()
                out = S.predict(net, geoms)[0] if mode == "warm" else None
                rho, u = S.initial_fields(geoms, out)
                S.apply_initial(b, rho, u)
                torch.cuda.synchronize()
                t_inf = time.perf_counter() - ti
            steps, conv, wall, n, rst = S.run_to_steady(b, tol=1e-6, max_steps=args.ws_max_steps, log=log,
                                                        label=f"{mode} batch {s0 // 50}", fallback=mode != "cold")
            restarts += int(rst.sum())
            all_steps.append(steps)
            all_conv.append(conv)
            # per-domain time: its steps at the batch's cost per domain-step, plus its share of the init
            all_time.append(steps * wall / (len(geoms) * max(n, 1)) + t_inf / len(geoms))
            wall_tot += wall
            inf_tot += t_inf
            b.close()
            del b
        st = np.concatenate(all_steps)
        cv = np.concatenate(all_conv)
        tm = np.concatenate(all_time)
        ok = st[cv]
        results[mode] = {"converged": int(cv.sum()), "not_converged": int((~cv).sum()),
                         "mean_steps": float(ok.mean()) if ok.size else None,
                         "median_steps": float(np.median(ok)) if ok.size else None,
                         "mean_time_s": float(tm[cv].mean()) if ok.size else None,
                         "median_time_s": float(np.median(tm[cv])) if ok.size else None,
                         "batch_wall_s": round(wall_tot, 1), "init_s": round(inf_tot, 3),
                         "cold_restarts": restarts,
                         "steps_per_domain": st.tolist()}
        record("eval", mode=mode, **{k: v for k, v in results[mode].items() if k != "steps_per_domain"})
    cold = np.array(results["cold"]["steps_per_domain"], dtype=float)
    for mode in ("prior", "warm"):
        st = np.array(results[mode]["steps_per_domain"], dtype=float)
        results[mode]["median_step_ratio_vs_cold"] = float(np.median(st / cold))
    results["warm"]["median_step_ratio_vs_prior"] = float(
        np.median(np.array(results["warm"]["steps_per_domain"], float) /
                  np.array(results["prior"]["steps_per_domain"], float)))
    return {"metric": "steps and time to a 1e-6 steady residual: cold vs Poiseuille prior vs surrogate warm start",
            "workload": "rD2Q9 NSE obstacle channels 512x256, dy = 0.5, Re 10-100, 1-8 obstacles, FP32-dev AA, "
                        "batches of 50 domains per launch",
            "train_fields": int(X.shape[0]), "train_tol": args.ws_train_tol, "generation_s": round(t_gen, 1),
            "training_s": round(t_train, 1), "test_fields": len(test), "max_steps": args.ws_max_steps,
            "results": results, "stages": stages}


if __name__ == "__main__":
    main()
