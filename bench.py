#!/usr/bin/env python3
"""Throughput of simulated annealing tomography with a PILA on one MI355X.

Workload: one annealing chain on a 256 x 256 slice (10 random ellipses),
180 angles in [0, 180), 367 unit bins, photon noise at I0 = 1e4 per ray,
circular support, best of M = 16 estimates per step, 5e6 steps, FP32
residual rebuilt in FP64 every 4096 accepted nonzero changes, T0 from
Eq. 8 (Q = 200) and T_N = T0 / 1e3 under linear cooling over 1000 stages.

One benchmark step is one pass of the whole path over that slice: PILA
build (pixel-major and ray-major), starting image, residual and Eq. 8, the
5e6-step chain with its resyncs.  Inputs are in device memory before the
timed region.  Reported value: SA estimates (proposals) evaluated per
second over the timed steps.  Beside it: steps/s, slices/s, per-slice
latency, final RMSE of the FP32 chain and of an FP64 chain with the same
seeds, the roofline of the chain kernel, and the CPU oracle timed on a
bounded sample of the same chain.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


def chain_kernel_bytes(n_steps: int, M: int, f_mean: float, accepts: int) -> float:
    """Algorithmic bytes of the chain kernel over a whole chain (FP32 PILA and residual).

    per estimate: support index 4, image value 8, row offsets 16, and per row
    entry ray index 4 + length 4 + residual 4; per accepted estimate: per row
    entry ray index 4 + length 4 + residual read 4 + write 4, image write 8.
    The FP64 rebuilds at the resyncs (per PILA entry pixel index 4 + length 4
    + image value 8, per ray 32) run in their own kernel and are not counted.
    """
    return n_steps * M * (28.0 + 12.0 * f_mean) + accepts * (8.0 + 16.0 * f_mean)


# HBM bytes per chain-kernel launch from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs of this benchmark, each scaled by the factor that makes the counter
# read the known size of a plain device copy in the same run; valid only for
# the kernel sources they were taken with (hash over the files below)
TRAFFIC_SOURCES = ("paper_1411_4622_amd/csrc/sat_chain.hpp", "paper_1411_4622_amd/csrc/sat.hip",
                   "paper_1411_4622_amd/csrc/common.hpp")
TRAFFIC = {"sources_sha256": "cec2281accac605fc0998dce270a3680c42776dae036492060191677cfa4a570",
           "bytes_per_launch": 143386283.5}


def sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cpu_baseline(sl, cfg, n_steps_cpu: int) -> dict:
    import oracle
    log("cpu baseline: oracle PILA for %dx%d, %d angles" % (sl.N, sl.N, sl.U))
    csr = oracle.pila(sl.N, sl.U, sl.K, sl.angles, sl.mask)
    kw = dict(seed=cfg["chain_seed"], chain_id=0, n_steps=n_steps_cpu, n_stages=cfg["n_stages"],
              m_cand=cfg["M"], T0=None, q_auto=cfg["q_auto"], tn_ratio=cfg["tn_ratio"],
              delta_max=cfg["delta_max"], f_min=cfg["f_min"], f_max=cfg["f_max"],
              precision=cfg["precision"], resync_every=cfg["resync_every"])
    log("cpu baseline: oracle chain, %d steps" % n_steps_cpu)
    t0 = time.perf_counter()
    oracle.sat_run(sl.N, sl.U, sl.K, csr, sl.sino, sl.f0, mask=sl.mask, trace=False, **kw)
    dt = time.perf_counter() - t0
    return {"value": n_steps_cpu * cfg["M"] / dt, "unit": "proposals/s", "cores": 1, "kind": "oracle",
            "sample": "the same chain (same slice, M, FP32 residual with FP64 resync) cut to its "
                      "first %d of %d steps, single thread, %.1f s; PILA build not timed"
                      % (n_steps_cpu, cfg["n_steps"], dt),
            "cpu": _cpu_model(), "nproc": os.cpu_count()}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chain-steps", type=int, default=None,
                    help="override the chain length (profiling runs); the reported config says so")
    ap.add_argument("--cpu-steps", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (counter "
                         "calibration for rocprofv3 --pmc runs)")
    ap.add_argument("--workload", default="c2", choices=("c2", "c3", "c4", "c5"),
                    help="c2 (default): the single-chain benchmark line; c3: batch of slices; "
                         "c4: 1024^2 slice, SAT M=32 and SIRT; c5: serving stream")
    ap.add_argument("--slices", type=int, default=512, help="c3: slices in the batch")
    ap.add_argument("--distinct", type=int, default=64,
                    help="c3: distinct phantoms generated (the rest repeat them with other seeds)")
    ap.add_argument("--requests", type=int, default=2000, help="c5: requests in the stream")
    ap.add_argument("--rate", type=float, default=200.0, help="c5: arrivals per second")
    ap.add_argument("--sweeps", type=float, default=None, help="c3/c5: steps = sweeps x support")
    ap.add_argument("--sat-steps", type=int, default=None, help="c4: chain steps")
    ap.add_argument("--mem-budget-gb", type=float, default=96.0, help="c5: server memory budget")
    ap.add_argument("--general-slots", type=int, default=16,
                    help="c5: server slots for the general body")
    ap.add_argument("--long-slots", type=int, default=60,
                    help="c5: server slots for the long-row body (720 angles)")
    ap.add_argument("--max-slots", type=int, default=0,
                    help="c5: server workgroups in all (0: the library's default)")
    ap.add_argument("--idle-ms", type=float, default=20.0,
                    help="c5: idle time after which the server's resident kernels end")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU: an annealing chain does not shard across GPUs, and this "
              "build measures the one-GPU path only (--gpus 1).", file=sys.stderr)
        return 2
    if args.workload != "c2":
        import bench_workloads
        return bench_workloads.run(args)

    import torch
    import datagen
    import paper_1411_4622_amd as P

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cfg = dict(datagen.CONFIGS["c2"])
    if args.chain_steps:
        cfg["n_steps"] = int(args.chain_steps)
    log("input: c2 slice (analytic ellipse sinogram + Poisson noise)")
    sl = datagen.config_slice("c2")
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32")
    sino = torch.from_numpy(sl.sino).to(dev)
    f0 = torch.from_numpy(sl.f0).to(dev)
    img = torch.empty_like(f0)
    prm = P.SatParams(n_steps=cfg["n_steps"], seed=cfg["chain_seed"], chain_id=0,
                      n_stages=cfg["n_stages"], m_cand=cfg["M"], T0=None, q_auto=cfg["q_auto"],
                      precision="f32", tn_ratio=cfg["tn_ratio"], delta_max=cfg["delta_max"],
                      f_min=cfg["f_min"], f_max=cfg["f_max"], resync_every=cfg["resync_every"])
    ws = P.sat_workspace(geom, prm, dev)
    stream = torch.cuda.current_stream()

    kernel_ms = []
    launch_stats = []
    last = {}

    def one_step():
        pl = P.pila_build(geom)
        img.copy_(f0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st, _ = P.sat_run(pl, sino, prm, img, workspace=ws)
        e1.record(stream)
        e1.synchronize()
        kernel_ms.append(e0.elapsed_time(e1))
        launch_stats.append((st["chain_launches"], st["chain_kernel_ms"]))
        last["stats"] = st
        last["pila"] = (pl.nnz, pl.n_support)

    for w in range(args.warmup):
        one_step()
        log("warmup %d/%d: chain %.1f ms" % (w + 1, args.warmup, kernel_ms[-1]))
    kernel_ms.clear()
    launch_stats.clear()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        one_step()
        lat.append(time.perf_counter() - ts)
        log("step %d/%d: %.3f s (chain kernel %.1f ms)" % (k + 1, args.steps, lat[-1], kernel_ms[-1]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    st = last["stats"]
    nnz, P_sup = last["pila"]
    proposals = args.steps * cfg["n_steps"] * cfg["M"]
    value = proposals / wall
    f32_img = img.cpu().numpy()
    rmse32 = datagen.rmse(f32_img, sl.truth)

    rmse64 = None
    if not args.no_fp64_reference:
        log("fp64 reference chain (same seeds, untimed)")
        g64 = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f64")
        pl64 = P.pila_build(g64)
        img64 = f0.clone()
        p64 = P.SatParams(**{**prm.__dict__, "precision": "f64", "resync_every": 0})
        P.sat_run(pl64, sino, p64, img64)
        torch.cuda.synchronize()
        rmse64 = datagen.rmse(img64.cpu().numpy(), sl.truth)
        del pl64

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d MiB read + %d MiB written per copy, 3 copies"
            % (args.copy_probe_mib, args.copy_probe_mib))
        del src, dst

    f_mean = nnz / P_sup
    # chain-kernel launches of the timed steps, each timed by the library with
    # HIP events on the chain's stream; every step runs the same chain
    launches = max(int(st["chain_launches"]), 1)
    launch_s = sum(ms for _, ms in launch_stats) / 1e3 / max(sum(n for n, _ in launch_stats), 1)
    alg_bytes = chain_kernel_bytes(cfg["n_steps"], cfg["M"], f_mean, st["accepts"]) / launches
    achieved = alg_bytes / launch_s / 1e9
    traffic = None
    if TRAFFIC and TRAFFIC.get("sources_sha256") == sources_hash() and not args.chain_steps:
        traffic = TRAFFIC["bytes_per_launch"]

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sl, cfg, args.cpu_steps)

    info = P.device_info()
    out = {
        "metric": "SA proposals evaluated/s + slices/s at fixed RMSE; p50/p99 slice latency",
        "value": value,
        "unit": "proposals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded 10-ellipse phantom, analytic line integrals, Poisson noise I0=1e4",
        "config": {"workload": "single SA chain, 256x256 slice, 180 angles, 367 bins, circular "
                               "support, BoME M=16, %d steps, FP32 residual with FP64 resync every "
                               "4096 accepts, Eq. 8 T0" % cfg["n_steps"],
                   "N": sl.N, "U": sl.U, "K": sl.K, "M": cfg["M"], "n_steps": cfg["n_steps"]},
        "steps_per_s": args.steps * cfg["n_steps"] / wall,
        "slices_per_s": args.steps / wall,
        "latency_s_p50": float(np.percentile(lat, 50)),
        "latency_s_p99": float(np.percentile(lat, 99)),
        "rmse_fp32": rmse32,
        "rmse_fp64": rmse64,
        "rmse_ratio_fp32_fp64": (rmse32 / rmse64) if rmse64 else None,
        "nrmse_fp32": rmse32 / float(np.mean(sl.truth)),
        "chain": {"accepts": st["accepts"], "accepts_nonzero": st["accepts_nonzero"],
                  "resyncs": st["resyncs"], "T0": st["T0_used"], "max_drift_r": st["max_drift_r"],
                  "max_drift_sse": st["max_drift_sse"], "cost_final": st["cost_final"]},
        "roofline": {"kernel": "sat_segment_kernel (one launch per resync segment of the chain)",
                     "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "launches_per_step": launches,
                     "avg_launch_ms": 1e3 * launch_s,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "chain_ms_per_step": statistics.mean(kernel_ms)},
        "cpu_baseline": cpu,
        "device": info,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
