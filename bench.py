#!/usr/bin/env python3
"""Throughput of simulated annealing tomography with a PILA on one MI355X.

Workload (default): a batch of 512 independent slices cut from one seeded
3-D volume of 32 random ellipsoids, each slice N x N with N drawn from
{128, 256, 512} and U angles from {90, 180, 360} in [0, 180), K =
ceil(sqrt(2) N) unit bins, photon noise at I0 = 1e4 per ray, circular
support; one annealing chain per slice: best of M = 8 estimates per step,
16 sweeps of the support (steps = 16 x support pixels), FP32 residual
rebuilt in FP64 every max(4096, nnz / 128) accepted nonzero changes, T0
from Eq. 8 (Q = 200), T_N = T0 / 1e3, linear cooling over 1000 stages.

One benchmark step is one pass of the whole path over that batch: the nine
PILAs (pixel-major and ray-major), the starting images, and the batched
chains (residuals, Eq. 8, the chains and their resyncs).  Inputs are in
device memory before the timed region.  Reported value: SA estimates
(proposals) evaluated per second over the timed steps.  Beside it: steps/s,
slices/s, per-slice latency inside a batch (p50/p99), final RMSE and NRMSE
of every slice and its ratio to an FP64 batch with the same seeds, the
batch against the same chains run one at a time (sat_run), the roofline of
the kernel that runs longest, the CPU oracle on a bounded sample of the same
chains, and the noise-free 64 x 64 quality check of section III-B.

Other workloads: --workload c2 (one chain, 256^2 x 180, M = 16), c3r (the
batch with repeated phantoms), c4 (1024^2 x 720: SAT M = 32 and SIRT), c5
(serving stream).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


def chain_bytes(n_steps: int, M: int, f_mean: float, accepts: int, len_bytes: int = 4) -> float:
    """Algorithmic bytes of one FP32 chain in a batch.

    per estimate: support index 4, image value 8, row offsets 16, and per row
    entry slot word 4 + length (4, or 1 for one-byte lengths) + residual 4;
    per accepted estimate: per row entry slot word 4 + length + residual read
    4 + write 4, image write 8.  In-group FP64 resyncs (per PILA entry pixel
    4 + length + image 8) are not counted.
    """
    return (n_steps * M * (28.0 + (8.0 + len_bytes) * f_mean)
            + accepts * (8.0 + (12.0 + len_bytes) * f_mean))


# HBM bytes per dispatch of the kernel the roofline reports, from two
# rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, then WRITE_SIZE, KiB
# per dispatch), each scaled by the factor that makes the counter read the
# known size of a plain device copy in the same run; valid only for the
# kernel sources they were taken with (hash over the files below)
TRAFFIC_SOURCES = ("paper_1411_4622_amd/csrc/sat_chain.hpp", "paper_1411_4622_amd/csrc/sat.hip",
                   "paper_1411_4622_amd/csrc/common.hpp", "bench_workloads.py")
TRAFFIC = {"kernel": "sat_batch_kernel<float,1,8>",
           "sources_sha256": "b70ca5d2de377365d7b6ceebbfdd3ddfd87111ddc20a1f37e16a83d509f7cdcc",
           "fetch_kib": 9659812400.5625, "fetch_factor": 524288.0 / 262155.5,
           "write_kib": 1120302595.90625, "write_factor": 524288.0 / 524288.0,
           "bytes_per_dispatch": 9659812400.5625 * 1024 * (524288.0 / 262155.5) + 1120302595.90625 * 1024 * (524288.0 / 524288.0),
           "profile": "profiles/sat_batch_kernel_c3_512slices.md"}


def sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _pool(procs):
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    return ProcessPoolExecutor(max_workers=procs, mp_context=mp.get_context("spawn"))


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the host cores, one process per chain
# ---------------------------------------------------------------------------

def _cpu_pila(arg):
    """Build one geometry's oracle PILA and save it (worker process)."""
    import datagen
    import oracle
    N, U, K, where = arg
    rp, col, ln = oracle.pila(N, U, K, datagen.angles_deg(U), datagen.circle_mask(N))
    np.save(where + "_rp.npy", rp)
    np.save(where + "_col.npy", col)
    np.save(where + "_len.npy", ln)
    return where


def _cpu_chain(arg):
    """One oracle chain, cut to its first steps (worker process)."""
    import datagen
    import oracle
    where, N, U, K, sino, f0, kw = arg
    csr = tuple(np.load(where + s, mmap_mode="r") for s in ("_rp.npy", "_col.npy", "_len.npy"))
    csr = tuple(np.ascontiguousarray(a) for a in csr)
    t0 = time.perf_counter()
    oracle.sat_run(N, U, K, csr, sino, f0, mask=datagen.circle_mask(N), trace=False, **kw)
    return time.perf_counter() - t0


class CpuBaseline:
    """The oracle (FP32 residual with FP64 resync, as the GPU chains) on a
    bounded sample of the batch's chains: those of the 128^2 and 256^2 slices
    (the oracle's ray-traced PILA of a 512^2 slice takes a minute to build),
    taken in turn from each geometry until there are two per host core, each
    cut to its first steps so that it does about 1.5e8 row entries of work.
    The PILAs are built first in a pool of their own; the chains then run
    one per process on the host cores and their wall time gives
    proposals/s.  Runs in the background while the GPU
    does other work."""

    def __init__(self, slices, params, cfg, procs):
        self.procs = procs
        self.tmp = tempfile.TemporaryDirectory(prefix="pila_cpu_")
        by_key = {}
        for c, sl in enumerate(slices):
            if sl.N <= 256:
                by_key.setdefault((sl.N, sl.U, sl.K), []).append(c)
        self.keys = sorted(by_key)
        self.chains = []
        M = cfg["M"]
        picks = []
        i = 0
        while len(picks) < 2 * procs and any(i < len(v) for v in by_key.values()):
            picks += [(key, by_key[key][i]) for key in self.keys if i < len(by_key[key])]
            i += 1
        for key, c in picks[:2 * procs]:
            F = 4.0 / math.pi * key[1]  # mean row length
            steps = int(min(params[c].n_steps, 1.5e8 / (M * F)))
            p = params[c]
            kw = dict(seed=p.seed, chain_id=p.chain_id, n_steps=steps, n_stages=p.n_stages,
                      m_cand=p.m_cand, T0=None, q_auto=p.q_auto, tn_ratio=p.tn_ratio,
                      delta_max=p.delta_max, f_min=p.f_min, f_max=p.f_max, precision="f32",
                      resync_every=p.resync_every)
            self.chains.append((key, slices[c].sino, slices[c].f0, kw, steps * M))
        self.ex = _pool(procs)

    def start(self):
        import threading
        self.result = None

        def work():
            t0 = time.perf_counter()
            where = {k: os.path.join(self.tmp.name, "%d_%d_%d" % k) for k in self.keys}
            list(self.ex.map(_cpu_pila, [(k[0], k[1], k[2], where[k]) for k in self.keys]))
            t_build = time.perf_counter() - t0
            t1 = time.perf_counter()
            secs = list(self.ex.map(_cpu_chain, [(where[k], k[0], k[1], k[2], s, f, kw)
                                                 for k, s, f, kw, _ in self.chains]))
            wall = time.perf_counter() - t1
            props = sum(c[4] for c in self.chains)
            used = min(self.procs, len(self.chains))
            self.result = {
                "value": props / wall, "unit": "proposals/s", "cores": used, "kind": "oracle",
                "sample": "%d chains of the batch (from its 128^2 and 256^2 geometries: %s), each cut "
                          "to its first steps (about 1.5e8 row entries of work; %d proposals in all), "
                          "one process per chain on %d host cores, %.1f s wall (%.1f s of chain CPU "
                          "time); oracle PILAs built beforehand in %.1f s, not timed"
                          % (len(self.chains), ", ".join("%dx%d" % (k[0], k[1]) for k in self.keys),
                             props, used, wall, sum(secs), t_build),
                "cpu": _cpu_model(), "nproc": os.cpu_count()}

        self.thread = threading.Thread(target=work, daemon=True)
        self.thread.start()

    def finish(self):
        self.thread.join()
        self.ex.shutdown()
        self.tmp.cleanup()
        return self.result


# ---------------------------------------------------------------------------
# the batch benchmark line
# ---------------------------------------------------------------------------

def run_c3(args) -> int:
    import torch
    import datagen
    import paper_1411_4622_amd as P
    from bench_workloads import _params
    from paper_1411_4622_amd import tune

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    cfg = datagen.CONFIGS["c3"]
    n = args.slices
    sweeps = cfg["sweeps"] if args.sweeps is None else args.sweeps
    M = cfg["M"]
    t0 = time.perf_counter()
    specs = datagen.batch_slice_specs(cfg["volume_seed"], n, cfg["sizes"], cfg["n_angles"], cfg["I0"],
                                      cfg["masked"])
    with _pool(16) as ex:
        slices = list(ex.map(datagen.slice_from_spec, specs, chunksize=4))
    log("c3: %d slices generated in %.1f s" % (len(slices), time.perf_counter() - t0))
    keys = sorted({(sl.N, sl.U) for sl in slices})
    geoms = {}
    for sl in slices:
        if (sl.N, sl.U) not in geoms:
            geoms[(sl.N, sl.U)] = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, args.lengths)
    sinos = [torch.from_numpy(sl.sino).to(dev) for sl in slices]
    f0s = [torch.from_numpy(sl.f0).to(dev) for sl in slices]
    imgs = [torch.empty_like(f) for f in f0s]
    pilas = {k: P.pila_build(geoms[k]) for k in keys}
    nnz = {k: pilas[k].nnz for k in keys}
    fmean = {k: pilas[k].nnz / pilas[k].n_support for k in keys}
    params = [_params(P, cfg, round(sweeps * int(sl.mask.sum())), cfg["chain_seed0"] + c, c,
                      nnz=nnz[(sl.N, sl.U)]) for c, sl in enumerate(slices)]
    steps_total = sum(p.n_steps for p in params)
    key_of = [(sl.N, sl.U) for sl in slices]

    waves_of = [0] * n

    def jobs_for(pl, prm=None, widths=None):
        return [P.Job(pl[key_of[c]], sinos[c], imgs[c], (prm or params)[c], (widths or waves_of)[c])
                for c in range(n)]

    # launch shape: each geometry's workgroup width from the stored tuning
    # table, or tuned now on 4096-step prefixes of the same chains
    info = P.device_info()
    jobs0 = jobs_for(pilas)
    stored = None if args.retune else tune.load_table(info["name"])
    per_cu = 1
    if stored and tune.apply_table(jobs0, stored):
        per_cu = int(stored["chains_per_cu"])
        tuning = {"source": "stored table (paper_1411_4622_amd/tuned_launch.json)",
                  "geometries": stored["geometries"]}
    else:
        for c in range(n):
            imgs[c].copy_(f0s[c])
        res = tune.tune_geometries(jobs0, waves=(8, 4), chains_per_cu=per_cu, sample_steps=4096)
        tune.apply_table(jobs0, {"geometries": res})
        tuning = {"source": "tuned in this run", "geometries": res}
        if args.tune_out:
            tune.save_table(res, info["name"], per_cu, 4096, args.tune_out)
    waves_of = [j.waves_per_chain for j in jobs0]
    waves = 8  # the launch default (every job carries its own width)
    log("c3: widths per geometry (%s): %s" % (tuning["source"], ", ".join(
        "%s -> %d" % (k, v["waves_per_chain"]) for k, v in sorted(tuning["geometries"].items()))))
    del pilas, jobs0

    def one_step():
        pl = {k: P.pila_build(geoms[k]) for k in keys}
        for c in range(n):
            imgs[c].copy_(f0s[c])
        groups = []
        st = P.sat_run_batch(jobs_for(pl), waves_per_chain=waves, chains_per_cu=per_cu, groups=groups)
        return st, groups

    for w in range(args.warmup):
        ts = time.perf_counter()
        one_step()
        log("warmup %d/%d: %.2f s" % (w + 1, args.warmup, time.perf_counter() - ts))
    torch.cuda.synchronize()
    lat_step, group_runs = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        st, groups = one_step()
        torch.cuda.synchronize()
        lat_step.append(time.perf_counter() - ts)
        group_runs.append(groups)
        log("step %d/%d: %.2f s (groups: %s)" % (k + 1, args.steps, lat_step[-1],
                                                 ", ".join("%d/%d,%d x%d %.0f ms" % (g["kind"], g["cpw"], g["e"],
                                                                                   g["chains"], g["ms"])
                                                           for g in groups)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    proposals = args.steps * steps_total * M
    value = proposals / wall
    f32_imgs = [im.cpu().numpy() for im in imgs]

    # per-slice latency inside the batch: device clock from the batch's first
    # chain start to each chain's end
    rate = info["wallclock_khz"] * 1e3
    t_first = min(s["t_begin"] for s in st)
    lat_slice = np.array([(s["t_end"] - t_first) / rate for s in st])

    # the plain one-chain form: each geometry's first chain alone (sat_run),
    # all its steps (later steps, with fewer accepted changes, are faster than
    # the first ones), then the serial time of all chains at those rates
    lone_us = {}
    for key in keys:
        c = key_of.index(key)
        steps1 = params[c].n_steps
        pl = P.pila_build(geoms[key])
        im = f0s[c].clone()
        prm1 = _params(P, cfg, steps1, cfg["chain_seed0"] + c, c, nnz=nnz[key])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        P.sat_run(pl, sinos[c], prm1, im, stats=False)
        e1.record()
        e1.synchronize()
        lone_us[key] = 1e3 * e0.elapsed_time(e1) / steps1
    serial_s = sum(params[c].n_steps * lone_us[key_of[c]] / 1e6 for c in range(n))
    log("c3: lone chains %s us/step; serial time of the batch's chains %.1f s"
        % (", ".join("%dx%d %.2f" % (k[0], k[1], v) for k, v in sorted(lone_us.items())), serial_s))

    # CPU oracle in the background while the GPU runs the FP64 reference batch
    cpu = None
    if not args.no_cpu_baseline:
        cpu_job = CpuBaseline(slices, params, cfg, procs=min(16, os.cpu_count() or 1))
        cpu_job.start()

    ratios, rm64 = None, None
    if not args.no_fp64_reference:
        log("c3: FP64 batch with the same seeds (untimed)")
        ts = time.perf_counter()
        g64 = {k: P.Geometry(geoms[k].n, geoms[k].angles, geoms[k].n_bins, geoms[k].mask, "f64") for k in keys}
        pl64 = {k: P.pila_build(g64[k]) for k in keys}
        prm64 = [_params(P, cfg, params[c].n_steps, cfg["chain_seed0"] + c, c, "f64") for c in range(n)]
        for c in range(n):
            imgs[c].copy_(f0s[c])
        P.sat_run_batch(jobs_for(pl64, prm=prm64, widths=[8] * n), waves_per_chain=8, chains_per_cu=1,
                        stats=False)
        torch.cuda.synchronize()
        rm64 = [datagen.rmse(imgs[c].cpu().numpy(), slices[c].truth) for c in range(n)]
        del pl64
        log("c3: FP64 batch in %.1f s" % (time.perf_counter() - ts))

    # the noise-free 64 x 64 check of section III-B: U = 60, N_e = 16, 2e6
    # steps over 1000 stages, Eq. 8 T0.  Noise-free here means data that the
    # pixel model can fit: the projections of the phantom's pixel image by
    # Eq. 1 (the exact line integrals of the continuous ellipses differ from
    # any pixel image's by a floor, cost 0.25 at this size).
    sanity = None
    if not args.no_sanity:
        N0, U0 = 64, 60
        K0 = datagen.n_bins_for(N0)
        ell = datagen.random_ellipses(106, N0, 10)
        sl0 = datagen.make_slice(N0, U0, K0, ell, masked=True, I0=None)
        pl0 = P.pila_build(P.Geometry(N0, sl0.angles, K0, sl0.mask, "f64"))
        truth0 = torch.from_numpy(sl0.truth * sl0.mask).to(dev)
        sino0 = P.pila_forward(pl0, truth0)
        f00 = torch.from_numpy(datagen.uniform_start(sino0.cpu().numpy(), sl0.mask, N0)).to(dev)
        im0 = f00.clone()
        p0 = P.SatParams(n_steps=2_000_000, seed=1006, chain_id=0, n_stages=1000, m_cand=16, T0=None,
                         q_auto=200, delta_max=0.05)
        ts = time.perf_counter()
        st0, _ = P.sat_run(pl0, sino0, p0, im0)
        torch.cuda.synchronize()
        f_s = im0.cpu().numpy()
        t_s = truth0.cpu().numpy()
        sanity = {"setting": "64x64 phantom of 10 ellipses, its pixel image projected by Eq. 1 (noise-free, "
                             "consistent data), U=60, K=91, circular support, N_e=16, 2e6 steps over 1000 "
                             "stages, change in [-0.05, 0.05) clamped to [0, 1], Eq. 8 T0, FP64",
                  "nrmse": datagen.nrmse(f_s, t_s), "rmse": datagen.rmse(f_s, t_s),
                  "cost_final": st0["cost_final"],
                  "paper": "NRMSE below 5% after N=200 of 1000 stages (section III-B, on its phantom)",
                  "seconds": time.perf_counter() - ts}
        log("c3: section III-B check: NRMSE %.4f" % sanity["nrmse"])

    if not args.no_cpu_baseline:
        cpu = cpu_job.finish()
        log("c3: cpu baseline %.3g proposals/s on %d cores" % (cpu["value"], cpu["cores"]))

    # roofline of the group kernel that runs longest (its chains' algorithmic
    # bytes over its duration from HIP events on its stream, averaged over
    # the timed steps); the whole batch beside it
    body_of = [s["body"] for s in st]
    acc = [s["accepts"] for s in st]
    lb = 1 if args.lengths == "u8" else 4
    b_chain = [chain_bytes(params[c].n_steps, M, fmean[key_of[c]], acc[c], lb) for c in range(n)]
    gdesc = [(g["kind"], g["cpw"], g["e"], g["waves"]) for g in group_runs[-1]]
    g_ms = {d: statistics.mean(next(g["ms"] for g in run if (g["kind"], g["cpw"], g["e"], g["waves"]) == d)
                                for run in group_runs) for d in gdesc}
    dom = max(g_ms, key=g_ms.get)

    def in_group(body, d):
        return ((body & 15) == d[0] and ((body >> 8) & 255) == d[1] and ((body >> 16) & 255) == d[2]
                and ((body >> 24) & 255) == d[3])

    dom_chains = [c for c in range(n) if in_group(body_of[c], dom)]
    dom_bytes = sum(b_chain[c] for c in dom_chains)
    achieved = dom_bytes / (g_ms[dom] / 1e3) / 1e9
    lt = ",LenQ" if args.lengths == "u8" else ""
    kname = {1: "sat_batch_kernel<float,%d,%d%s>" % (dom[1], dom[2], lt),
             2: "sat_batch_long_kernel<float,16%s>" % lt,
             3: "sat_batch_simple_kernel<float%s>" % lt}[dom[0]]
    traffic = None
    if TRAFFIC and TRAFFIC.get("sources_sha256") == sources_hash() and TRAFFIC.get("kernel") == kname \
            and args.slices == 512 and args.sweeps is None:
        traffic = TRAFFIC["bytes_per_dispatch"]
    rm32 = [datagen.rmse(f32_imgs[c], slices[c].truth) for c in range(n)]
    nrm32 = [datagen.nrmse(f32_imgs[c], slices[c].truth) for c in range(n)]
    ratio = [rm32[c] / rm64[c] for c in range(n)] if rm64 else None
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
        "data": "synthetic: 512 slices of a seeded 32-ellipsoid volume, analytic line integrals, "
                "Poisson noise I0=1e4",
        "config": {"workload": "batch of %d independent slices in persistent launches: N in {128,256,512}, "
                               "U in {90,180,360}, K=ceil(sqrt2 N), circular support, BoME M=8, %g sweeps "
                               "(steps = sweeps x support), FP32 residual with FP64 resync, Eq. 8 T0, "
                               "tuned launch shape" % (n, sweeps),
                   "n_slices": n, "sweeps": sweeps, "M": M, "steps_total": steps_total,
                   "lengths": {"f32": "FP32", "u8": "one byte, round(180 l)"}[args.lengths],
                   "geometries": {"%dx%d" % k: key_of.count(k) for k in keys}},
        "steps_per_s": args.steps * steps_total / wall,
        "slices_per_s": args.steps * n / wall,
        "latency_s_p50": float(np.percentile(lat_slice, 50)),
        "latency_s_p99": float(np.percentile(lat_slice, 99)),
        "latency_note": "per slice inside one batch: device clock from the batch's first chain start "
                        "to the slice's chain end",
        "batch_s_per_step": statistics.mean(lat_step),
        "rmse_fp32_mean": statistics.mean(rm32),
        "nrmse_fp32_mean": statistics.mean(nrm32),
        "rmse_ratio_fp32_fp64": None if ratio is None else
        {"slices": len(ratio), "min": min(ratio), "max": max(ratio), "mean": statistics.mean(ratio),
         "within_1pct": sum(1 for r in ratio if abs(r - 1.0) <= 0.01)},
        "max_drift_r": max(s["max_drift_r"] for s in st),
        "max_drift_sse": max(s["max_drift_sse"] for s in st),
        "resyncs": sum(s["resyncs"] for s in st),
        "batch_over_single": {"value": serial_s / (wall / args.steps), "serial_s": serial_s,
                              "lone_us_per_step": {"%dx%d" % k: v for k, v in sorted(lone_us.items())},
                              "how": "the same chains one at a time with sat_run, each geometry's "
                                     "per-step time from one whole chain of it"},
        "launch": {"chains_per_cu": per_cu, "tuning": tuning, "groups": group_runs[-1]},
        "roofline": {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_ms": g_ms[dom], "algorithmic_bytes_per_launch": dom_bytes,
                     "chains": len(dom_chains),
                     "batch_achieved_gbs": sum(b_chain) / (wall / args.steps) / 1e9},
        "cpu_baseline": cpu,
        "sanity_section_3b": sanity,
        "device": info,
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=("c2", "c3", "c3r", "c4", "c5", "bome", "drt"),
                    help="c3 (default): the batch line; c2: one chain; c3r: batch with repeated "
                         "phantoms; c4: 1024^2 slice, SAT M=32 and SIRT; c5: serving stream; bome: "
                         "N_e and cooling-schedule sweeps; drt: PILA against the bilinear DRT")
    ap.add_argument("--slices", type=int, default=512, help="c3: slices in the batch")
    ap.add_argument("--lengths", default="f32", choices=("f32", "u8"),
                    help="c3: PILA lengths as FP32 or as one byte each (section II-B)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--no-sanity", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="c3: tune the workgroup width per geometry even when a stored table exists")
    ap.add_argument("--tune-out", default=None,
                    help="c3: write the tuning results to this JSON file (when tuning)")
    ap.add_argument("--chain-steps", type=int, default=None,
                    help="c2: override the chain length (profiling runs); the reported config says so")
    ap.add_argument("--cpu-steps", type=int, default=1_000_000, help="c2: oracle steps timed")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (counter "
                         "calibration for rocprofv3 --pmc runs)")
    ap.add_argument("--distinct", type=int, default=64, help="c3r: distinct phantoms generated")
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
    if args.workload == "c3":
        rc = run_c3(args)
        if args.copy_probe_mib > 0:
            import torch
            import bench_workloads
            bench_workloads.copy_probe(args, torch)
        return rc
    import bench_workloads
    return bench_workloads.run(args)


if __name__ == "__main__":
    sys.exit(main())
