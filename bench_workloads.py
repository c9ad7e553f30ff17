"""Workloads beside the batch benchmark line (bench.py --workload ...).

c2  one chain: 256 x 256 slice, 180 angles, 367 bins, M = 16, 5e6 steps, FP32
    residual against an FP64 chain with the same seeds.

c3r batch with repeated phantoms: slices cut from one seeded ellipsoid volume (N in {128, 256, 512},
    90/180/360 angles, K = ceil(sqrt(2) N), Poisson noise I0 = 1e4, circular
    support), M = 8, FP32 residual with FP64 resync every 4096 accepted
    nonzero changes, 16 sweeps of the support, all chains in one persistent
    launch whose shape the tuner picks.  --distinct phantoms are generated and
    repeated with other chain seeds up to --slices chains.
c4  one 1024 x 1024 slice (30 ellipses, 720 angles, 1449 bins, I0 = 1e4,
    circular support): the PILA build, a SAT chain at M = 32 (FP32 residual,
    FP64 resync) and 200 SIRT iterations (relaxation 0.1).
c5  serving: requests arrive by a Poisson process; each is a slice with N in
    {128, 256, 384, 512, 768, 1024}, 90/180/360/720 angles and an ellipse
    phantom with Poisson noise at I0 drawn in [1e3, 1e5]; the server admits
    them against its memory budget and runs them as workgroups free up.

Every input is synthetic and seeded.  Each workload prints one JSON line.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import statistics
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _pool_map(fn, items, procs=16):
    procs = max(1, min(procs, len(items), os.cpu_count() or 1))
    if procs == 1:
        return [fn(x) for x in items]
    with ProcessPoolExecutor(max_workers=procs) as ex:
        return list(ex.map(fn, items, chunksize=1))


def resync_interval(cfg, nnz):
    """Accepted nonzero changes between FP64 resyncs for the batch and serving
    workloads, which do not fix it: at least the configured 4096, and at
    least nnz / 128.  Their resyncs run inside the chain's workgroup, where a
    full-PILA rebuild takes about 1.1 ns per entry (one CU, bound by its
    image gathers: 100 ms at 512^2 x 360) against about 4 us per step, so
    nnz / 128 keeps the rebuilds near 4% of the chain's time."""
    return max(int(cfg["resync_every"]), int(nnz) // 128)


def _params(P, cfg, n_steps, seed, chain_id, precision="f32", nnz=0):
    return P.SatParams(n_steps=int(n_steps), seed=seed, chain_id=chain_id, n_stages=cfg["n_stages"],
                       m_cand=cfg["M"], T0=None, q_auto=cfg["q_auto"], precision=precision,
                       tn_ratio=cfg["tn_ratio"], delta_max=cfg["delta_max"], f_min=cfg["f_min"],
                       f_max=cfg["f_max"],
                       resync_every=resync_interval(cfg, nnz) if precision == "f32" else 0)


def copy_probe(args, torch):
    """Three device copies of a buffer of --copy-probe-mib MiB: the known-size
    kernel that rocprofv3 --pmc runs scale FETCH_SIZE / WRITE_SIZE by."""
    if not getattr(args, "copy_probe_mib", 0):
        return
    n = args.copy_probe_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy probe: %d MiB read + %d MiB written per copy, 3 copies"
        % (args.copy_probe_mib, args.copy_probe_mib))


def _chain_bytes(n_steps, M, f_mean, accepts):
    # the single-chain kernel's per-estimate and per-accept bytes (FP32)
    return n_steps * M * (28.0 + 12.0 * f_mean) + accepts * (8.0 + 16.0 * f_mean)


# ---------------------------------------------------------------------------
# c2: one chain, FP32 residual against FP64
# ---------------------------------------------------------------------------

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


def cpu_baseline_c2(sl, cfg, n_steps_cpu: int) -> dict:
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



def run_c2(args, P, torch, datagen):
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

    # the same chain from a HIP graph captured once (its launch sequence:
    # one segment per possible resync, the rebuilds and finishes), replayed
    # on the same buffers; the image must come out with the same bits
    pl_g = P.pila_build(geom)
    graph = P.sat_graph(pl_g, sino, prm, img, workspace=ws)
    graph_ms = []
    same = True
    for _ in range(3):
        img.copy_(f0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        graph.launch()
        e1.record(stream)
        e1.synchronize()
        graph_ms.append(e0.elapsed_time(e1))
        same = same and bool(np.array_equal(img.cpu().numpy(), f32_img))
    graph.close()
    log("graph replay: chain %.1f ms (eager %.1f ms), same image: %s"
        % (statistics.mean(graph_ms), statistics.mean(kernel_ms), same))

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
        cpu = cpu_baseline_c2(sl, cfg, args.cpu_steps)

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
        "graph": {"chain_ms_eager": statistics.mean(kernel_ms), "chain_ms_graph": statistics.mean(graph_ms),
                  "replays": len(graph_ms), "same_image_bits": same},
        "cpu_baseline": cpu,
        "device": info,
    }
    print(json.dumps(out), flush=True)
    return 0


# ---------------------------------------------------------------------------
# c3 with repeated phantoms (the default benchmark line is bench.run_c3)
# ---------------------------------------------------------------------------

def run_c3_repeat(args, P, torch, datagen):
    from paper_1411_4622_amd.tune import tune_batch
    cfg = datagen.CONFIGS["c3"]
    sweeps = args.sweeps if args.sweeps is not None else cfg["sweeps"]
    n_dist = min(args.distinct, args.slices)
    specs = datagen.batch_slice_specs(cfg["volume_seed"], n_dist, cfg["sizes"], cfg["n_angles"],
                                      cfg["I0"], cfg["masked"])
    t0 = time.perf_counter()
    slices = _pool_map(datagen.slice_from_spec, specs)
    log("c3: %d distinct slices generated in %.1f s" % (len(slices), time.perf_counter() - t0))
    geoms, pilas = {}, {}
    for sl in slices:
        key = (sl.N, sl.U)
        if key not in pilas:
            g = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32")
            geoms[key], pilas[key] = g, P.pila_build(g)
    dev = torch.device("cuda", 0)
    sinos = [torch.from_numpy(sl.sino).to(dev) for sl in slices]
    jobs = []
    for c in range(args.slices):
        sl = slices[c % n_dist]
        P_sup = int(sl.mask.sum())
        pl = pilas[(sl.N, sl.U)]
        prm = _params(P, cfg, round(sweeps * P_sup), cfg["chain_seed0"] + c, c, nnz=pl.nnz)
        jobs.append(P.Job(pl, sinos[c % n_dist],
                          torch.from_numpy(sl.f0.copy()).to(dev), prm))
    f0s = [j.image.clone() for j in jobs]
    (waves, per_cu), table = tune_batch(jobs, sample_steps=4096)
    log("c3: tuned launch shape %d waves/chain, %d chains/CU: %s"
        % (waves, per_cu, ", ".join("(%d,%d) %.3g/s" % (r["waves_per_chain"], r["chains_per_cu"],
                                                          r["proposals_per_s"]) for r in table)))
    for j, f in zip(jobs, f0s):
        j.image.copy_(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = P.sat_run_batch(jobs, waves_per_chain=waves, chains_per_cu=per_cu)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = sum(j.params.n_steps for j in jobs)
    M = cfg["M"]
    rm32 = [datagen.rmse(j.image.cpu().numpy(), slices[c % n_dist].truth) for c, j in enumerate(jobs)]
    drift = max(s["max_drift_r"] for s in stats)
    # FP64 chains with the same seeds on a sample of slices, for the RMSE ratio
    sample = list(range(0, len(jobs), max(1, len(jobs) // 8)))[:8]
    jobs64, keys64 = [], []
    for c in sample:
        sl = slices[c % n_dist]
        g64 = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f64")
        key = (sl.N, sl.U)
        if key not in keys64:
            keys64.append(key)
        pl64 = P.pila_build(g64)
        prm = _params(P, cfg, jobs[c].params.n_steps, cfg["chain_seed0"] + c, c, "f64")
        jobs64.append(P.Job(pl64, sinos[c % n_dist], f0s[c].clone(), prm))
    log("c3: %d FP64 reference chains" % len(jobs64))
    P.sat_run_batch(jobs64, waves_per_chain=8, chains_per_cu=1)
    torch.cuda.synchronize()
    ratios = []
    for c, j64 in zip(sample, jobs64):
        r64 = datagen.rmse(j64.image.cpu().numpy(), slices[c % n_dist].truth)
        ratios.append(rm32[c] / r64 if r64 > 0 else float("nan"))
    # the plain one-chain GPU form at the same M on the most common geometry
    common = max(pilas, key=lambda k: sum(1 for c in range(len(jobs))
                                          if (slices[c % n_dist].N, slices[c % n_dist].U) == k))
    c0 = next(c for c in range(len(jobs)) if (slices[c % n_dist].N, slices[c % n_dist].U) == common)
    single_steps = min(jobs[c0].params.n_steps, 200_000)
    img = f0s[c0].clone()
    prm1 = _params(P, cfg, single_steps, cfg["chain_seed0"] + c0, c0, nnz=pilas[common].nnz)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    P.sat_run(pilas[common], sinos[c0 % n_dist], prm1, img)
    e1.record()
    e1.synchronize()
    single_rate = single_steps * M / (e0.elapsed_time(e1) / 1e3)
    f_mean = statistics.mean(pl.nnz / pl.n_support for pl in pilas.values())
    alg = sum(_chain_bytes(j.params.n_steps, M, j.pila.nnz / j.pila.n_support, s["accepts"])
              for j, s in zip(jobs, stats))
    out = {
        "workload": "c3",
        "metric": "SA proposals evaluated/s + slices/s (batch of independent slices)",
        "value": steps * M / wall, "unit": "proposals/s",
        "slices": len(jobs), "distinct_phantoms": n_dist, "sweeps": sweeps, "M": M,
        "steps_total": steps, "wall_s": wall, "slices_per_s": len(jobs) / wall,
        "launch_shape": {"waves_per_chain": waves, "chains_per_cu": per_cu, "tuner": table},
        "single_chain_proposals_per_s": single_rate,
        "single_chain_geometry": {"N": common[0], "U": common[1]},
        "batch_over_single": steps * M / wall / single_rate,
        "rmse_fp32_mean": statistics.mean(rm32),
        "rmse_ratio_fp32_fp64_sample": ratios, "max_drift_r": drift,
        "roofline": {"kernel": "sat_batch_kernel", "bound": "hbm",
                     "achieved": alg / wall / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg / wall / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": alg,
                     "mean_row": f_mean},
        "data": "synthetic: slices of a seeded 32-ellipsoid volume, analytic line integrals, "
                "Poisson noise I0=1e4",
    }
    print(json.dumps(out), flush=True)
    return 0


# ---------------------------------------------------------------------------
# c4: large slice, SAT M=32 and SIRT
# ---------------------------------------------------------------------------

def run_c4(args, P, torch, datagen):
    cfg = datagen.CONFIGS["c4"]
    t0 = time.perf_counter()
    sl = datagen.config_slice("c4")
    log("c4: slice generated in %.1f s" % (time.perf_counter() - t0))
    dev = torch.device("cuda", 0)
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl = P.pila_build(geom)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log("c4: PILA nnz %d (%.2f GB per order) built in %.2f s" % (pl.nnz, pl.nnz * 8 / 1e9, build_s))
    sino = torch.from_numpy(sl.sino).to(dev)
    f0 = torch.from_numpy(sl.f0).to(dev)
    # SIRT
    n_it, lam = cfg["sirt_iters"], cfg["sirt_lambda"]
    img = f0.clone()
    P.sirt_run(pl, sino, 2, lam, img, cost=False)  # warm-up
    img.copy_(f0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    costs = P.sirt_run(pl, sino, n_it, lam, img, cost=False)
    e1.record()
    e1.synchronize()
    sirt_s = e0.elapsed_time(e1) / 1e3
    rm_sirt = datagen.rmse(img.cpu().numpy(), sl.truth)
    G = sl.U * sl.K
    NP = sl.N * sl.N
    # per iteration: both PILA orders (ray or pixel index 4 + length 4 per entry),
    # both offset arrays, image read twice and written once, residual written and read
    sirt_bytes = n_it * (2 * 8.0 * pl.nnz + 8.0 * (G + NP) + 3 * 8.0 * NP + 2 * 8.0 * G)
    log("c4: SIRT %d iterations in %.3f s (%.1f GB/s algorithmic)"
        % (n_it, sirt_s, sirt_bytes / sirt_s / 1e9))
    # SAT chain (--sat-steps 0 skips it)
    steps = cfg["n_steps"] if args.sat_steps is None else args.sat_steps
    sat_s, rm_sat = float("nan"), float("nan")
    st = {"accepts": 0, "resyncs": 0, "max_drift_r": 0.0}
    if steps > 0:
        prm = _params(P, cfg, steps, cfg["chain_seed"], 0)  # c4 keeps resync every 4096
        img.copy_(f0)
        e0.record()
        st, _ = P.sat_run(pl, sino, prm, img)
        e1.record()
        e1.synchronize()
        sat_s = e0.elapsed_time(e1) / 1e3
        rm_sat = datagen.rmse(img.cpu().numpy(), sl.truth)
    # the same chain in FP64 (FP64 PILA, same seeds) for the RMSE ratio
    rm64, sat64_s = float("nan"), float("nan")
    if steps > 0 and not getattr(args, "no_fp64_reference", False):
        pl64 = P.pila_build(P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f64"))
        prm64 = _params(P, cfg, steps, cfg["chain_seed"], 0, "f64")
        img.copy_(f0)
        e0.record()
        P.sat_run(pl64, sino, prm64, img)
        e1.record()
        e1.synchronize()
        sat64_s = e0.elapsed_time(e1) / 1e3
        rm64 = datagen.rmse(img.cpu().numpy(), sl.truth)
        del pl64
        log("c4: FP64 chain in %.1f s" % sat64_s)
    out = {
        "workload": "c4", "N": sl.N, "U": sl.U, "K": sl.K, "nnz": pl.nnz, "max_row": pl.max_row,
        "pila_build_s": build_s,
        "sirt": {"iterations": n_it, "lambda": lam, "seconds": sirt_s, "ms_per_iteration":
                 1e3 * sirt_s / n_it, "rmse": rm_sirt,
                 "roofline": {"kernel": "ray_tile_part_kernel + tile_back_kernel (whole iteration)",
                              "bound": "hbm",
                              "achieved": sirt_bytes / sirt_s / 1e9, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": sirt_bytes / sirt_s / 1e9 / HBM_PEAK_GBS,
                              "algorithmic_bytes": sirt_bytes}},
        "sat": {"steps": steps, "M": cfg["M"], "seconds": sat_s,
                "proposals_per_s": steps * cfg["M"] / sat_s if steps else None,
                "us_per_step": 1e6 * sat_s / steps if steps else None,
                "accepts": st["accepts"], "resyncs": st["resyncs"], "max_drift_r": st["max_drift_r"],
                "rmse": rm_sat, "rmse_fp64": rm64, "rmse_ratio_fp32_fp64": rm_sat / rm64,
                "fp64_seconds": sat64_s},
        "data": "synthetic: seeded 30-ellipse phantom, analytic line integrals, Poisson noise I0=1e4",
    }
    copy_probe(args, torch)
    print(json.dumps(out), flush=True)
    return 0


# ---------------------------------------------------------------------------
# c5: serving stream
# ---------------------------------------------------------------------------

def _c5_pool_item(arg):
    import datagen
    N, U, ph, seed = arg
    ell = datagen.random_ellipses(seed, N, 10)
    K = datagen.n_bins_for(N)
    sino = datagen.radon_ellipses(ell, N, datagen.angles_deg(U), K)
    truth = datagen.rasterize(ell, N)
    return (N, U, ph, sino, truth)


def run_c5(args, P, torch, datagen):
    cfg = datagen.CONFIGS["c5"]
    sweeps = args.sweeps if args.sweeps is not None else 1.0
    rng = np.random.default_rng(cfg["seed"])
    n_req = args.requests
    sizes, angs = cfg["sizes"], cfg["n_angles"]
    n_ph = 2  # phantoms per geometry in the pool
    items = [(N, U, ph, cfg["seed"] * 100000 + N * 1000 + U * 3 + ph) for N in sizes for U in angs
             for ph in range(n_ph)]
    t0 = time.perf_counter()
    pool = _pool_map(_c5_pool_item, items)
    log("c5: %d clean sinograms generated in %.1f s" % (len(pool), time.perf_counter() - t0))
    clean = {(N, U, ph): (sino, truth) for N, U, ph, sino, truth in pool}
    masks = {N: datagen.circle_mask(N) for N in sizes}
    geoms = {(N, U): P.Geometry(N, datagen.angles_deg(U), datagen.n_bins_for(N), masks[N], "f32")
             for N in sizes for U in angs}
    # requests: arrival time, geometry, phantom, I0, noise seed
    gaps = rng.exponential(1.0 / args.rate, size=n_req)
    arrive = np.cumsum(gaps)
    reqs = []
    for i in range(n_req):
        N = int(rng.choice(sizes))
        U = int(rng.choice(angs))
        ph = int(rng.integers(n_ph))
        I0 = float(rng.uniform(*cfg["I0_range"]))
        reqs.append((float(arrive[i]), N, U, ph, I0, cfg["seed"] * 1000003 + i))
    # noisy sinograms: a few noise levels per (geometry, phantom) reused across requests
    dev = torch.device("cuda", 0)
    noisy = {}
    levels = np.geomspace(cfg["I0_range"][0], cfg["I0_range"][1], 4)
    for (N, U, ph), (sino, _) in clean.items():
        for li, I0 in enumerate(levels):
            s = datagen.poisson_noise(sino, N, float(I0), cfg["seed"] + 7919 * li + N + U + ph)
            f0 = datagen.uniform_start(s, masks[N], N, cfg["f_min"], cfg["f_max"])
            noisy[(N, U, ph, li)] = (torch.from_numpy(s).to(dev), torch.from_numpy(f0).to(dev))
    log("c5: %d noisy sinograms on the device" % len(noisy))

    budget = int(args.mem_budget_gb * (1 << 30))
    srv = P.Server(mem_budget=budget, max_slots=args.max_slots, idle_us=int(args.idle_ms * 1000),
                   general_slots=args.general_slots, long_slots=args.long_slots)
    t0 = time.perf_counter()
    for g in geoms.values():
        srv.prepare(g)
    prep_s = time.perf_counter() - t0
    st0 = srv.status()
    log("c5: %d PILAs prepared in %.1f s (%.1f GB)" % (st0["pila_cached"], prep_s, st0["bytes_used"] / 1e9))

    torch.cuda.current_stream().synchronize()
    lat, done_at, steps_done, props, rm = [], [], 0, 0, []
    waiting = []  # arrived, not yet admitted
    by_queue, by_geom = {}, {}  # latencies per server queue and per geometry
    inflight = {}
    nxt = 0
    busy_retries = 0
    start = time.perf_counter()
    last_log = start
    while nxt < n_req or waiting or inflight:
        now = time.perf_counter() - start
        while nxt < n_req and reqs[nxt][0] <= now:
            waiting.append(reqs[nxt])
            nxt += 1
        while waiting:
            a, N, U, ph, I0, seed = waiting[0]
            li = int(np.argmin(np.abs(np.log(levels) - math.log(I0))))
            sino, f0 = noisy[(N, U, ph, li)]
            img = f0.clone()
            torch.cuda.current_stream().synchronize()
            P_sup = int(masks[N].sum())
            prm = _params(P, cfg, max(1, round(sweeps * P_sup)), seed, 0,
                          nnz=int(P_sup * U * 4 / math.pi))
            t = srv.submit(geoms[(N, U)], sino, img, prm)
            if t is None:
                busy_retries += 1
                break
            waiting.pop(0)
            inflight[t] = (a, N, U, ph, img, prm.n_steps)
            by_queue.setdefault(t & 3, [])
        for t in list(inflight):
            st = srv.poll(t)
            if st is None:
                continue
            a, N, U, ph, img, n_steps = inflight.pop(t)
            fin = time.perf_counter() - start
            lat.append(fin - a)
            by_queue[t & 3].append(fin - a)
            by_geom.setdefault("%dx%d" % (N, U), []).append(fin - a)
            done_at.append(fin)
            steps_done += n_steps
            props += n_steps * cfg["M"]
            if len(rm) < 200:
                rm.append((N, datagen.rmse(img.cpu().numpy(), clean[(N, U, ph)][1])))
        if time.perf_counter() - last_log > 5:
            last_log = time.perf_counter()
            log("c5: t=%.1f s arrived %d done %d in flight %d waiting %d"
                % (now, nxt, len(lat), len(inflight), len(waiting)))
        time.sleep(0.0005)
    span = max(done_at) - reqs[0][0]
    stat = srv.status()
    srv.close()
    lat_ms = np.array(lat) * 1e3
    out = {
        "workload": "c5",
        "metric": "slices/s and p50/p99 latency of a Poisson request stream (continuous batching)",
        "requests": n_req, "rate_per_s": args.rate, "sweeps": sweeps, "M": cfg["M"],
        "server_idle_ms": args.idle_ms, "server_max_slots": args.max_slots,
        "slices_per_s": n_req / span, "proposals_per_s": props / span, "steps_per_s": steps_done / span,
        "latency_ms_p50": float(np.percentile(lat_ms, 50)),
        "latency_ms_p99": float(np.percentile(lat_ms, 99)),
        "latency_ms_mean": float(lat_ms.mean()),
        "span_s": span, "pila_prepare_s": prep_s, "busy_retries": busy_retries,
        "kernel_launches": stat["launches"], "bytes_used_peak_after_prepare": st0["bytes_used"],
        "latency_s_by_queue": {["pipelined", "general", "long-row"][q]:
                               {"n": len(v), "p50": float(np.percentile(v, 50)),
                                "p99": float(np.percentile(v, 99))}
                               for q, v in sorted(by_queue.items()) if v},
        "latency_s_p50_by_geometry": {k: float(np.percentile(v, 50)) for k, v in sorted(by_geom.items())},
        "rmse_by_N_sample": {str(N): float(np.mean([r for n, r in rm if n == N]))
                             for N in sorted({n for n, _ in rm})},
        "data": "synthetic: seeded 10-ellipse phantoms (2 per geometry), analytic line integrals, "
                "Poisson noise at 4 levels in [1e3, 1e5] (each request takes the level nearest "
                "its drawn I0)",
    }
    print(json.dumps(out), flush=True)
    return 0


# ---------------------------------------------------------------------------
# BoME and cooling schedules (sections III-B, III-C)
# ---------------------------------------------------------------------------

def _consistent_slice(P, torch, datagen, N, U, seed, n_ell=10):
    """A phantom's pixel image and its Eq. 1 projections (noise-free data the
    pixel model can fit), FP64 PILA, uniform start."""
    K = datagen.n_bins_for(N)
    ell = datagen.random_ellipses(seed, N, n_ell)
    sl = datagen.make_slice(N, U, K, ell, masked=True, I0=None)
    pl = P.pila_build(P.Geometry(N, sl.angles, K, sl.mask, "f64"))
    truth = torch.from_numpy(sl.truth * sl.mask).cuda()
    sino = P.pila_forward(pl, truth)
    f0 = torch.from_numpy(datagen.uniform_start(sino.cpu().numpy(), sl.mask, N)).cuda()
    return sl, pl, truth.cpu().numpy(), sino, f0


def run_bome(args, P, torch, datagen):
    """N_e and cooling-schedule sweeps on noise-free 64 x 64 data (U = 60):
    1000 stages of 2000 steps, Eq. 8 T0, FP64; cost C (Eq. 4) at stages
    100, 200, 500 and 1000 from the chain's trace and the final NRMSE; the
    N_e = 1 chain with four times the steps of N_e = 4 (same evaluations);
    and the final cost after 200 stages of one sweep each (steps = 200 x
    support) for N = 32, 64, 128 with U = N."""
    t_all = time.perf_counter()
    sl, pl, truth, sino, f0 = _consistent_slice(P, torch, datagen, 64, 60, 106)
    stages = 1000

    def chain(Ne, schedule, steps, seed=1006):
        im = f0.clone()
        prm = P.SatParams(n_steps=steps, seed=seed, chain_id=Ne, n_stages=stages, m_cand=Ne, T0=None,
                          q_auto=200, delta_max=0.05, schedule=schedule)
        ts = time.perf_counter()
        st, tr = P.sat_run(pl, sino, prm, im, trace=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - ts
        acc = tr["accept"].cpu().numpy().astype(bool)
        dc = tr["dC"].cpu().numpy()
        # C after each step: the start cost plus the accepted changes
        c_start = st["cost_final"] - float(np.sum(dc[acc]))
        c_path = c_start + np.cumsum(np.where(acc, dc, 0.0))
        at = {str(k): float(c_path[k * steps // stages - 1]) for k in (100, 200, 500, 1000)}
        f = im.cpu().numpy()
        return {"N_e": Ne, "schedule": schedule, "steps": steps, "cost_at_stage": at,
                "cost_final": st["cost_final"], "nrmse": datagen.nrmse(f, truth), "accepts": st["accepts"],
                "T0": st["T0_used"], "seconds": dt}

    sweep = []
    for schedule in ("linear", "exp", "cubic"):
        for Ne in (1, 2, 4, 8, 16, 32):
            r = chain(Ne, schedule, 2_000_000)
            sweep.append(r)
            log("bome: %s N_e=%d NRMSE %.4f C %.3g (stage 200: %.3g) %.1f s" % (
                schedule, Ne, r["nrmse"], r["cost_final"], r["cost_at_stage"]["200"], r["seconds"]))
    same_evals = chain(1, "linear", 8_000_000)
    log("bome: N_e=1 with 8e6 steps: NRMSE %.4f" % same_evals["nrmse"])

    # final cost against N_e for three sizes, all chains in one batch
    sizes = []
    jobs, meta = [], []
    for N in (32, 64, 128):
        sl2, pl2, truth2, sino2, f02 = _consistent_slice(P, torch, datagen, N, N, 200 + N)
        sup = int(sl2.mask.sum())
        for Ne in (1, 2, 4, 8, 16, 32):
            im = f02.clone()
            prm = P.SatParams(n_steps=200 * sup, seed=77, chain_id=Ne, n_stages=200, m_cand=Ne, T0=None,
                              q_auto=200, delta_max=0.05)
            jobs.append(P.Job(pl2, sino2, im, prm))
            meta.append((N, Ne, truth2))
    ts = time.perf_counter()
    st = P.sat_run_batch(jobs, waves_per_chain=8, chains_per_cu=1)
    torch.cuda.synchronize()
    for (N, Ne, truth2), j, s_ in zip(meta, jobs, st):
        sizes.append({"N": N, "U": N, "N_e": Ne, "steps": j.params.n_steps, "cost_final": s_["cost_final"],
                      "nrmse": datagen.nrmse(j.image.cpu().numpy(), truth2)})
    log("bome: size sweep (18 chains, one batch) in %.1f s" % (time.perf_counter() - ts))
    out = {"metric": "final NRMSE and cost C (Eq. 4) against N_e and cooling schedule",
           "workload": "noise-free 64x64 (10 ellipses, its pixel image projected by Eq. 1), U=60, K=91, "
                       "1000 stages x 2000 steps, change in [-0.05, 0.05) clamped to [0, 1], Eq. 8 T0, FP64",
           "sweep": sweep, "N_e1_same_evaluations_as_N_e4": same_evals,
           "size_sweep": {"setting": "200 stages of one sweep each (steps = 200 x support), U = N, Eq. 8 T0",
                          "results": sizes},
           "seconds": time.perf_counter() - t_all}
    print(json.dumps(out), flush=True)
    return 0


# ---------------------------------------------------------------------------
# the PILA against the bilinear DRT (section III-A, Fig. 3)
# ---------------------------------------------------------------------------

def run_drt(args, P, torch, datagen):
    """Time per SA step with the PILA (sat_run, N_e = 1; FP64, and FP32 with
    FP64 resyncs) and with the bilinear discrete Radon transform of the
    whole image per estimate (sat_drt_run, FP64), for N = 64 .. 512 and U =
    90, 180, 360: 200 steps as in the paper (N = 1, M = 200) for the DRT
    chain, the PILA chains timed on 20000 steps for a stable rate; the gain
    is the ratio of the per-step times, and also of the 200-step totals with
    the FP64 PILA build included."""
    res = []
    for N in (64, 128, 256, 512):
        for U in (90, 180, 360):
            K = datagen.n_bins_for(N)
            ell = datagen.random_ellipses(300 + N, N, 8)
            sl = datagen.make_slice(N, U, K, ell, masked=True, I0=1e4, noise_seed=N + U)
            sino = torch.from_numpy(sl.sino).cuda()
            f0 = torch.from_numpy(sl.f0).cuda()
            geom = P.Geometry(N, sl.angles, K, sl.mask, "f64")
            torch.cuda.synchronize()
            ts = time.perf_counter()
            pl = P.pila_build(geom)
            torch.cuda.synchronize()
            t_build = time.perf_counter() - ts

            pl32 = P.pila_build(P.Geometry(N, sl.angles, K, sl.mask, "f32"))

            def pila_time(steps, prec="f64"):
                im = f0.clone()
                prm = P.SatParams(n_steps=steps, seed=5, m_cand=1, T0=1e-2, TN=1e-6, n_stages=100,
                                  precision=prec, resync_every=4096 if prec == "f32" else 0)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                P.sat_run(pl if prec == "f64" else pl32, sino, prm, im, stats=False)
                e1.record()
                e1.synchronize()
                return e0.elapsed_time(e1) / 1e3

            pila_time(2000)
            pila_time(2000, "f32")
            t_pila_200 = pila_time(200)
            t_pila = pila_time(20000) / 20000
            t_pila32 = pila_time(20000, "f32") / 20000
            im = f0.clone()
            prm = P.SatParams(n_steps=200, seed=5, m_cand=1, T0=1e-2, TN=1e-6, n_stages=100)
            P.sat_drt_run(geom, sino, prm, im)  # warm-up
            im = f0.clone()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            P.sat_drt_run(geom, sino, prm, im)
            torch.cuda.synchronize()
            t_drt = (time.perf_counter() - ts) / 200
            r = {"N": N, "U": U, "K": K, "pila_nnz": pl.nnz, "pila_build_s": t_build,
                 "pila_us_per_step": 1e6 * t_pila, "pila_f32_us_per_step": 1e6 * t_pila32,
                 "drt_us_per_step": 1e6 * t_drt,
                 "gain_per_step": t_drt / t_pila, "gain_per_step_f32": t_drt / t_pila32,
                 "gain_200_steps_with_build": 200 * t_drt / (t_pila_200 + t_build)}
            res.append(r)
            log("drt: N=%d U=%d: PILA %.2f us/step (FP32 %.2f), DRT %.1f us/step, gain %.0fx (FP32 %.0fx; "
                "%.0fx with the build)" % (N, U, r["pila_us_per_step"], r["pila_f32_us_per_step"],
                                           r["drt_us_per_step"], r["gain_per_step"], r["gain_per_step_f32"],
                                           r["gain_200_steps_with_build"]))
            del pl, pl32
    out = {"metric": "SA step time: PILA against the bilinear DRT (section III-A)",
           "setting": "one chain, N_e=1, given T0/TN, Poisson I0=1e4 data; DRT chain (FP64) 200 steps "
                      "(N=1, M=200), PILA chains (FP64; FP32 with FP64 resync) timed on 20000 steps",
           "paper": "gain over 300x for the largest sizes on its CPU (Fig. 3)", "results": res}
    print(json.dumps(out), flush=True)
    return 0


def run(args) -> int:
    import torch
    import datagen
    import paper_1411_4622_amd as P
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    return {"c2": run_c2, "c3r": run_c3_repeat, "c4": run_c4, "c5": run_c5, "bome": run_bome,
            "drt": run_drt}[args.workload](args, P, torch, datagen)
