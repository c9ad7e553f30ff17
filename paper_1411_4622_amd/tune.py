"""Launch-shape tuner for batches of chains (sat_run_batch).

A batch's speed depends on how many wavefronts serve one chain and how many
chains share a compute unit: more wavefronts shorten each step, more chains
per CU overlap their latencies but split the CU's registers and LDS.  The
tuner runs every candidate shape on a short prefix of the same chains (the
first sample_steps steps of each, on copies of the images) and keeps the
shape with the most proposals per second.  Results do not depend on the
shape, only the time does.

Widths can also be tuned per geometry (image side, angles, estimates,
precision) and stored in tuned_launch.json beside this file; a batch then
gives each chain its geometry's width (sat_job.waves_per_chain), and its
groups of chains run with their own widths.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import replace
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from ._binding import Job, _torch, sat_run_batch

# (waves per chain, chains per CU)
DEFAULT_SHAPES: Tuple[Tuple[int, int], ...] = ((8, 1), (4, 1), (4, 2), (2, 2), (2, 4))


def tune_batch(jobs: Sequence[Job], shapes: Iterable[Tuple[int, int]] = DEFAULT_SHAPES,
               sample_steps: int = 4096, repeats: int = 1) -> Tuple[Tuple[int, int], List[dict]]:
    """Time each launch shape on the jobs cut to sample_steps steps.

    Returns the fastest (waves_per_chain, chains_per_cu) and one record per
    shape: proposals, seconds, proposals/s.
    """
    torch = _torch()
    table = []
    best, best_rate = None, -1.0
    for waves, per_cu in shapes:
        rate = 0.0
        secs = []
        for _ in range(max(1, repeats)):
            sample = [Job(j.pila, j.sino, j.image.clone(),
                          replace(j.params, n_steps=min(j.params.n_steps, sample_steps)), 0)
                      for j in jobs]
            props = sum(j.params.n_steps * j.params.m_cand for j in sample)
            torch.cuda.current_stream().synchronize()
            t0 = time.perf_counter()
            sat_run_batch(sample, waves_per_chain=waves, chains_per_cu=per_cu)
            torch.cuda.current_stream().synchronize()
            secs.append(time.perf_counter() - t0)
        dt = min(secs)
        rate = props / dt
        table.append({"waves_per_chain": waves, "chains_per_cu": per_cu, "proposals": props,
                      "seconds": dt, "proposals_per_s": rate})
        if rate > best_rate:
            best, best_rate = (waves, per_cu), rate
    return best, table


# ---------------------------------------------------------------------------
# per-geometry tuning with stored results
# ---------------------------------------------------------------------------

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_launch.json")


def geometry_key(job: Job) -> str:
    """Tuning key of a chain: image side, angles, estimates per step, precision."""
    g = job.pila.geom
    return "%d,%d,%d,%s" % (g.n, g.n_angles, job.params.m_cand,
                            "f32" if job.params.precision in ("f32", 1) else "f64")


def tune_geometries(jobs: Sequence[Job], waves: Iterable[int] = (8, 4), chains_per_cu: int = 1,
                    sample_steps: int = 4096, max_chains: int = 64) -> Dict[str, dict]:
    """Time each workgroup width per geometry: up to max_chains of a
    geometry's chains, cut to sample_steps steps, run as a batch of their own
    at every width.  Returns {key: {"waves_per_chain": best, "table": [...]}}."""
    by_key: Dict[str, List[Job]] = {}
    for j in jobs:
        by_key.setdefault(geometry_key(j), []).append(j)
    out = {}
    for key, js in sorted(by_key.items()):
        best, table = tune_batch(js[:max_chains], [(w, chains_per_cu) for w in waves], sample_steps)
        out[key] = {"waves_per_chain": best[0],
                    "table": [{"waves_per_chain": r["waves_per_chain"], "proposals_per_s": r["proposals_per_s"]}
                              for r in table]}
    return out


def save_table(results: Dict[str, dict], device: str, chains_per_cu: int, sample_steps: int,
               path: str = TABLE_PATH) -> None:
    with open(path, "w") as fh:
        json.dump({"device": device, "chains_per_cu": chains_per_cu, "sample_steps": sample_steps,
                   "geometries": results}, fh, indent=1, sort_keys=True)
        fh.write("\n")


def load_table(device: str, path: str = TABLE_PATH) -> Optional[dict]:
    """The stored table if it was tuned on this kind of device, else None."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("device", "").split(":")[0] != device.split(":")[0]:
        return None
    return t


def apply_table(jobs: Sequence[Job], table: dict) -> bool:
    """Give every job the width stored for its geometry; False (nothing set)
    when some geometry is missing from the table."""
    geo = table.get("geometries", {})
    keys = [geometry_key(j) for j in jobs]
    if any(k not in geo for k in keys):
        return False
    for j, k in zip(jobs, keys):
        j.waves_per_chain = int(geo[k]["waves_per_chain"])
    return True
