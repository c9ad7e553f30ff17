"""Launch-shape tuner for batches of chains (sat_run_batch).

A batch's speed depends on how many wavefronts serve one chain and how many
chains share a compute unit: more wavefronts shorten each step, more chains
per CU overlap their latencies but split the CU's registers and LDS.  The
tuner runs every candidate shape on a short prefix of the same chains (the
first sample_steps steps of each, on copies of the images) and keeps the
shape with the most proposals per second.  Results do not depend on the
shape, only the time does.
"""
from __future__ import annotations

import time
from dataclasses import replace
from typing import Iterable, List, Sequence, Tuple

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
                          replace(j.params, n_steps=min(j.params.n_steps, sample_steps)))
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
