"""Autotuner for the gridding work decomposition (tile edge, chunk size).

For one coverage, every candidate (tile, chunk) plan is built and one fused
PPD iteration (forward FFT, degridding with the dual update, gridding, fold,
inverse FFT, SARA, primal update) is timed by graph replay on the GPU; the
fastest candidate wins.  Results are cached in a JSON file keyed by the image
size, the number of visibilities and blocks, a digest of the coverage and
the device name, so a workload is tuned once per machine.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Iterable, Optional, Tuple

import numpy as np

from . import ppd as P

DEFAULT_CANDIDATES = ((8, 128), (8, 256), (16, 256), (16, 512), (16, 1024), (32, 512), (32, 1024))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ppd_mi355x_tune.json")


def _key(nx, ny, wu, wv, block_off, device_name: str) -> str:
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(wu, np.float32).tobytes())
    h.update(np.ascontiguousarray(wv, np.float32).tobytes())
    h.update(np.ascontiguousarray(block_off, np.int64).tobytes())
    return f"{nx}x{ny}:M{len(wu)}:d{len(block_off) - 1}:{h.hexdigest()[:16]}:{device_name}"


def time_iteration(plan: "P.Plan", reps: int = 20) -> float:
    """Microseconds per fused iteration (graph replay) on a synthetic state."""
    import torch
    y = torch.ones(plan.M, dtype=torch.complex64, device="cuda")
    U = torch.ones(plan.M, dtype=torch.float64, device="cuda")
    eps = np.full(plan.d, 1e-3)
    st = P.PPDState(plan, y)
    P.ppd_iterate(plan, st, y, U, eps, 3, eta=1e-4, use_graph=True, stats=False)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(plan.stream)
    P.ppd_iterate(plan, st, y, U, eps, reps, eta=1e-4, use_graph=True, stats=False)
    b.record(plan.stream)
    torch.cuda.synchronize()
    return 1000.0 * a.elapsed_time(b) / reps


def autotune(nx: int, ny: int, wu, wv, block_off, stream, candidates: Iterable[Tuple[int, int]] = DEFAULT_CANDIDATES,
             cache: Optional[str] = DEFAULT_CACHE, levels: int = 3, verbose: bool = False):
    """Return ((tile, chunk), {candidate: us}) for this coverage."""
    import torch
    key = _key(nx, ny, wu, wv, block_off, torch.cuda.get_device_name(0))
    table = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if key in table:
        best = tuple(table[key]["best"])
        return best, {tuple(map(int, k.split(","))): v for k, v in table[key]["us"].items()}
    timings = {}
    for tile, chunk in candidates:
        if tile > 2 * min(nx, ny):
            continue
        plan = P.Plan(nx, ny, wu, wv, block_off, tile=tile, chunk=chunk, levels=levels, stream=stream)
        timings[(tile, chunk)] = time_iteration(plan)
        if verbose:
            print(f"tune tile={tile} chunk={chunk}: {timings[(tile, chunk)]:.1f} us/iteration", flush=True)
        plan.close()
    best = min(timings, key=timings.get)
    if cache:
        table[key] = {"best": list(best), "us": {f"{t},{c}": v for (t, c), v in timings.items()}}
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        except OSError:
            pass
    return best, timings
