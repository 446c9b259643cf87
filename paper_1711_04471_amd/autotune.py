"""Autotuner for the batched ensemble: one band height per size class.

Instances are grouped by width into size classes; for each class the candidate band
heights are timed on that class's instances alone (a batch of them, HIP-event timed
steps after a warm-up). A candidate is only eligible if the state it produces is
bitwise equal to every other candidate's (the parity guard: the band height may change
speed, never results). Results are cached in a JSON file keyed by GPU architecture, steps
per pass, class bounds, candidate set and a digest of the member shapes, so a different
ensemble never reuses another's choice.
"""

from __future__ import annotations

import hashlib
import json
import os

import torch

CLASSES = ((128, 256), (256, 512), (512, 1025))
CANDIDATES = (8, 16, 32, 64)
# with several steps per pass the band halo grows by 2 rows per step, so taller bands pay
CANDIDATES_BY_K = {1: CANDIDATES, 2: (16, 32, 48, 64), 3: (16, 32, 48, 64, 96)}


def size_class(nx: int):
    for lo, hi in CLASSES:
        if lo <= nx < hi:
            return (lo, hi)
    return None


def _shapes(cases) -> str:
    """Digest of the members' grid sizes, in member order (part of every cache key)."""
    return hashlib.sha1(",".join(f"{int(c.nx)}x{int(c.ny)}" for c in cases).encode()).hexdigest()[:12]


def _digest(batch) -> str:
    torch.cuda.synchronize(batch.device)
    h = hashlib.sha1()
    for k in range(batch.n):
        for t in batch.state(k):
            h.update(t.contiguous().cpu().numpy().tobytes())
    return h.hexdigest()


def _arch(device) -> str:
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name)


def tune(cases, candidates=None, cache_path=None, steps=24, warmup=6, device="cuda",
         default_rows=16, log=None, steps_per_pass=1, whole=False):
    """Band height per instance (list of ints), tuned per size class for the batched kernel
    at ``steps_per_pass`` steps per pass (steps and warmup must be multiples of it). With
    ``whole``, the tuned assignment is then timed against each uniform height on the whole
    batch and the fastest kept."""
    if candidates is None:
        candidates = CANDIDATES_BY_K[steps_per_pass]
    from .sw2d import Sw2dBatch
    dev = torch.device(device)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    arch = _arch(dev)
    by_class = {}
    for i, c in enumerate(cases):
        by_class.setdefault(size_class(int(c.nx)), []).append(i)
    rows = [default_rows] * len(cases)
    for cls, idx in by_class.items():
        if cls is None:
            continue
        sub = [cases[i] for i in idx]
        key = f"{arch}|K{steps_per_pass}|{cls[0]}-{cls[1]}|{','.join(map(str, candidates))}|{_shapes(sub)}"
        if key not in cache:
            timing, digests = {}, {}
            for cand in candidates:
                with Sw2dBatch(sub, band_rows=[cand] * len(sub), device=dev) as b:
                    b.set_time_blocking(steps_per_pass)
                    b.step(warmup)
                    timing[cand] = b.step_timed(steps)
                    digests[cand] = _digest(b)
            if len(set(digests.values())) != 1:
                raise RuntimeError(f"parity guard: band heights {candidates} disagree on {cls}")
            best = min(timing, key=timing.get)
            cache[key] = {"rows": int(best), "ms_per_step": {str(k): v for k, v in timing.items()},
                          "instances": len(idx)}
            if log:
                log(f"autotune {cls}: {cache[key]}")
        for i in idx:
            rows[i] = int(cache[key]["rows"])
    if whole and len(by_class) > 1:
        # the classes share one grid, so the best heights class by class need not be the best
        # together: time the tuned assignment against each uniform height on the whole batch
        key = f"{arch}|K{steps_per_pass}|whole|{len(cases)}|{','.join(map(str, candidates))}|" \
              f"{hashlib.sha1(json.dumps(rows).encode()).hexdigest()[:12]}|{_shapes(cases)}"
        if key not in cache:
            options = {"tuned": rows}
            options.update({str(c): [c] * len(cases) for c in candidates})
            timing, digests = {}, {}
            for name, opt in options.items():
                with Sw2dBatch(cases, band_rows=[min(r, int(c.ny)) for r, c in zip(opt, cases)], device=dev) as b:
                    b.set_time_blocking(steps_per_pass)
                    b.step(warmup)
                    timing[name] = b.step_timed(steps)
                    digests[name] = _digest(b)
            if len(set(digests.values())) != 1:
                raise RuntimeError("parity guard: band-height assignments disagree on the whole batch")
            best = min(timing, key=timing.get)
            cache[key] = {"choice": best, "rows": [int(r) for r in options[best]],
                          "ms_per_step": timing}
            if log:
                log(f"autotune whole batch: {best} {timing}")
        rows = [int(r) for r in cache[key]["rows"]]
    if cache_path:
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return rows
