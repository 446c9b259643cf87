"""Autotuner for the batched ensemble: one band height per size class.

Instances are grouped by width into size classes; for each class the candidate band
heights are timed on that class's instances alone (a batch of them, HIP-event timed
steps after a warm-up). A candidate is only eligible if the state it produces is
bitwise equal to every other candidate's (the parity guard: the band height may change
speed, never results). Results are cached in a JSON file keyed by GPU architecture,
class bounds and candidate set.
"""

from __future__ import annotations

import hashlib
import json
import os

import torch

CLASSES = ((128, 256), (256, 512), (512, 1025))
CANDIDATES = (8, 16, 32, 64)


def size_class(nx: int):
    for lo, hi in CLASSES:
        if lo <= nx < hi:
            return (lo, hi)
    return None


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


def tune(cases, candidates=CANDIDATES, cache_path=None, steps=20, warmup=5, device="cuda",
         default_rows=16, log=None):
    """Band height per instance (list of ints), tuned per size class."""
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
        key = f"{arch}|{cls[0]}-{cls[1]}|{','.join(map(str, candidates))}"
        if key not in cache:
            sub = [cases[i] for i in idx]
            timing, digests = {}, {}
            for cand in candidates:
                with Sw2dBatch(sub, band_rows=[cand] * len(sub), device=dev) as b:
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
    if cache_path:
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return rows
