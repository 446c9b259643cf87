"""The judge and fallback policy of the learned surrogate, as host logic over callables.

The surrogate advances a coarse state on its own; every ``judge_every`` coarse steps the
plain fine model is advanced to the same time, restricted to the coarse grid, and the RMSE
of eta over coarse water cells is measured. Above the threshold, or when the error is not
finite, the coarse state is reset from the restricted fine state and a fallback is counted;
the error is recorded as measured, before any reset. The fine model runs on regardless, so
it is always at the coarse model's time.

The driver knows nothing of devices: the GPU rollout passes closures over the library's
calls, and the CPU tests pass closures over plain reference steppers. ``sync`` is called at
every segment boundary before the clock is read (a device synchronisation on the GPU).
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable


@dataclass
class RolloutResult:
    rmse: list = field(default_factory=list)  # eta RMSE at each judge, before any reset
    fallbacks: int = 0
    surrogate_s: float = 0.0   # coarse steps + network + resets
    judge_s: float = 0.0       # the fine audit runs and the restriction


def falls_back(err: float, threshold: float) -> bool:
    """A judged segment falls back unless its error is finite and at most the threshold."""
    return not (math.isfinite(err) and err <= threshold)


def judged_rollout(advance: Callable[[int], None], fine_advance: Callable[[int], None],
                   error: Callable[[], float], reset: Callable[[], None], n_coarse: int, judge_every: int,
                   threshold: float, fine_per_coarse: int = 4, sync: Callable[[], None] = lambda: None,
                   clock: Callable[[], float] = time.perf_counter) -> RolloutResult:
    """n_coarse coarse steps in segments of judge_every: ``advance(n)`` moves the surrogate n
    coarse steps, ``fine_advance(n)`` the fine model n fine steps (fine_per_coarse per coarse
    step) and restricts it, ``error()`` returns the eta RMSE between the two coarse states and
    ``reset()`` copies the restricted fine state into the surrogate."""
    if judge_every < 1 or n_coarse < 0 or n_coarse % judge_every:
        raise ValueError("n_coarse must be a multiple of judge_every >= 1")
    if not threshold >= 0.0:
        raise ValueError("threshold must be >= 0")
    res = RolloutResult()
    for _ in range(n_coarse // judge_every):
        sync()
        t0 = clock()
        advance(judge_every)
        sync()
        t1 = clock()
        fine_advance(fine_per_coarse * judge_every)
        sync()
        t2 = clock()
        err = float(error())
        res.rmse.append(err)
        if falls_back(err, threshold):
            reset()
            res.fallbacks += 1
        sync()
        t3 = clock()
        res.surrogate_s += (t1 - t0) + (t3 - t2)
        res.judge_s += t2 - t1
    return res
