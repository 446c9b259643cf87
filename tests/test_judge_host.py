"""The surrogate's judge and fallback policy on the CPU, with the FP64 oracle as both the fine
and the coarse model and stub corrections in place of the network: no fallback when the
threshold is out of reach, one per judge at threshold 0 (each reset restarting the coarse
model from the restricted fine state), a NaN planted by the correction caught and cleared,
and a coarse model pushed past its stability limit caught by the judge."""
import math

import numpy as np
import pytest

from oracle import cnn_ref, sw2d_ref
from paper_1711_04471_amd import inputs
from paper_1711_04471_amd.judge import falls_back, judged_rollout

FINE = 64  # 64^2 fine basin with a 4-cell land border -> 16^2 coarse


def _case(seed=50400):
    return inputs.seeded_basin(f"judge_{seed}", FINE, FINE, 500.0, seed=seed, n_bumps=2, steps=0, border=4)


class OraclePair:
    """Fine and coarse oracle models; ``correction(state, k)`` (a stub) may alter the coarse
    state after its k-th coarse step. ``dt_factor`` scales the coarse time step."""

    def __init__(self, case, correction=None, dt_factor=1.0):
        self.c = case
        self.fine = [np.asarray(case.eta, np.float64), np.asarray(case.u, np.float64), np.asarray(case.v, np.float64)]
        self.ref = list(cnn_ref.restrict4(*self.fine, case.H, case.mask))
        self.Hc, self.mc = self.ref[3], self.ref[4]
        self.coarse = [a.copy() for a in self.ref[:3]]
        self.correction = correction
        self.dt_c = 4 * case.dt * dt_factor
        self.k = 0

    def advance(self, n):
        c = self.c
        for _ in range(n):
            try:
                e, u, v, _ = sw2d_ref.run(FINE // 4, FINE // 4, 4 * c.dx, 4 * c.dy, c.g, self.dt_c, c.eps, self.Hc,
                                          self.mc, *self.coarse, 1, reductions=False)
            except sw2d_ref.DryCellError:  # a blown-up coarse model: its state is lost
                e = u = v = np.full_like(self.Hc, np.nan)
            self.coarse = [e, u, v]
            self.k += 1
            if self.correction is not None:
                self.coarse = self.correction(self.coarse, self.k)

    def fine_advance(self, n):
        c = self.c
        e, u, v, _ = sw2d_ref.run(c.nx, c.ny, c.dx, c.dy, c.g, c.dt, c.eps, c.H, c.mask, *self.fine, n,
                                  reductions=False)
        self.fine = [e, u, v]
        self.ref = list(cnn_ref.restrict4(e, u, v, c.H, c.mask))

    def error(self):
        e = self.coarse[0]
        if not np.all(np.isfinite(e)):
            return math.nan
        return cnn_ref.rmse_wet(e, self.ref[0], self.mc)

    def reset(self):
        self.coarse = [a.copy() for a in self.ref[:3]]

    def run(self, n_coarse, judge_every, threshold, **kw):
        return judged_rollout(self.advance, self.fine_advance, self.error, self.reset, n_coarse, judge_every,
                              threshold, **kw)


def test_falls_back_rule():
    assert not falls_back(0.0, 0.0) and not falls_back(1e-3, 1e-3)
    assert falls_back(1.0000001e-3, 1e-3)
    assert falls_back(math.nan, 1e9) and falls_back(math.inf, 1e9)


def test_no_fallback_below_an_unreachable_threshold():
    """Threshold out of reach: the coarse model runs alone and each judge's error is the one
    of an independent coarse-only run against the restricted fine model at that time."""
    case = _case()
    r = OraclePair(case).run(12, 4, 1e9)
    assert r.fallbacks == 0 and len(r.rmse) == 3
    # the same errors from one coarse run of 12 steps and one fine run of 48, read every 4 / 16
    c = case
    fine = [np.asarray(a, np.float64) for a in (c.eta, c.u, c.v)]
    e0, u0, v0, Hc, mc = cnn_ref.restrict4(*fine, c.H, c.mask)
    coarse = [e0, u0, v0]
    expect = []
    for _ in range(3):
        coarse = list(sw2d_ref.run(16, 16, 4 * c.dx, 4 * c.dy, c.g, 4 * c.dt, c.eps, Hc, mc, *coarse, 4,
                                   reductions=False)[:3])
        fine = list(sw2d_ref.run(c.nx, c.ny, c.dx, c.dy, c.g, c.dt, c.eps, c.H, c.mask, *fine, 16,
                                 reductions=False)[:3])
        expect.append(cnn_ref.rmse_wet(coarse[0], cnn_ref.restrict4(*fine, c.H, c.mask)[0], mc))
    assert r.rmse == pytest.approx(expect, rel=1e-12, abs=0)
    assert all(x > 0 for x in r.rmse)


def test_every_judge_falls_back_at_threshold_zero():
    """Threshold 0: every judge falls back, and each reset leaves the coarse state equal to the
    restricted fine state, so each segment's error is that of a fresh start from it."""
    case = _case()
    pair = OraclePair(case)
    r = pair.run(12, 4, 0.0)
    assert r.fallbacks == 3 and len(r.rmse) == 3
    for a, b in zip(pair.coarse, pair.ref[:3]):
        assert np.array_equal(a, b)
    # segment 2 restarted from R(fine after 16 fine steps)
    c = case
    fine = list(sw2d_ref.run(c.nx, c.ny, c.dx, c.dy, c.g, c.dt, c.eps, c.H, c.mask, c.eta, c.u, c.v, 16,
                             reductions=False)[:3])
    e0, u0, v0, Hc, mc = cnn_ref.restrict4(*fine, c.H, c.mask)
    co = sw2d_ref.run(16, 16, 4 * c.dx, 4 * c.dy, c.g, 4 * c.dt, c.eps, Hc, mc, e0, u0, v0, 4, reductions=False)[0]
    fine = list(sw2d_ref.run(c.nx, c.ny, c.dx, c.dy, c.g, c.dt, c.eps, c.H, c.mask, *fine, 16,
                             reductions=False)[:3])
    ref = cnn_ref.restrict4(*fine, c.H, c.mask)[0]
    assert r.rmse[1] == pytest.approx(cnn_ref.rmse_wet(co, ref, mc), rel=1e-12)


def test_a_planted_nan_is_caught_and_cleared():
    """A correction that writes NaN into eta after coarse step 6 (second segment): that judge
    sees a non-finite error and falls back; the reset clears it, the next segment is finite."""
    def corrupt(state, k):
        if k == 6:
            e = state[0].copy()
            e[8, 8] = np.nan
            return [e, state[1], state[2]]
        return state

    r = OraclePair(_case(), correction=corrupt).run(12, 4, 1e9)
    assert r.fallbacks == 1
    assert math.isfinite(r.rmse[0]) and math.isnan(r.rmse[1]) and math.isfinite(r.rmse[2])


def test_a_biased_correction_falls_back_and_the_timings_add_up():
    """A stub correction adding 1 cm to every water cell of eta each coarse step: above a 1 mm
    threshold at every judge. With a counting clock each segment adds 2 ticks of surrogate
    time (advance; error, reset) and 1 of judge time."""
    pair = OraclePair(_case())
    wet = pair.mc != 0
    pair.correction = lambda state, k: [state[0] + 0.01 * wet, state[1], state[2]]
    ticks = iter(range(10 ** 6))
    r = pair.run(8, 4, 1e-3, clock=lambda: float(next(ticks)))
    assert r.fallbacks == 2 and all(x > 0.03 for x in r.rmse)
    assert r.surrogate_s == 4.0 and r.judge_s == 2.0


def test_blow_up_past_the_stability_limit_is_caught():
    """The coarse oracle at three times its stable step: the state grows without bound (or a
    cell dries out and the model is lost) and the judge falls back; the fine model, at its
    own stable step, stays finite and bounded."""
    case = _case()
    stable = OraclePair(case).run(40, 20, 1e9)
    assert all(math.isfinite(x) and x < 0.2 for x in stable.rmse), stable.rmse
    pair = OraclePair(case, dt_factor=3.0)
    r = pair.run(40, 20, 1e-3)
    assert r.fallbacks == 2
    assert any((not math.isfinite(x)) or x > 1.0 for x in r.rmse), r.rmse
    assert np.all(np.isfinite(pair.fine[0])) and np.abs(pair.fine[0]).max() < 2.0


def test_bad_arguments():
    pair = OraclePair(_case())
    with pytest.raises(ValueError):
        pair.run(10, 4, 1e-3)
    with pytest.raises(ValueError):
        pair.run(8, 0, 1e-3)
    with pytest.raises(ValueError):
        pair.run(8, 4, -1.0)
