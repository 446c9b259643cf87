"""The batched persistent form: every instance bitwise equal to the same basin stepped alone
through sw2d_step, graph replays equal eager launches, folds equal the single-grid folds up
to summation order and the oracle's to 1e-5, and a barrier deadline is reported."""
import numpy as np
import pytest

from oracle import sw2d_ref
from paper_1711_04471_amd import _lib, inputs
from paper_1711_04471_amd.sw2d import Sw2d, Sw2dBatch
from tests.helpers import gpu_run, rel_l2

pytestmark = pytest.mark.gpu

SHAPES = [(70, 65), (130, 257), (241, 90), (128, 128), (300, 301), (61, 200), (1024, 130),
          (517, 333), (200, 200), (90, 700), (3, 3), (9, 40)]


def _cases(shapes, steps=37):
    out = []
    for k, (nx, ny) in enumerate(shapes):
        if min(nx, ny) < 12:
            c = inputs.small_basin(40, 40, seed=900 + k, steps=steps)
            sl = (slice(0, ny), slice(0, nx))
            c.nx, c.ny = nx, ny
            c.H, c.mask, c.eta, c.u, c.v = (np.ascontiguousarray(a[sl]) for a in
                                            (c.H, c.mask, c.eta, c.u, c.v))
            c.mask[0], c.mask[-1], c.mask[:, 0], c.mask[:, -1] = 0, 0, 0, 0
            if not c.mask.any():
                c.mask[1, 1] = 1
            c.eta[c.mask == 0] = 0
        else:
            c = inputs.small_basin(nx, ny, seed=900 + k, steps=steps, n_bumps=2)
        out.append(c)
    return out


def test_batch_is_bitwise_equal_to_single_runs():
    cases = _cases(SHAPES)
    rows = [8, 16, 24, 8, 32, 8, 16, 64, 8, 16, 8, 8]
    n = 37
    with Sw2dBatch(cases, band_rows=rows) as b:
        b.set_launch(steps_per_launch=10, use_graph=True)
        b.step(n)
        red = b.reduce()
        states = [b.state_numpy(k) for k in range(b.n)]
    assert (red["step"] == n).all()
    for k, c in enumerate(cases):
        e, u, v, sred = gpu_run(c, nsteps=n, k=1)
        for g, s in zip(states[k], (e, u, v)):
            assert np.array_equal(g, s), f"instance {k} {c.nx}x{c.ny}"
        np.testing.assert_allclose(red["vol_disp"][k], sred["vol_disp"][-1], rtol=1e-12,
                                   atol=1e-9 * c.dx * c.dy)
        assert red["max_abs_u"][k] == sred["max_abs_u"][-1]
        assert red["max_abs_v"][k] == sred["max_abs_v"][-1]
    for k in (0, 4, 9):
        c = cases[k]
        oe, ou, ov, ored = sw2d_ref.run_case(c, nsteps=n)
        assert max(rel_l2(states[k][0], oe), rel_l2(states[k][1], ou), rel_l2(states[k][2], ov)) <= 1e-5
        np.testing.assert_allclose(red["vol_disp"][k], ored[-1, 1], rtol=1e-5)


def test_graph_replays_equal_eager_launches():
    cases = _cases(SHAPES[:6], steps=60)
    with Sw2dBatch(cases) as g, Sw2dBatch(cases) as e:
        g.set_launch(steps_per_launch=7, use_graph=True)
        e.set_launch(steps_per_launch=7, use_graph=False)
        for rep in range(3):
            g.step(20)
            e.step(20)
            rg, re_ = g.reduce(), e.reduce()
            assert np.array_equal(rg, re_), rep
            for k in range(len(cases)):
                for x, y in zip(g.state_numpy(k), e.state_numpy(k)):
                    assert np.array_equal(x, y), (rep, k)


def test_launch_shape_changes_no_bit():
    cases = _cases(SHAPES[:5], steps=30)
    ref = None
    for spl, grid in ((1, 0), (13, 0), (50, 0), (30, 64)):
        with Sw2dBatch(cases) as b:
            b.set_launch(steps_per_launch=spl, use_graph=True, grid=grid)
            b.step(30)
            got = [b.state_numpy(k) for k in range(b.n)]
        if ref is None:
            ref = got
        for k in range(len(cases)):
            for x, y in zip(got[k], ref[k]):
                assert np.array_equal(x, y), (spl, grid, k)


def test_barrier_deadline_is_reported():
    cases = _cases(SHAPES[:4], steps=10)
    with Sw2dBatch(cases) as b:
        b.set_barrier_timeout(0.0)
        b.step(5)
        with pytest.raises(_lib.Sw2dError) as ei:
            b.reduce()
        assert ei.value.code == _lib.SW2D_EHIP


def test_batch_rejects_bad_instance():
    cases = _cases(SHAPES[:3], steps=10)
    cases[1].mask[0, 5] = 1  # wet border
    with pytest.raises(_lib.Sw2dError) as ei:
        Sw2dBatch(cases)
    assert ei.value.code == _lib.SW2D_EINVAL


def test_full_ensemble_as_benchmarked(tmp_path):
    """The 256-member ensemble (sides 128..1024) exactly as the benchmark runs it: autotuned
    band heights, the steps per pass and steps per launch of the benchmark, HIP graph replay,
    999 steps. Sampled members (the smallest, the largest and two others) bitwise equal to
    the same basins stepped alone; the smallest and the largest against the oracle; every
    member's folds finite and its displaced volume conserved to 1e-5."""
    import bench
    from paper_1711_04471_amd import autotune
    K, launch = bench.BATCH_PASS, bench.BATCH_LAUNCH_PASSES * bench.BATCH_PASS
    steps = 999 // K * K
    cases = inputs.ensemble(steps=steps)
    print(f"ensemble cells {sum(c.nx * c.ny for c in cases)}, K={K}, {launch} steps per launch", flush=True)
    rows = autotune.tune(cases, cache_path=str(tmp_path / "tune.json"), steps_per_pass=K, whole=True)
    print(f"autotuned rows {sorted(set(rows))}", flush=True)
    with Sw2dBatch(cases, band_rows=rows) as b:
        b.set_time_blocking(K)
        b.set_launch(steps_per_launch=launch, use_graph=True)
        b.step(steps)
        red = b.reduce()
        sizes = [c.nx * c.ny for c in cases]
        picks = [int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 100]
        got = {k: b.state_numpy(k) for k in picks}
    assert (red["step"] == steps).all()
    assert np.isfinite(red["vol_total"]).all() and np.isfinite(red["max_abs_u"]).all()
    for k, c in enumerate(cases):
        v0 = sw2d_ref.reduce(c.nx, c.ny, c.dx, c.dy, c.H, c.mask, c.eta, c.u, c.v)
        assert abs(red["vol_disp"][k] - v0[1]) <= 1e-5 * abs(v0[1]), (k, red["vol_disp"][k], v0[1])
    for k in picks:
        e, u, v, _ = gpu_run(cases[k], nsteps=steps, k=1)
        for x, y in zip(got[k], (e, u, v)):
            assert np.array_equal(x, y), k
    for k in picks[:2]:
        print(f"oracle member {k} {cases[k].nx}x{cases[k].ny}", flush=True)
        oe, ou, ov, ored = sw2d_ref.run_case(cases[k], nsteps=steps, nthreads=8)
        assert max(rel_l2(got[k][0], oe), rel_l2(got[k][1], ou), rel_l2(got[k][2], ov)) <= 1e-5, k
        np.testing.assert_allclose(red["vol_disp"][k], ored[-1, 1], rtol=1e-5)
        np.testing.assert_allclose(red["max_abs_u"][k], ored[-1, 2], rtol=1e-5)
        np.testing.assert_allclose(red["max_abs_v"][k], ored[-1, 3], rtol=1e-5)


def test_autotuner_parity_guard_and_cache(tmp_path):
    from paper_1711_04471_amd import autotune
    cases = _cases([(150, 140), (160, 200), (300, 260), (600, 333)], steps=10)
    path = str(tmp_path / "tune.json")
    rows = autotune.tune(cases, candidates=(8, 16, 32), cache_path=path, steps=5, warmup=2)
    assert len(rows) == 4 and all(r in (8, 16, 32) for r in rows)
    again = autotune.tune(cases, candidates=(8, 16, 32), cache_path=path, steps=5, warmup=2)
    assert again == rows


@pytest.mark.parametrize("K", [2, 3])
def test_multi_step_passes_equal_single_runs(K):
    """K steps per pass in the batched kernel: every instance bitwise equal to single steps,
    the folds of every step kept (the last K ring entries checked against single runs)."""
    cases = _cases(SHAPES)
    rows = [8, 16, 24, 8, 32, 8, 16, 64, 8, 16, 8, 8]
    n = 12 * K
    with Sw2dBatch(cases, band_rows=rows) as b:
        b.set_time_blocking(K)
        assert b.time_blocking == K
        b.set_launch(steps_per_launch=5 * K, use_graph=True)
        b.step(n - 2 * K)
        b.step(K)
        b.step(K)
        red = b.reduce()
        states = [b.state_numpy(k) for k in range(b.n)]
        with pytest.raises(_lib.Sw2dError):
            b.step(K + 1)
    assert (red["step"] == n).all()
    for k, c in enumerate(cases):
        e, u, v, sred = gpu_run(c, nsteps=n, k=1)
        for g, s in zip(states[k], (e, u, v)):
            assert np.array_equal(g, s), f"K={K} instance {k} {c.nx}x{c.ny}"
        np.testing.assert_allclose(red["vol_disp"][k], sred["vol_disp"][-1], rtol=1e-12,
                                   atol=1e-9 * c.dx * c.dy)
        assert red["max_abs_u"][k] == sred["max_abs_u"][-1]
        assert red["max_abs_v"][k] == sred["max_abs_v"][-1]


def test_switching_steps_per_pass_mid_run():
    cases = _cases(SHAPES[:6], steps=30)
    with Sw2dBatch(cases) as b:
        b.step(5)
        b.set_time_blocking(3)
        b.step(9)
        b.set_time_blocking(2)
        b.step(4)
        b.set_time_blocking(1)
        b.step(3)
        states = [b.state_numpy(k) for k in range(b.n)]
        red = b.reduce()
    assert (red["step"] == 21).all()
    for k, c in enumerate(cases):
        e, u, v, _ = gpu_run(c, nsteps=21, k=1)
        for g, s in zip(states[k], (e, u, v)):
            assert np.array_equal(g, s), k
