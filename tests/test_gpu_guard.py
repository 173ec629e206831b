"""Non-finite guard: a scene whose parameters go non-finite between round
boundaries gets back the poses of the snapshot its last round started from
and takes no further steps; the other scenes of the context go on, and the
call that found it returns FEA_ENONFINITE.  The non-finite value is written
from the host through fea_set_params_dev (device tensors), so every kernel
still runs on finite or NaN arithmetic only (no fault is provoked)."""
import math

import numpy as np
import pytest

from paper_2605_18052_amd import fastea, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _two_scenes(**opt):
    scenes = [synth.tiny_scene(n_cams=6, n_pts=80, seed=11, sigma=0.5, outlier_frac=0.1),
              synth.tiny_scene(n_cams=5, n_pts=70, seed=12, sigma=0.5, outlier_frac=0.1)]
    cat, cam_scene, offs = synth.concat_scenes(scenes)
    ctx = fastea.Context(0, fastea.default_options(**opt))
    ctx.load_intrinsics(cat["f_init"], cat["cx"], cat["cy"])
    ctx.set_scenes(cam_scene)
    ctx.load_matches(cat["x1"], cat["y1"], cat["x2"], cat["y2"], cat["cam1"], cat["cam2"])
    ctx.init_poses(cat["R_init"], cat["t_init"])
    return ctx, offs


@pytest.mark.parametrize("inner_loop", [0, 1])
def test_guard_restores_and_stops_the_scene(inner_loop):
    import torch
    ctx, offs = _two_scenes(inner_loop=inner_loop, tile_matches=8192 if inner_loop else 1024)
    a, b = slice(offs[0], offs[1]), slice(offs[1], offs[2])
    ctx.begin_round(64.0)
    R0, t0, f0 = ctx.get_poses()  # the poses the round's snapshot holds
    ctx.step(7)
    R1, t1, f1 = ctx.get_poses()
    assert not np.allclose(R1[a], R0[a])  # the steps moved both scenes
    a6, t, logf = ctx.get_params()
    t[offs[0] + 2, 1] = math.nan
    ctx.set_params_dev(a6, t, logf)
    with pytest.raises(fastea.FeaError) as err:
        ctx.begin_round(32.0)
    assert err.value.status == fastea.FEA_ENONFINITE
    np.testing.assert_array_equal(ctx.scene_nonfinite(), [1, -1])
    R2, t2, f2 = ctx.get_poses()
    np.testing.assert_allclose(R2[a], R0[a], rtol=0, atol=1e-12)
    np.testing.assert_allclose(t2[a], t0[a], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(f2[a], f0[a], rtol=1e-14)
    np.testing.assert_array_equal(R2[b], R1[b])  # the other scene is untouched
    # the stopped scene takes no further steps, the other one does
    ctx.step(10)
    R3, t3, f3 = ctx.get_poses()
    np.testing.assert_array_equal(R3[a], R2[a])
    np.testing.assert_array_equal(t3[a], t2[a])
    assert not np.allclose(R3[b], R2[b])
    assert np.isfinite(R3).all() and np.isfinite(t3).all() and np.isfinite(f3).all()
    # found once: the next boundary does not report it again
    ctx.begin_round(16.0)
    # a solve from here keeps it stopped and reports it
    rep = ctx.epipolar_adjust()
    assert rep["scenes_nonfinite"] == 1
    np.testing.assert_array_equal(ctx.get_poses()[0][a], R2[a])
    ctx.close()


def test_guard_stops_a_solve_and_reports(monkeypatch):
    """A single-scene solve whose parameters are made non-finite before the
    solve's first round boundary: fea_epipolar_adjust returns
    FEA_ENONFINITE with the report filled and the last finite poses."""
    sc = synth.tiny_scene(n_cams=6, n_pts=80, seed=13, sigma=0.5, outlier_frac=0.1)
    ctx = fastea.Context(0, fastea.default_options(rounds=3, iters_per_round=5))
    ctx.load_intrinsics(sc.f_init, sc.cx, sc.cy)
    ctx.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
    ctx.init_poses(sc.R_init, sc.t_init)
    ctx.begin_round(64.0)
    R0, t0, _ = ctx.get_poses()
    a6, t, logf = ctx.get_params()
    a6[1, 0] = math.inf
    ctx.set_params_dev(a6, t, logf)
    with pytest.raises(fastea.FeaError) as err:
        ctx.epipolar_adjust()
    assert err.value.status == fastea.FEA_ENONFINITE
    assert err.value.report["scenes_nonfinite"] == 1 and err.value.report["rounds_run"] == 3
    R, t2, f = ctx.get_poses()
    np.testing.assert_allclose(R, R0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(t2, t0, rtol=1e-12, atol=1e-12)
    assert ctx.scene_nonfinite()[0] == 1
    ctx.close()


def test_guard_is_silent_on_finite_solves():
    ctx, _ = _two_scenes(rounds=3, iters_per_round=5)
    rep = ctx.epipolar_adjust()
    assert rep["scenes_nonfinite"] == 0
    np.testing.assert_array_equal(ctx.scene_nonfinite(), [-1, -1])
    ctx.close()
