"""Batching row: several independent scenes in one context (one launch of
each kernel for all of them) give the same result as solving each alone."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import fastea, metrics, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _scenes():
    return [synth.sphere_scene(n_cams=12, n_pts=800, seed=31, name="a"),
            synth.trajectory_scene(n_cams=40, n_pts=8000, knn=8, target_matches=150_000, seed=32,
                                   name="b", calib_sample=8000),
            synth.sphere_scene(n_cams=7, n_pts=3000, seed=33, p_det=0.8, name="c"),
            synth.trajectory_scene(n_cams=25, n_pts=5000, knn=6, target_matches=60_000, seed=34,
                                   name="d", calib_sample=5000)]


def _opts(inner_loop=0):
    return fastea.default_options(rounds=4, iters_per_round=15, tile_matches=2048, inner_loop=inner_loop)


def _solo(sc, inner_loop=0):
    ctx = fastea.Context(0, _opts(inner_loop))
    ctx.load_intrinsics(sc.f_init, sc.cx, sc.cy)
    ctx.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
    ctx.init_poses(sc.R_init, sc.t_init)
    rep = ctx.epipolar_adjust()
    R, t, f = ctx.get_poses()
    mask, _ = ctx.get_mask()
    ctx.close()
    return R, t, f, mask, rep


@pytest.mark.parametrize("inner_loop", [0, 1])
def test_batched_equals_individual(inner_loop):
    """Per match and with the quadratic form (whose per-scene counts and
    normalisers are summed on the device): each scene of the batch ends as
    it does when solved alone."""
    scenes = _scenes()
    cat, cam_scene, offs = synth.concat_scenes(scenes)
    ctx = fastea.Context(0, _opts(inner_loop))
    ctx.load_intrinsics(cat["f_init"], cat["cx"], cat["cy"])
    ctx.set_scenes(cam_scene)
    ctx.load_matches(cat["x1"], cat["y1"], cat["x2"], cat["y2"], cat["cam1"], cat["cam2"])
    ctx.init_poses(cat["R_init"], cat["t_init"])
    ctx.epipolar_adjust()
    R, t, f = ctx.get_poses()
    mask, _ = ctx.get_mask()
    stats = ctx.scene_stats()
    assert ctx.info()["n_scenes"] == len(scenes)
    ctx.close()
    m0 = 0
    for k, sc in enumerate(scenes):
        Rs, ts, fs, ms, rep = _solo(sc, inner_loop)
        sl = slice(offs[k], offs[k + 1])
        np.testing.assert_allclose(R[sl], Rs, rtol=0, atol=1e-12)
        np.testing.assert_allclose(t[sl], ts, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(f[sl], fs, rtol=1e-12)
        assert np.array_equal(mask[m0:m0 + sc.n_matches], ms)
        assert stats["retained"][k] == rep["inliers"][-1]
        m0 += sc.n_matches


def test_batch_rejects_cross_scene_matches_and_groups():
    scenes = _scenes()[:2]
    cat, cam_scene, offs = synth.concat_scenes(scenes)
    ctx = fastea.Context(0, _opts())
    ctx.load_intrinsics(cat["f_init"], cat["cx"], cat["cy"])
    ctx.set_scenes(cam_scene)
    c2 = cat["cam2"].copy()
    c2[0] = offs[1] if cat["cam1"][0] < offs[1] else 0
    with pytest.raises(fastea.FeaError) as e:
        ctx.load_matches(cat["x1"], cat["y1"], cat["x2"], cat["y2"], cat["cam1"], c2)
    assert e.value.status == fastea.FEA_EINVAL
    groups = np.arange(len(cam_scene), dtype=np.int32)
    groups[offs[1]] = 0  # first camera of scene 1 shares scene 0's group
    ctx.load_intrinsics(cat["f_init"], cat["cx"], cat["cy"], groups)
    with pytest.raises(fastea.FeaError) as e:
        ctx.set_scenes(cam_scene)
    assert e.value.status == fastea.FEA_EINVAL
    ctx.close()


def test_autotuner_choice_is_reused_in_process():
    """The timed pick of the work-item shape is remembered per size class:
    a second context on a problem of the same size gets the same shape."""
    sc = synth.trajectory_scene(n_cams=60, n_pts=20000, knn=8, target_matches=400_000, seed=36,
                                name="tune", calib_sample=8000)
    picks = []
    for _ in range(2):
        ctx = fastea.Context(0, fastea.default_options(tile_matches=0))
        ctx.load_intrinsics(sc.f_init, sc.cx, sc.cy)
        ctx.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
        ctx.init_poses(sc.R_init, sc.t_init)
        ctx.begin_round(128.0)
        info = ctx.info()
        picks.append((info["tile_matches"], info["tile_threads"]))
        ctx.close()
    assert picks[0] == picks[1] and picks[0][0] in (1024, 2048, 4096, 8192)


@pytest.mark.parametrize("inner_loop", [0, 1])
def test_batch_solve_equals_solo_solves(inner_loop):
    """fea_batch_solve over separately loaded contexts: each context ends
    with the poses its solo solve reaches, and its report holds that solve's
    per-round loss and retained matches."""
    scenes = _scenes()
    ctxs, solo = [], []
    for sc in scenes:
        c = fastea.Context(0, _opts(inner_loop))
        c.load_intrinsics(sc.f_init, sc.cx, sc.cy)
        c.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
        c.init_poses(sc.R_init, sc.t_init)
        ctxs.append(c)
        solo.append(_solo(sc, inner_loop))
    reps = fastea.batch_solve(ctxs)
    for c, (Rs, ts, fs, _, rep_s), rep in zip(ctxs, solo, reps):
        R, t, f = c.get_poses()
        np.testing.assert_allclose(R, Rs, rtol=0, atol=1e-12)
        np.testing.assert_allclose(t, ts, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(f, fs, rtol=1e-12)
        assert rep["rounds_run"] == rep_s["rounds_run"] and rep["iters_run"] == rep_s["iters_run"]
        np.testing.assert_array_equal(rep["inliers"], rep_s["inliers"])
        np.testing.assert_allclose(rep["loss"], rep_s["loss"], rtol=1e-10)
        assert rep["scenes_converged"] == 0
        c.close()


def test_batch_solve_rejects_bad_arguments():
    sc = _scenes()[0]
    c = fastea.Context(0, _opts())
    c.load_intrinsics(sc.f_init, sc.cx, sc.cy)
    c.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
    with pytest.raises(fastea.FeaError) as e:
        fastea.batch_solve([c])  # no poses yet
    assert e.value.status == fastea.FEA_ESTATE
    c.init_poses(sc.R_init, sc.t_init)
    with pytest.raises(fastea.FeaError) as e:
        fastea.batch_solve([c, c])
    assert e.value.status == fastea.FEA_EINVAL
    with pytest.raises(fastea.FeaError) as e:
        fastea.batch_solve([c], fastea.default_options(tile_matches=3000))
    assert e.value.status == fastea.FEA_EINVAL
    c.close()
