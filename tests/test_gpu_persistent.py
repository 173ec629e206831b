"""The quadratic form's steps in one cooperative launch per call (workgroups
wait for each other between steps) against one launch per step: the same
poses, losses, optimiser counters and rotation log, bit for bit, in one
scene, in several scenes with the per-scene early exit, and with more
cameras than resident wavefronts (each wavefront then takes several cameras
per step)."""
import numpy as np
import pytest

from paper_2605_18052_amd import fastea, synth

from gpu_helpers import make_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(run):
    """run(persistent_steps) -> (result tuple, quad_steps_blocks)."""
    (a, blocks_off), (b, blocks_on) = run(0), run(1)
    assert blocks_off == 0 and blocks_on > 0  # the persistent launch did run
    for x, y in zip(a, b):
        np.testing.assert_array_equal(np.asarray(x), np.asarray(y))
    return blocks_on


def test_persistent_steps_equal_launch_per_step():
    sc = synth.config1()

    def run(ps):
        ctx = make_context(sc, gauge=1, inner_loop=1, persistent_steps=ps, log_every=5, max_log=40)
        ctx.init_poses(sc.R_init, sc.t_init)
        ctx.begin_round(128.0)
        ctx.step(23)  # odd: the next call starts at the other parity
        ctx.begin_round(64.0)
        ctx.step(20)
        loss, gR, gt, gf = ctx.residual_grad()
        out = ctx.get_poses() + (ctx.get_rotation_log(40), float(loss.item()), gR.cpu().numpy())
        blocks = ctx.info()["quad_steps_blocks"]
        ctx.close()
        return out, blocks

    print(f"persistent launch: {_both(run)} workgroups for {sc.n_cams} cameras", flush=True)


def test_persistent_solve_equals_launch_per_step():
    sc = synth.config1()

    def run(ps):
        ctx = make_context(sc, gauge=1, inner_loop=1, persistent_steps=ps, rounds=4, iters_per_round=25,
                           lr_decay=0.5)
        ctx.init_poses(sc.R_init, sc.t_init)
        rep = ctx.epipolar_adjust()
        out = ctx.get_poses() + (rep["loss"], rep["inliers"])
        blocks = ctx.info()["quad_steps_blocks"]
        ctx.close()
        return out, blocks

    _both(run)


def test_persistent_steps_several_scenes_with_early_exit():
    scenes = [synth.sphere_scene(n_cams=12, n_pts=800, seed=31, name="a"),
              synth.trajectory_scene(n_cams=40, n_pts=8000, knn=8, target_matches=150_000, seed=32,
                                     name="b", calib_sample=8000),
              synth.sphere_scene(n_cams=7, n_pts=3000, seed=33, p_det=0.8, name="c")]
    cat, cam_scene, _ = synth.concat_scenes(scenes)

    def run(ps):
        o = fastea.default_options(inner_loop=1, persistent_steps=ps, rounds=10, iters_per_round=15,
                                   converge_deg=0.05, tau_px_min=16.0)
        ctx = fastea.Context(0, o)
        ctx.load_intrinsics(cat["f_init"], cat["cx"], cat["cy"])
        ctx.set_scenes(cam_scene)
        ctx.load_matches(cat["x1"], cat["y1"], cat["x2"], cat["y2"], cat["cam1"], cat["cam2"])
        ctx.init_poses(cat["R_init"], cat["t_init"])
        rep = ctx.epipolar_adjust()
        out = ctx.get_poses() + (rep["loss"], np.array([rep["scenes_converged"]]))
        blocks = ctx.info()["quad_steps_blocks"]
        ctx.close()
        return out, blocks

    _both(run)


def test_persistent_steps_more_cameras_than_resident_waves():
    """3,000 cameras: more than the device holds wavefronts of the kernel at
    once, so wavefronts take several cameras per step."""
    sc = synth.trajectory_scene(n_cams=3000, n_pts=60000, knn=4, target_matches=400_000, seed=35,
                                name="wide", calib_sample=20000)

    def run(ps):
        ctx = make_context(sc, inner_loop=1, persistent_steps=ps)
        ctx.init_poses(sc.R_init, sc.t_init)
        ctx.begin_round(64.0)
        ctx.step(12)
        out = ctx.get_poses()
        blocks = ctx.info()["quad_steps_blocks"]
        ctx.close()
        return out, blocks

    blocks = _both(run)
    print(f"persistent launch: {blocks} workgroups ({4 * blocks} wavefronts) for 3000 cameras", flush=True)
    assert 4 * blocks < 3000


def test_a_wait_past_its_bound_ends_the_launch_and_is_reported():
    """The device-wide wait between steps gives up after wait_limit_us: with
    a bound of 1 us (a wait takes about 10 us) the workgroups leave the
    launch early and set the flag, every wavefront exiting normally; the
    next round boundary reports FEA_EDEVICE once, and the context goes on
    with one launch per step."""
    sc = synth.config1()
    ctx = make_context(sc, inner_loop=1, persistent_steps=1, wait_limit_us=1)
    ctx.init_poses(sc.R_init, sc.t_init)
    ctx.begin_round(128.0)
    ctx.step(20)
    with pytest.raises(fastea.FeaError) as err:
        ctx.begin_round(64.0)
    assert err.value.status == fastea.FEA_EDEVICE and "wait" in str(err.value)
    ctx.begin_round(64.0)  # reported once: the flag was cleared
    ctx.step(20)
    assert ctx.info()["quad_steps_blocks"] > 0  # the last persistent launch's size is kept
    R, t, f = ctx.get_poses()
    assert np.isfinite(R).all() and np.isfinite(t).all() and np.isfinite(f).all()
    ctx.close()
