"""Checkpoint / resume: a context restored from fea_get_state continues bit
for bit as the saved one does (plain and learned weights, several scenes),
and states that do not fit the loaded problem are rejected."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import fastea, synth

from gpu_helpers import make_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _soft_inlier_mlp():
    W1 = np.zeros((64, 8))
    W1[0, 0] = 1.0
    W2 = np.zeros((64, 64))
    W2[0, 0] = 1.0
    w3 = np.zeros(64)
    w3[0] = -8.0
    return oracle.mlp_pack(W1, np.zeros(64), W2, np.zeros(64), w3, [5.0]).astype(np.float32)


def _continue(ctx):
    """The same continuation for both contexts: rest of a round, a new round."""
    ctx.step(23)
    ctx.begin_round(32.0)
    ctx.step(11)
    R, t, f = ctx.get_poses()
    mask, z = ctx.get_mask()
    return R, t, f, mask, z, ctx.info()


def _same(a, b):
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)
    assert a[4] == b[4]
    for k in ("round", "step", "n_retained", "n_items", "tile_matches"):
        assert a[5][k] == b[5][k], k


@pytest.mark.parametrize("weight_mode,inner_loop", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_resume_is_bit_identical(weight_mode, inner_loop):
    sc = synth.config1()
    # learned weights with the quadratic form take its default 8192-match items
    tile = 0 if (weight_mode and inner_loop) else 2048
    mk = lambda: make_context(sc, gauge=1, weight_mode=weight_mode, inner_loop=inner_loop,
                              tile_matches=tile)
    a = mk()
    if weight_mode:
        a.set_mlp(_soft_inlier_mlp())
    a.init_poses(sc.R_init, sc.t_init)
    a.begin_round(128.0)
    a.step(17)
    a.begin_round(64.0)
    a.step(9)
    state = a.get_state()
    ref = _continue(a)
    a.close()

    b = mk()
    if weight_mode:
        b.set_mlp(_soft_inlier_mlp())
    b.set_state(state)
    assert b.info()["round"] == 1 and b.info()["step"] == 9
    got = _continue(b)
    b.close()
    _same(ref, got)


def test_resume_several_scenes_and_before_first_round():
    scenes = [synth.sphere_scene(n_cams=9, n_pts=600, seed=41, name="a"),
              synth.sphere_scene(n_cams=6, n_pts=900, seed=42, p_det=0.7, name="b")]
    cat, cam_scene, _ = synth.concat_scenes(scenes)

    def mk():
        ctx = fastea.Context(0, fastea.default_options(tile_matches=1024))
        ctx.load_intrinsics(cat["f_init"], cat["cx"], cat["cy"])
        ctx.set_scenes(cam_scene)
        ctx.load_matches(cat["x1"], cat["y1"], cat["x2"], cat["y2"], cat["cam1"], cat["cam2"])
        return ctx

    a = mk()
    a.init_poses(cat["R_init"], cat["t_init"])
    s0 = a.get_state()  # before any round
    a.begin_round(128.0)
    a.step(30)
    s1 = a.get_state()
    ref = _continue(a)
    a.close()
    b = mk()
    b.set_state(s1)
    _same(ref, _continue(b))
    # the state before the first round: the same solve from the start
    b.set_state(s0)
    b.begin_round(128.0)
    b.step(30)
    _same(ref, _continue(b))
    b.close()


def test_mismatched_states_are_rejected():
    sc = synth.config1()
    a = make_context(sc)
    with pytest.raises(fastea.FeaError) as e:
        a.get_state()
    assert e.value.status == fastea.FEA_ESTATE
    a.init_poses(sc.R_init, sc.t_init)
    a.begin_round(math.inf)
    state = a.get_state()
    with pytest.raises(fastea.FeaError) as e:
        a.set_state(state[:-1])
    assert e.value.status == fastea.FEA_EINVAL
    bad = bytearray(state)
    bad[0] ^= 0xFF
    with pytest.raises(fastea.FeaError) as e:
        a.set_state(bytes(bad))
    assert e.value.status == fastea.FEA_EINVAL
    a.close()
    # same sizes, matches in another order: another sorted order
    rng = np.random.default_rng(0)
    p = rng.permutation(sc.n_matches)
    o = fastea.Context(0, fastea.default_options())
    o.load_intrinsics(sc.f_init, sc.cx, sc.cy)
    o.load_matches(sc.x1[p], sc.y1[p], sc.x2[p], sc.y2[p], sc.cam1[p], sc.cam2[p])
    with pytest.raises(fastea.FeaError) as e:
        o.set_state(state)
    assert e.value.status == fastea.FEA_EINVAL
    o.close()
    # a learned state needs the network
    l = make_context(sc, weight_mode=1)
    l.set_mlp(_soft_inlier_mlp())
    l.init_poses(sc.R_init, sc.t_init)
    l.begin_round(128.0)
    ls = l.get_state()
    l.close()
    m = make_context(sc, weight_mode=1)
    with pytest.raises(fastea.FeaError) as e:
        m.set_state(ls)
    assert e.value.status == fastea.FEA_ESTATE
    m.close()


def test_kernel_timing_leaves_results_unchanged():
    """Steps timed with per-launch HIP events (no graph replay) give the same
    poses bit for bit as untimed steps replayed from graphs; every timed
    launch is reported and the per-launch durations add up to the total."""
    sc = synth.config1()
    out = []
    for timed in (False, True):
        ctx = make_context(sc)
        ctx.init_poses(sc.R_init, sc.t_init)
        ctx.begin_round(16.0)
        ctx.set_kernel_timing(timed)
        ctx.step(25)
        if timed:
            total, n = ctx.kernel_timing()
            each = ctx.kernel_times()
            assert n == 25 and len(each) == 25
            assert np.all(each > 0)
            assert abs(each.sum() - total) <= 1e-6 * total
            ctx.set_kernel_timing(False)
            assert ctx.kernel_timing() == (0.0, 0) and len(ctx.kernel_times()) == 0
        out.append(ctx.get_poses())
        ctx.close()
    for x, y in zip(out[0], out[1]):
        assert np.array_equal(x, y)
