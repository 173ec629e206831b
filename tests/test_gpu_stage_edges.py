"""Empty and minimal inputs of the stages before the adjustment, through
the C-ABI: no matches for the search, one candidate for the vote, two
cameras and one pair for global rotation and for the alignment."""
import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import fastea, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def test_search_with_no_matches_returns_nothing():
    ctx = fastea.Context(0)
    ctx.load_intrinsics(np.full(3, 500.0), np.full(3, 320.0), np.full(3, 240.0))
    e = np.zeros(0, np.float32)
    ctx.load_matches(e, e, e, e, np.zeros(0, np.int32), np.zeros(0, np.int32))
    got = ctx.relative_translations(np.stack([np.eye(3)] * 3), synth.sphere_candidates(16))
    ctx.close()
    assert got["t_rel"].shape == (0, 3) and got["best"].shape == (0,)


def test_vote_with_one_candidate_returns_it():
    sc = synth.trajectory_scene(n_cams=20, n_pts=2000, target_matches=20_000, seed=13, name="one")
    pc = sc.pairs().astype(np.int32)
    F = synth.fundamental_matrices(sc, pc, noise=1e-2, seed=2)
    ctx = fastea.Context(0)
    got = ctx.focal_vote(sc.n_cams, pc, F, [640.0], 0.05, votes=True)
    ctx.close()
    ref_v, _ = oracle.focal_vote(pc, F, np.zeros(sc.n_cams, int), [0.0], [640.0], 0.05)
    assert got["f_best"][0] == 640.0 and got["k_best"][0] == 0
    assert got["votes"][0, 0] == pytest.approx(ref_v[0, 0], rel=1e-6)


def test_two_cameras_one_pair():
    """Rotation: the initialisation gives the second camera's rotation
    relative to the first exactly (up to the global gauge), and the
    optimisation keeps the loss near 0.  Alignment: the two aligned centres
    are opposite unit vectors along the target (to the final learning
    rate)."""
    R = synth.rotation_from_axis_angle(np.array([[0.3, -0.2, 1.0], [1.0, 0.5, -0.3]]), np.array([0.4, 1.1]))
    pc = np.array([[0, 1]], np.int32)
    Rrel = (R[1] @ R[0].T)[None]
    ctx = fastea.Context(0)
    v0 = np.random.default_rng(1).normal(size=(2, 2, 3))
    # the initialisation alone is exact (Adam's first step moves every
    # parameter by about lr even at the optimum)
    ra0 = ctx.rotation_averaging(2, pc, Rrel, v0=v0, options=fastea.ra_default_options(iters=0))
    np.testing.assert_allclose(ra0["R"][1] @ ra0["R"][0].T, Rrel[0], atol=1e-9)
    ra = ctx.rotation_averaging(2, pc, Rrel, v0=v0)
    assert ra["loss"] < 1e-3
    t = np.array([[0.6, 0.0, 0.8]])
    al = ctx.translation_align(pc, R, t, synth.random_centres(2, 2, 2))
    ctx.close()
    target = -R[1].T @ t[0]
    d = al["o"][1] - al["o"][0]
    np.testing.assert_allclose(d / np.linalg.norm(d), target, atol=1e-4)
    np.testing.assert_allclose(al["o"].sum(0), 0.0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(al["o"], axis=1), 1.0, atol=1e-12)
