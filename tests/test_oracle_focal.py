"""Pins of the oracle's focal-length vote (Method > Focal Length
Estimation, Eq. fastmap-focal-vote): a 3x3 matrix is essential exactly when
its two non-zero singular values are equal, so at the true focal length
every pair's term is exp(0) = 1."""
import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import synth


@pytest.fixture(scope="module")
def shared_scene():
    """A 40-camera trajectory with one focal length (700 px) for all."""
    sc = synth.trajectory_scene(n_cams=40, n_pts=5000, target_matches=100_000, seed=7,
                                f_range=(700.0, 700.0), name="shared700")
    return sc, sc.pairs().astype(np.int32)


def test_true_focal_length_scores_one_per_pair_and_wins(shared_scene):
    sc, pc = shared_scene
    F = synth.fundamental_matrices(sc, pc)
    cand = np.sort(np.concatenate([synth.focal_candidates(300, 200, 3000), [700.0]]))
    votes, best = oracle.focal_vote(pc, F, np.zeros(sc.n_cams, int), [0.0], cand, 0.05)
    k = np.nonzero(cand == 700.0)[0][0]
    assert votes[0, k] == pytest.approx(len(pc), rel=1e-9)
    assert best[0] == 700.0
    others = np.delete(votes[0], k)
    assert others.max() < len(pc) - 1e-3


def test_votes_ignore_the_scale_and_sign_of_each_fundamental_matrix(shared_scene):
    sc, pc = shared_scene
    F = synth.fundamental_matrices(sc, pc, noise=1e-2, seed=3)
    s = np.random.default_rng(4).uniform(0.1, 10.0, len(pc)) * np.where(np.arange(len(pc)) % 2, -1, 1)
    cand = synth.focal_candidates(100, 300, 1500)
    v0, b0 = oracle.focal_vote(pc, F, np.zeros(sc.n_cams, int), [0.0], cand, 0.05)
    v1, b1 = oracle.focal_vote(pc, F * s[:, None, None], np.zeros(sc.n_cams, int), [0.0], cand, 0.05)
    np.testing.assert_allclose(v1, v0, rtol=1e-12)
    assert b1[0] == b0[0]


def test_per_camera_vote_finds_each_true_focal_length():
    """One group per camera, the other cameras at their true focal lengths:
    each camera's vote at its own true focal length equals its number of
    pairs, the maximum."""
    sc = synth.trajectory_scene(n_cams=30, n_pts=4000, target_matches=80_000, seed=8, name="percam")
    pc = sc.pairs().astype(np.int32)
    F = synth.fundamental_matrices(sc, pc)
    for c in (0, 7, 19):
        cand = np.sort(np.concatenate([synth.focal_candidates(120, 300, 1500), [sc.f_gt[c]]]))
        votes, best = oracle.focal_vote(pc, F, np.arange(sc.n_cams), sc.f_gt, cand, 0.05)
        deg = np.sum((pc[:, 0] == c) | (pc[:, 1] == c))
        assert best[c] == sc.f_gt[c]
        assert votes[c].max() == pytest.approx(deg, rel=1e-9)


def test_intersecting_optical_axes_leave_the_focal_length_open():
    """Cameras all looking at one point: a known degeneracy of focal length
    from the fundamental matrix (the optical axes intersect), so candidates
    other than the true one also make every pair's matrix essential."""
    sc = synth.sphere_scene(n_cams=12, n_pts=200, p_det=0.6, seed=5, focal=600.0, name="axes")
    pc = sc.pairs().astype(np.int32)
    F = synth.fundamental_matrices(sc, pc)
    cand = np.concatenate([synth.focal_candidates(200), [600.0]])
    votes, _ = oracle.focal_vote(pc, F, np.zeros(sc.n_cams, int), [0.0], cand, 0.05)
    full = np.abs(votes[0] - len(pc)) < 1e-6
    assert full[-1] and full[:-1].sum() >= 1
