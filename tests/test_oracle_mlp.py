"""Pins of the FP64 oracle's learned-weight MLP and its features."""
import math

import numpy as np
import pytest

from paper_2605_18052_amd import synth


def _rand_params(orc, rng, scale=0.3):
    return rng.normal(scale=scale, size=orc.MLP_NPARAM)


def test_zero_network_closed_form(orc):
    """All-zero weights: y = sigmoid(b3); BCE with b3 = 0 is log 2 and only
    b3 has a gradient, equal to mean(0.5 - t)."""
    rng = np.random.default_rng(0)
    x = rng.normal(size=(50, 8))
    t = rng.random(50)
    p = np.zeros(orc.MLP_NPARAM)
    np.testing.assert_allclose(orc.mlp_forward(x, p), 0.5, rtol=0, atol=0)
    loss, g = orc.mlp_bce_grad(x, t, p)
    assert abs(loss - math.log(2.0)) < 1e-15
    np.testing.assert_allclose(g[:-1], 0.0, atol=0)
    assert abs(g[-1] - np.mean(0.5 - t)) < 1e-15
    p[-1] = 1.7
    np.testing.assert_allclose(orc.mlp_forward(x, p), 1 / (1 + math.exp(-1.7)), rtol=1e-15)


def test_hand_built_network(orc):
    """y = sigmoid(2 relu(x0) - 1): one path through each layer."""
    W1 = np.zeros((64, 8))
    W1[0, 0] = 1.0
    W2 = np.zeros((64, 64))
    W2[0, 0] = 1.0
    w3 = np.zeros(64)
    w3[0] = 2.0
    p = orc.mlp_pack(W1, np.zeros(64), W2, np.zeros(64), w3, [-1.0])
    x = np.zeros((3, 8))
    x[:, 0] = [0.5, -1.0, 2.0]
    # sigmoid(0) = 0.5; sigmoid(-1) (ReLU clips); sigmoid(3)
    np.testing.assert_allclose(orc.mlp_forward(x, p),
                               [0.5, 0.2689414213699951, 0.9525741268224334], rtol=1e-15)


def test_bce_gradient_finite_differences(orc):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(40, 8))
    t = (rng.random(40) < 0.6).astype(float)
    p = _rand_params(orc, rng)
    loss, g = orc.mlp_bce_grad(x, t, p)
    bounds = np.cumsum([0, 512, 64, 4096, 64, 64, 1])
    picks = np.concatenate([rng.choice(np.arange(a, b), size=min(12, b - a), replace=False)
                            for a, b in zip(bounds[:-1], bounds[1:])])
    for k in picks:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (orc.mlp_bce_grad(x, t, pp)[0] - orc.mlp_bce_grad(x, t, pm)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_bce_is_stable_for_large_logits(orc):
    W1 = np.zeros((64, 8))
    p = orc.mlp_pack(W1, np.zeros(64), np.zeros((64, 64)), np.zeros(64), np.zeros(64), [800.0])
    loss, g = orc.mlp_bce_grad(np.zeros((2, 8)), np.array([0.0, 1.0]), p)
    assert math.isfinite(loss) and abs(loss - 400.0) < 1e-9  # (800 + 0)/2
    assert np.all(np.isfinite(g))


def test_features_special_cases(orc):
    sc = synth.tiny_scene(n_cams=5, n_pts=60, seed=3)
    pb = orc.OracleProblem.from_scene(sc)
    snaps = [(sc.R_gt, sc.t_gt, sc.f_gt)] * 3
    feat = orc.mlp_features(pb, snaps)
    # zero residual at ground truth up to the float32 rounding of keypoints
    # (|eps| < 5e-7, i.e. < 3e-4 px, and g(e) <= e_px / log(257))
    assert np.abs(feat[:, :3]).max() < 6e-5
    assert np.all(np.abs(feat[:, 3:7]) <= 1.0)
    # away from truth the residual features are positive and ordered by round
    feat2 = orc.mlp_features(pb, [(sc.R_init, sc.t_init, sc.f_gt), (sc.R_gt, sc.t_gt, sc.f_gt),
                                   (sc.R_gt, sc.t_gt, sc.f_gt)])
    assert feat2[:, 0].max() > 0.1 and np.abs(feat2[:, 1:3]).max() < 6e-5
    # 256 px of epipolar error maps to 1: a residual of 256/fbar
    # keypoint coordinates: centre -> 0, corners -> -1 / +1
    R = np.stack([np.eye(3), np.eye(3)])
    t = np.array([[0.0, 0, 0], [-1.0, 0, 0]])
    f = np.array([500.0, 500.0])
    x1 = np.array([320.0, 0.0, 640.0])
    y1 = np.array([240.0, 0.0, 480.0])
    q = orc.OracleProblem(x1, y1, x1, y1, np.zeros(3, np.int32), np.ones(3, np.int32),
                          [320.0, 320.0], [240.0, 240.0])
    ft = orc.mlp_features(q, [(R, t, f)] * 3)
    np.testing.assert_allclose(ft[:, 3:7], [[0, 0, 0, 0], [-1, -1, -1, -1], [1, 1, 1, 1]], atol=0)
    assert np.all(ft[:, 7] == 0.0)  # parallel optical axes
    # each keypoint is scaled by its own camera's image size
    q3 = orc.OracleProblem([320.0], [240.0], [640.0], [480.0], np.zeros(1, np.int32),
                           np.ones(1, np.int32), [320.0, 640.0], [240.0, 480.0])
    np.testing.assert_allclose(orc.mlp_features(q3, [(R, t, f)] * 3)[0, 3:7], 0.0, atol=0)
    q4 = orc.OracleProblem([640.0], [480.0], [640.0], [480.0], np.ones(1, np.int32),
                           np.zeros(1, np.int32), [320.0, 640.0], [240.0, 480.0])
    # a match given as (camera 1, camera 0) is read in the pair's orientation:
    # the keypoint in camera 0 (640, 480 -> 1, 1) comes first
    np.testing.assert_allclose(orc.mlp_features(q4, [(R, t, f)] * 3)[0, 3:7], [1, 1, 0, 0], atol=0)
    # rectified stereo with y2 - y1 = 256 px at f = 500: g = 1 exactly
    q2 = orc.OracleProblem([100.0], [100.0], [80.0], [356.0], np.zeros(1, np.int32),
                           np.ones(1, np.int32), [320.0, 320.0], [240.0, 240.0])
    assert abs(orc.mlp_features(q2, [(R, t, f)] * 3)[0, 0] - 1.0) < 1e-12
    # perpendicular optical axes -> 1
    Ry = synth.rotation_from_axis_angle(np.array([[0.0, 1.0, 0.0]]), np.array([np.pi / 2]))[0]
    R2 = np.stack([np.eye(3), Ry])
    assert abs(orc.mlp_features(q2, [(R2, t, f)] * 3)[0, 7] - 1.0) < 1e-12


def test_features_invariant_to_match_orientation(orc):
    """Swapping a match's cameras and keypoints leaves all 8 features (and the
    residual) unchanged."""
    sc = synth.tiny_scene(n_cams=6, n_pts=80, seed=7, sigma=1.0, outlier_frac=0.2)
    pb = orc.OracleProblem.from_scene(sc)
    rng = np.random.default_rng(2)
    flip = rng.random(sc.n_matches) < 0.5
    sw = lambda a, b: np.where(flip, b, a)
    pb2 = orc.OracleProblem(sw(sc.x1, sc.x2), sw(sc.y1, sc.y2), sw(sc.x2, sc.x1), sw(sc.y2, sc.y1),
                            sw(sc.cam1, sc.cam2).astype(np.int32),
                            sw(sc.cam2, sc.cam1).astype(np.int32), sc.cx, sc.cy)
    snaps = [(sc.R_init, sc.t_init, sc.f_init), (sc.R_gt, sc.t_gt, sc.f_gt),
             (sc.R_init, sc.t_gt, sc.f_gt)]
    a = orc.mlp_features(pb, snaps)
    b = orc.mlp_features(pb2, snaps)
    assert flip.any() and (~flip).any()
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)
