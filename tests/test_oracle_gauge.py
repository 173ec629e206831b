"""Pins of the oracle's gauge normalisation (the similarity freedom of the
epipolar objective: Method > Epipolar Adjustment builds E from global poses
only, so a rotation, translation and positive scale of the whole scene leave
every residual unchanged; Global Translation fixes the same freedom by
centring and scaling the camera centres).

The oracle moves the camera centres o_i = -R_i^T t_i to mean 0 and scales
them so that the median distance between the centres of matched pairs is 1,
and epipolar_adjust maps its result back to the caller's frame.  Every check
below computes the expected value with numpy from the definition (mean,
median of pair distances, o = -R^T t), not with the oracle's own code, and
the hand-built cases separate the median from the mean, the scale from its
inverse and the shift from its opposite.
"""
import numpy as np

from paper_2605_18052_amd import synth


def _centres(R, t):
    return -np.einsum("nji,nj->ni", R, t)


def _t_of(R, o):
    return -np.einsum("nij,nj->ni", R, o)


def test_two_cameras_closed_form(orc):
    """Centres (0,0,0) and (2,0,0) with R = I: mean (1,0,0), one pair of
    length 2, so the new centres are (-1/2,0,0), (1/2,0,0) and t = -o'."""
    R = np.stack([np.eye(3), np.eye(3)])
    t = _t_of(R, np.array([[0.0, 0, 0], [2.0, 0, 0]]))
    t2, center, scale = orc.gauge_normalize(R, t, np.array([[0, 1]], np.int32))
    np.testing.assert_allclose(center, [1.0, 0.0, 0.0], atol=1e-15)
    assert scale == 2.0
    np.testing.assert_allclose(t2, [[0.5, 0, 0], [-0.5, 0, 0]], atol=1e-15)


def test_median_not_mean_of_pair_lengths(orc):
    """Four cameras on a line at 0, 1, 3, 13 with pairs of lengths 1, 2, 10:
    the median is 2 (the mean would be 13/3).  With a fourth pair of length
    3 the median of an even count is the mean of the middle two, 2.5."""
    rng = np.random.default_rng(0)
    R = synth.rotation_from_axis_angle(rng.normal(size=(4, 3)), rng.uniform(0.1, 3.0, 4))
    o = np.array([[0.0, 0, 0], [1.0, 0, 0], [3.0, 0, 0], [13.0, 0, 0]])
    t = _t_of(R, o)
    pc3 = np.array([[0, 1], [1, 2], [2, 3]], np.int32)
    _, center, scale = orc.gauge_normalize(R, t, pc3)
    np.testing.assert_allclose(center, [17.0 / 4, 0, 0], atol=1e-14)
    np.testing.assert_allclose(scale, 2.0, rtol=1e-14)
    pc4 = np.array([[0, 1], [1, 2], [2, 3], [0, 2]], np.int32)
    _, _, scale4 = orc.gauge_normalize(R, t, pc4)
    np.testing.assert_allclose(scale4, 2.5, rtol=1e-14)


def test_normalised_frame_properties(orc):
    """On a scene with random poses: the new centres (computed here as
    -R^T t) have mean 0, the median matched-pair distance is 1, the
    rotations are unchanged, and the returned centre and scale are the mean
    centre and the median pair distance of the input."""
    sc = synth.config1()
    pc = sc.pairs().astype(np.int32)
    R, t = sc.R_init, sc.t_init
    o = _centres(R, t)
    t2, center, scale = orc.gauge_normalize(R, t, pc)
    o2 = _centres(R, t2)
    np.testing.assert_allclose(o2.mean(0), 0.0, atol=1e-13)
    d2 = np.linalg.norm(o2[pc[:, 0]] - o2[pc[:, 1]], axis=1)
    np.testing.assert_allclose(np.median(d2), 1.0, rtol=1e-13)
    np.testing.assert_allclose(center, o.mean(0), rtol=1e-13, atol=1e-13)
    d = np.linalg.norm(o[pc[:, 0]] - o[pc[:, 1]], axis=1)
    np.testing.assert_allclose(scale, np.median(d), rtol=1e-13)
    # the map is o -> (o - center) / scale, camera by camera
    np.testing.assert_allclose(o2, (o - center) / scale, rtol=0, atol=1e-12)


def test_residuals_unchanged(orc):
    """A positive scale and a shift of all centres leave every epipolar
    residual exactly where it was (unit translation direction in E)."""
    sc = synth.tiny_scene(n_cams=6, n_pts=60, seed=21, sigma=1.0, outlier_frac=0.2)
    pb = orc.OracleProblem.from_scene(sc)
    pc = sc.pairs().astype(np.int32)
    R, t, f = sc.R_init, sc.t_init, sc.f_gt
    # move the scene far away and make it large, so that the normalisation
    # has a real shift and scale to undo
    t_far = 40.0 * t - np.einsum("nij,j->ni", R, np.array([300.0, -120.0, 55.0]))
    eps = orc.residuals(pb, R, t_far, f)
    t2, center, scale = orc.gauge_normalize(R, t_far, pc)
    assert scale > 10.0 and np.linalg.norm(center) > 100.0
    np.testing.assert_allclose(orc.residuals(pb, R, t2, f), eps, rtol=0, atol=1e-12)


def test_round_trip_to_callers_frame(orc):
    """Undoing the normalisation (o = scale * o' + center) returns the
    caller's translations; and a solve with no rounds, which normalises on
    entry and maps back on exit, returns its input poses."""
    sc = synth.tiny_scene(n_cams=5, n_pts=50, seed=22, sigma=1.0)
    pc = sc.pairs().astype(np.int32)
    R = sc.R_init
    t = 7.0 * sc.t_init + np.array([3.0, -2.0, 11.0])
    t2, center, scale = orc.gauge_normalize(R, t, pc)
    back = _t_of(R, scale * _centres(R, t2) + center)
    np.testing.assert_allclose(back, t, rtol=0, atol=1e-12 * np.abs(t).max())
    pb = orc.OracleProblem.from_scene(sc)
    out = orc.epipolar_adjust(pb, R, t, sc.f_init,
                              options=orc.default_options(rounds=0, gauge_normalize=1))
    np.testing.assert_allclose(out["t"], t, rtol=0, atol=1e-12 * np.abs(t).max())
    np.testing.assert_allclose(out["R"], R, rtol=0, atol=1e-14)
