"""Pins of the oracle's early exit (a batching addition: the paper runs a
fixed schedule of re-weighting rounds whose threshold decreases to a
minimum, Method > Epipolar Adjustment).  The rule: at the start of round
r >= 1 whose threshold equals round r-1's, the solve stops if the cameras'
mean rotation over round r-1 (geodesic distance between the round's
snapshot and the current rotation) is below converge_deg degrees and their
mean |log f| change below converge_deg pi/180.

The expected stopping round is computed here from a run without the exit:
its rotation log (one entry per round end) gives every round's mean
camera rotation, measured with numpy through the rotation angle of
R_a^T R_b from its eigen-decomposition's complex eigenvalues (not the trace
formula the oracle uses), and the threshold schedule gives the eligible
rounds.
"""
import numpy as np

from paper_2605_18052_amd import synth


def _schedule(opt):
    r = np.arange(opt.rounds)
    return np.maximum(opt.tau_px_init * opt.tau_decay ** r, opt.tau_px_min)


def _angle_deg(Ra, Rb):
    """Rotation angle of Ra^T Rb from the argument of its complex eigenvalue."""
    Q = np.einsum("nji,njk->nik", Ra, Rb)
    ev = np.linalg.eigvals(Q)
    return np.degrees(np.max(np.abs(np.angle(ev)), axis=1))


def _scene():
    return synth.sphere_scene(n_cams=8, n_pts=600, seed=21, name="conv")


def test_off_runs_every_round(orc):
    sc = _scene()
    pb = orc.OracleProblem.from_scene(sc)
    opt = orc.default_options(rounds=9, iters_per_round=10, gauge_normalize=0)
    out = orc.epipolar_adjust(pb, sc.R_init, sc.t_init, sc.f_init, options=opt)
    assert out["rounds_run"] == 9 and len(out["loss"]) == 9 and np.all(out["inliers"] >= 0)


def test_frozen_poses_stop_at_the_first_round_of_the_floor(orc):
    """With zero learning rates nothing moves, so the exit fires at the
    first round whose threshold repeats: 128 px halving to a 4 px floor
    gives thresholds 128, 64, 32, 16, 8, 4, 4, ... -- round 6."""
    sc = _scene()
    pb = orc.OracleProblem.from_scene(sc)
    opt = orc.default_options(rounds=12, iters_per_round=5, gauge_normalize=0, lr_rot=0.0, lr_t=0.0,
                              lr_logf=0.0, converge_deg=1e-9)
    tau = _schedule(opt)
    first = int(np.nonzero(tau[1:] == tau[:-1])[0][0]) + 1
    assert first == 6
    out = orc.epipolar_adjust(pb, sc.R_init, sc.t_init, sc.f_init, options=opt)
    assert out["rounds_run"] == first
    # a schedule that never repeats never exits
    opt2 = orc.default_options(rounds=5, iters_per_round=5, gauge_normalize=0, lr_rot=0.0, lr_t=0.0,
                               lr_logf=0.0, converge_deg=1e9)
    assert orc.epipolar_adjust(pb, sc.R_init, sc.t_init, sc.f_init, options=opt2)["rounds_run"] == 5


def test_stopping_round_from_the_logged_trajectory(orc):
    """The exit round equals the first eligible round whose previous round's
    mean rotation (from the no-exit run's log) is below the tolerance,
    for tolerances placed between the measured per-round figures; the poses
    at the exit equal the no-exit run's poses at that round's start."""
    sc = _scene()
    pb = orc.OracleProblem.from_scene(sc)
    K, rounds = 10, 16
    base = dict(rounds=rounds, iters_per_round=K, gauge_normalize=0, optimize_focal=0)
    ref = orc.epipolar_adjust(pb, sc.R_init, sc.t_init, sc.f_init, options=orc.default_options(**base),
                              log_every=K, max_log=rounds)
    R0 = np.stack([orc.rot6d_to_R(orc.R_to_rot6d(r)) for r in sc.R_init])
    ends = np.concatenate([R0[None], ref["log_R"]])  # ends[k] = rotations at the start of round k
    change = np.array([_angle_deg(ends[r - 1], ends[r]).mean() for r in range(1, rounds + 1)])
    # change[r-1]: mean rotation over round r-1, known at the start of round r
    tau = _schedule(orc.default_options(**base))
    eligible = [r for r in range(1, rounds) if tau[r] == tau[r - 1]]
    figures = np.sort(change[[r - 1 for r in eligible]])
    cuts = [np.sqrt(a * b) for a, b in zip(figures[:-1], figures[1:]) if b > 1.05 * a]
    assert len(cuts) >= 2
    for tol in cuts[:3] + [figures[-1] * 1.5]:
        want = next(r for r in eligible if change[r - 1] < tol)
        out = orc.epipolar_adjust(pb, sc.R_init, sc.t_init, sc.f_init,
                                  options=orc.default_options(converge_deg=float(tol), **base),
                                  log_every=K, max_log=rounds)
        assert out["rounds_run"] == want, (tol, want, out["rounds_run"])
        np.testing.assert_allclose(out["R"], ends[want], atol=1e-13)
        np.testing.assert_array_equal(out["inliers"], ref["inliers"][:want])


def test_focal_change_blocks_the_exit(orc):
    """A scene whose focal lengths still move by more than the tolerance
    per round does not exit even when its rotations have settled: with the
    rotation and translation learning rates at zero and a large focal one,
    the exit waits for the focal lengths."""
    sc = _scene()
    pb = orc.OracleProblem.from_scene(sc)
    opt = orc.default_options(rounds=12, iters_per_round=10, gauge_normalize=0, lr_rot=0.0, lr_t=0.0,
                              lr_logf=5e-2, lr_decay=1.0, converge_deg=1e-3)
    out = orc.epipolar_adjust(pb, sc.R_init, sc.t_init, sc.f_init * 1.3, options=opt)
    assert out["rounds_run"] > 6
    frozen = orc.default_options(rounds=12, iters_per_round=10, gauge_normalize=0, lr_rot=0.0, lr_t=0.0,
                                 lr_logf=0.0, converge_deg=1e-3)
    assert orc.epipolar_adjust(pb, sc.R_init, sc.t_init, sc.f_init * 1.3, options=frozen)["rounds_run"] == 6
