"""GPU parity of the Global Translation stages against the FP64 oracle:
the relative-translation candidate search (matrix-core scoring, selection,
cheirality sign) and the camera-centre alignment with multiple random
initialisations, through the C-ABI."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import fastea, metrics, synth

from gpu_helpers import check_search, make_context, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def _cand32(k):
    """Candidates rounded to fp32 and given to both sides in that form."""
    return synth.sphere_candidates(k).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("K,tau_px", [(1, math.inf), (700, 32.0), (2048, math.inf), (3000, 32.0)])
def test_search_matches_oracle_several_items_per_pair(K, tau_px):
    """Six cameras, 20k points: pairs of ~4-8k matches span several
    2048-match work items with a ragged tail; 10% outliers, rotations 2-5
    degrees off; K = 1 (no choice), 700 (a ragged candidate group of 1024),
    2048 (two full groups) and 3000 (two full and a ragged one); the plain
    mean and the mean capped at 32 px (over the median focal length)."""
    sc = synth.sphere_scene(n_cams=6, n_pts=20000, p_det=0.5, sigma=0.5, outlier_frac=0.1, seed=31,
                            name="search6")
    cand = _cand32(K)
    ctx = make_context(sc)
    got = ctx.relative_translations(sc.R_init, cand, f=sc.f_gt, tau_px=tau_px, scores=True)
    _, _, pc, seg = ctx.get_segments()
    ctx.close()
    assert np.diff(seg).max() > 2 * 2048 and np.any(np.diff(seg) % 2048 != 0)
    ref = oracle.rel_trans(oracle_problem(sc), sc.R_init, sc.f_gt, cand, scores=True,
                           tau=tau_px / np.median(sc.f_gt))
    np.testing.assert_array_equal(ref["pair_cams"], pc)
    agree, _ = check_search(got, ref, K)
    print(f"K={K}, cap {tau_px} px: {len(pc)} pairs, choice agrees on {agree:.3f}", flush=True)


def test_search_sphere_scene_all_pairs():
    """The 20-camera, 190-pair scene (a few hundred matches per pair, one
    item each) with its initial rotations and 4096 candidates."""
    sc = synth.config1()
    cand = _cand32(4096)
    ctx = make_context(sc)
    got = ctx.relative_translations(sc.R_init, cand, scores=True, timing=True)
    ctx.close()
    assert got["score_ms"] > 0
    ref = oracle.rel_trans(oracle_problem(sc), sc.R_init, sc.f_init, cand, scores=True)
    check_search(got, ref, 4096)


def test_search_returns_the_true_direction_on_noiseless_matches():
    sc = synth.sphere_scene(n_cams=12, n_pts=600, p_det=0.7, sigma=0.0, outlier_frac=0.0, seed=11,
                            name="clean")
    ctx = make_context(sc)
    _, _, pc, seg = ctx.get_segments()
    gt = synth.relative_translations_gt(sc, pc)
    folded = np.where(gt[:, 2:3] >= 0, gt, -gt).astype(np.float32).astype(np.float64)
    cand = np.concatenate([_cand32(500), folded])
    got = ctx.relative_translations(sc.R_gt, cand, f=sc.f_gt)
    ctx.close()
    P = len(pc)
    np.testing.assert_array_equal(got["best"], 500 + np.arange(P))
    np.testing.assert_array_equal(got["vote"], np.diff(seg))
    np.testing.assert_allclose(got["t_rel"], gt, atol=2e-7)  # fp32 candidates


def test_search_rejects_bad_input():
    sc = synth.tiny_scene()
    ctx = fastea.Context(0)
    with pytest.raises(fastea.FeaError, match="load matches"):
        ctx.relative_translations(sc.R_gt, _cand32(8))
    ctx.close()
    ctx = make_context(sc)
    cand = _cand32(8)
    cand[3] *= 1.01
    with pytest.raises(fastea.FeaError, match="unit"):
        ctx.relative_translations(sc.R_gt, cand)
    cand = _cand32(8)
    cand[0, 0] = np.nan
    with pytest.raises(fastea.FeaError):
        ctx.relative_translations(sc.R_gt, cand)
    with pytest.raises(fastea.FeaError, match="focal"):
        ctx.relative_translations(sc.R_gt, _cand32(8), f=-sc.f_gt)
    with pytest.raises(fastea.FeaError, match="tau_px"):
        ctx.relative_translations(sc.R_gt, _cand32(8), tau_px=0.0)
    ctx.close()


# ---- camera centres ------------------------------------------------------------

def _object_graph(n, angle, seed):
    return synth.object_pair_graph(n, angle, seed)


def _aligned(o):
    o = o - o.mean(0)
    return o / np.linalg.norm(o, axis=1).mean()


def test_alignment_trajectory_matches_oracle():
    """Forty Adam steps of three runs from random centres with noisy (2 degree)
    relative translations, the merge, twenty final steps: every intermediate
    the oracle returns agrees to 1e-10.  Both sides are fp64; the library sums
    each camera's pair terms across a wave, multiplies by reciprocals where
    the oracle divides and keeps running products for the bias-correction and
    learning-rate powers (pow in the oracle): rounding-level differences."""
    pc, R, tij, c = _object_graph(120, 65.0, 3)
    rng = np.random.default_rng(4)
    tn = tij + np.deg2rad(2) * rng.normal(size=tij.shape) / np.sqrt(3)
    init = synth.random_centres(9, 3, len(c))
    kw = dict(iters_run=40, iters_final=20)
    ctx = fastea.Context(0)
    got = ctx.translation_align(pc, R, tn, init, fastea.ta_default_options(**kw), details=True)
    ctx.close()
    tg = oracle.ta_targets(len(c), pc, R, tn)
    ref = oracle.ta_solve(pc, tg, init, oracle.ta_default_options(**kw))
    np.testing.assert_allclose(got["run_o"], ref["run_o"], atol=1e-10)
    np.testing.assert_allclose(got["cam_loss"], ref["cam_loss"], atol=1e-10)
    np.testing.assert_allclose(got["run_loss"], ref["run_loss"], rtol=1e-10)
    srt = np.sort(ref["cam_loss"], axis=0)
    sep = srt[1] - srt[0] > 1e-8
    np.testing.assert_array_equal(got["run_of_cam"][sep], ref["run_of_cam"][sep])
    assert sep.mean() > 0.9
    if sep.all():
        np.testing.assert_allclose(got["o"], ref["o"], atol=1e-10)
    assert got["final_loss"] == pytest.approx(ref["final_loss"], rel=1e-9)


def test_alignment_merge_removes_outliers_like_the_oracle():
    """The full default schedule on 500 cameras with pairs within 60 degrees
    (~31k pairs): from this random start one run leaves a few cameras far off
    and two runs recover every centre, on the GPU as in the oracle; the
    results agree to 1e-6 (near convergence the L1 signs flip at rounding
    level, so the last steps differ at the scale of the final learning rate)."""
    pc, R, tij, c = _object_graph(500, 60.0, 0)
    init = synth.random_centres(7, 2, len(c))
    ctx = fastea.Context(0)
    one = ctx.translation_align(pc, R, tij, init[:1])
    two = ctx.translation_align(pc, R, tij, init)
    ctx.close()
    tg = oracle.ta_targets(len(c), pc, R, tij)
    ref1 = oracle.ta_solve(pc, tg, init[:1])
    ref2 = oracle.ta_solve(pc, tg, init)
    truth = _aligned(c)
    e1 = np.linalg.norm(one["o"] - truth, axis=1)
    r1 = np.linalg.norm(ref1["o"] - truth, axis=1)
    np.testing.assert_array_equal(e1 > 0.05, r1 > 0.05)
    assert 1 <= (e1 > 0.05).sum() <= 10
    assert np.linalg.norm(two["o"] - truth, axis=1).max() < 1e-5
    np.testing.assert_allclose(two["o"], ref2["o"], atol=1e-6)
    print(f"alignment: 1 run {(e1 > 0.05).sum()} outliers, 2 runs max error "
          f"{np.linalg.norm(two['o'] - truth, axis=1).max():.2e}, {two['ms']:.1f} ms", flush=True)


def test_alignment_edge_cases():
    """A camera without pairs keeps its aligned initial centre in the merge
    (all runs score 0 for it, run 0 wins); invalid input is refused."""
    pc, R, tij, c = _object_graph(30, 80.0, 5)
    N = len(c) + 1  # camera 30 has no pairs
    R = np.concatenate([R, np.eye(3)[None]])
    init = synth.random_centres(2, 2, N)
    ctx = fastea.Context(0)
    got = ctx.translation_align(pc, R, tij, init, fastea.ta_default_options(iters_final=0), details=True)
    assert got["run_of_cam"][N - 1] == 0
    assert np.all(got["cam_loss"][:, N - 1] == 0)
    tg = oracle.ta_targets(N, pc, R, tij)
    ref = oracle.ta_solve(pc, tg, init, oracle.ta_default_options(iters_final=0))
    np.testing.assert_allclose(got["o"][N - 1], ref["o"][N - 1], atol=1e-6)
    for bad, msg in ((dict(pair_cams=np.array([[0, 0]])), "pair"),
                     (dict(t_rel=np.zeros((1, 3))), "zero"),
                     (dict(o_init=np.zeros((65, N, 3))), "n_runs")):
        args = dict(pair_cams=pc[:1], R=R, t_rel=tij[:1], o_init=init)
        args.update(bad)
        with pytest.raises(fastea.FeaError, match=msg):
            ctx.translation_align(**args)
    with pytest.raises(fastea.FeaError, match="coincide"):
        ctx.translation_align(pc, R, tij, np.zeros((1, N, 3)), fastea.ta_default_options(iters_run=0))
    ctx.close()


def test_search_alignment_and_adjustment_compose():
    """The three stages on an object-centric capture (60 cameras, pairs
    within 70 degrees, 0.5 px noise, no outliers) from rotations 2-5 degrees
    off and no translations: candidate search, alignment with two random
    starts, then epipolar adjustment from those centres reaches <= 1 degree
    mean rotation error and recovers the centres.  The oracle runs the same
    three stages from the same scene, candidates and starts; the adjustment's
    fixed schedule leaves the centres short of their optimum by an amount that
    is the method's, not the library's (0.022 of the mean centre distance in
    the oracle's chain), so the library's centre error is bounded by the
    oracle's: the two chains part only where fp32 scoring breaks a near-tie
    between candidates differently."""
    sc = synth.sphere_scene(n_cams=60, n_pts=3000, p_det=0.35, sigma=0.5, outlier_frac=0.0, seed=41,
                            pair_angle_deg=70.0, name="object60")
    cand = _cand32(4096)
    starts = synth.random_centres(3, 2, sc.n_cams)
    ctx = make_context(sc, gauge=1)
    rt = ctx.relative_translations(sc.R_init, cand, tau_px=32.0)
    _, _, pc, _ = ctx.get_segments()
    al = ctx.translation_align(pc, sc.R_init, rt["t_rel"], starts)
    o = al["o"]
    t0 = -np.einsum("nab,nb->na", sc.R_init, o)
    ctx.init_poses(sc.R_init, t0)
    ctx.epipolar_adjust()
    R, t, _ = ctx.get_poses()
    ctx.close()
    err0 = metrics.mean_rotation_error_deg(sc.R_init, sc.R_gt)
    err1 = metrics.mean_rotation_error_deg(R, sc.R_gt)
    truth = _aligned(-np.einsum("nba,nb->na", sc.R_gt, sc.t_gt))
    c_ta = np.linalg.norm(o - truth, axis=1)
    c_ea = np.linalg.norm(_aligned(-np.einsum("nba,nb->na", R, t)) - truth, axis=1)
    # the oracle's chain
    pb = oracle_problem(sc)
    ort = oracle.rel_trans(pb, sc.R_init, sc.f_init, cand, tau=32.0 / np.median(sc.f_init))
    tg = oracle.ta_targets(sc.n_cams, ort["pair_cams"], sc.R_init, ort["t_rel"])
    oo = oracle.ta_solve(ort["pair_cams"], tg, starts)["o"]
    out = oracle.epipolar_adjust(pb, sc.R_init, -np.einsum("nab,nb->na", sc.R_init, oo), sc.f_init,
                                 options=oracle.default_options(gauge_normalize=1))
    c_ta_ref = np.linalg.norm(oo - truth, axis=1)
    c_ea_ref = np.linalg.norm(_aligned(-np.einsum("nba,nb->na", out["R"], out["t"])) - truth, axis=1)
    print(f"pipeline: rotation error {err0:.2f} -> {err1:.3f} deg (oracle "
          f"{metrics.mean_rotation_error_deg(out['R'], sc.R_gt):.3f}); median centre error after "
          f"alignment {np.median(c_ta):.4f} (oracle {np.median(c_ta_ref):.4f}), after adjustment "
          f"{np.median(c_ea):.4f} (oracle {np.median(c_ea_ref):.4f})", flush=True)
    assert err1 <= 1.0 < err0
    assert np.median(c_ea) < np.median(c_ta)
    assert np.median(c_ea) <= 1.1 * np.median(c_ea_ref)
