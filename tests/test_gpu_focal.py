"""GPU parity of the focal-length vote (Method > Focal Length Estimation,
Eq. fastmap-focal-vote) against the numpy oracle, through the C-ABI."""
import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import fastea, synth

from gpu_helpers import vote_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def check(got, ref_votes, ref_best, cand, tau, n_pairs):
    v = got["votes"]
    tol = vote_tol(ref_votes, tau, n_pairs)
    bad = np.abs(v - ref_votes) > tol
    assert not bad.any(), (np.argwhere(bad)[:5], np.abs(v - ref_votes)[bad][:5])
    srt = np.sort(ref_votes, axis=1)
    sep = srt[:, -1] - srt[:, -2] > 2 * vote_tol(srt[:, -1], tau, n_pairs)
    np.testing.assert_array_equal(got["f_best"][sep], ref_best[sep])
    kk = np.searchsorted(cand, got["f_best"]) if np.all(np.diff(cand) > 0) else None
    if kk is not None:
        chosen = ref_votes[np.arange(len(kk)), kk]
        assert np.all(chosen >= srt[:, -1] - 2 * vote_tol(srt[:, -1], tau, n_pairs))


@pytest.mark.parametrize("noise", [0.0, 1e-2])
def test_shared_focal_vote_matches_oracle(noise):
    sc = synth.trajectory_scene(n_cams=40, n_pts=5000, target_matches=100_000, seed=7,
                                f_range=(700.0, 700.0), name="shared700")
    pc = sc.pairs().astype(np.int32)
    F = synth.fundamental_matrices(sc, pc, noise=noise, seed=1)
    cand = np.sort(np.concatenate([synth.focal_candidates(600, 200, 3000), [700.0]]))
    ctx = fastea.Context(0)
    got = ctx.focal_vote(sc.n_cams, pc, F, cand, 0.05, votes=True)
    ctx.close()
    ref_v, ref_b = oracle.focal_vote(pc, F, np.zeros(sc.n_cams, int), [0.0], cand, 0.05)
    check(got, ref_v, ref_b, cand, 0.05, len(pc))
    if noise == 0.0:
        assert got["f_best"][0] == 700.0
        assert got["votes"][0].max() == pytest.approx(len(pc), rel=1e-6)
    else:
        assert abs(got["f_best"][0] / 700.0 - 1) < 0.01


def test_per_camera_vote_matches_oracle():
    """One group per camera, the others at their initial (10% off) focal
    lengths; 1% noise on the essential matrices; 400 candidates."""
    sc = synth.trajectory_scene(n_cams=60, n_pts=6000, target_matches=150_000, seed=9, name="percam60")
    pc = sc.pairs().astype(np.int32)
    F = synth.fundamental_matrices(sc, pc, noise=1e-2, seed=2)
    cand = synth.focal_candidates(400, 200, 3000)
    groups = np.arange(sc.n_cams, dtype=np.int32)
    ctx = fastea.Context(0)
    got = ctx.focal_vote(sc.n_cams, pc, F, cand, 0.05, group=groups, f_cur=sc.f_init, votes=True)
    ctx.close()
    ref_v, ref_b = oracle.focal_vote(pc, F, groups, sc.f_init, cand, 0.05)
    check(got, ref_v, ref_b, cand, 0.05, len(pc))
    print("per-camera vote: median f_best / f_true", float(np.median(got["f_best"] / sc.f_gt)), flush=True)


def test_mixed_groups_and_errors():
    """Three intrinsics groups with pairs inside and across groups, the true
    focal lengths among the candidates: each group's vote at its own true
    value is its pair count; invalid input is refused."""
    sc = synth.trajectory_scene(n_cams=30, n_pts=4000, target_matches=80_000, seed=11, name="groups")
    groups = (np.arange(sc.n_cams) % 3).astype(np.int32)
    f_true = np.array([500.0, 800.0, 1100.0])
    sc.f_gt = f_true[groups]
    pc = sc.pairs().astype(np.int32)
    F = synth.fundamental_matrices(sc, pc)
    cand = np.sort(np.concatenate([synth.focal_candidates(300, 200, 3000), f_true]))
    ctx = fastea.Context(0)
    got = ctx.focal_vote(sc.n_cams, pc, F, cand, 0.05, group=groups, f_cur=f_true, votes=True)
    ref_v, ref_b = oracle.focal_vote(pc, F, groups, f_true, cand, 0.05)
    check(got, ref_v, ref_b, cand, 0.05, len(pc))
    np.testing.assert_array_equal(got["f_best"], f_true)
    for g in range(3):
        deg = np.sum((groups[pc[:, 0]] == g) | (groups[pc[:, 1]] == g))
        assert got["votes"][g].max() == pytest.approx(deg, rel=1e-6)
    with pytest.raises(fastea.FeaError, match="tau"):
        ctx.focal_vote(sc.n_cams, pc, F, cand, 0.0)
    with pytest.raises(fastea.FeaError, match="f_cur"):
        ctx.focal_vote(sc.n_cams, pc, F, cand, 0.05, group=groups)
    with pytest.raises(fastea.FeaError, match="candidate"):
        ctx.focal_vote(sc.n_cams, pc, F, -cand, 0.05)
    with pytest.raises(fastea.FeaError, match="pair"):
        ctx.focal_vote(sc.n_cams, np.array([[1, 1]]), F[:1], cand, 0.05)
    ctx.close()
