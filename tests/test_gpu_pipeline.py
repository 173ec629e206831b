"""The stages before the adjustment and the adjustment itself, chained on
one scene: focal-length vote (Focal Length Estimation), global rotation
(Global Rotation), relative-translation search and camera-centre alignment
(Global Translation), then epipolar adjustment (Epipolar Adjustment), all
through the C-ABI.  The inputs the paper's earlier stages would supply
(fundamental matrices, relative rotations) are the true ones with noise."""
import numpy as np
import pytest

from paper_2605_18052_amd import fastea, metrics, synth

from gpu_helpers import make_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _aligned(o):
    o = o - o.mean(0)
    return o / np.linalg.norm(o, axis=1).mean()


def test_stages_chain_from_two_view_geometry_to_adjusted_poses():
    """60 cameras on a trajectory, each paired with its 30 nearest (a pair
    graph dense enough for random starts), 1 px noise and 20% outliers in the
    matches, focal lengths in [400, 1200] px known only to 10%."""
    sc = synth.trajectory_scene(n_cams=60, n_pts=6000, knn=30, target_matches=400_000, seed=12, name="pipe")
    N = sc.n_cams
    pc = sc.pairs().astype(np.int32)
    rng = np.random.default_rng(7)
    ctx = fastea.Context(0)
    # focal lengths: two per-camera sweeps of the vote from the initial ones
    F = synth.fundamental_matrices(sc, pc, noise=5e-3, seed=1)
    cand = synth.focal_candidates(1024, 200.0, 3000.0)
    f = sc.f_init.copy()
    for _ in range(2):
        f = ctx.focal_vote(N, pc, F, cand, 0.05, group=np.arange(N, dtype=np.int32), f_cur=f)["f_best"]
    f_err = np.abs(f / sc.f_gt - 1)
    # rotations from relative rotations with |N(0, 1 deg)| of noise
    Q = synth.rotation_from_axis_angle(rng.normal(size=(len(pc), 3)), np.deg2rad(1.0) * np.abs(rng.normal(size=len(pc))))
    Rrel = Q @ np.einsum("pab,pcb->pac", sc.R_gt[pc[:, 1]], sc.R_gt[pc[:, 0]])
    ra = ctx.rotation_averaging(N, pc, Rrel, v0=rng.normal(size=(2, N, 3)))
    R = ra["R"]
    ctx.close()
    # relative translations over the matches, then the centres
    ea = make_context(sc, gauge=1, f=f)
    _, _, pcm, _ = ea.get_segments()
    rt = ea.relative_translations(R, synth.sphere_candidates(4096).astype(np.float32).astype(np.float64),
                                  f=f, tau_px=32.0)
    al = ea.translation_align(pcm, R, rt["t_rel"], synth.random_centres(3, 2, N))
    t0 = -np.einsum("nab,nb->na", R, al["o"])
    # the adjustment from there
    ea.init_poses(R, t0)
    ea.epipolar_adjust()
    R1, t1, f1 = ea.get_poses()
    ea.close()
    e_rot = metrics.mean_rotation_error_deg(R, sc.R_gt)
    e_fin = metrics.mean_rotation_error_deg(R1, sc.R_gt)
    # centres compared after the rotation gauge of the global rotation stage
    c_true = -np.einsum("nba,nb->na", sc.R_gt, sc.t_gt)
    c_ta = al["o"]
    c_ea = -np.einsum("nba,nb->na", R1, t1)
    # align the estimated frames to the true one by the rotation that maps
    # the estimated rotations onto the true ones (R_est = R_true W)
    W = np.einsum("nba,nbc->ac", sc.R_gt, R)
    U, _, Vt = np.linalg.svd(W)
    W = U @ Vt
    ce_ta = np.median(np.linalg.norm(_aligned(c_ta @ W.T) - _aligned(c_true), axis=1))
    ce_ea = np.median(np.linalg.norm(_aligned(c_ea @ W.T) - _aligned(c_true), axis=1))
    print(f"pipeline: focal error median {np.median(f_err):.4f}; rotation {e_rot:.3f} deg after averaging, "
          f"{e_fin:.3f} after adjustment; centre error {ce_ta:.4f} after alignment, {ce_ea:.4f} after adjustment; "
          f"focal after adjustment {np.median(np.abs(f1 / sc.f_gt - 1)):.4f}", flush=True)
    assert np.median(f_err) < 0.03
    assert e_fin <= 1.0
    assert ce_ea < 0.05
