"""Parity at the benchmark's own size: the ~20M-match, 500-camera trajectory
scene in its first IRLS round at the default threshold, the per-match kernel
in the tile the autotuner picks and in each fixed tile, every camera's
gradient against the FP64 oracle evaluated over all matches."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import fastea, synth

from gpu_helpers import check_search, make_context, per_camera_close, vote_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bench_scene():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sc = synth.config2()
    rng = np.random.default_rng(21)
    dR = synth.rotation_from_axis_angle(rng.normal(size=(sc.n_cams, 3)), np.deg2rad(0.5) * np.ones(sc.n_cams))
    R = dR @ sc.R_init
    t = sc.t_init + rng.normal(scale=0.01, size=sc.t_init.shape)
    f = sc.f_init * np.exp(rng.uniform(-0.01, 0.01, sc.n_cams))
    pb = oracle.OracleProblem.from_scene(sc)
    tau = fastea.default_options().tau_px_init / np.median(sc.f_init)
    mask, Z = oracle.update_mask(pb, sc.R_init, sc.t_init, sc.f_init, tau, np.ones(sc.n_matches, bool))
    eps = np.abs(oracle.residuals(pb, sc.R_init, sc.t_init, sc.f_init))
    print(f"bench scene: {sc.n_matches} matches, {Z} retained at tau {tau:.4g}", flush=True)
    return sc, pb, (R, t, f), tau, mask, Z, eps


@pytest.mark.parametrize("tile,persistent", [(0, 0), (1024, 0), (2048, 0), (4096, 0), (8192, 0), (1024, 1),
                                             (2048, 1), (4096, 1)])
def test_bench_workload_gradient_vs_oracle(bench_scene, tile, persistent):
    sc, pb, (R, t, f), tau, mask_ref, Z_ref, eps = bench_scene
    opt = fastea.default_options()
    ctx = make_context(sc, gauge=0, tile_matches=tile, tile_persistent=persistent)
    ctx.init_poses(sc.R_init, sc.t_init)
    ctx.begin_round(opt.tau_px_init)
    info = ctx.info()
    assert tile == 0 or (info["tile_matches"] == tile and info["tile_persistent"] == persistent)
    ctx.set_poses(R, t, f)
    loss, gR, gt, gf = ctx.residual_grad()
    mask, Z = ctx.get_mask()
    ctx.close()
    # the retained set: identical except within rounding of the threshold
    diff = np.flatnonzero(mask != mask_ref)
    assert np.all(np.abs(eps[diff] - tau) <= 1e-9 * tau), diff[:10]
    assert Z == int(mask.sum())
    # both sides with the same retained set and Z
    lr, gRr, gtr, gfr = (oracle.loss_grad(pb, R, t, f, sc.R_init, sc.t_init, sc.f_init, mask, delta=opt.delta)
                         if len(diff) else bench_scene_ref(bench_scene, opt.delta))
    l = float(loss.item())
    assert abs(l - lr) <= 1e-5 * abs(lr), (l, lr)
    for a, b in ((gR.cpu().numpy(), gRr), (gt.cpu().numpy(), gtr), (gf.cpu().numpy()[:, None], gfr[:, None])):
        ok, worst = per_camera_close(a, b)
        assert ok, (info["tile_matches"], worst)


_REF = {}


def bench_scene_ref(bench_scene, delta):
    """The oracle's loss and gradient with its own retained set (computed once)."""
    if "ref" not in _REF:
        sc, pb, (R, t, f), tau, mask_ref, Z_ref, eps = bench_scene
        _REF["ref"] = oracle.loss_grad(pb, R, t, f, sc.R_init, sc.t_init, sc.f_init, mask_ref, delta=delta)
    return _REF["ref"]


def test_bench_workload_quadratic_form_vs_oracle(bench_scene):
    """The quadratic-form inner loop on the same scene and round (the forms
    built once per round by one wavefront per 8192-match item): every
    camera's gradient against the FP64 oracle's per-match sum."""
    sc, pb, (R, t, f), tau, mask_ref, Z_ref, eps = bench_scene
    opt = fastea.default_options()
    ctx = make_context(sc, gauge=0, inner_loop=1)
    ctx.init_poses(sc.R_init, sc.t_init)
    ctx.begin_round(opt.tau_px_init)
    assert ctx.info()["tile_matches"] == 8192
    ctx.set_poses(R, t, f)
    loss, gR, gt, gf = ctx.residual_grad()
    mask, Z = ctx.get_mask()
    ctx.close()
    diff = np.flatnonzero(mask != mask_ref)
    assert np.all(np.abs(eps[diff] - tau) <= 1e-9 * tau), diff[:10]
    lr, gRr, gtr, gfr = (oracle.loss_grad(pb, R, t, f, sc.R_init, sc.t_init, sc.f_init, mask, delta=opt.delta)
                         if len(diff) else bench_scene_ref(bench_scene, opt.delta))
    l = float(loss.item())
    assert abs(l - lr) <= 1e-5 * abs(lr), (l, lr)
    for a, b in ((gR.cpu().numpy(), gRr), (gt.cpu().numpy(), gtr), (gf.cpu().numpy()[:, None], gfr[:, None])):
        ok, worst = per_camera_close(a, b)
        assert ok, worst


def test_bench_workload_learned_weights_vs_oracle(bench_scene):
    """The shipped inlier network on the 20M-match scene after three round
    snapshots: the weights of 100,000 sampled matches against the FP64
    network on the oracle's features, to 1e-2 absolute (the bound for the
    reduced-precision mode).  The arithmetic: the features enter as fp16
    hi + lo parts (about 2^-22 relative), the weights and the two hidden
    layers' activations are fp16 rounded to nearest (2^-12 relative) in
    64-term dot products; on this network that puts at most ~0.02 on the
    logit and a quarter of it on the weight (an fp64 emulation of exactly
    these roundings gives 4.9e-3 at most over 200,000 feature vectors), and
    the fp16 storage of the weight adds at most 2.5e-4."""
    from paper_2605_18052_amd import learned
    sc = bench_scene[0]
    params = learned.load_weights()
    rng = np.random.default_rng(23)
    snaps = []
    for k, deg in enumerate((0.0, 0.5, 1.0)):
        Rk = synth.rotation_from_axis_angle(rng.normal(size=(sc.n_cams, 3)),
                                            np.deg2rad(deg) * np.ones(sc.n_cams)) @ sc.R_init
        snaps.append((Rk, sc.t_init + 0.01 * k, sc.f_init))
    ctx = make_context(sc, gauge=0, weight_mode=1)
    ctx.set_mlp(params.astype(np.float32))
    ctx.init_poses(snaps[0][0], snaps[0][1])
    ctx.begin_round(math.inf)
    for Rk, tk, fk in snaps[1:]:
        ctx.set_poses(Rk, tk, fk)
        ctx.begin_round(math.inf)
    w = ctx.learned_weights()
    ctx.close()
    sel = np.sort(rng.choice(sc.n_matches, size=100_000, replace=False))
    feat = oracle.mlp_features(oracle.OracleProblem.from_scene(sc, sel), [snaps[2], snaps[1], snaps[0]])
    ref = oracle.mlp_forward(feat, params.astype(np.float32).astype(np.float64))
    err = np.abs(w[sel] - ref)
    print(f"learned weights at full size: max |err| {err.max():.3g}, mean {err.mean():.3g}", flush=True)
    assert err.max() < 1e-2 and err.mean() < 1e-3, (err.max(), err.mean())
    assert ref.std() > 0.05


def test_bench_workload_relative_translations_vs_oracle(bench_scene):
    """The relative-translation search in bench.py's configuration (the
    20M-match scene, true rotations and focal lengths, 2,048 candidates, the
    32 px cap, 2,048-match work items) against the FP64 oracle on 16 sampled
    pairs: scores within the fp32 bound, the choice where separated, vote
    and signed direction where the choice agrees."""
    sc = bench_scene[0]
    cand = synth.sphere_candidates(2048).astype(np.float32).astype(np.float64)
    ctx = make_context(sc)
    got = ctx.relative_translations(sc.R_gt, cand, f=sc.f_gt, tau_px=32.0, scores=True)
    _, _, pc, _ = ctx.get_segments()
    ctx.close()
    pick = np.sort(np.random.default_rng(31).choice(len(pc), 16, replace=False))
    i = np.minimum(sc.cam1, sc.cam2).astype(np.int64)
    j = np.maximum(sc.cam1, sc.cam2).astype(np.int64)
    sel = np.nonzero(np.isin(i * sc.n_cams + j, pc[pick, 0].astype(np.int64) * sc.n_cams + pc[pick, 1]))[0]
    ref = oracle.rel_trans(oracle.OracleProblem.from_scene(sc, sel), sc.R_gt, sc.f_gt, cand, scores=True,
                           tau=32.0 / np.median(sc.f_gt))
    np.testing.assert_array_equal(ref["pair_cams"], pc[pick])
    sub = {k: got[k][pick] for k in ("scores", "best", "vote", "t_rel", "score_best")}
    agree, _ = check_search(sub, ref, 2048)
    print(f"search at full size: choice agrees on {agree:.3f} of 16 sampled pairs", flush=True)


def test_bench_workload_focal_vote_vs_oracle(bench_scene):
    """The focal vote in bench.py's configuration (one group per camera of the
    20M-match scene, the others at their initial focal lengths, 1% noise on
    the essential matrices, 1,024 candidates) against the oracle on 25
    sampled cameras (all of their pairs)."""
    sc = bench_scene[0]
    pc = sc.pairs().astype(np.int32)
    F = synth.fundamental_matrices(sc, pc, noise=1e-2, seed=1)
    cand = synth.focal_candidates(1024, 200.0, 3000.0)
    groups = np.arange(sc.n_cams, dtype=np.int32)
    ctx = fastea.Context(0)
    got = ctx.focal_vote(sc.n_cams, pc, F, cand, 0.05, group=groups, f_cur=sc.f_init, votes=True)
    ctx.close()
    cams = np.sort(np.random.default_rng(32).choice(sc.n_cams, 25, replace=False))
    keep = np.isin(pc[:, 0], cams) | np.isin(pc[:, 1], cams)
    ref_v, _ = oracle.focal_vote(pc[keep], F[keep], groups, sc.f_init, cand, 0.05)
    v = got["votes"][cams]
    r = ref_v[cams]
    assert np.all(np.abs(v - r) <= vote_tol(r, 0.05, len(pc)))
    srt = np.sort(r, axis=1)
    sep = srt[:, -1] - srt[:, -2] > 2 * vote_tol(srt[:, -1], 0.05, len(pc))
    np.testing.assert_array_equal(got["f_best"][cams][sep], cand[np.argmax(r, axis=1)][sep])


def test_bench_workload_rotation_steps_vs_oracle(bench_scene):
    """Global rotation on bench.py's pair graph and noise (500 cameras, 5,181
    pairs, |N(0, 2 deg)| per pair): twenty Adam steps from the oracle's
    initialisation, the same rotations to 1e-9."""
    sc = bench_scene[0]
    pc = sc.pairs().astype(np.int32)
    rng = np.random.default_rng(3)
    Q = synth.rotation_from_axis_angle(rng.normal(size=(len(pc), 3)),
                                       np.deg2rad(2.0) * np.abs(rng.normal(size=len(pc))))
    Rrel = Q @ np.einsum("pab,pcb->pac", sc.R_gt[pc[:, 1]], sc.R_gt[pc[:, 0]])
    a6, _ = oracle.ra_init(pc, Rrel, sc.n_cams)
    ctx = fastea.Context(0)
    got = ctx.rotation_averaging(sc.n_cams, pc, Rrel, a6_init=a6, options=fastea.ra_default_options(iters=20))
    ctx.close()
    _, Rref, Lref = oracle.ra_solve(pc, Rrel, a6, iters=20)
    np.testing.assert_allclose(got["R"], Rref, atol=1e-9)
    assert got["loss"] == pytest.approx(Lref, rel=1e-9)
