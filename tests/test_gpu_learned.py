"""Learned-weight row: MLP features and MFMA inference, training kernels and
the judge, against the FP64 oracle.  Snapshots are built by the test with
fea_set_poses, so no oracle input comes from the GPU path."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import fastea, metrics, synth

from gpu_helpers import make_context, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def _rand_mlp(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    W1 = rng.normal(scale=scale, size=(64, 8))
    b1 = rng.normal(scale=0.1, size=64)
    W2 = rng.normal(scale=scale / 4, size=(64, 64))
    b2 = rng.normal(scale=0.1, size=64)
    w3 = rng.normal(scale=scale, size=64)
    return oracle.mlp_pack(W1, b1, W2, b2, w3, [0.2])


def _three_snapshots(sc):
    rng = np.random.default_rng(9)
    snaps = []
    for k, deg in enumerate((0.0, 0.7, 1.5)):
        R = synth.rotation_from_axis_angle(rng.normal(size=(sc.n_cams, 3)),
                                           np.deg2rad(deg) * np.ones(sc.n_cams)) @ sc.R_init
        snaps.append((R, sc.t_init + 0.01 * k, sc.f_init))
    return snaps  # oldest first


def _ctx_with_history(sc, params, weight_mode=1):
    snaps = _three_snapshots(sc)
    ctx = make_context(sc, gauge=0, weight_mode=weight_mode, tile_matches=2048)
    ctx.set_mlp(params.astype(np.float32))
    ctx.init_poses(snaps[0][0], snaps[0][1])
    ctx.begin_round(math.inf)
    for R, t, f in snaps[1:]:
        ctx.set_poses(R, t, f)
        ctx.begin_round(math.inf)
    return ctx, snaps


def test_features_match_oracle():
    sc = synth.config1()
    params = _rand_mlp(1)
    ctx, snaps = _ctx_with_history(sc, params)
    feat, pos = ctx.mlp_features()
    perm, _, _, _ = ctx.get_segments()
    feat = feat.cpu().numpy()
    pos = pos.cpu().numpy()
    ctx.close()
    ok = pos >= 0
    order = perm[pos[ok]]
    ref = oracle.mlp_features(oracle_problem(sc), [snaps[2], snaps[1], snaps[0]])[order]
    got = feat[ok]
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6)


def test_mfma_inference_matches_oracle():
    """fp16 activations on the matrix cores vs the FP64 network: the weight
    agrees to 1e-2."""
    sc = synth.config1()
    params = _rand_mlp(2)
    ctx, snaps = _ctx_with_history(sc, params)
    w = ctx.learned_weights()
    ctx.close()
    feat = oracle.mlp_features(oracle_problem(sc), [snaps[2], snaps[1], snaps[0]])
    ref = oracle.mlp_forward(feat, params.astype(np.float32).astype(np.float64))
    err = np.abs(w - ref)
    print(f"learned weight vs FP64 network: max |err| {err.max():.3g}, mean {err.mean():.3g}, "
          f"max rel {(err / np.maximum(ref, 1e-3)).max():.3g}", flush=True)
    # the features enter as fp16 hi + lo parts (about 22 significand bits);
    # weights and hidden activations keep fp16's 11 (rounded to nearest), a
    # few times that on the logit, at most 1/4 of it on the sigmoid, plus
    # the fp16 storage of the weight (<= 2.5e-4); the weight lies in [0, 1],
    # so the bound is absolute
    assert err.max() < 1e-2 and err.mean() < 2.5e-3, (err.max(), err.mean())
    assert ref.std() > 0.05  # the network is not constant on these inputs


def test_set_mlp_rejects_weights_beyond_fp16():
    """Inference takes W1, W2 and w3 as fp16: a weight above 65504 would turn
    infinite there, so the call refuses it; the fp32 biases may be larger."""
    sc = synth.config1()
    ctx = make_context(sc, gauge=0, weight_mode=1)
    try:
        base = _rand_mlp(7).astype(np.float32)
        for off in (3, 576 + 100, 4736 + 5):  # one entry of W1, W2, w3
            p = base.copy()
            p[off] = 7e4
            with pytest.raises(fastea.FeaError, match="fp16"):
                ctx.set_mlp(p)
        p = base.copy()
        p[512] = 7e4  # b1
        p[4800] = -7e4  # b3
        p[576 + 7] = 65504.0  # the largest finite fp16 is accepted
        ctx.set_mlp(p)
    finally:
        ctx.close()


def test_training_gradient_matches_oracle():
    import torch
    rng = np.random.default_rng(4)
    n = 5000
    x = rng.normal(size=(n, 8)).astype(np.float32)
    t = (rng.random(n) < 0.7).astype(np.float32)
    p = _rand_mlp(3).astype(np.float32)
    loss, g = fastea.mlp_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(),
                              torch.from_numpy(p).cuda())
    lref, gref = oracle.mlp_bce_grad(x.astype(np.float64), t.astype(np.float64),
                                     p.astype(np.float64))
    assert abs(loss - lref) <= 1e-5 * lref
    g = g.cpu().numpy().astype(np.float64)
    bounds = np.cumsum([0, 512, 64, 4096, 64, 64, 1])
    for a, b in zip(bounds[:-1], bounds[1:]):
        assert np.linalg.norm(g[a:b] - gref[a:b]) <= 1e-5 * np.linalg.norm(gref[a:b]) + 1e-12, (a, b)


def test_training_reduces_loss():
    import torch
    rng = np.random.default_rng(5)
    n = 60000
    x = rng.normal(size=(n, 8)).astype(np.float32)
    t = ((x[:, 0] + 0.5 * x[:, 3] > 0.2) ^ (x[:, 7] > 1.5)).astype(np.float32)
    p = torch.from_numpy(_rand_mlp(6, scale=0.3).astype(np.float32)).cuda()
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    l0, _ = fastea.mlp_grad(xd, td, p)
    losses = fastea.mlp_train(xd, td, p, epochs=6, batch=4096, lr=3e-3, seed=1)
    l1, _ = fastea.mlp_grad(xd, td, p)
    assert np.all(np.isfinite(losses)) and l1 < 0.5 * l0 and l1 < 0.2, (l0, losses, l1)
    # the trained network, run through the oracle, classifies the data
    y = oracle.mlp_forward(x.astype(np.float64), p.cpu().numpy().astype(np.float64))
    assert np.mean((y > 0.5) == (t > 0.5)) > 0.93


def _inverted_mlp():
    """Weight ~1 for large residuals, ~0 for small ones: the opposite of an
    inlier detector."""
    W1 = np.zeros((64, 8))
    W1[0, 0] = 1.0
    W2 = np.zeros((64, 64))
    W2[0, 0] = 1.0
    w3 = np.zeros(64)
    w3[0] = 60.0
    return oracle.mlp_pack(W1, np.zeros(64), W2, np.zeros(64), w3, [-6.0])


def _inlier_mlp():
    """A soft inlier detector on the current snapshot's residual feature g:
    logit 5 - 8 g, i.e. weight 0.98 at 1 px, 0.5 at 32 px, 0.12 at 128 px."""
    W1 = np.zeros((64, 8))
    W1[0, 0] = 1.0
    W2 = np.zeros((64, 64))
    W2[0, 0] = 1.0
    w3 = np.zeros(64)
    w3[0] = -8.0
    return oracle.mlp_pack(W1, np.zeros(64), W2, np.zeros(64), w3, [5.0])


def test_judge_falls_back_on_a_harmful_network():
    sc = synth.config1()
    res = {}
    for name, p in (("inverted", _inverted_mlp()), ("inlier", _inlier_mlp())):
        ctx = make_context(sc, gauge=1, weight_mode=1)
        ctx.set_mlp(p.astype(np.float32))
        ctx.init_poses(sc.R_init, sc.t_init)
        rep = ctx.epipolar_adjust()
        R, _, _ = ctx.get_poses()
        res[name] = (rep["fallbacks"], metrics.mean_rotation_error_deg(R, sc.R_gt),
                     ctx.scene_stats()["learned"][0])
        ctx.close()
    assert res["inverted"][0] >= 1 and res["inverted"][2] == 0
    assert res["inverted"][1] < 1.0  # the plain fallback still converges
    assert res["inlier"][1] < 1.0


@pytest.mark.parametrize("inner_loop", [0, 1])
def test_judge_losses_against_the_oracle(inner_loop):
    """The two plain objectives the judge compares after a learned round come
    from one pass over the matches: the objective at the round's end, and at
    its snapshot from the same pass's snapshot residuals.  Both against the
    FP64 oracle's loss with that round's plain weights (the threshold filter
    at the snapshot, 1/Z over the retained matches) at the snapshot and at
    the poses the round ended with."""
    sc = synth.config1()
    o = fastea.default_options()
    ctx = make_context(sc, weight_mode=1, inner_loop=inner_loop, rounds=1, iters_per_round=30)
    ctx.set_mlp(_inlier_mlp().astype(np.float32))
    ctx.init_poses(sc.R_init, sc.t_init)
    R0, t0, f0 = ctx.get_poses()
    l0, l1 = ctx.judge_losses()
    assert not l0.any() and not l1.any()  # no learned round yet
    ctx.epipolar_adjust()
    l0, l1 = ctx.judge_losses()
    assert ctx.scene_stats()["learned"][0] == 1  # kept: the poses are the round's end
    R1, t1, f1 = ctx.get_poses()
    ctx.close()
    pb = oracle_problem(sc)
    mask, _ = oracle.update_mask(pb, R0, t0, f0, o.tau_px_init / np.median(f0), np.ones(sc.n_matches, bool))
    ref0 = oracle.loss_grad(pb, R0, t0, f0, R0, t0, f0, mask, delta=o.delta)[0]
    ref1 = oracle.loss_grad(pb, R1, t1, f1, R0, t0, f0, mask, delta=o.delta)[0]
    assert abs(l0[0] - ref0) <= 1e-5 * abs(ref0), (l0[0], ref0)
    assert abs(l1[0] - ref1) <= 1e-5 * abs(ref1), (l1[0], ref1)
    assert l1[0] < l0[0]


def _auc(score, label):
    """Probability that a random inlier scores above a random outlier."""
    order = np.argsort(score, kind="stable")
    rank = np.empty(len(score))
    rank[order] = np.arange(1, len(score) + 1)
    npos = label.sum()
    nneg = len(label) - npos
    return (rank[label].sum() - npos * (npos + 1) / 2) / (npos * nneg)


def test_trained_network_gain_on_heldout_scene():
    """The shipped network (trained on the GPU from plain solves of 500-camera
    scenes with 20% outliers, paper_2605_18052_amd/weights) on a held-out
    scene with 30% outliers: what it gains over the method without it.
    (1) Among the matches the threshold keeps, it separates true inliers from
    outliers far better than the plain method's own signal, the snapshot
    residual |eps_hat| (area under the ROC curve, ground-truth labels).
    (2) The first rounds of the learned solve reach a lower rotation error."""
    from paper_2605_18052_amd import learned
    params = learned.load_weights()
    sc = synth.trajectory_scene(n_cams=300, n_pts=120_000, knn=12, target_matches=3_000_000,
                                outlier_frac=0.3, seed=5180, name="heldout")
    pb = oracle_problem(sc)
    o = fastea.default_options(weight_mode=1)
    ctx = make_context(sc, gauge=1, weight_mode=1)
    ctx.set_mlp(params)
    ctx.init_poses(sc.R_init, sc.t_init)
    gains = []
    for r in range(3):
        ctx.begin_round(max(o.tau_px_init * o.tau_decay ** r, o.tau_px_min))
        w = ctx.learned_weights()
        mask, _ = ctx.get_mask()
        R, t, f = ctx.get_poses()
        eps = np.abs(oracle.residuals(pb, R, t, f))
        a_net = _auc(w[mask], sc.inlier[mask])
        a_res = _auc(-eps[mask], sc.inlier[mask])
        gains.append((a_net, a_res))
        ctx.step(o.iters_per_round)
    ctx.close()
    print("AUC (network, -|eps_hat|) per round:", [(round(a, 4), round(b, 4)) for a, b in gains])
    for a_net, a_res in gains:
        assert a_net > a_res + 0.05, gains

    def early_error(mode):
        ctx = make_context(sc, gauge=1, weight_mode=mode, log_every=50, max_log=20)
        if mode:
            ctx.set_mlp(params)
        ctx.init_poses(sc.R_init, sc.t_init)
        for r in range(3):
            ctx.begin_round(max(o.tau_px_init * o.tau_decay ** r, o.tau_px_min))
            ctx.step(o.iters_per_round)
        log = ctx.get_rotation_log(3)
        ctx.close()
        return [metrics.mean_rotation_error_deg(R, sc.R_gt) for R in log]

    plain, lrn = early_error(0), early_error(1)
    print("rotation error after rounds 1-3, plain:", np.round(plain, 3), "learned:", np.round(lrn, 3))
    assert lrn[1] < plain[1] and lrn[2] < plain[2], (plain, lrn)
