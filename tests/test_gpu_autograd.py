"""Autograd row: EpipolarLoss (torch.autograd.Function over the C ABI's
fea_loss_dev / fea_adjoint_dev) against the FP64 oracle and finite
differences, and as the backward pass a torch optimiser uses."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import fastea, synth

from gpu_helpers import make_context, oracle_problem, per_camera_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def _setup(sc, tau_px=math.inf):
    ctx = make_context(sc, gauge=0)
    ctx.init_poses(sc.R_init, sc.t_init)
    ctx.begin_round(tau_px)
    return ctx


def _perturb_params(a6, t, logf, seed=0):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    da = 0.01 * torch.randn(a6.shape, generator=g, dtype=torch.float64)
    dt = 0.02 * torch.randn(t.shape, generator=g, dtype=torch.float64)
    dl = 0.02 * torch.randn(logf.shape, generator=g, dtype=torch.float64)
    return ((a6.cpu() + da).cuda().contiguous(), (t.cpu() + dt).cuda().contiguous(),
            (logf.cpu() + dl).cuda().contiguous())


def _oracle_reference(sc, a6, t, logf, mask=None):
    """Loss and parameter gradients from the oracle's own functions."""
    a6 = a6.cpu().numpy()
    t = t.cpu().numpy()
    f = np.exp(logf.cpu().numpy())
    R = np.stack([oracle.rot6d_to_R(a) for a in a6])
    pb = oracle_problem(sc)
    loss, gR, gt, gf = oracle.loss_grad(pb, R, t, f, sc.R_init, sc.t_init, sc.f_init, mask,
                                        delta=fastea.default_options().delta)
    ga6 = np.stack([oracle.rot6d_backward(a6[c], gR[c]) for c in range(sc.n_cams)])
    return loss, ga6, gt, gf * f


@pytest.mark.parametrize("name", ["sphere20_m60k", "tiny_focals"])
def test_epipolar_loss_matches_oracle(name):
    import torch

    from paper_2605_18052_amd.autograd import EpipolarLoss
    sc = synth.config1() if name == "sphere20_m60k" else synth.tiny_scene(
        n_cams=6, n_pts=70, seed=5, sigma=1.0, outlier_frac=0.2)
    ctx = _setup(sc)
    a6, t, logf = ctx.get_params()
    a6, t, logf = _perturb_params(a6, t, logf)
    for x in (a6, t, logf):
        x.requires_grad_(True)
    loss = EpipolarLoss.apply(a6, t, logf, ctx)
    loss.backward()
    lref, ga6r, gtr, glr = _oracle_reference(sc, a6.detach(), t.detach(), logf.detach())
    assert abs(loss.item() - lref) <= 1e-5 * abs(lref)
    ok, worst = per_camera_close(a6.grad.cpu().numpy(), ga6r)
    assert ok, worst
    ok, worst = per_camera_close(t.grad.cpu().numpy(), gtr)
    assert ok, worst
    ok, worst = per_camera_close(logf.grad.cpu().numpy()[:, None], glr[:, None])
    assert ok, worst
    # upstream gradient scales the adjoint
    a6.grad = t.grad = logf.grad = None
    (3.0 * EpipolarLoss.apply(a6, t, logf, ctx)).backward()
    ok, worst = per_camera_close(a6.grad.cpu().numpy(), 3.0 * ga6r)
    assert ok, worst
    ctx.close()


def test_epipolar_loss_orders_on_the_callers_stream():
    """Parameters produced by torch work still queued on a side stream (no
    host synchronisation in between) give bit-identical loss and gradients
    to a fully synchronised call: the library's stream waits for torch's
    current stream and torch's waits for the library's, through events."""
    import torch

    from paper_2605_18052_amd.autograd import EpipolarLoss
    sc = synth.config1()
    ctx = _setup(sc)
    a6, t, logf = ctx.get_params()
    a6p, tp, lp = _perturb_params(a6, t, logf)
    ref = []
    for x in (a6p, tp, lp):
        x.requires_grad_(True)
    loss = EpipolarLoss.apply(a6p, tp, lp, ctx)
    loss.backward()
    torch.cuda.synchronize()
    ref = [loss.detach().cpu(), a6p.grad.cpu(), tp.grad.cpu(), lp.grad.cpu()]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        # a few milliseconds of queued work that the parameters depend on
        big = torch.randn(4096, 4096, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
        for _ in range(12):
            big = torch.tanh(big @ big)
        z = (big.sum() * 0.0).double()
        a6s = (a6p.detach() + z).contiguous().requires_grad_(True)
        ts = (tp.detach() + z).contiguous().requires_grad_(True)
        ls = (lp.detach() + z).contiguous().requires_grad_(True)
        loss2 = EpipolarLoss.apply(a6s, ts, ls, ctx)
        loss2.backward()
        got = [loss2.detach().clone(), a6s.grad.clone(), ts.grad.clone(), ls.grad.clone()]
    torch.cuda.synchronize()
    ctx.close()
    for a, b in zip(got, ref):
        assert torch.equal(a.cpu(), b)


def test_epipolar_loss_finite_differences():
    """Central differences of the forward agree with the adjoint (loose: the
    forward accumulates in fp32)."""
    import torch

    from paper_2605_18052_amd.autograd import EpipolarLoss
    sc = synth.config1()
    ctx = _setup(sc)
    a6, t, logf = ctx.get_params()
    a6, t, logf = _perturb_params(a6, t, logf, seed=1)
    for x in (a6, t, logf):
        x.requires_grad_(True)
    EpipolarLoss.apply(a6, t, logf, ctx).backward()
    grads = [a6.grad.clone(), t.grad.clone(), logf.grad.clone()]
    rng = np.random.default_rng(0)
    with torch.no_grad():
        for which, (p, g) in enumerate(zip((a6, t, logf), grads)):
            scale = g.abs().max().item()
            for _ in range(6):
                idx = tuple(int(rng.integers(s)) for s in p.shape)
                h = 1e-4
                p[idx] += h
                lp = EpipolarLoss.apply(a6, t, logf, ctx).item()
                p[idx] -= 2 * h
                lm = EpipolarLoss.apply(a6, t, logf, ctx).item()
                p[idx] += h
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx].item()) <= 2e-3 * scale + 1e-3 * abs(fd), (which, idx, fd,
                                                                                  g[idx].item())
    ctx.close()


def test_torch_adam_through_adjoint_matches_library_steps():
    """torch.optim.Adam driven by EpipolarLoss's backward takes the same steps
    as the library's own fused step (same adjoint kernels, same update)."""
    import torch

    from paper_2605_18052_amd.autograd import EpipolarLoss
    sc = synth.config1()
    o = fastea.default_options(gauge_normalize=0)
    ctx = _setup(sc)
    a6, t, logf = ctx.get_params()
    params = [a6.clone().requires_grad_(True), t.clone().requires_grad_(True),
              logf.clone().requires_grad_(True)]
    opt = torch.optim.Adam([{"params": [params[0]], "lr": o.lr_rot},
                            {"params": [params[1]], "lr": o.lr_t},
                            {"params": [params[2]], "lr": o.lr_logf}],
                           betas=(o.beta1, o.beta2), eps=o.adam_eps)
    for _ in range(4):
        opt.zero_grad()
        EpipolarLoss.apply(*params, ctx).backward()
        opt.step()
    ctx.step(4)
    a6_lib, t_lib, logf_lib = ctx.get_params()
    ctx.close()
    assert torch.allclose(params[0].detach(), a6_lib, rtol=0, atol=1e-9)
    assert torch.allclose(params[1].detach(), t_lib, rtol=0, atol=1e-9)
    assert torch.allclose(params[2].detach(), logf_lib, rtol=0, atol=1e-9)


def test_adjoint_at_scale_vs_fp64_finite_differences():
    """100M-match scene (3,000 cameras, 30 neighbours): the hand-written
    adjoint for 1% of the cameras (30, all 10 parameters each) against
    central differences of the FP64 oracle.  Each camera's derivative only
    involves its incident pairs, so the oracle evaluates those matches; the
    loss normalisation 1/Z is rescaled from the subset's Z to the full Z."""
    import torch

    from paper_2605_18052_amd.autograd import EpipolarLoss
    sc = synth.config3()
    ctx = make_context(sc, gauge=0)
    ctx.init_poses(sc.R_init, sc.t_init)
    ctx.begin_round(math.inf)
    Z = ctx.info()["n_retained"]
    a6, t, logf = ctx.get_params()
    for x in (a6, t, logf):
        x.requires_grad_(True)
    EpipolarLoss.apply(a6, t, logf, ctx).backward()
    ga6 = a6.grad.cpu().numpy()
    gt = t.grad.cpu().numpy()
    gl = logf.grad.cpu().numpy()
    ctx.close()
    a6n = a6.detach().cpu().numpy()
    tn = t.detach().cpu().numpy()
    lfn = logf.detach().cpu().numpy()
    rng = np.random.default_rng(3)
    cams = rng.choice(sc.n_cams, size=sc.n_cams // 100, replace=False)
    R0 = np.stack([oracle.rot6d_to_R(a) for a in a6n])
    f0 = np.exp(lfn)
    worst = 0.0
    for c in cams:
        sel = (sc.cam1 == c) | (sc.cam2 == c)
        pb = oracle.OracleProblem.from_scene(sc, sel)
        scale = sel.sum() / Z

        def L(a6c=None, tc=None, lfc=None):
            R = R0.copy()
            tt = tn.copy()
            f = f0.copy()
            if a6c is not None:
                R[c] = oracle.rot6d_to_R(a6c)
            if tc is not None:
                tt[c] = tc
            if lfc is not None:
                f[c] = np.exp(lfc)
            return scale * oracle.loss_grad(pb, R, tt, f, R0, tn, f0)[0]

        fd = np.zeros(10)
        for k in range(6):
            h = 1e-6
            ap, am = a6n[c].copy(), a6n[c].copy()
            ap[k] += h
            am[k] -= h
            fd[k] = (L(a6c=ap) - L(a6c=am)) / (2 * h)
        for k in range(3):
            h = 1e-6 * max(1.0, abs(tn[c, k]))
            tp_, tm_ = tn[c].copy(), tn[c].copy()
            tp_[k] += h
            tm_[k] -= h
            fd[6 + k] = (L(tc=tp_) - L(tc=tm_)) / (2 * h)
        h = 1e-6
        fd[9] = (L(lfc=lfn[c] + h) - L(lfc=lfn[c] - h)) / (2 * h)
        an = np.concatenate([ga6[c], gt[c], [gl[c]]])
        for blk in (slice(0, 6), slice(6, 9), slice(9, 10)):
            err = np.linalg.norm(an[blk] - fd[blk])
            ref = np.linalg.norm(fd[blk])
            worst = max(worst, err / ref)
            assert err <= 1e-5 * ref + 1e-12, (c, blk, an[blk], fd[blk])
    print(f"adjoint vs FP64 FD on {len(cams)} cameras: worst relative error {worst:.2e}")
