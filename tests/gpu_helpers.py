"""Shared set-up for the GPU parity tests (host side only)."""
import numpy as np

import oracle
from paper_2605_18052_amd import fastea


def make_context(sc, gauge=0, f=None, groups=None, **opt):
    o = fastea.default_options(gauge_normalize=gauge, **opt)
    ctx = fastea.Context(0, o)
    ctx.load_intrinsics(sc.f_init if f is None else f, sc.cx, sc.cy, groups)
    ctx.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
    return ctx


def per_camera_close(g_gpu, g_ref, rel=1e-5, floor=1e-3):
    """||g_gpu,c - g_ref,c|| <= rel * max(||g_ref,c||, floor * max_c' ||g_ref,c'||)."""
    g_gpu = np.asarray(g_gpu).reshape(len(g_gpu), -1)
    g_ref = np.asarray(g_ref).reshape(len(g_ref), -1)
    nr = np.linalg.norm(g_ref, axis=1)
    err = np.linalg.norm(g_gpu - g_ref, axis=1)
    bound = rel * np.maximum(nr, floor * nr.max())
    return bool(np.all(err <= bound)), float((err / np.maximum(bound / rel, 1e-300)).max())


def tau_in_gap(abs_eps, target):
    """A threshold near `target` that no |eps| comes within 1e-7 relative of."""
    v = np.sort(abs_eps)
    k = np.searchsorted(v, target)
    for d in range(0, len(v)):
        for kk in (k + d, k - d):
            if 1 <= kk < len(v):
                lo, hi = v[kk - 1], v[kk]
                if hi - lo > 1e-6 * hi:
                    return 0.5 * (lo + hi)
    return target


def oracle_problem(sc):
    return oracle.OracleProblem.from_scene(sc)


def score_tol(ref):
    """Bound on |fp32 score - fp64 score|: the per-match n = (R x1) x x2 in fp32
    from fp32 inputs carries <= ~1e-6 absolute (normalised coordinates below
    ~1.5, a few roundings of 2^-24 each), the matrix-core dot products a few
    ulps more; each lane sums at most 128 terms, then at most 4 such sums, in
    fp32 (<= 132 * 2^-24 = 8e-6 relative) before the fp64 cross-lane sum."""
    return 1e-6 + 1e-5 * np.abs(ref)


def check_search(got, ref, K):
    """Scores to the bound; the choice equal where the oracle's best is
    separated from its runner-up by more than the bound, else a valid
    near-tie; vote and signed direction equal where the choice agrees."""
    sg, sr = got["scores"].astype(np.float64), ref["scores"]
    tol = score_tol(sr)
    bad = np.abs(sg - sr) > tol
    assert not bad.any(), (np.argwhere(bad)[:5], np.abs(sg - sr)[bad][:5], sr[bad][:5])
    P = len(sr)
    order = np.sort(sr, axis=1)
    sep = order[:, 1] - order[:, 0] > 2 * score_tol(order[:, 0]) if K > 1 else np.ones(P, bool)
    assert np.array_equal(got["best"][sep], ref["best"][sep])
    chosen = sr[np.arange(P), got["best"]]
    assert np.all(chosen <= order[:, 0] + 2 * score_tol(order[:, 0]))
    same = got["best"] == ref["best"]
    assert np.all(np.abs(got["vote"][same] - ref["vote"][same]) <= 2)
    sgn = np.sign(got["vote"]) == np.sign(ref["vote"])
    m = same & (sgn | (np.abs(ref["vote"]) > 2))
    np.testing.assert_array_equal(got["t_rel"][same & sgn], ref["t_rel"][same & sgn])
    np.testing.assert_allclose(got["score_best"], chosen, rtol=1e-5, atol=1e-6)
    return same.mean(), m.mean()


def vote_tol(ref, tau, n_pairs):
    """The closed-form eigenvalues fix s1/s2 to ~1.5e-8 (sqrt of the fp64
    epsilon: the gap of two nearly equal eigenvalues from the cubic's
    invariants), so each term exp((1 - s1/s2)/tau) to ~1.5e-8/tau relative;
    a factor 10 of margin, plus an absolute floor for terms near zero."""
    return 10 * 1.5e-8 / tau * np.abs(ref) + 1e-12 * n_pairs
