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
