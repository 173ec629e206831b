"""Seeded synthetic scenes shaped like the FastMap epipolar-adjustment workloads.

This module only builds inputs: cameras, 3D points, their noisy projections,
matches between image pairs, outliers and a perturbed starting pose.  It holds
none of the epipolar-adjustment arithmetic (no essential matrix, residual,
weight or gradient); both the HIP library's tests/benchmarks and the FP64
oracle draw their inputs from here.

Camera model (FastMap, Method > Intrinsics Estimation): pinhole, principal
point fixed at the image centre (continuous convention: pixel (0,0) is the
image corner, so the centre of a W x H image is (W/2, H/2)), one focal length
per camera.  Poses are world-to-camera: X_cam = R X + t, camera centre
o = -R^T t.

Randomness that must be identical no matter how the scene is traversed (which
camera sees which point, the pixel noise of one observation, outlier draws)
comes from a counter-based hash of (seed, stream, a, b); the bulk layout
(camera placement, point cloud, match shuffle) comes from numpy's PCG64.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014), vectorised over uint64."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _workers() -> int:
    """Host threads for scene generation (numpy releases the GIL in the bulk
    array work; every result is assembled in a fixed order, so the scene does
    not depend on the thread count)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _pmap(fn, items):
    """fn over items on the generation threads, results in item order."""
    items = list(items)
    if len(items) <= 1 or _workers() == 1:
        return [fn(x) for x in items]
    # one BLAS thread per worker: the small products here gain nothing from
    # BLAS's own threads, which would contend with the workers
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1, user_api="blas"), ThreadPoolExecutor(max_workers=_workers()) as ex:
        return list(ex.map(fn, items))


def _ranges(n: int, parts: int):
    """Contiguous [lo, hi) ranges splitting range(n) into about `parts` pieces."""
    parts = max(1, min(parts, n))
    cuts = np.linspace(0, n, parts + 1).astype(np.int64)
    return [(int(cuts[k]), int(cuts[k + 1])) for k in range(parts) if cuts[k + 1] > cuts[k]]


def hash_u01(seed: int, stream: int, a, b) -> np.ndarray:
    """Uniform [0,1) doubles from a counter hash of (seed, stream, a, b)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    with np.errstate(over="ignore"):
        k = _splitmix64(np.uint64(seed) * np.uint64(0x100000001B3) + np.uint64(stream))
        h = _splitmix64(k ^ _splitmix64(a * np.uint64(0x9E3779B1) + np.uint64(0x632BE5AB)))
        h = _splitmix64(h ^ b)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def hash_normal(seed: int, stream: int, a, b) -> np.ndarray:
    """Standard normals by Box-Muller from two hashed uniforms."""
    u1 = hash_u01(seed, 2 * stream, a, b)
    u2 = hash_u01(seed, 2 * stream + 1, a, b)
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


def rotation_from_axis_angle(axis: np.ndarray, angle: np.ndarray) -> np.ndarray:
    """Rodrigues' formula, batched: axis [...,3] (unit), angle [...] radians."""
    axis = np.asarray(axis, dtype=np.float64)
    angle = np.asarray(angle, dtype=np.float64)
    k = axis / np.linalg.norm(axis, axis=-1, keepdims=True)
    K = np.zeros(k.shape[:-1] + (3, 3))
    K[..., 0, 1], K[..., 0, 2] = -k[..., 2], k[..., 1]
    K[..., 1, 0], K[..., 1, 2] = k[..., 2], -k[..., 0]
    K[..., 2, 0], K[..., 2, 1] = -k[..., 1], k[..., 0]
    s = np.sin(angle)[..., None, None]
    c = np.cos(angle)[..., None, None]
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + s * K + (1.0 - c) * (K @ K)


def look_at(center: np.ndarray, target: np.ndarray) -> np.ndarray:
    """World-to-camera rotations whose +z axis points from center to target.

    Rows of R are the camera x, y, z axes in world coordinates; the world up
    vector is +z unless the viewing direction is nearly vertical.
    """
    center = np.atleast_2d(center)
    z = target - center
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    up = np.tile(np.array([0.0, 0.0, 1.0]), (len(z), 1))
    vertical = np.abs(z @ np.array([0.0, 0.0, 1.0])) > 0.95
    up[vertical] = np.array([0.0, 1.0, 0.0])
    x = np.cross(up, z)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=1)


@dataclass
class Scene:
    """One synthetic epipolar-adjustment problem (all arrays host numpy)."""

    name: str
    seed: int
    width: np.ndarray  # float64 [N]
    height: np.ndarray  # float64 [N]
    f_gt: np.ndarray  # float64 [N]
    f_init: np.ndarray  # float64 [N]
    intr_group: np.ndarray  # int32 [N]
    R_gt: np.ndarray  # float64 [N,3,3] world-to-camera
    t_gt: np.ndarray  # float64 [N,3]
    R_init: np.ndarray
    t_init: np.ndarray
    x1: np.ndarray  # float32 [M] pixel coordinates in camera cam1
    y1: np.ndarray
    x2: np.ndarray  # float32 [M] pixel coordinates in camera cam2
    y2: np.ndarray
    cam1: np.ndarray  # int32 [M]
    cam2: np.ndarray  # int32 [M]
    inlier: np.ndarray  # bool [M]
    radius: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n_cams(self) -> int:
        return int(self.f_gt.shape[0])

    @property
    def n_matches(self) -> int:
        return int(self.x1.shape[0])

    @property
    def cx(self) -> np.ndarray:
        return self.width / 2.0

    @property
    def cy(self) -> np.ndarray:
        return self.height / 2.0

    def pairs(self) -> np.ndarray:
        """Distinct unordered camera pairs (i<j) present in the matches."""
        i = np.minimum(self.cam1, self.cam2).astype(np.int64)
        j = np.maximum(self.cam1, self.cam2).astype(np.int64)
        key = np.unique(i * self.n_cams + j)
        return np.stack([key // self.n_cams, key % self.n_cams], axis=1)


def _observe(R, t, f, cx, cy, X):
    """Noise-free pinhole projection of X [K,3] into one camera."""
    Xc = X @ R.T + t
    z = Xc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = f * Xc[:, 0] / z + cx
        v = f * Xc[:, 1] / z + cy
    return u, v, z


def _visible(u, v, z, width, height):
    return (z > 1e-3) & (u >= 0.0) & (u < width) & (v >= 0.0) & (v < height)


def _perturb_init(rng, R_gt, t_gt, rot_sigma_deg, rot_min_deg, center_frac, pairs):
    """Starting poses standing in for the output of global rotation and
    translation alignment: GT rotation times a random-axis rotation of angle
    |N(0, rot_sigma)| + rot_min; camera centres plus isotropic Gaussian noise
    whose sigma is `center_frac` times the median baseline of the matched
    pairs (so relative translation directions start a few degrees off)."""
    n = len(R_gt)
    axis = rng.normal(size=(n, 3))
    ang = np.deg2rad(np.abs(rng.normal(0.0, rot_sigma_deg, size=n)) + rot_min_deg)
    R_init = rotation_from_axis_angle(axis, ang) @ R_gt
    centers = -np.einsum("nji,nj->ni", R_gt, t_gt)
    pairs = np.asarray(pairs).reshape(-1, 2)
    base = np.median(np.linalg.norm(centers[pairs[:, 0]] - centers[pairs[:, 1]], axis=1))
    centers_init = centers + rng.normal(0.0, center_frac * base, size=centers.shape)
    t_init = -np.einsum("nij,nj->ni", R_init, centers_init)
    return R_init, t_init


def _emit_matches(seed, pair_list, det_ids, det_u, det_v, n_cams, width, height,
                  outlier_frac, rng):
    """Matches for every pair: the points detected by both cameras.

    det_ids[c] is the sorted array of point ids detected by camera c and
    det_u/det_v their noisy pixel coordinates.  An outlier keeps the first
    keypoint and moves the second one to a uniformly random pixel of the
    second image.  Each match is then emitted in a random orientation and the
    whole list is shuffled, so callers must canonicalise and sort.
    """
    pairs = np.asarray(pair_list, dtype=np.int64).reshape(-1, 2)
    sizes = np.array([len(d) for d in det_ids], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    n_pts = int(max((d.max() + 1 for d in det_ids if len(d)), default=0))
    all_ids = np.concatenate(det_ids) if n_pts else np.zeros(0, np.int64)
    all_u = np.concatenate(det_u) if n_pts else np.zeros(0)
    all_v = np.concatenate(det_v) if n_pts else np.zeros(0)
    # visit pairs grouped by their second camera, with a dense point -> slot
    # map of that camera; runs of whole groups go to the threads and their
    # parts are joined in visiting order
    order = np.argsort(pairs[:, 1], kind="stable")
    heads = np.flatnonzero(np.diff(pairs[order, 1], prepend=-1)) if len(order) else np.zeros(0, np.int64)
    bounds = np.append(heads, len(order))

    def visit(span):
        g0, g1 = span
        pos = np.full(max(n_pts, 1), -1, dtype=np.int64)
        a_parts, b_parts, k_parts = [], [], []
        for g in range(g0, g1):
            ks = order[bounds[g]:bounds[g + 1]]
            j = int(pairs[ks[0], 1])
            pos[det_ids[j]] = np.arange(len(det_ids[j]))
            for k in ks:
                i = int(pairs[k, 0])
                h = pos[det_ids[i]]
                hit = np.flatnonzero(h >= 0)
                if len(hit) == 0:
                    continue
                a_parts.append(offs[i] + hit)
                b_parts.append(offs[j] + h[hit])
                k_parts.append(np.full(len(hit), k, dtype=np.int64))
            pos[det_ids[j]] = -1
        return a_parts, b_parts, k_parts

    spans = _ranges(len(heads), 8 * _workers())
    a_parts, b_parts, k_parts = [], [], []
    for a, b, k in _pmap(visit, spans):
        a_parts += a
        b_parts += b
        k_parts += k
    if not a_parts:
        e = np.zeros(0, np.float32)
        ei = np.zeros(0, np.int32)
        return e, e, e, e, ei, ei, np.zeros(0, bool)
    A = np.concatenate(a_parts)
    B = np.concatenate(b_parts)
    K = np.concatenate(k_parts)
    del a_parts, b_parts, k_parts
    n = len(A)
    ax, ay, bx, by = (np.empty(n) for _ in range(4))
    c1 = np.empty(n, np.int32)
    c2 = np.empty(n, np.int32)
    inl = np.empty(n, bool)

    def emit(span):
        lo, hi = span
        Ak, Bk, Kk = A[lo:hi], B[lo:hi], K[lo:hi]
        ci, cj = pairs[Kk, 0], pairs[Kk, 1]
        pts = all_ids[Ak]
        x1, y1 = all_u[Ak], all_v[Ak]
        x2, y2 = all_u[Bk], all_v[Bk]
        key = ci.astype(np.uint64) * np.uint64(n_cams) + cj.astype(np.uint64)
        out = hash_u01(seed, 40, key, pts) < outlier_frac
        x2[out] = hash_u01(seed, 41, key[out], pts[out]) * width[cj[out]]
        y2[out] = hash_u01(seed, 42, key[out], pts[out]) * height[cj[out]]
        flip = hash_u01(seed, 43, key, pts) < 0.5
        c1[lo:hi] = np.where(flip, cj, ci)
        c2[lo:hi] = np.where(flip, ci, cj)
        ax[lo:hi], ay[lo:hi] = np.where(flip, x2, x1), np.where(flip, y2, y1)
        bx[lo:hi], by[lo:hi] = np.where(flip, x1, x2), np.where(flip, y1, y2)
        inl[lo:hi] = ~out

    _pmap(emit, _ranges(n, 4 * _workers()))
    del A, B, K
    perm = rng.permutation(n)
    res = (np.empty(n, np.float32), np.empty(n, np.float32), np.empty(n, np.float32),
           np.empty(n, np.float32), np.empty(n, np.int32), np.empty(n, np.int32), np.empty(n, bool))

    def gather(span):
        lo, hi = span
        pk = perm[lo:hi]
        for dst, src in zip(res, (ax, ay, bx, by, c1, c2, inl)):
            dst[lo:hi] = src[pk]

    _pmap(gather, _ranges(n, 4 * _workers()))
    return res


def _detect(seed, R, t, f, cx, cy, width, height, X, p_det, sigma):
    """Per camera: sorted detected point ids and their noisy pixels."""
    n = len(R)
    ids_all = np.arange(len(X), dtype=np.int64)

    def one(c):
        u, v, z = _observe(R[c], t[c], f[c], cx[c], cy[c], X)
        vis = _visible(u, v, z, width[c], height[c])
        ids = ids_all[vis]
        if p_det < 1.0:
            keep = hash_u01(seed, 10, c, ids) < p_det
            ids = ids[keep]
        uu = u[ids]
        vv = v[ids]
        if sigma > 0:
            uu = uu + sigma * hash_normal(seed, 11, c, ids)
            vv = vv + sigma * hash_normal(seed, 12, c, ids)
        return ids, uu, vv

    res = _pmap(one, range(n))
    return [r[0] for r in res], [r[1] for r in res], [r[2] for r in res]


def sphere_scene(n_cams=20, n_pts=2000, radius=4.0, focal=500.0, width=640.0,
                 height=480.0, p_det=0.4, sigma=0.5, outlier_frac=0.1, seed=1,
                 extent=1.0, rot_sigma_deg=3.0, rot_min_deg=2.0, center_frac=0.05,
                 name="sphere", pair_angle_deg=None) -> Scene:
    """Cameras at seeded uniform directions on a sphere, looking at the origin,
    points uniform in a cube of side `extent`; all camera pairs matched, or
    with pair_angle_deg only the pairs whose viewing directions are less than
    that angle apart (an object-centric capture's pair graph)."""
    rng = np.random.default_rng(seed)
    dirs = rng.normal(size=(n_cams, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    centers = radius * dirs
    R = look_at(centers, np.zeros(3))
    t = -np.einsum("nij,nj->ni", R, centers)
    X = rng.uniform(-extent / 2, extent / 2, size=(n_pts, 3))
    f = np.broadcast_to(np.asarray(focal, dtype=np.float64), (n_cams,)).copy()
    W = np.full(n_cams, float(width))
    H = np.full(n_cams, float(height))
    det = _detect(seed, R, t, f, W / 2, H / 2, W, H, X, p_det, sigma)
    if pair_angle_deg is None:
        pair_list = [(i, j) for i in range(n_cams) for j in range(i + 1, n_cams)]
    else:
        ii, jj = np.nonzero(np.triu(dirs @ dirs.T > np.cos(np.deg2rad(pair_angle_deg)), 1))
        pair_list = list(zip(ii.tolist(), jj.tolist()))
    x1, y1, x2, y2, c1, c2, inl = _emit_matches(seed, pair_list, *det, n_cams, W, H,
                                                outlier_frac, rng)
    R0, t0 = _perturb_init(rng, R, t, rot_sigma_deg, rot_min_deg, center_frac,
                           pair_list)
    return Scene(name=name, seed=seed, width=W, height=H, f_gt=f, f_init=f.copy(),
                 intr_group=np.arange(n_cams, dtype=np.int32), R_gt=R, t_gt=t,
                 R_init=R0, t_init=t0, x1=x1, y1=y1, x2=x2, y2=y2, cam1=c1, cam2=c2,
                 inlier=inl, radius=radius,
                 meta=dict(n_pts=n_pts, p_det=p_det, sigma=sigma, outlier_frac=outlier_frac))


def _knn_pairs(centers: np.ndarray, k: int) -> np.ndarray:
    n = len(centers)
    k = min(k, n - 1)
    pairs = set()
    for s in range(0, n, 512):
        d = np.linalg.norm(centers[s:s + 512, None, :] - centers[None, :, :], axis=2)
        d[np.arange(len(d)), np.arange(s, s + len(d))] = np.inf
        nn = np.argpartition(d, k - 1, axis=1)[:, :k]
        for r, row in enumerate(nn):
            i = s + r
            for j in row:
                pairs.add((min(i, int(j)), max(i, int(j))))
    return np.array(sorted(pairs), dtype=np.int64).reshape(-1, 2)


def trajectory_scene(n_cams=500, n_pts=200_000, radius=6.0, height_wave=1.0,
                     center_noise=0.1, jitter_deg=5.0, box=(4.0, 4.0, 2.0), knn=20,
                     target_matches=20_000_000, sigma=1.0, outlier_frac=0.2,
                     f_range=(400.0, 1200.0), f_init_spread=0.1, width=640.0,
                     height=480.0, seed=2, rot_sigma_deg=3.0, rot_min_deg=2.0,
                     center_frac=0.05, calib_sample=50_000, name="trajectory") -> Scene:
    """Cameras on a noisy closed loop around a box of points, each matched to
    its `knn` nearest neighbours by centre; the detection probability is set
    so that the expected match count is `target_matches`."""
    rng = np.random.default_rng(seed)
    th = 2.0 * np.pi * np.arange(n_cams) / n_cams
    centers = np.stack([radius * np.cos(th), radius * np.sin(th),
                        height_wave * np.sin(3.0 * th)], axis=1)
    centers += rng.normal(0.0, center_noise, size=centers.shape)
    R = look_at(centers, np.zeros(3))
    jitter = rotation_from_axis_angle(rng.normal(size=(n_cams, 3)),
                                      np.deg2rad(rng.normal(0.0, jitter_deg, size=n_cams)))
    R = jitter @ R
    t = -np.einsum("nij,nj->ni", R, centers)
    X = rng.uniform(-0.5, 0.5, size=(n_pts, 3)) * np.asarray(box)
    f = rng.uniform(f_range[0], f_range[1], size=n_cams)
    f_init = f * np.exp(rng.uniform(-f_init_spread, f_init_spread, size=n_cams))
    W = np.full(n_cams, float(width))
    H = np.full(n_cams, float(height))
    pair_arr = _knn_pairs(centers, knn)
    # Calibrate the detection probability on a point sample: the expected
    # number of matches is p^2 * sum over pairs of co-visible points.
    samp = rng.choice(n_pts, size=min(calib_sample, n_pts), replace=False)
    Xs = X[samp]

    def seen(c):
        u, v, z = _observe(R[c], t[c], f[c], W[c] / 2, H[c] / 2, Xs)
        return _visible(u, v, z, W[c], H[c])

    vis = np.stack(_pmap(seen, range(n_cams))) if n_cams else np.zeros((0, len(samp)), bool)
    packed = np.packbits(vis, axis=1)
    covis = 0
    for s in range(0, len(pair_arr), 4096):
        pa = pair_arr[s:s + 4096]
        covis += int(np.bitwise_count(packed[pa[:, 0]] & packed[pa[:, 1]]).sum())
    covis *= n_pts / len(samp)
    p_det = float(min(1.0, np.sqrt(target_matches / max(covis, 1.0))))
    det = _detect(seed, R, t, f, W / 2, H / 2, W, H, X, p_det, sigma)
    x1, y1, x2, y2, c1, c2, inl = _emit_matches(seed, [tuple(p) for p in pair_arr], *det,
                                                n_cams, W, H, outlier_frac, rng)
    R0, t0 = _perturb_init(rng, R, t, rot_sigma_deg, rot_min_deg, center_frac, pair_arr)
    return Scene(name=name, seed=seed, width=W, height=H, f_gt=f, f_init=f_init,
                 intr_group=np.arange(n_cams, dtype=np.int32), R_gt=R, t_gt=t,
                 R_init=R0, t_init=t0, x1=x1, y1=y1, x2=x2, y2=y2, cam1=c1, cam2=c2,
                 inlier=inl, radius=radius,
                 meta=dict(n_pts=n_pts, p_det=p_det, sigma=sigma,
                           outlier_frac=outlier_frac, n_pairs=len(pair_arr), knn=knn))


# Workload presets.  Sizes follow the FastMap scene scales (hundreds to a few
# thousand images, 5k-500k image pairs in the kernel-fusion ablation).
def config1(seed: int = 1) -> Scene:
    """20 cameras on a radius-4 sphere, 2,000 points in the unit cube, f=500,
    640x480, all 190 pairs, detection 0.4 (~60.8k matches), sigma 0.5 px,
    10% outliers."""
    return sphere_scene(seed=seed, name="sphere20_m60k")


def config2(seed: int = 2, target_matches: int = 20_000_000) -> Scene:
    """500 cameras on a noisy loop, 200k points, 20 nearest neighbours,
    ~20M matches, sigma 1 px, 20% outliers, f in [400,1200] px."""
    return trajectory_scene(seed=seed, target_matches=target_matches,
                            name="traj500_m20M")


def config3(seed: int = 3, target_matches: int = 100_000_000) -> Scene:
    """3,000 cameras, 1M points, 30 nearest neighbours, ~100M matches,
    sigma 1 px, 25% outliers."""
    return trajectory_scene(n_cams=3000, n_pts=1_000_000, knn=30,
                            target_matches=target_matches, outlier_frac=0.25,
                            seed=seed, name="traj3000_m100M")


def config5(seed: int = 5100, target_matches: int = 30_000_000) -> Scene:
    """Held-out scene of the learned-weight workload: 1,000 cameras on the
    noisy loop, 400k points, 20 nearest neighbours, ~30M matches, sigma
    1 px, 30% outliers, f in [400,1200] px.  The network is trained on the
    500-camera, 20%-outlier scenes of seeds 5000-5003 and validated on 5004;
    the test scenes are seeds 5100-5102."""
    return trajectory_scene(n_cams=1000, n_pts=400_000, knn=20, target_matches=target_matches,
                            outlier_frac=0.3, seed=seed, name=f"traj1000_m30M_s{seed}")


def tiny_scene(n_cams=4, n_pts=40, seed=7, sigma=0.0, outlier_frac=0.0,
               p_det=1.0, focal=500.0, distinct_focals=True) -> Scene:
    """Small sphere scene for brute-force checks; optional distinct focals."""
    if distinct_focals:
        focal = np.random.default_rng(seed + 1000).uniform(0.8 * focal, 1.2 * focal,
                                                           size=n_cams)
    return sphere_scene(n_cams=n_cams, n_pts=n_pts, p_det=p_det, sigma=sigma,
                        outlier_frac=outlier_frac, seed=seed, focal=focal, name="tiny")


def random_poses(rng, n_cams, radius=4.0):
    """Random (not necessarily realistic) poses for gradient checks."""
    R = rotation_from_axis_angle(rng.normal(size=(n_cams, 3)),
                                 rng.uniform(0, np.pi, size=n_cams))
    centers = rng.normal(size=(n_cams, 3)) * radius
    t = -np.einsum("nij,nj->ni", R, centers)
    return R, t


def config4(n_scenes: int = 64, seed: int = 4000, total_matches: float = 120e6,
            cams_range=(20, 1000), matches_range=(5e4, 1e7)) -> list:
    """64 independent trajectory scenes of uneven size: camera counts drawn
    log-uniformly in [20, 1000] and match counts log-uniformly in
    [5e4, 1e7] (rescaled so that the batch holds about `total_matches`)."""
    rng = np.random.default_rng(seed)
    n_cams = np.round(np.exp(rng.uniform(np.log(cams_range[0]), np.log(cams_range[1]),
                                         n_scenes))).astype(int)
    m = np.exp(rng.uniform(np.log(matches_range[0]), np.log(matches_range[1]), n_scenes))
    m = np.clip(m * total_matches / m.sum(), matches_range[0], matches_range[1])
    scenes = []
    for s in range(n_scenes):
        n = int(n_cams[s])
        knn = min(20, n - 1)
        pts = int(np.clip(m[s] / 100, 2_000, 200_000))
        scenes.append(trajectory_scene(n_cams=n, n_pts=pts, knn=knn, target_matches=int(m[s]),
                                       seed=seed + s, name=f"batch{s:02d}",
                                       calib_sample=min(50_000, pts)))
    return scenes


def concat_scenes(scenes: list):
    """One multi-scene problem: cameras of scene s get ids offset by the
    camera counts of the scenes before it.  Returns (arrays dict, cam_scene,
    camera offsets)."""
    offs = np.concatenate([[0], np.cumsum([s.n_cams for s in scenes])]).astype(np.int64)
    cat = lambda name: np.concatenate([getattr(s, name) for s in scenes])
    out = dict(x1=cat("x1"), y1=cat("y1"), x2=cat("x2"), y2=cat("y2"),
               cam1=np.concatenate([s.cam1 + offs[k] for k, s in enumerate(scenes)]).astype(np.int32),
               cam2=np.concatenate([s.cam2 + offs[k] for k, s in enumerate(scenes)]).astype(np.int32),
               f_init=cat("f_init"), cx=np.concatenate([s.cx for s in scenes]),
               cy=np.concatenate([s.cy for s in scenes]), R_init=cat("R_init"), t_init=cat("t_init"),
               R_gt=cat("R_gt"))
    cam_scene = np.concatenate([np.full(s.n_cams, k, np.int32) for k, s in enumerate(scenes)])
    return out, cam_scene, offs


def sphere_candidates(n: int) -> np.ndarray:
    """n unit directions spread evenly over the upper hemisphere (z > 0): a
    Fibonacci lattice, z_k = 1 - (k + 1/2)/n, azimuth k times the golden
    angle.  Candidate relative-translation directions; a direction and its
    opposite score the same, so one hemisphere suffices.  float64 [n, 3]."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (k + 0.5) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * np.pi * (3.0 - np.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def random_centres(seed: int, n_runs: int, n_cams: int) -> np.ndarray:
    """Independent random initial camera centres for translation alignment:
    standard normal per coordinate, float64 [n_runs, n_cams, 3]."""
    return np.random.default_rng(seed).normal(size=(n_runs, n_cams, 3))


def relative_translations_gt(sc: "Scene", pair_cams: np.ndarray) -> np.ndarray:
    """Ground-truth unit relative translations t^{i->j} (camera j frame) of the
    given pairs, from the scene's true poses.  float64 [P, 3]."""
    i, j = pair_cams[:, 0], pair_cams[:, 1]
    Rij = np.einsum("pab,pcb->pac", sc.R_gt[j], sc.R_gt[i])
    t = sc.t_gt[j] - np.einsum("pab,pb->pa", Rij, sc.t_gt[i])
    return t / np.linalg.norm(t, axis=1, keepdims=True)


def object_pair_graph(n_cams: int = 500, angle_deg: float = 60.0, seed: int = 0, radius: float = 4.0):
    """An object-centric capture's pair graph without matches: cameras at
    seeded uniform directions on a sphere looking at the origin, pairs whose
    viewing directions are less than angle_deg apart.  Returns pair_cams
    int32 [P, 2] (i < j), world-to-camera rotations [N, 3, 3], the true unit
    relative translations t^{i->j} [P, 3] (camera j frame) and the camera
    centres [N, 3]."""
    rng = np.random.default_rng(seed)
    dirs = rng.normal(size=(n_cams, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    ii, jj = np.nonzero(np.triu(dirs @ dirs.T > np.cos(np.deg2rad(angle_deg)), 1))
    pc = np.stack([ii, jj], 1).astype(np.int32)
    c = radius * dirs
    R = look_at(c, np.zeros(3))
    t = -np.einsum("nij,nj->ni", R, c)
    i, j = pc[:, 0], pc[:, 1]
    Rij = np.einsum("pab,pcb->pac", R[j], R[i])
    tij = t[j] - np.einsum("pab,pb->pa", Rij, t[i])
    return pc, R, tij / np.linalg.norm(tij, axis=1, keepdims=True), c


def fundamental_matrices(sc: "Scene", pair_cams: np.ndarray, noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """Fundamental matrices of the given pairs from the scene's true poses and
    focal lengths, in centred pixel coordinates (p_j^T F p_i = 0 with
    p = (x - cx, y - cy, 1)), each scaled to unit Frobenius norm.  With noise,
    the essential matrix (unit Frobenius norm, calibrated coordinates, where
    all entries have comparable scale) gets seeded Gaussian noise of that
    size on every entry and is projected back to rank 2 before the focal
    lengths are applied.  float64 [P, 3, 3]."""
    i, j = pair_cams[:, 0], pair_cams[:, 1]
    Rij = np.einsum("pab,pcb->pac", sc.R_gt[j], sc.R_gt[i])
    t = sc.t_gt[j] - np.einsum("pab,pb->pa", Rij, sc.t_gt[i])
    tx = np.zeros((len(t), 3, 3))
    tx[:, 0, 1], tx[:, 0, 2], tx[:, 1, 2] = -t[:, 2], t[:, 1], -t[:, 0]
    tx[:, 1, 0], tx[:, 2, 0], tx[:, 2, 1] = t[:, 2], -t[:, 1], t[:, 0]
    E = tx @ Rij
    E /= np.linalg.norm(E, axis=(1, 2), keepdims=True)
    if noise > 0:
        E = E + noise * np.random.default_rng(seed).normal(size=E.shape)
        U, s, Vt = np.linalg.svd(E)
        s[:, 2] = 0.0
        E = U @ (s[:, :, None] * Vt)
    di = np.stack([1 / sc.f_gt[i], 1 / sc.f_gt[i], np.ones(len(i))], 1)
    dj = np.stack([1 / sc.f_gt[j], 1 / sc.f_gt[j], np.ones(len(j))], 1)
    F = dj[:, :, None] * E * di[:, None, :]
    return F / np.linalg.norm(F, axis=(1, 2), keepdims=True)


def focal_candidates(n: int, lo: float = 100.0, hi: float = 5000.0) -> np.ndarray:
    """n focal lengths spaced evenly in log between lo and hi (pixels)."""
    return np.exp(np.linspace(np.log(lo), np.log(hi), n))
