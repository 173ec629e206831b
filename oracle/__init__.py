"""FP64 CPU oracle for FastMap epipolar adjustment and the stages before it
(focal-length vote, global rotation, relative-translation search,
camera-centre alignment with multiple initialisations).  The C parts go
through ctypes; the focal vote and the global rotation are plain numpy
(singular values from numpy's SVD, eigenvectors from its eigh).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg use it to check and time the GPU library.  The
library itself never imports it.  The arithmetic lives in ``fea_oracle.c``
(plain C, double precision); this module only marshals numpy arrays.

Parity status: see the per-function notes in ``fea_oracle.h``; the IRLS
threshold schedule and optimiser constants are not fixed by the paper
("parity unpinned" for those constants: they are pinned only by outcome).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over image pairs)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-o", _LIB_PATH + ".tmp", os.path.join(_HERE, "fea_oracle.c"), "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Problem(C.Structure):
    _fields_ = [("n_matches", C.c_int64), ("n_cams", C.c_int32),
                ("x1", C.c_void_p), ("y1", C.c_void_p), ("x2", C.c_void_p),
                ("y2", C.c_void_p), ("cam1", C.c_void_p), ("cam2", C.c_void_p),
                ("cx", C.c_void_p), ("cy", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("iters_per_round", C.c_int32),
                ("tau_px_init", C.c_double), ("tau_px_min", C.c_double),
                ("tau_decay", C.c_double), ("delta", C.c_double),
                ("lr_rot", C.c_double), ("lr_t", C.c_double), ("lr_logf", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("adam_eps", C.c_double),
                ("optimize_focal", C.c_int32), ("gauge_normalize", C.c_int32),
                ("lr_decay", C.c_double), ("reset_moments", C.c_int32),
                ("converge_deg", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        _lib.orc_segment.argtypes = [C.c_int64, C.c_int32, P, P, P, P, P, P, P]
        _lib.orc_segment.restype = C.c_int
        _lib.orc_rot6d_to_R.argtypes = [P, P]
        _lib.orc_rot6d_backward.argtypes = [P, P, P]
        _lib.orc_R_to_rot6d.argtypes = [P, P]
        _lib.orc_pair_F.argtypes = [P, P, C.c_double, P, P, C.c_double, P]
        _lib.orc_pair_F.restype = C.c_int
        _lib.orc_residuals.argtypes = [P, P, P, P, P]
        _lib.orc_residuals.restype = C.c_int
        _lib.orc_update_mask.argtypes = [P, P, P, P, C.c_double, P]
        _lib.orc_update_mask.restype = C.c_int64
        _lib.orc_loss_grad.argtypes = [P, P, P, P, P, P, P, P, C.c_double, P, P, P, P]
        _lib.orc_loss_grad.restype = C.c_int
        _lib.orc_loss_grad_weighted.argtypes = [P, P, P, P, P, P, P, P, P, C.c_double, P, P, P, P]
        _lib.orc_loss_grad_weighted.restype = C.c_int
        _lib.orc_adam.argtypes = [C.c_int64, P, P, P, P, C.c_int64, C.c_double, C.c_double,
                                  C.c_double, C.c_double]
        _lib.orc_gauge_normalize.argtypes = [C.c_int32, P, P, C.c_int64, P, P, P]
        _lib.orc_epipolar_adjust.argtypes = [P, P, P, P, P, P, P, P, P, P, P, C.c_int32,
                                             C.c_int32, P, P, P]
        _lib.orc_epipolar_adjust.restype = C.c_int
        _lib.orc_default_options.argtypes = [P]
        _lib.orc_mlp_features.argtypes = [P] + [P] * 9 + [P]
        _lib.orc_mlp_features.restype = C.c_int
        _lib.orc_mlp_forward.argtypes = [C.c_int64, P, P, P]
        _lib.orc_mlp_bce_grad.argtypes = [C.c_int64, P, P, P, P]
        _lib.orc_mlp_bce_grad.restype = C.c_double
        _lib.orc_rel_trans.argtypes = [P, P, P, C.c_int32, P, C.c_double, P, P, P, P, P, P]
        _lib.orc_rel_trans.restype = C.c_int
        _lib.orc_ta_targets.argtypes = [C.c_int32, C.c_int64, P, P, P, P, P]
        _lib.orc_ta_targets.restype = C.c_int
        _lib.orc_ta_loss_grad.argtypes = [C.c_int32, C.c_int64, P, P, P, P, P, P]
        _lib.orc_ta_loss_grad.restype = C.c_double
        _lib.orc_ta_default_options.argtypes = [P]
        _lib.orc_ta_solve.argtypes = [C.c_int32, C.c_int64, P, P, P, C.c_int32, P, P, P, P, P,
                                      P, P, P]
        _lib.orc_ta_solve.restype = C.c_int
        _lib.orc_num_threads.restype = C.c_int
        _lib.orc_set_threads.argtypes = [C.c_int]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleProblem:
    """Holds contiguous copies of a scene's matches for the C oracle."""

    def __init__(self, x1, y1, x2, y2, cam1, cam2, cx, cy):
        self.x1 = np.ascontiguousarray(x1, np.float32)
        self.y1 = np.ascontiguousarray(y1, np.float32)
        self.x2 = np.ascontiguousarray(x2, np.float32)
        self.y2 = np.ascontiguousarray(y2, np.float32)
        self.cam1 = np.ascontiguousarray(cam1, np.int32)
        self.cam2 = np.ascontiguousarray(cam2, np.int32)
        self.cx = _f64(cx)
        self.cy = _f64(cy)
        self.n_cams = len(self.cx)
        self.s = Problem(len(self.x1), self.n_cams, _p(self.x1).value, _p(self.y1).value,
                         _p(self.x2).value, _p(self.y2).value, _p(self.cam1).value,
                         _p(self.cam2).value, _p(self.cx).value, _p(self.cy).value)

    @classmethod
    def from_scene(cls, sc, sel=None):
        if sel is None:
            return cls(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2, sc.cx, sc.cy)
        return cls(sc.x1[sel], sc.y1[sel], sc.x2[sel], sc.y2[sel], sc.cam1[sel],
                   sc.cam2[sel], sc.cx, sc.cy)

    @property
    def ref(self):
        return C.byref(self.s)

    @property
    def n_matches(self):
        return len(self.x1)


def default_options(**kw) -> Options:
    o = Options()
    lib().orc_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def segment(cam1, cam2, n_cams):
    cam1 = np.ascontiguousarray(cam1, np.int32)
    cam2 = np.ascontiguousarray(cam2, np.int32)
    n = len(cam1)
    perm = np.zeros(max(n, 1), np.int32)
    swapped = np.zeros(max(n, 1), np.uint8)
    pair_cams = np.zeros(2 * max(n, 1), np.int32)
    seg_off = np.zeros(max(n, 1) + 1, np.int64)
    npairs = C.c_int64(0)
    rc = lib().orc_segment(n, n_cams, _p(cam1), _p(cam2), _p(perm), _p(swapped),
                           _p(pair_cams), _p(seg_off), C.byref(npairs))
    if rc:
        raise ValueError("oracle segment rejected the matches")
    P = npairs.value
    return (perm[:n], swapped[:n].astype(bool), pair_cams[:2 * P].reshape(P, 2),
            seg_off[:P + 1])


def rot6d_to_R(a6):
    a6 = _f64(a6)
    R = np.zeros(9)
    lib().orc_rot6d_to_R(_p(a6), _p(R))
    return R.reshape(3, 3)


def R_to_rot6d(R):
    R = _f64(R)
    a6 = np.zeros(6)
    lib().orc_R_to_rot6d(_p(R), _p(a6))
    return a6


def rot6d_backward(a6, gR):
    a6, gR = _f64(a6), _f64(gR)
    g = np.zeros(6)
    lib().orc_rot6d_backward(_p(a6), _p(gR), _p(g))
    return g


def pair_F(Ri, ti, fi, Rj, tj, fj):
    F = np.zeros(9)
    Ri, ti, Rj, tj = _f64(Ri), _f64(ti), _f64(Rj), _f64(tj)
    if lib().orc_pair_F(_p(Ri), _p(ti), float(fi), _p(Rj), _p(tj), float(fj), _p(F)):
        raise ValueError("degenerate pair (t_ij = 0)")
    return F.reshape(3, 3)


def residuals(pb: OracleProblem, R, t, f):
    R, t, f = _f64(R), _f64(t), _f64(f)
    eps = np.zeros(max(pb.n_matches, 1))
    rc = lib().orc_residuals(pb.ref, _p(R), _p(t), _p(f), _p(eps))
    if rc:
        raise ValueError(f"oracle residuals failed ({rc})")
    return eps[:pb.n_matches]


def update_mask(pb: OracleProblem, Rh, th, fh, tau, mask):
    Rh, th, fh = _f64(Rh), _f64(th), _f64(fh)
    mask = np.ascontiguousarray(mask, np.uint8).copy()
    Z = lib().orc_update_mask(pb.ref, _p(Rh), _p(th), _p(fh), float(tau), _p(mask))
    if Z < 0:
        raise ValueError("oracle update_mask failed")
    return mask.astype(bool), int(Z)


def loss_grad(pb: OracleProblem, R, t, f, Rh=None, th=None, fh=None, mask=None,
              delta=1e-4, weights=None):
    """Loss and (dL/dR [N,3,3], dL/dt [N,3], dL/df [N]) at (R,t,f); with
    `weights` (one per match, input order) each match's IRLS factor is scaled
    by its weight and Z is the sum of the retained matches' weights."""
    N = pb.n_cams
    R, t, f = _f64(R), _f64(t), _f64(f)
    Rh = R if Rh is None else _f64(Rh)
    th = t if th is None else _f64(th)
    fh = f if fh is None else _f64(fh)
    if mask is None:
        mask = np.ones(pb.n_matches, np.uint8)
    mask = np.ascontiguousarray(mask, np.uint8)
    loss = C.c_double(0.0)
    gR = np.zeros(9 * N)
    gt = np.zeros(3 * N)
    gf = np.zeros(N)
    if weights is None:
        rc = lib().orc_loss_grad(pb.ref, _p(R), _p(t), _p(f), _p(Rh), _p(th), _p(fh), _p(mask),
                                 float(delta), C.byref(loss), _p(gR), _p(gt), _p(gf))
    else:
        w = _f64(weights)
        if w.shape != (pb.n_matches,):
            raise ValueError("one weight per match")
        rc = lib().orc_loss_grad_weighted(pb.ref, _p(R), _p(t), _p(f), _p(Rh), _p(th), _p(fh),
                                          _p(mask), _p(w), float(delta), C.byref(loss), _p(gR),
                                          _p(gt), _p(gf))
    if rc:
        raise ValueError(f"oracle loss_grad failed ({rc})")
    return loss.value, gR.reshape(N, 3, 3), gt.reshape(N, 3), gf


def adam(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-12):
    p, m, v, g = _f64(p).copy(), _f64(m).copy(), _f64(v).copy(), _f64(g)
    lib().orc_adam(len(p), _p(p), _p(m), _p(v), _p(g), int(step), lr, beta1, beta2, eps)
    return p, m, v


def gauge_normalize(R, t, pair_cams):
    """Centres to mean 0, median matched-pair baseline to 1."""
    R = _f64(R)
    t = _f64(t).copy()
    pc = np.ascontiguousarray(pair_cams, np.int32)
    center = np.zeros(3)
    scale = C.c_double(0.0)
    lib().orc_gauge_normalize(len(R), _p(R), _p(t), len(pc), _p(pc), _p(center),
                              C.byref(scale))
    return t, center, scale.value


def epipolar_adjust(pb: OracleProblem, R0, t0, f0, intr_group=None, options=None,
                    log_every=0, max_log=0):
    """Run the whole EA loop; returns dict with R, t, f, losses, inliers, logs."""
    N = pb.n_cams
    opt = options if options is not None else default_options()
    R0, t0, f0 = _f64(R0), _f64(t0), _f64(f0)
    ig = None if intr_group is None else np.ascontiguousarray(intr_group, np.int32)
    R = np.zeros(9 * N)
    t = np.zeros(3 * N)
    f = np.zeros(N)
    losses = np.zeros(max(opt.rounds, 1))
    inl = np.zeros(max(opt.rounds, 1), np.int64)
    logR = np.zeros((max(max_log, 1), N, 9)) if max_log > 0 else None
    nlog = C.c_int32(0)
    mask = np.zeros(max(pb.n_matches, 1), np.uint8)
    rc = lib().orc_epipolar_adjust(pb.ref, C.byref(opt), _p(R0), _p(t0), _p(f0), _p(ig),
                                   _p(R), _p(t), _p(f), _p(losses), _p(inl), log_every,
                                   max_log, _p(logR), C.byref(nlog), _p(mask))
    if rc:
        raise ValueError(f"oracle epipolar_adjust failed ({rc})")
    run = int(np.sum(inl[:opt.rounds] >= 0))  # rounds before an early exit
    out = dict(R=R.reshape(N, 3, 3), t=t.reshape(N, 3), f=f, loss=losses[:run],
               inliers=inl[:run], mask=mask[:pb.n_matches].astype(bool), rounds_run=run)
    if logR is not None:
        out["log_R"] = logR[:nlog.value].reshape(-1, N, 3, 3)
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


MLP_NFEAT = 8
MLP_HIDDEN = 64
MLP_NPARAM = 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1


def mlp_pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(w3),
                           np.ravel(b3)]).astype(np.float64)


def mlp_unpack(p):
    p = np.asarray(p)
    o = 0
    out = []
    for shape in ((64, 8), (64,), (64, 64), (64,), (64,), (1,)):
        k = int(np.prod(shape))
        out.append(p[o:o + k].reshape(shape))
        o += k
    return out


def mlp_features(pb: OracleProblem, snaps):
    """snaps: [(R, t, f)] for rounds r, r-1, r-2 (3 entries)."""
    args = []
    for R, t, f in snaps:
        args += [_f64(R), _f64(t), _f64(f)]
    feat = np.zeros((max(pb.n_matches, 1), MLP_NFEAT))
    if lib().orc_mlp_features(pb.ref, *[_p(a) for a in args], _p(feat)):
        raise ValueError("oracle mlp_features failed")
    return feat[:pb.n_matches]


def mlp_forward(feat, params):
    feat = _f64(feat)
    params = _f64(params)
    y = np.zeros(max(len(feat), 1))
    lib().orc_mlp_forward(len(feat), _p(feat), _p(params), _p(y))
    return y[:len(feat)]


def mlp_bce_grad(feat, target, params):
    feat, target, params = _f64(feat), _f64(target), _f64(params)
    g = np.zeros(MLP_NPARAM)
    loss = lib().orc_mlp_bce_grad(len(feat), _p(feat), _p(target), _p(params), _p(g))
    return loss, g


# ---- Global Translation -----------------------------------------------------

class TaOptions(C.Structure):
    _fields_ = [("iters_run", C.c_int32), ("iters_final", C.c_int32), ("lr", C.c_double),
                ("lr_final", C.c_double), ("lr_end_frac", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("adam_eps", C.c_double)]


def ta_default_options(**kw) -> TaOptions:
    o = TaOptions()
    lib().orc_ta_default_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def rel_trans(pb: OracleProblem, R, f, cand, scores=False, tau=np.inf):
    """Relative-translation candidate search (see orc_rel_trans); tau caps
    each match's |eps| (normalised units; inf: the plain mean).  Returns a
    dict with pair_cams [P,2], best [P], t_rel [P,3], vote [P] and, with
    scores=True, the mean capped |eps| of every candidate [P, K]."""
    _, _, pc, _ = segment(pb.cam1, pb.cam2, pb.n_cams)
    P = len(pc)
    cand = _f64(cand).reshape(-1, 3)
    K = len(cand)
    R = _f64(R).reshape(-1, 9)
    f = _f64(f)
    pair_cams = np.zeros((max(P, 1), 2), np.int32)
    sc = np.zeros((max(P, 1), K)) if scores else None
    best = np.zeros(max(P, 1), np.int32)
    t_rel = np.zeros((max(P, 1), 3))
    vote = np.zeros(max(P, 1), np.int64)
    n_pairs = C.c_int64(0)
    if lib().orc_rel_trans(pb.ref, _p(R), _p(f), K, _p(cand), float(tau), C.byref(n_pairs), _p(pair_cams),
                           _p(sc), _p(best), _p(t_rel), _p(vote)):
        raise ValueError("oracle rel_trans rejected its input")
    assert n_pairs.value == P
    out = dict(pair_cams=pair_cams[:P], best=best[:P], t_rel=t_rel[:P], vote=vote[:P])
    if scores:
        out["scores"] = sc[:P]
    return out


def ta_targets(n_cams, pair_cams, R, t_rel):
    pc = np.ascontiguousarray(pair_cams, np.int32).reshape(-1, 2)
    pi, pj = np.ascontiguousarray(pc[:, 0]), np.ascontiguousarray(pc[:, 1])
    t_rel = _f64(t_rel).reshape(-1, 3)
    tg = np.zeros((max(len(pc), 1), 3))
    if lib().orc_ta_targets(n_cams, len(pc), _p(pi), _p(pj), _p(_f64(R).reshape(-1, 9)),
                            _p(t_rel), _p(tg)):
        raise ValueError("oracle ta_targets rejected its input")
    return tg[:len(pc)]


def ta_loss_grad(pair_cams, target, o):
    pc = np.ascontiguousarray(pair_cams, np.int32).reshape(-1, 2)
    pi, pj = np.ascontiguousarray(pc[:, 0]), np.ascontiguousarray(pc[:, 1])
    o = _f64(o).reshape(-1, 3)
    g = np.zeros_like(o)
    pl = np.zeros(max(len(pc), 1))
    L = lib().orc_ta_loss_grad(len(o), len(pc), _p(pi), _p(pj), _p(_f64(target).reshape(-1, 3)),
                               _p(o), _p(g), _p(pl))
    return L, g, pl[:len(pc)]


def ta_solve(pair_cams, target, o_init, options=None):
    """Multiple-initialisation translation alignment (see orc_ta_solve).
    o_init [runs, N, 3]."""
    pc = np.ascontiguousarray(pair_cams, np.int32).reshape(-1, 2)
    pi, pj = np.ascontiguousarray(pc[:, 0]), np.ascontiguousarray(pc[:, 1])
    o_init = _f64(o_init)
    runs, N = o_init.shape[0], o_init.shape[1]
    opt = options if options is not None else ta_default_options()
    o = np.zeros((N, 3))
    run_o = np.zeros((runs, N, 3))
    cam_loss = np.zeros((runs, N))
    run_of_cam = np.zeros(N, np.int32)
    run_loss = np.zeros(runs)
    final = C.c_double(0.0)
    if lib().orc_ta_solve(N, len(pc), _p(pi), _p(pj), _p(_f64(target).reshape(-1, 3)), runs,
                          _p(o_init), C.byref(opt), _p(o), _p(run_o), _p(cam_loss),
                          _p(run_of_cam), _p(run_loss), C.byref(final)):
        raise ValueError("oracle ta_solve failed")
    return dict(o=o, run_o=run_o, cam_loss=cam_loss, run_of_cam=run_of_cam, run_loss=run_loss,
                final_loss=final.value)


# ---- Focal Length Estimation ---------------------------------------------------

def focal_vote(pair_cams, F, group, f_cur, cand_f, tau):
    """Focal-length vote (Method > Focal Length Estimation,
    Eq. fastmap-focal-vote), plain numpy.  For intrinsics group g and
    candidate f: v_g(f) = sum over the pairs touching g of
    exp((1 - s1/s2) / tau), s1 >= s2 the two largest singular values of
    E = K_j^T F K_i with K = diag(f, f, 1) in centred pixel coordinates; the
    cameras of group g take the candidate, the others their group's f_cur
    (reading: with one group for all cameras this is the paper's
    shared-intrinsics vote).  F [P, 3, 3] maps camera i's centred point to a
    line of camera j (p_j^T F p_i = 0).  Returns votes [G, K] and the best
    candidate per group (highest vote, ties: the lower index)."""
    pc = np.asarray(pair_cams).reshape(-1, 2)
    F = np.asarray(F, dtype=np.float64).reshape(-1, 3, 3)
    group = np.asarray(group)
    cand_f = np.asarray(cand_f, dtype=np.float64)
    f_cur = np.asarray(f_cur, dtype=np.float64)
    G = int(group.max()) + 1
    votes = np.zeros((G, len(cand_f)))
    gi, gj = group[pc[:, 0]], group[pc[:, 1]]
    for g in range(G):
        sel = np.nonzero((gi == g) | (gj == g))[0]
        if len(sel) == 0:
            continue
        for k, f in enumerate(cand_f):
            fi = np.where(gi[sel] == g, f, f_cur[gi[sel]])
            fj = np.where(gj[sel] == g, f, f_cur[gj[sel]])
            Ki = np.zeros((len(sel), 3, 3))
            Kj = np.zeros((len(sel), 3, 3))
            Ki[:, 0, 0] = Ki[:, 1, 1] = fi
            Kj[:, 0, 0] = Kj[:, 1, 1] = fj
            Ki[:, 2, 2] = Kj[:, 2, 2] = 1.0
            E = np.transpose(Kj, (0, 2, 1)) @ F[sel] @ Ki
            s = np.linalg.svd(E, compute_uv=False)
            ratio = np.where(s[:, 1] > 0, s[:, 0] / np.where(s[:, 1] > 0, s[:, 1], 1.0), np.inf)
            votes[g, k] = np.sum(np.exp((1.0 - ratio) / tau))
    best = cand_f[np.argmax(votes, axis=1)]  # argmax takes the first of equal maxima
    return votes, best


# ---- Global Rotation -----------------------------------------------------------

def geodesic(Ra, Rb):
    """d(Ra, Rb) = arccos((tr(Ra^T Rb) - 1) / 2), the argument clamped to
    [-1, 1] (Global Rotation; reading: clamp)."""
    x = (np.einsum("...ab,...ab->...", Ra, Rb) - 1.0) / 2.0
    return np.arccos(np.clip(x, -1.0, 1.0))


def ra_loss_grad(pair_cams, R_rel, a6):
    """Eq. fastmap-rotation-objective: L_R = (1/|P|) sum d(R_j, R^{i->j} R_i)
    over the pairs, R_i from the 6D parameters a6 [N, 6] (columns a1, a2;
    Gram-Schmidt).  Returns L_R and dL_R/da6 [N, 6].  The derivative of
    arccos is taken where its argument lies strictly inside (-1, 1) and is
    zero elsewhere (a pair already at distance 0 or pi)."""
    pc = np.asarray(pair_cams).reshape(-1, 2)
    a6 = _f64(a6).reshape(-1, 6)
    N, P = len(a6), len(pc)
    R = np.stack([rot6d_to_R(a6[k]) for k in range(N)])
    Rr = _f64(R_rel).reshape(-1, 3, 3)
    i, j = pc[:, 0], pc[:, 1]
    Ri_t = Rr @ R[i]  # the prediction of R_j
    x = (np.einsum("pab,pab->p", R[j], Ri_t) - 1.0) / 2.0
    L = np.sum(np.arccos(np.clip(x, -1.0, 1.0))) / P
    inside = np.abs(x) < 1.0
    dx = np.where(inside, -1.0 / np.sqrt(np.where(inside, 1.0 - x * x, 1.0)), 0.0) / P
    # tr(R_j^T R_rel R_i): d/dR_j = R_rel R_i, d/dR_i = R_rel^T R_j; x = (tr - 1)/2
    gR = np.zeros((N, 3, 3))
    np.add.at(gR, j, 0.5 * dx[:, None, None] * Ri_t)
    np.add.at(gR, i, 0.5 * dx[:, None, None] * (np.transpose(Rr, (0, 2, 1)) @ R[j]))
    g6 = np.stack([rot6d_backward(a6[k], gR[k].ravel()) for k in range(N)])
    return L, g6


def ra_init(pair_cams, R_rel, n_cams, details=False):
    """Initialisation (Global Rotation > Initialization details, after
    Martinec and Pajdla): the first columns c1 minimise
    sum |c1_j - R^{i->j} c1_i|^2 over unit-norm stacked vectors (the smallest
    eigenvector of the 3N x 3N normal matrix, numpy's eigh), each then
    normalised; the second columns minimise the same over the pairs / |P|
    plus sum (c1_i^T c2_i)^2 / |I|, then are normalised and made orthogonal
    to c1 (Gram-Schmidt); the third column is c1 x c2.  Returns a6 [N, 6]
    (c1, c2) and R [N, 3, 3]; with details also the second problem's raw
    solution [N, 3] (before the per-camera steps)."""
    pc = np.asarray(pair_cams).reshape(-1, 2)
    Rr = _f64(R_rel).reshape(-1, 3, 3)
    N, P = n_cams, len(pc)
    M = np.zeros((3 * N, 3 * N))
    for p, (i, j) in enumerate(pc):
        A = np.zeros((3, 3 * N))
        A[:, 3 * j:3 * j + 3] = np.eye(3)
        A[:, 3 * i:3 * i + 3] = -Rr[p]
        M += A.T @ A
    _, V = np.linalg.eigh(M)
    c1 = V[:, 0].reshape(N, 3)
    c1 /= np.linalg.norm(c1, axis=1, keepdims=True)
    B = np.zeros((3 * N, 3 * N))
    for k in range(N):
        B[3 * k:3 * k + 3, 3 * k:3 * k + 3] = np.outer(c1[k], c1[k])
    _, V2 = np.linalg.eigh(M / P + B / N)
    raw2 = V2[:, 0].reshape(N, 3).copy()
    c2 = raw2.copy()
    c2 -= np.sum(c1 * c2, axis=1, keepdims=True) * c1
    c2 /= np.linalg.norm(c2, axis=1, keepdims=True)
    a6 = np.concatenate([c1, c2], axis=1)
    R = np.stack([rot6d_to_R(a6[k]) for k in range(N)])
    return (a6, R, raw2) if details else (a6, R)


def ra_solve(pair_cams, R_rel, a6_0, iters=1000, lr=1e-2, lr_end_frac=1e-2, beta1=0.9, beta2=0.999,
             eps=1e-12):
    """Adam on the 6D parameters of L_R from a6_0 (reading: the learning rate
    of step k is lr * lr_end_frac^(k/iters)).  Returns a6, R and the loss."""
    a6 = _f64(a6_0).reshape(-1, 6).copy()
    m = np.zeros(a6.size)
    v = np.zeros(a6.size)
    for k in range(iters):
        _, g = ra_loss_grad(pair_cams, R_rel, a6)
        p, m, v = adam(a6.ravel(), m, v, g.ravel(), k + 1, lr * lr_end_frac ** (k / iters), beta1, beta2, eps)
        a6 = p.reshape(-1, 6)
    L, _ = ra_loss_grad(pair_cams, R_rel, a6)
    return a6, np.stack([rot6d_to_R(a6[k]) for k in range(len(a6))]), L
