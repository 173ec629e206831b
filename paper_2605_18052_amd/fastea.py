"""ctypes binding of libfastea (the C ABI declared in include/fastea.h).

Argument marshalling only: every step of epipolar adjustment runs in the HIP
kernels of the library.  The raw ``fea_*`` functions keep the C names; the
``Context`` class wraps them for numpy (host) and torch (device) arrays.
Loading fails loudly when the library has not been built -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastea.so")

FEA_OK, FEA_EINVAL, FEA_ENOMEM, FEA_EDEVICE, FEA_ESTATE, FEA_EDEGENERATE, FEA_ENONFINITE = (
    0, -1, -2, -3, -4, -5, -6)


class fea_options(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("iters_per_round", C.c_int32),
                ("tau_px_init", C.c_double), ("tau_px_min", C.c_double),
                ("tau_decay", C.c_double), ("delta", C.c_double), ("lr_rot", C.c_double),
                ("lr_t", C.c_double), ("lr_logf", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("adam_eps", C.c_double),
                ("optimize_focal", C.c_int32), ("gauge_normalize", C.c_int32),
                ("log_every", C.c_int32), ("max_log", C.c_int32),
                ("lr_decay", C.c_double), ("reset_moments", C.c_int32),
                ("tile_matches", C.c_int32), ("use_graphs", C.c_int32),
                ("weight_mode", C.c_int32), ("inner_loop", C.c_int32),
                ("tile_persistent", C.c_int32), ("persistent_steps", C.c_int32),
                ("wait_limit_us", C.c_int32),
                ("converge_deg", C.c_double)]


class fea_report(C.Structure):
    _fields_ = [("rounds_run", C.c_int32), ("iters_run", C.c_int32),
                ("inliers_per_round", C.c_int64 * 64), ("loss_per_round", C.c_double * 64),
                ("ms_total", C.c_double), ("n_logged", C.c_int32), ("fallbacks", C.c_int32),
                ("scenes_converged", C.c_int32), ("scenes_nonfinite", C.c_int32),
                ("reserved", C.c_int32 * 4)]


class fea_info(C.Structure):
    _fields_ = [("n_cams", C.c_int32), ("n_groups", C.c_int32), ("n_matches", C.c_int64),
                ("n_pairs", C.c_int64), ("n_retained", C.c_int64), ("n_items", C.c_int64),
                ("layout_matches", C.c_int64), ("round", C.c_int32), ("step", C.c_int32),
                ("gauge_center", C.c_double * 3), ("gauge_scale", C.c_double),
                ("tau", C.c_double), ("tile_matches", C.c_int32),
                ("tile_threads", C.c_int32), ("n_scenes", C.c_int32),
                ("tile_persistent", C.c_int32), ("quad_steps_blocks", C.c_int32),
                ("reserved", C.c_int32 * 3)]


class FeaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fastea error {status}: {msg}")
        self.status = status


_lib = None
_P = C.c_void_p
_SIGNATURES = {
    "fea_version": ([], C.c_int32),
    "fea_status_string": ([C.c_int], C.c_char_p),
    "fea_default_options": ([_P], C.c_int),
    "fea_check_options": ([_P, _P, C.c_size_t], C.c_int),
    "fea_create": ([_P, C.c_int32, _P, _P], C.c_int),
    "fea_destroy": ([_P], None),
    "fea_last_error": ([_P], C.c_char_p),
    "fea_set_options": ([_P, _P], C.c_int),
    "fea_load_intrinsics": ([_P, C.c_int32, _P, _P, _P, _P], C.c_int),
    "fea_set_scenes": ([_P, C.c_int32, _P], C.c_int),
    "fea_get_scene_stats": ([_P, _P, _P, _P, _P, _P], C.c_int),
    "fea_get_judge_losses": ([_P, _P, _P], C.c_int),
    "fea_get_scene_convergence": ([_P, _P, _P], C.c_int),
    "fea_get_scene_nonfinite": ([_P, _P], C.c_int),
    "fea_set_params_dev": ([_P, _P, _P, _P], C.c_int),
    "fea_batch_solve": ([C.c_int32, _P, _P, _P], C.c_int),
    "fea_set_mlp": ([_P, _P], C.c_int),
    "fea_mlp_features_dev": ([_P, _P, _P], C.c_int),
    "fea_get_learned_weights": ([_P, _P], C.c_int),
    "fea_mlp_train": ([C.c_int32, _P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_double, C.c_uint64, _P,
                       _P], C.c_int),
    "fea_mlp_grad": ([C.c_int32, _P, _P, C.c_int64, _P, _P, _P], C.c_int),
    "fea_mlp_grad_noalloc": ([C.c_int32, _P, _P, _P, C.c_int64, _P, _P, _P], C.c_int),
    "fea_load_matches": ([_P, C.c_int64, _P, _P, _P, _P, _P, _P], C.c_int),
    "fea_load_matches_device": ([_P, C.c_int64, _P, _P, _P, _P, _P, _P], C.c_int),
    "fea_init_poses": ([_P, _P, _P], C.c_int),
    "fea_set_poses": ([_P, _P, _P, _P], C.c_int),
    "fea_begin_round": ([_P, C.c_double], C.c_int),
    "fea_residual_grad": ([_P, _P, _P, _P, _P], C.c_int),
    "fea_step": ([_P, C.c_int32], C.c_int),
    "fea_get_params_dev": ([_P, _P, _P, _P], C.c_int),
    "fea_loss_dev": ([_P, _P, _P, _P, _P], C.c_int),
    "fea_adjoint_dev": ([_P, _P, _P, _P, _P, _P, _P, _P], C.c_int),
    "fea_epipolar_adjust": ([_P, _P], C.c_int),
    "fea_get_poses": ([_P, _P, _P, _P], C.c_int),
    "fea_get_segments": ([_P, _P, _P, _P, _P], C.c_int),
    "fea_get_mask": ([_P, _P, _P], C.c_int),
    "fea_get_info": ([_P, _P], C.c_int),
    "fea_get_state": ([_P, _P, _P], C.c_int),
    "fea_ablation": ([_P, C.c_int32, C.c_int32, _P, _P], C.c_int),
    "fea_set_state": ([_P, _P, C.c_size_t], C.c_int),
    "fea_synchronize": ([_P], C.c_int),
    "fea_get_tile_timings": ([_P, _P, C.c_int32, _P], C.c_int),
    "fea_get_stream": ([_P, _P], C.c_int),
    "fea_get_rotation_log": ([_P, _P, _P], C.c_int),
    "fea_set_kernel_timing": ([_P, C.c_int32], C.c_int),
    "fea_hbm_probe": ([C.c_int32, C.c_int64, C.c_int32, _P, _P], C.c_int),
    "fea_get_kernel_timing": ([_P, _P, _P], C.c_int),
    "fea_get_kernel_times": ([_P, _P, C.c_int64, _P], C.c_int),
    "fea_relative_translations": ([_P, _P, _P, C.c_double, C.c_int32, _P, _P, _P, _P, _P, _P, _P], C.c_int),
    "fea_ta_default_options": ([_P], C.c_int),
    "fea_ra_default_options": ([_P], C.c_int),
    "fea_rotation_averaging": ([_P, C.c_int32, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P], C.c_int),
    "fea_focal_vote": ([_P, C.c_int32, C.c_int64, _P, _P, _P, _P, _P, C.c_int32, _P, C.c_double, _P, _P, _P,
                        _P], C.c_int),
    "fea_translation_align": ([_P, C.c_int32, C.c_int64, _P, _P, _P, _P, C.c_int32, _P, _P, _P, _P, _P,
                               _P, _P, _P, _P], C.c_int),
}


class fea_ta_options(C.Structure):
    _fields_ = [("iters_run", C.c_int32), ("iters_final", C.c_int32), ("lr", C.c_double),
                ("lr_final", C.c_double), ("lr_end_frac", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("adam_eps", C.c_double)]


def lib():
    """Load libfastea.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_18052_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = res
        _lib = h
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


def hbm_probe(device=0, nbytes=1 << 30, reps=5):
    """(read GB/s, copy GB/s) of plain streaming kernels on `device`."""
    r = C.c_double(0.0)
    w = C.c_double(0.0)
    rc = lib().fea_hbm_probe(int(device), int(nbytes), int(reps), C.byref(r), C.byref(w))
    if rc != FEA_OK:
        raise FeaError(rc, lib().fea_status_string(rc).decode())
    return r.value, w.value


MLP_FEATURES = 8
MLP_PARAMS = 4801


def mlp_train(feat, target, params, epochs=3, batch=16384, lr=1e-3, seed=0, device=0):
    """Train in place on torch device tensors (feat [n,8] f32, target [n] f32,
    params [4801] f32); returns the mean loss per epoch."""
    import torch
    n = int(feat.shape[0])
    for x in (feat, target, params):
        if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
            raise ValueError("feat, target and params must be contiguous float32 CUDA tensors")
    losses = np.zeros(max(epochs, 1))
    torch.cuda.current_stream().synchronize()
    rc = lib().fea_mlp_train(int(device), C.c_void_p(feat.data_ptr()), C.c_void_p(target.data_ptr()),
                             n, int(epochs), int(batch), float(lr), int(seed),
                             C.c_void_p(params.data_ptr()), losses.ctypes.data_as(_P))
    if rc != FEA_OK:
        raise FeaError(rc, lib().fea_status_string(rc).decode())
    return losses[:epochs]


def mlp_grad(feat, target, params, device=0):
    """(mean BCE loss, gradient [4801] torch tensor) over all samples."""
    import torch
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feat.device)
    loss = C.c_double(0.0)
    torch.cuda.current_stream().synchronize()
    rc = lib().fea_mlp_grad(int(device), C.c_void_p(feat.data_ptr()), C.c_void_p(target.data_ptr()),
                            int(feat.shape[0]), C.c_void_p(params.data_ptr()),
                            C.c_void_p(grad.data_ptr()), C.byref(loss))
    if rc != FEA_OK:
        raise FeaError(rc, lib().fea_status_string(rc).decode())
    return loss.value, grad


class fea_ra_options(C.Structure):
    _fields_ = [("init_iters", C.c_int32), ("iters", C.c_int32), ("lr", C.c_double),
                ("lr_end_frac", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("adam_eps", C.c_double)]


def ra_default_options(**kw) -> fea_ra_options:
    o = fea_ra_options()
    lib().fea_ra_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def ta_default_options(**kw) -> fea_ta_options:
    o = fea_ta_options()
    lib().fea_ta_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def default_options(**kw) -> fea_options:
    o = fea_options()
    lib().fea_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _report(rep):
    r = rep.rounds_run
    return dict(rounds_run=r, iters_run=rep.iters_run,
                inliers=np.array(rep.inliers_per_round[:min(r, 64)]),
                loss=np.array(rep.loss_per_round[:min(r, 64)]), ms_total=rep.ms_total,
                n_logged=rep.n_logged, fallbacks=rep.fallbacks,
                scenes_converged=rep.scenes_converged, scenes_nonfinite=rep.scenes_nonfinite)


def batch_solve(contexts, options: fea_options | None = None):
    """fea_batch_solve over Context objects (each with one scene, poses
    initialised, all on one device): one batched solve, each context's poses
    then hold its result.  Returns one report dict per context."""
    n = len(contexts)
    arr = (C.c_void_p * n)(*[c._h.value for c in contexts])
    reps = (fea_report * n)()
    popt = C.byref(options) if options is not None else None
    rc = lib().fea_batch_solve(n, arr, popt, reps)
    if rc != FEA_OK:
        msg = lib().fea_last_error(contexts[0]._h).decode() if n else ""
        raise FeaError(rc, msg)
    return [_report(r) for r in reps]


def check_options(opt: fea_options):
    """(status, reason) of fea_check_options: whether a context would accept
    these options (needs no GPU)."""
    buf = C.create_string_buffer(256)
    rc = lib().fea_check_options(C.byref(opt), buf, len(buf))
    return rc, buf.value.decode()


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class Context:
    """One solver context on one GPU (wraps a fea_ctx*)."""

    def __init__(self, device: int = 0, options: fea_options | None = None, stream=None):
        self._h = C.c_void_p()
        opt = options if options is not None else default_options()
        st = C.c_void_p(stream) if stream else None
        rc = lib().fea_create(C.byref(self._h), int(device), C.byref(opt), st)
        if rc != FEA_OK:
            raise FeaError(rc, lib().fea_status_string(rc).decode())
        self.device = device
        self.n_cams = 0

    def _check(self, rc):
        if rc != FEA_OK:
            raise FeaError(rc, lib().fea_last_error(self._h).decode())

    def close(self):
        if self._h:
            lib().fea_destroy(self._h)
            self._h = C.c_void_p()
        self._tstream = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_options(self, options: fea_options):
        self._check(lib().fea_set_options(self._h, C.byref(options)))

    def load_intrinsics(self, f, cx, cy, groups=None):
        f, pf = _host(f, np.float64)
        cx, pcx = _host(cx, np.float64)
        cy, pcy = _host(cy, np.float64)
        pg = None
        if groups is not None:
            groups, pg = _host(groups, np.int32)
        self._check(lib().fea_load_intrinsics(self._h, len(f), pf, pcx, pcy, pg))
        self.n_cams = len(f)

    def set_scenes(self, cam_scene):
        cam_scene, p = _host(cam_scene, np.int32)
        self._check(lib().fea_set_scenes(self._h, int(cam_scene.max()) + 1, p))

    def scene_stats(self):
        S = self.info()["n_scenes"]
        loss = np.zeros(S)
        ret = np.zeros(S, np.int64)
        gc = np.zeros((S, 3))
        gs = np.zeros(S)
        lm = np.zeros(S, np.int32)
        self._check(lib().fea_get_scene_stats(self._h, loss.ctypes.data_as(_P), ret.ctypes.data_as(_P),
                                              gc.ctypes.data_as(_P), gs.ctypes.data_as(_P),
                                              lm.ctypes.data_as(_P)))
        return dict(loss=loss, retained=ret, gauge_center=gc, gauge_scale=gs, learned=lm)

    def judge_losses(self):
        """Per scene, the plain objective at the last learned round's snapshot
        and at its end, as the judge compared them (zeros before any)."""
        S = self.info()["n_scenes"]
        l0, l1 = np.zeros(S), np.zeros(S)
        self._check(lib().fea_get_judge_losses(self._h, l0.ctypes.data_as(_P), l1.ctypes.data_as(_P)))
        return l0, l1

    def scene_nonfinite(self):
        """Per scene: the round at whose start the non-finite guard stopped
        it (the number of rounds run if at the end of the solve), or -1."""
        S = self.info()["n_scenes"]
        out = np.zeros(S, dtype=np.int32)
        self._check(lib().fea_get_scene_nonfinite(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params_dev(self, a6, t, logf):
        """Replaces the parameters with float64 device tensors (a6 [N,6], t
        [N,3], logf [G]) in the context's gauge; ordered after torch's
        current stream, no host wait."""
        import torch
        cur = torch.cuda.current_stream(a6.device)
        ls = self.torch_stream()
        if ls.cuda_stream != cur.cuda_stream:
            ls.wait_stream(cur)
        self._check(lib().fea_set_params_dev(self._h, self._dev(a6), self._dev(t), self._dev(logf)))
        if ls.cuda_stream != cur.cuda_stream:
            cur.wait_stream(ls)

    def scene_convergence(self):
        """(round each scene converged at or -1 [S], mean camera rotation over
        the last round in degrees [S])."""
        S = self.info()["n_scenes"]
        rd = np.zeros(S, np.int32)
        ch = np.zeros(S)
        self._check(lib().fea_get_scene_convergence(self._h, rd.ctypes.data_as(_P), ch.ctypes.data_as(_P)))
        return rd, ch

    # -- learned inlier weights --
    def set_mlp(self, params):
        params, p = _host(params, np.float32)
        if params.size != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters")
        self._check(lib().fea_set_mlp(self._h, p))

    def mlp_features(self):
        """(features [layout,8], slot position [layout]) torch device tensors."""
        import torch
        L = self.info()["layout_matches"]
        dev = torch.device("cuda", self.device)
        feat = torch.empty(max(L, 1), MLP_FEATURES, dtype=torch.float32, device=dev)
        pos = torch.empty(max(L, 1), dtype=torch.int32, device=dev)
        torch.cuda.current_stream().synchronize()
        self._check(lib().fea_mlp_features_dev(self._h, self._dev(feat), self._dev(pos)))
        self.synchronize()
        return feat[:L], pos[:L]

    def learned_weights(self):
        M = self.info()["n_matches"]
        w = np.zeros(max(M, 1), np.float32)
        self._check(lib().fea_get_learned_weights(self._h, w.ctypes.data_as(_P)))
        return w[:M]

    def load_matches(self, x1, y1, x2, y2, cam1, cam2):
        if _is_torch(x1) and x1.is_cuda:
            import torch
            arrs = [x1, y1, x2, y2, cam1, cam2]
            dts = [torch.float32] * 4 + [torch.int32] * 2
            arrs = [a.to(dtype=d).contiguous() for a, d in zip(arrs, dts)]
            torch.cuda.current_stream().synchronize()
            ptrs = [C.c_void_p(a.data_ptr()) for a in arrs]
            self._check(lib().fea_load_matches_device(self._h, arrs[0].numel(), *ptrs))
            return
        keep = [_host(x1, np.float32), _host(y1, np.float32), _host(x2, np.float32),
                _host(y2, np.float32), _host(cam1, np.int32), _host(cam2, np.int32)]
        self._check(lib().fea_load_matches(self._h, len(keep[0][0]), *[p for _, p in keep]))

    def init_poses(self, R, t):
        R, pR = _host(R, np.float64)
        t, pt = _host(t, np.float64)
        self._check(lib().fea_init_poses(self._h, pR, pt))

    def set_poses(self, R, t, f=None):
        R, pR = _host(R, np.float64)
        t, pt = _host(t, np.float64)
        pf = None
        if f is not None:
            f, pf = _host(f, np.float64)
        self._check(lib().fea_set_poses(self._h, pR, pt, pf))

    def begin_round(self, tau_px=math.inf):
        self._check(lib().fea_begin_round(self._h, float(tau_px)))

    def residual_grad(self):
        """Loss and dL/dR [N,3,3], dL/dt [N,3], dL/df [N] as torch device tensors."""
        import torch
        N = self.n_cams
        dev = torch.device("cuda", self.device)
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        gR = torch.empty(N, 3, 3, dtype=torch.float64, device=dev)
        gt = torch.empty(N, 3, dtype=torch.float64, device=dev)
        gf = torch.empty(N, dtype=torch.float64, device=dev)
        torch.cuda.current_stream().synchronize()
        self._check(lib().fea_residual_grad(self._h, C.c_void_p(loss.data_ptr()),
                                            C.c_void_p(gR.data_ptr()), C.c_void_p(gt.data_ptr()),
                                            C.c_void_p(gf.data_ptr())))
        self.synchronize()
        return loss, gR, gt, gf

    # -- parameters as torch device tensors (autograd support) --
    def _dev(self, a):
        return C.c_void_p(a.data_ptr()) if a is not None else None

    def get_params(self):
        """(a6 [N,6], t [N,3], logf [G]) float64 torch tensors on the GPU."""
        import torch
        dev = torch.device("cuda", self.device)
        inf = self.info()
        a6 = torch.empty(inf["n_cams"], 6, dtype=torch.float64, device=dev)
        t = torch.empty(inf["n_cams"], 3, dtype=torch.float64, device=dev)
        logf = torch.empty(inf["n_groups"], dtype=torch.float64, device=dev)
        torch.cuda.current_stream().synchronize()
        self._check(lib().fea_get_params_dev(self._h, self._dev(a6), self._dev(t), self._dev(logf)))
        self.synchronize()
        return a6, t, logf

    def loss_dev(self, a6, t, logf, out):
        self._check(lib().fea_loss_dev(self._h, self._dev(a6), self._dev(t), self._dev(logf),
                                       self._dev(out)))

    def adjoint_dev(self, a6, t, logf, gout, ga6, gt, glogf):
        self._check(lib().fea_adjoint_dev(self._h, self._dev(a6), self._dev(t), self._dev(logf),
                                          self._dev(gout), self._dev(ga6), self._dev(gt),
                                          self._dev(glogf)))

    def step(self, n=1):
        self._check(lib().fea_step(self._h, int(n)))

    def synchronize(self):
        self._check(lib().fea_synchronize(self._h))

    def tile_timings(self):
        """The autotuner's mean per-pass time (ms) of each candidate shape at
        its last tuning on this context (empty if none was timed)."""
        n = C.c_int32(0)
        ms = np.zeros(64, dtype=np.float32)
        self._check(lib().fea_get_tile_timings(self._h, ms.ctypes.data_as(_P), 64, C.byref(n)))
        return ms[:n.value].copy()

    def stream_handle(self) -> int:
        """The context's hipStream_t as an integer."""
        h = C.c_void_p()
        self._check(lib().fea_get_stream(self._h, C.byref(h)))
        return int(h.value or 0)

    def torch_stream(self):
        """The context's stream as a torch stream object (for event ordering
        against torch's streams); the context keeps ownership."""
        import torch
        if getattr(self, "_tstream", None) is None:
            self._tstream = torch.cuda.ExternalStream(self.stream_handle(),
                                                      device=torch.device("cuda", self.device))
        return self._tstream

    def epipolar_adjust(self):
        """Runs the solve; returns its report.  If the non-finite guard
        stopped a scene, raises FeaError(FEA_ENONFINITE) whose `report`
        attribute holds the report (the other scenes ran to the end)."""
        rep = fea_report()
        rc = lib().fea_epipolar_adjust(self._h, C.byref(rep))
        if rc == FEA_ENONFINITE:
            err = FeaError(rc, lib().fea_last_error(self._h).decode())
            err.report = _report(rep)
            raise err
        self._check(rc)
        return _report(rep)

    def get_poses(self):
        N = self.n_cams
        R = np.zeros((N, 3, 3))
        t = np.zeros((N, 3))
        f = np.zeros(N)
        self._check(lib().fea_get_poses(self._h, R.ctypes.data_as(_P), t.ctypes.data_as(_P),
                                        f.ctypes.data_as(_P)))
        return R, t, f

    def relative_translations(self, R, cand, f=None, tau_px=math.inf, scores=False, timing=False):
        """Relative-translation candidate search over the loaded matches (see
        fea_relative_translations).  R [N,3,3], cand [K,3] unit vectors,
        tau_px the cap of each match's error in pixels (inf: plain mean).
        Returns t_rel [P,3], best [P], vote [P], score_best [P], optionally
        scores [P,K] (float32) and score_ms."""
        R, pR = _host(np.asarray(R).reshape(-1, 9), np.float64)
        cand, pc = _host(np.asarray(cand).reshape(-1, 3), np.float64)
        pf = None
        if f is not None:
            f, pf = _host(f, np.float64)
        P = self.info()["n_pairs"]
        t_rel = np.zeros((max(P, 1), 3))
        best = np.zeros(max(P, 1), np.int32)
        vote = np.zeros(max(P, 1), np.int32)
        sb = np.zeros(max(P, 1))
        sc = np.zeros((max(P, 1), len(cand)), np.float32) if scores else None
        ms = C.c_float(0.0)
        self._check(lib().fea_relative_translations(
            self._h, pR, pf, float(tau_px), len(cand), pc, t_rel.ctypes.data_as(_P), best.ctypes.data_as(_P),
            vote.ctypes.data_as(_P), sb.ctypes.data_as(_P),
            sc.ctypes.data_as(_P) if scores else None, C.byref(ms) if timing else None))
        out = dict(t_rel=t_rel[:P], best=best[:P], vote=vote[:P], score_best=sb[:P])
        if scores:
            out["scores"] = sc[:P]
        if timing:
            out["score_ms"] = ms.value
        return out

    def translation_align(self, pair_cams, R, t_rel, o_init, options=None, details=False):
        """Camera centres from unit relative translations with multiple random
        initialisations (see fea_translation_align).  pair_cams [P,2],
        R [N,3,3], t_rel [P,3], o_init [runs,N,3]."""
        pc = np.ascontiguousarray(np.asarray(pair_cams).reshape(-1, 2), np.int32)
        pi, ppi = _host(pc[:, 0], np.int32)
        pj, ppj = _host(pc[:, 1], np.int32)
        R, pR = _host(np.asarray(R).reshape(-1, 9), np.float64)
        t_rel, pt = _host(np.asarray(t_rel).reshape(-1, 3), np.float64)
        o_init, po = _host(o_init, np.float64)
        runs, N = o_init.shape[0], o_init.shape[1]
        opt = options if options is not None else ta_default_options()
        o = np.zeros((N, 3))
        run_of_cam = np.zeros(N, np.int32)
        run_loss = np.zeros(runs)
        final = C.c_double(0.0)
        run_o = np.zeros((runs, N, 3)) if details else None
        cam_loss = np.zeros((runs, N)) if details else None
        ms = C.c_float(0.0)
        self._check(lib().fea_translation_align(
            self._h, N, len(pc), ppi, ppj, pR, pt, runs, po, C.byref(opt), o.ctypes.data_as(_P),
            run_of_cam.ctypes.data_as(_P), run_loss.ctypes.data_as(_P), C.byref(final),
            run_o.ctypes.data_as(_P) if details else None,
            cam_loss.ctypes.data_as(_P) if details else None, C.byref(ms)))
        out = dict(o=o, run_of_cam=run_of_cam, run_loss=run_loss, final_loss=final.value, ms=ms.value)
        if details:
            out.update(run_o=run_o, cam_loss=cam_loss)
        return out

    def rotation_averaging(self, n_cams, pair_cams, R_rel, v0=None, a6_init=None, options=None):
        """Global rotations from relative rotations (see
        fea_rotation_averaging).  pair_cams [P,2], R_rel [P,3,3] with
        R_j ~ R_rel R_i, v0 [2,N,3] random start vectors of the
        initialisation, or a6_init [N,6] to start the optimisation there."""
        pc = np.ascontiguousarray(np.asarray(pair_cams).reshape(-1, 2), np.int32)
        pi, ppi = _host(pc[:, 0], np.int32)
        pj, ppj = _host(pc[:, 1], np.int32)
        Rr, pR = _host(np.asarray(R_rel).reshape(-1, 9), np.float64)
        pv = pa = None
        if v0 is not None:
            v0, pv = _host(np.asarray(v0).reshape(-1), np.float64)
        if a6_init is not None:
            a6_init, pa = _host(np.asarray(a6_init).reshape(-1), np.float64)
        opt = options if options is not None else ra_default_options()
        R = np.zeros((n_cams, 3, 3))
        R0 = np.zeros((n_cams, 3, 3))
        loss = np.zeros(2)
        ms = C.c_float(0.0)
        self._check(lib().fea_rotation_averaging(self._h, int(n_cams), len(pc), ppi, ppj, pR, pv, pa, C.byref(opt),
                                                 R.ctypes.data_as(_P), R0.ctypes.data_as(_P),
                                                 loss.ctypes.data_as(_P), C.byref(ms)))
        return dict(R=R, R_init=R0, loss_init=loss[0], loss=loss[1], ms=ms.value)

    def focal_vote(self, n_cams, pair_cams, F, cand_f, tau, group=None, f_cur=None, votes=False):
        """Focal-length vote (see fea_focal_vote).  pair_cams [P,2], F [P,3,3]
        in centred pixel coordinates, cand_f [K]; group [N] (None: one group),
        f_cur [G].  Returns f_best [G], k_best [G], optionally votes [G,K], and
        the vote kernel's ms."""
        pc = np.ascontiguousarray(np.asarray(pair_cams).reshape(-1, 2), np.int32)
        pi, ppi = _host(pc[:, 0], np.int32)
        pj, ppj = _host(pc[:, 1], np.int32)
        F, pF = _host(np.asarray(F).reshape(-1, 9), np.float64)
        cand, pc_ = _host(cand_f, np.float64)
        pg = pfc = None
        G = 1
        if group is not None:
            group, pg = _host(group, np.int32)
            G = int(group.max()) + 1
        if f_cur is not None:
            f_cur, pfc = _host(f_cur, np.float64)
        fb = np.zeros(G)
        kb = np.zeros(G, np.int32)
        v = np.zeros((G, len(cand))) if votes else None
        ms = C.c_float(0.0)
        self._check(lib().fea_focal_vote(self._h, int(n_cams), len(pc), ppi, ppj, pF, pg, pfc, len(cand), pc_,
                                         float(tau), fb.ctypes.data_as(_P), kb.ctypes.data_as(_P),
                                         v.ctypes.data_as(_P) if votes else None, C.byref(ms)))
        out = dict(f_best=fb, k_best=kb, ms=ms.value)
        if votes:
            out["votes"] = v
        return out

    def info(self) -> dict:
        i = fea_info()
        self._check(lib().fea_get_info(self._h, C.byref(i)))
        return {k: (list(getattr(i, k)) if k == "gauge_center" else getattr(i, k))
                for k, _ in fea_info._fields_ if k != "reserved"}

    def get_segments(self):
        inf = self.info()
        M, P = inf["n_matches"], inf["n_pairs"]
        perm = np.zeros(max(M, 1), np.int32)
        sw = np.zeros(max(M, 1), np.uint8)
        pc = np.zeros(2 * max(P, 1), np.int32)
        so = np.zeros(P + 1, np.int64)
        self._check(lib().fea_get_segments(self._h, perm.ctypes.data_as(_P), sw.ctypes.data_as(_P),
                                           pc.ctypes.data_as(_P), so.ctypes.data_as(_P)))
        return perm[:M], sw[:M].astype(bool), pc[:2 * P].reshape(P, 2), so

    def get_mask(self):
        M = self.info()["n_matches"]
        mask = np.zeros(max(M, 1), np.uint8)
        z = C.c_int64(0)
        self._check(lib().fea_get_mask(self._h, mask.ctypes.data_as(_P), C.byref(z)))
        return mask[:M].astype(bool), z.value

    def ablation(self, variant, reps=5):
        """(mean ms per pass, per-pair sums [P, 10]) of ablation `variant`."""
        P = self.info()["n_pairs"]
        ms = C.c_double(0.0)
        sums = np.zeros((max(P, 1), 10), np.float32)
        self._check(lib().fea_ablation(self._h, int(variant), int(reps), C.byref(ms),
                                       sums.ctypes.data_as(_P)))
        return ms.value, sums[:P]

    def get_state(self):
        """Checkpoint of the solver state (bytes)."""
        n = C.c_size_t(0)
        self._check(lib().fea_get_state(self._h, None, C.byref(n)))
        buf = np.zeros(n.value, np.uint8)
        self._check(lib().fea_get_state(self._h, buf.ctypes.data_as(_P), C.byref(n)))
        return buf.tobytes()

    def set_state(self, state):
        buf = np.frombuffer(state, np.uint8)
        self._check(lib().fea_set_state(self._h, buf.ctypes.data_as(_P), len(buf)))

    def set_kernel_timing(self, enable=True):
        self._check(lib().fea_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_timing(self):
        """(summed ms, launches) of the timed per-match kernel launches."""
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(lib().fea_get_kernel_timing(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def kernel_times(self):
        """Per-launch durations (ms, launch order) of the timed per-match kernel launches."""
        n = C.c_int64(0)
        self._check(lib().fea_get_kernel_times(self._h, None, 0, C.byref(n)))
        out = np.zeros(max(n.value, 1), np.float32)
        self._check(lib().fea_get_kernel_times(self._h, out.ctypes.data_as(_P), n.value, C.byref(n)))
        return out[:n.value].astype(np.float64)

    def get_rotation_log(self, max_log):
        N = self.n_cams
        buf = np.zeros((max(max_log, 1), N, 3, 3))
        n = C.c_int32(0)
        self._check(lib().fea_get_rotation_log(self._h, buf.ctypes.data_as(_P), C.byref(n)))
        return buf[:n.value]
