"""Benchmark: one epipolar-adjustment step of FastMap on one MI355X.

A step is one pass of the whole hot path over the retained matches of the
first IRLS round: the fused residual / IRLS-weight / dL/dF kernel over every
match, the per-camera adjoint and Adam update, and the pose table of the next
step.  The default workload is the 3,000-camera trajectory scene (1M points,
30 nearest neighbours, ~100M matches, sigma 1 px, 25% outliers, unknown focal
lengths in [400, 1200] px): 1.4 GB of retained coordinates per pass, 5.5x the
256 MB Infinity Cache, so the pass streams from HBM.  It is generated
synthetically and resident in HBM before timing; `--workload traj500_m20M`
times the 500-camera, ~20M-match scene instead.

Prints ONE JSON line on stdout (progress goes to stderr):
  value       retained matches processed per second (whole job = 1 GPU), from
              the timed steps as the library runs them (runs of 10 steps
              replayed as HIP graphs)
  roofline    the per-match kernel: algorithmic bytes (16 B/match) / its
              mean HIP-event duration over a second, per-dispatch-timed run of
              the same steps, against the 8 TB/s HBM peak
  cpu_baseline the FP64 oracle timed on the host on a 6M-match sample
  solve       wall time until the mean rotation error first drops to <= 1 deg
              on the held-out learned-weight scenes (1,000 cameras, ~30M
              matches, 30% outliers): the per-match inner loop, the pairs'
              quadratic forms, and learned weights with the quadratic forms
  batch       64 uneven scenes (~120M matches) solved in one context against
              one after another, with per-scene early exit and convergence
  translation the stages before the adjustment on the first held-out scene:
              the focal-length vote and global rotation on its pair graph,
              the relative-translation candidate search over its matches (the
              scoring kernel against its roofline) and the multi-start
              camera-centre alignment on a 500-camera object-centric pair
              graph, each with the oracle timed beside it
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "residual+grad matches/s and HBM GB/s vs peak; wall time to ≤1° mean rot error"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense fp32 matrix-core peak of the MI355X
# VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
BYTES_PER_MATCH = 16  # x1, y1, x2, y2 as fp32: the algorithmic minimum per match
SETTLE_S = 0.3  # untimed device work before the timed steps, seconds
# per-scene early exit of the batched solves: a scene whose cameras rotate by
# less than this many degrees on average over a round at the threshold floor
# stops
BATCH_CONVERGE_DEG = 0.01

# HBM bytes per launch of the per-match kernel at round 0 of each workload,
# from two rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE; KiB per dispatch
# scaled by what the same counters read for a 1 GiB plain copy: x2.0, x1.0),
# summarised in profiles/k_resgrad_traj3000_m100M_hbm_traffic.md.  They hold
# only for the kernel source they were taken on (hashed below) and are keyed
# by the retained-match count and the work-item shape, which the autotuner
# may pick differently per run.
# The sources that define the kernel's device code (its file, the device
# helpers and the layout constants; the host-side context is not hashed).
KERNEL_SOURCES = ("paper_2605_18052_amd/csrc/fea_resgrad.hip", "paper_2605_18052_amd/csrc/fea_device.h",
                  "paper_2605_18052_amd/csrc/fea_layout.h")
PMC_TRAFFIC = {
    "sources_sha256": "0da24db5ded85a54879b5459a4eb845c5d1291db8ce787a3be8fa4edbe0aa79d",
    # retained matches per launch -> "matches x threads" -> fetched + written bytes
    "bytes_per_launch": {
        87275962: {  # traj3000_m100M, round 0
            "2048x256": 1448063047, "1024x256": 1484844646,
        },
    },
}


def measured_traffic(tile, Z):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != PMC_TRAFFIC["sources_sha256"]:
        return None
    return PMC_TRAFFIC["bytes_per_launch"].get(Z, {}).get(tile)


WORKLOADS = {
    "traj500_m20M": ("500 cameras, 200k points, 20-NN pairs, ~20M matches, sigma 1 px, 20% outliers, "
                     "f in [400,1200] px", "config2", 20_000_000),
    "traj3000_m100M": ("3,000 cameras, 1M points, 30-NN pairs, ~100M matches, sigma 1 px, 25% outliers, "
                       "f in [400,1200] px", "config3", 100_000_000),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="traj3000_m100M",
                    help="scene the step is timed on (the 100M-match scene streams 1.4 GB per pass, "
                         "far beyond the 256 MB Infinity Cache)")
    ap.add_argument("--matches", type=int, default=0, help="target match count (0: the workload's own)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-1-degree solves")
    ap.add_argument("--solve-seeds", default="5100,5101,5102",
                    help="seeds of the held-out learned-weight scenes the solves run on")
    ap.add_argument("--solve-per-match-seeds", type=int, default=1,
                    help="how many of those scenes also run the per-match inner loop")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-scene batch (batched against one after another)")
    ap.add_argument("--no-translation", action="store_true",
                    help="skip the relative-translation search and camera-centre alignment")
    ap.add_argument("--candidates", type=int, default=2048,
                    help="candidate directions of the relative-translation search")
    ap.add_argument("--search-cap-px", type=float, default=8.0,
                    help="cap of each match's error in the search, pixels (inf: the plain mean)")
    ap.add_argument("--search-cpu-pairs", type=int, default=400,
                    help="pairs of the scene the CPU oracle searches for its baseline")
    ap.add_argument("--cpu-sample", type=int, default=6_000_000)
    ap.add_argument("--cpu-iters", type=int, default=200)
    ap.add_argument("--ablation", action="store_true",
                    help="also time the per-match pass with each design choice taken back")
    ap.add_argument("--tile-matches", type=int, default=0,
                    help="matches per work item of the per-match kernel (0: the autotuner picks)")
    ap.add_argument("--tile-persistent", type=int, default=0,
                    help="with --tile-matches: 1 for the persistent launch of that item size")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    return ap.parse_args()


def cpu_baseline(sc, n_sample, iters):
    """The FP64 oracle, timed as it stands, on a random sample of matches."""
    import oracle
    oracle.build(force=False)
    rng = np.random.default_rng(12345)
    sel = np.sort(rng.choice(sc.n_matches, size=min(n_sample, sc.n_matches), replace=False))
    pb = oracle.OracleProblem.from_scene(sc, sel)
    opt = oracle.default_options(rounds=1, iters_per_round=iters,
                                 tau_px_init=oracle.default_options().tau_px_init)
    t0 = time.perf_counter()
    oracle.epipolar_adjust(pb, sc.R_init, sc.t_init, sc.f_init, options=opt)
    dt = time.perf_counter() - t0
    # the same on one host thread, on a tenth of the sample and a fifth of the steps
    threads = oracle.num_threads()
    sel1 = sel[: max(len(sel) // 10, 1)]
    pb1 = oracle.OracleProblem.from_scene(sc, sel1)
    opt1 = oracle.default_options(rounds=1, iters_per_round=max(iters // 5, 1),
                                  tau_px_init=oracle.default_options().tau_px_init)
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.epipolar_adjust(pb1, sc.R_init, sc.t_init, sc.f_init, options=opt1)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": pb.n_matches * iters / dt, "unit": "matches/s",
            "cores": threads, "cpu_model": model, "kind": "oracle",
            "value_1thread": pb1.n_matches * opt1.iters_per_round / dt1,
            "sample": f"{pb.n_matches} random matches of the same scene, 1 round x {iters} "
                      f"steps of the FP64 C oracle incl. its one-time segmenting, "
                      f"{dt:.1f} s wall on {threads} threads; value_1thread: "
                      f"{pb1.n_matches} matches x {opt1.iters_per_round} steps on one thread, {dt1:.1f} s"}


def time_to_one_degree(sc, fastea, metrics, every=10, **options):
    """Wall time of fea_epipolar_adjust from the initial poses until the mean
    rotation error is <= 1 deg.  A first solve keeps every `every`-th step's
    rotations in the device-side log (ground truth never enters the solver;
    errors are computed afterwards); a second, fresh solve runs the rounds up
    to the one containing the first logged step at <= 1 deg and is timed,
    with nothing read back until it returns."""
    mlp = options.pop("mlp", None)

    def setup(**extra):
        opt = fastea.default_options(**{**options, **extra})
        ctx = fastea.Context(0, opt)
        ctx.load_intrinsics(sc.f_init, sc.cx, sc.cy)
        ctx.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
        if mlp is not None:
            ctx.set_mlp(mlp)
        ctx.init_poses(sc.R_init, sc.t_init)
        ctx.synchronize()
        return ctx, opt

    base = fastea.default_options(**options)
    total_iters = base.rounds * base.iters_per_round
    ctx, opt = setup(log_every=every, max_log=max(total_iters // every, 1))
    t0 = time.perf_counter()
    rep = ctx.epipolar_adjust()
    ctx.synchronize()
    full = time.perf_counter() - t0
    log_R = ctx.get_rotation_log(total_iters // every)
    ctx.close()
    errs = [metrics.mean_rotation_error_deg(R, sc.R_gt) for R in log_R]
    k = next((i for i, e in enumerate(errs) if e <= 1.0), None)
    out = {"wall_to_1deg_s": None, "iters_to_1deg": None, "rounds_timed": None,
           "init_rot_err_deg": round(metrics.mean_rotation_error_deg(sc.R_init, sc.R_gt), 4),
           "final_rot_err_deg": round(errs[-1], 4) if errs else None,
           "solve_wall_s": round(full, 4), "iters": total_iters, "judge_fallbacks": rep["fallbacks"],
           "note": f"fea_epipolar_adjust; rotations logged on the device every {every} steps; the "
                   "timed solve runs whole rounds up to the first logged step at <= 1 deg"}
    if k is not None:
        n = (k + 1) * every
        rounds = -(-n // base.iters_per_round)
        ctx, opt = setup(rounds=rounds)
        t0 = time.perf_counter()
        ctx.epipolar_adjust()
        ctx.synchronize()
        out["wall_to_1deg_s"] = round(time.perf_counter() - t0, 4)
        out["iters_to_1deg"] = n
        out["rounds_timed"] = rounds
        ctx.close()
    return out


def batched_vs_sequential(scenes, fastea, metrics, synth, sequential=True, **options):
    """Independent scenes of uneven size solved in one context (every kernel
    launch covers all scenes, steps replayed as HIP graphs, a scene that has
    converged takes no further steps) against the same scenes solved one
    after another with the same options.  Loading and segmenting are outside
    the timed regions; per-scene convergence and final rotation error are
    reported."""
    cat, cam_scene, offs = synth.concat_scenes(scenes)
    mlp = options.pop("mlp", None)
    ctx = fastea.Context(0, fastea.default_options(**options))
    ctx.load_intrinsics(cat["f_init"], cat["cx"], cat["cy"])
    ctx.set_scenes(cam_scene)
    if mlp is not None:
        ctx.set_mlp(mlp)
    ctx.load_matches(cat["x1"], cat["y1"], cat["x2"], cat["y2"], cat["cam1"], cat["cam2"])
    ctx.init_poses(cat["R_init"], cat["t_init"])
    ctx.synchronize()
    t1 = time.perf_counter()
    rep = ctx.epipolar_adjust()
    ctx.synchronize()
    batched = time.perf_counter() - t1
    R, _, _ = ctx.get_poses()
    done, _ = ctx.scene_convergence()
    learned_scenes = int(sum(ctx.scene_stats()["learned"])) if mlp is not None else None
    ctx.close()
    per_scene = [metrics.mean_rotation_error_deg(R[offs[k]:offs[k + 1]], sc.R_gt)
                 for k, sc in enumerate(scenes)]
    seq, seq_err = (0.0, []) if sequential else (None, None)
    for sc in (scenes if sequential else []):
        c = fastea.Context(0, fastea.default_options(**options))
        c.load_intrinsics(sc.f_init, sc.cx, sc.cy)
        if mlp is not None:
            c.set_mlp(mlp)
        c.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
        c.init_poses(sc.R_init, sc.t_init)
        c.synchronize()
        t1 = time.perf_counter()
        c.epipolar_adjust()
        c.synchronize()
        seq += time.perf_counter() - t1
        Rs, _, _ = c.get_poses()
        seq_err.append(metrics.mean_rotation_error_deg(Rs, sc.R_gt))
        c.close()
    rounds = fastea.default_options(**options).rounds
    return {"scenes": len(scenes), "matches": int(sum(s.n_matches for s in scenes)),
            "batched_s": round(batched, 4), "sequential_s": None if seq is None else round(seq, 4),
            "speedup": None if not seq else round(seq / batched, 2),
            "rounds_run": rep["rounds_run"], "scenes_converged": rep["scenes_converged"],
            "per_scene_rounds": [int(d) if d >= 0 else rounds for d in done],
            "learned_scenes_at_end": learned_scenes,
            "judge_fallbacks": rep["fallbacks"] if mlp is not None else None,
            "per_scene_final_rot_err_deg": [round(e, 3) for e in per_scene],
            "scenes_at_or_below_1deg": int(sum(e <= 1.0 for e in per_scene)),
            "sequential_scenes_at_or_below_1deg": None if seq_err is None else int(sum(e <= 1.0 for e in seq_err)),
            "options": ({**options, "weight_mode": "learned"} if mlp is not None else options) or "defaults"}


def translation_stages(sc, fastea, synth, n_cand, with_cpu, cap_px=8.0, cpu_pairs=400, reps=5):
    """Relative-translation search over the scene's matches (the true
    rotations and focal lengths are its inputs, so that the stage is judged
    on its own; global rotation and the focal vote are timed beside it from
    their own perturbed starts; each match's error capped at cap_px) and
    camera-centre alignment (2 random starts, default schedule) on a
    500-camera object graph (pairs within 60 degrees, true directions with 2
    degrees of noise)."""
    from paper_2605_18052_amd import metrics
    cand = synth.sphere_candidates(n_cand)
    ctx = fastea.Context(0)
    ctx.load_intrinsics(sc.f_init, sc.cx, sc.cy)
    ctx.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
    ctx.relative_translations(sc.R_gt, cand, f=sc.f_gt, tau_px=cap_px)
    ms, walls = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = ctx.relative_translations(sc.R_gt, cand, f=sc.f_gt, tau_px=cap_px, timing=True)
        walls.append(time.perf_counter() - t0)
        ms.append(r["score_ms"])
    _, _, pc, _ = ctx.get_segments()
    ctx.close()
    gt = synth.relative_translations_gt(sc, pc)
    ang = np.degrees(np.arccos(np.clip(np.sum(r["t_rel"] * gt, axis=1), -1.0, 1.0)))
    k_ms = float(np.mean(ms))
    flop = 6.0 * sc.n_matches * n_cand  # 3 multiply-adds per (candidate, match)
    achieved = flop / (k_ms / 1e3) / 1e12
    cm_rate = sc.n_matches * n_cand / (k_ms / 1e3)
    mfma = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_MFMA_PEAK_TFLOPS, "traffic": None, "flop_per_launch": flop,
            "note": "6 flop per (candidate, match); the fp32 16x16x4 matrix instruction spends a fourth "
                    "depth slot on zero padding, so the reachable fraction is 0.75"}
    if math.isfinite(cap_px):
        # capped score: per (candidate, match) one v_min_f32 and one v_add_f32 lane operation
        peak_cm = VALU_LANE_OPS_PER_S / 2
        roof = {"bound": "alu", "achieved": cm_rate / 1e12, "peak": peak_cm / 1e12,
                "unit": "T candidate-matches/s", "frac": cm_rate / peak_cm, "traffic": None,
                "note": "two VALU lane operations per (candidate, match), the cap and the sum, against "
                        "256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz; the matrix-core products run beside them",
                "mfma": mfma}
    else:
        roof = mfma
    search = {
        "candidates": n_cand, "pairs": int(len(pc)), "matches": sc.n_matches,
        "cap_px": cap_px if math.isfinite(cap_px) else None,
        "kernel": "k_rt_score", "kernel_ms": k_ms, "kernel_ms_all": [round(x, 4) for x in ms],
        "call_ms": 1e3 * float(np.median(walls)),
        "candidate_matches_per_s": cm_rate,
        "roofline": roof,
        "direction_error_deg_median": float(np.median(ang)),
        "sign_correct": float(np.mean(ang < 90.0)),
    }
    pcg, R, tij, c = synth.object_pair_graph(500, 60.0, 0)
    rng = np.random.default_rng(1)
    tn = tij + np.deg2rad(2.0) * rng.normal(size=tij.shape) / np.sqrt(3.0)
    init = synth.random_centres(7, 2, len(c))
    actx = fastea.Context(0)
    actx.translation_align(pcg, R, tn, init)
    a_ms = []
    for _ in range(reps):
        a = actx.translation_align(pcg, R, tn, init)
        a_ms.append(a["ms"])
    actx.close()
    truth = c - c.mean(0)
    truth /= np.linalg.norm(truth, axis=1).mean()
    opts = fastea.ta_default_options()
    steps = opts.iters_run + opts.iters_final
    align = {"cameras": len(c), "pairs": int(len(pcg)), "runs": 2, "steps_per_run": opts.iters_run,
             "final_steps": opts.iters_final, "ms": float(np.median(a_ms)),
             "us_per_step": 1e3 * float(np.median(a_ms)) / steps, "final_loss": a["final_loss"],
             "centre_error_median": float(np.median(np.linalg.norm(a["o"] - truth, axis=1))),
             "bound": "latency: O(runs x pairs) fp64 work per step, one wave per (run, camera)"}
    # focal-length vote on the same scene's pair graph: one group per camera,
    # the others at their initial focal lengths, 1% noise on the true
    # essential matrices, 1,024 candidates from 200 to 3,000 px
    fF = synth.fundamental_matrices(sc, pc, noise=1e-2, seed=1)
    fcand = synth.focal_candidates(1024, 200.0, 3000.0)
    groups = np.arange(sc.n_cams, dtype=np.int32)
    fctx = fastea.Context(0)
    fctx.focal_vote(sc.n_cams, pc, fF, fcand, 0.05, group=groups, f_cur=sc.f_init)
    f_ms = []
    for _ in range(reps):
        fv = fctx.focal_vote(sc.n_cams, pc, fF, fcand, 0.05, group=groups, f_cur=sc.f_init)
        f_ms.append(fv["ms"])
    fctx.close()
    n_eval = 2 * len(pc) * len(fcand)  # each pair votes for both of its cameras' groups
    ratio = fv["f_best"] / sc.f_gt
    focal = {"cameras": sc.n_cams, "pairs": int(len(pc)), "candidates": len(fcand), "tau": 0.05,
             "kernel": "k_fv_vote", "kernel_ms": float(np.median(f_ms)),
             "matrices_per_s": n_eval / (float(np.median(f_ms)) / 1e3),
             "bound": "latency: one wave per (camera, 64 candidates), lanes over candidates, ~20 pairs each, fp64 closed-form 3x3",
             "f_best_over_true_median": float(np.median(ratio)),
             "within_5pct": float(np.mean(np.abs(ratio - 1) < 0.05))}
    # global rotation on the same scene's pair graph: true relative rotations
    # with |N(0, 2 deg)| of noise each, random start vectors, default schedule
    rng = np.random.default_rng(3)
    Q = synth.rotation_from_axis_angle(rng.normal(size=(len(pc), 3)),
                                       np.deg2rad(2.0) * np.abs(rng.normal(size=len(pc))))
    Rrel = Q @ np.einsum("pab,pcb->pac", sc.R_gt[pc[:, 1]], sc.R_gt[pc[:, 0]])
    v0 = np.random.default_rng(4).normal(size=(2, sc.n_cams, 3))
    rctx = fastea.Context(0)
    rctx.rotation_averaging(sc.n_cams, pc, Rrel, v0=v0)
    r_ms = []
    for _ in range(reps):
        ra = rctx.rotation_averaging(sc.n_cams, pc, Rrel, v0=v0)
        r_ms.append(ra["ms"])
    rctx.close()
    ropt = fastea.ra_default_options()
    rotation = {"cameras": sc.n_cams, "pairs": int(len(pc)), "init_iters_cap": ropt.init_iters,
                "iters": ropt.iters, "ms": float(np.median(r_ms)),
                "error_init_deg": metrics.mean_rotation_error_deg(ra["R_init"], sc.R_gt),
                "error_deg": metrics.mean_rotation_error_deg(ra["R"], sc.R_gt),
                "loss_init": ra["loss_init"], "loss": ra["loss"],
                "bound": "latency: six launches per Lanczos step (operator, two projection and two "
                         "subtraction passes, normalisation; host check every 16 steps) and one per Adam step, "
                         "O(pairs) fp64 each"}
    out = {"relative_translations": search, "alignment": align, "focal_vote": focal, "rotation": rotation}
    if with_cpu:
        import oracle
        oracle.build(force=False)
        sel_pairs = np.random.default_rng(5).choice(len(pc), size=min(cpu_pairs, len(pc)), replace=False)
        i = np.minimum(sc.cam1, sc.cam2)
        j = np.maximum(sc.cam1, sc.cam2)
        key = i.astype(np.int64) * sc.n_cams + j
        want = pc[sel_pairs, 0].astype(np.int64) * sc.n_cams + pc[sel_pairs, 1]
        sel = np.nonzero(np.isin(key, want))[0]
        pb = oracle.OracleProblem.from_scene(sc, sel)
        t0 = time.perf_counter()
        oracle.rel_trans(pb, sc.R_gt, sc.f_gt, cand, tau=cap_px / np.median(sc.f_gt))
        dt = time.perf_counter() - t0
        tg = oracle.ta_targets(len(c), pcg, R, tn)
        t1 = time.perf_counter()
        oracle.ta_solve(pcg, tg, init)
        dt1 = time.perf_counter() - t1
        search["cpu_baseline"] = {
            "value": len(sel) * n_cand / dt, "unit": "candidate-matches/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{len(sel_pairs)} random pairs ({len(sel)} matches) x {n_cand} candidates, FP64 C "
                      f"oracle (OpenMP over pairs), {dt:.1f} s wall"}
        keep = (pc[:, 0] < 50) & (pc[:, 1] < 50)  # the pairs among the first 50 cameras
        t2 = time.perf_counter()
        oracle.focal_vote(pc[keep], fF[keep], groups, sc.f_init, fcand, 0.05)
        dt2 = time.perf_counter() - t2
        focal["cpu_baseline"] = {"value": 2 * int(keep.sum()) * len(fcand) / dt2, "unit": "matrices/s", "cores": 1,
                                 "kind": "oracle",
                                 "sample": f"the per-camera votes over the {int(keep.sum())} pairs among 50 "
                                           f"cameras x {len(fcand)} candidates in the numpy oracle, "
                                           f"{dt2:.1f} s wall"}
        t3 = time.perf_counter()
        a6o, _ = oracle.ra_init(pc, Rrel, sc.n_cams)
        oracle.ra_solve(pc, Rrel, a6o, iters=100)
        dt3 = time.perf_counter() - t3
        rotation["cpu_baseline"] = {"value": 1e3 * dt3, "unit": "ms", "cores": 1, "kind": "oracle",
                                    "sample": f"the numpy oracle's initialisation (dense eigh of the {3 * sc.n_cams:,} x "
                                              f"{3 * sc.n_cams:,} normal matrices) and 100 of the "
                                              f"{ropt.iters:,} Adam steps, {dt3:.1f} s wall"}
        align["cpu_baseline"] = {"value": 1e3 * dt1, "unit": "ms", "cores": 1, "kind": "oracle",
                                 "sample": "the same alignment (2 runs, default schedule) in the FP64 C "
                                           f"oracle, one thread, {dt1:.1f} s wall"}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "design is described in DESIGN.md and is not built", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2605_18052_amd import fastea, metrics, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    t0 = time.perf_counter()
    desc, gen, default_m = WORKLOADS[args.workload]
    sc = getattr(synth, gen)(target_matches=args.matches or default_m)
    log(f"[bench] scene {sc.name}: {sc.n_cams} cams, {sc.n_matches} matches, "
        f"{len(sc.pairs())} pairs ({time.perf_counter() - t0:.1f} s)")

    opt = fastea.default_options(tile_matches=args.tile_matches, tile_persistent=args.tile_persistent)
    ctx = fastea.Context(0, opt)
    ctx.load_intrinsics(sc.f_init, sc.cx, sc.cy)
    t1 = time.perf_counter()
    ctx.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
    ctx.synchronize()
    seg_s = time.perf_counter() - t1
    ctx.init_poses(sc.R_init, sc.t_init)
    ctx.begin_round(opt.tau_px_init)
    info = ctx.info()
    Z = info["n_retained"]
    tile = f"{info['tile_matches']}x{info['tile_threads']}" + ("p" if info["tile_persistent"] else "")
    tune_ms = [round(float(x), 5) for x in ctx.tile_timings()]
    log(f"[bench] loaded and segmented in {seg_s:.2f} s; round 0: {Z} of {sc.n_matches} matches retained, "
        f"{info['n_items']} items of {tile}")
    # W warm-up steps, then an untimed settle: runs of 10 steps (even, so the
    # parity stays that of the timed steps, whose step graph is captured here)
    # for at least SETTLE_S of device work, so that the timed steps see the
    # device at its sustained clocks rather than fresh from the host-side
    # scene generation
    ctx.step(args.warmup)
    ctx.synchronize()
    settle_steps, t_settle = 0, time.perf_counter()
    while settle_steps < 20 or time.perf_counter() - t_settle < SETTLE_S:
        ctx.step(10)
        ctx.synchronize()
        settle_steps += 10
    torch.cuda.synchronize()
    # timed region: the steps as the library issues them (runs of 10 steps
    # replayed as HIP graphs), nothing read back until the end
    t_start = time.perf_counter()
    ctx.step(args.steps)
    ctx.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_step = 1e3 * wall / args.steps
    value = Z * args.steps / wall
    # second pass over the same steps, issued one by one, each dispatch of the
    # per-match kernel bracketed by a pair of HIP events on the library's stream
    ctx.set_kernel_timing(True)
    t_k = time.perf_counter()
    ctx.step(args.steps)
    ctx.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t_k) / args.steps
    k_ms, k_n = ctx.kernel_timing()
    k_each = ctx.kernel_times()
    ctx.set_kernel_timing(False)
    ctx.close()
    k_avg_s = k_ms / 1e3 / max(k_n, 1)
    achieved = BYTES_PER_MATCH * Z / k_avg_s / 1e9
    log(f"[bench] {args.steps} steps in {wall:.4f} s ({ms_step:.4f} ms/step, graph replay; "
        f"{eager_ms:.4f} ms/step issued one by one with kernel timing); "
        f"k_resgrad {1e3 * k_avg_s:.4f} ms avg over {k_n} launches = {achieved:.1f} GB/s")

    read_peak, copy_peak = fastea.hbm_probe(0, 1 << 30, 5)
    log(f"[bench] HBM probe (1 GiB): read {read_peak:.0f} GB/s, copy {copy_peak:.0f} GB/s")

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.calib_copy_mib} MiB read + written, 3 launches")

    ablation = None
    if args.ablation:
        names = {0: "library kernel: pose table, DPP reduction, per-item partials",
                 1: "pose block built per workgroup and staged in LDS",
                 2: "per-match global atomics (sorted layout)",
                 3: "unsorted input order, pair id per match, per-match atomics"}
        actx = fastea.Context(0, fastea.default_options(tile_matches=2048))
        actx.load_intrinsics(sc.f_init, sc.cx, sc.cy)
        actx.load_matches(sc.x1, sc.y1, sc.x2, sc.y2, sc.cam1, sc.cam2)
        actx.init_poses(sc.R_init, sc.t_init)
        actx.begin_round(opt.tau_px_init)
        actx.step(3)
        Za = actx.info()["n_retained"]
        ablation = {}
        for v, name in names.items():
            ms, _ = actx.ablation(v, reps=10)
            ablation[name] = {"kernel_ms": round(ms, 4), "GB_per_s_at_16B_per_match": round(16 * Za / ms / 1e6, 1)}
            log(f"[bench] ablation {v}: {ms:.4f} ms ({name})")
        actx.close()

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(sc, args.cpu_sample, args.cpu_iters)
        log(f"[bench] cpu: {cpu}")
    del sc

    # held-out learned-weight scenes: the solves and the stages before them
    solve, translation, held = None, None, None
    if not (args.no_solve and args.no_translation):
        seeds = [int(x) for x in args.solve_seeds.split(",") if x.strip()] or [5100]
        from paper_2605_18052_amd import learned
        mlp = learned.load_weights()
        solve = {"scenes": [], "variants": {}} if not args.no_solve else None
        for k, seed in enumerate(seeds if not args.no_solve else seeds[:1]):
            t0 = time.perf_counter()
            held = synth.config5(seed=seed)
            log(f"[bench] held-out scene {held.name}: {held.n_cams} cams, {held.n_matches} matches "
                f"({time.perf_counter() - t0:.1f} s)")
            if solve is not None:
                solve["scenes"].append(held.name)
                variants = [("quadratic_form", {"inner_loop": 1}),
                            ("learned_quadratic_form", {"inner_loop": 1, "weight_mode": 1, "mlp": mlp})]
                if k < args.solve_per_match_seeds:
                    variants.insert(0, ("per_match", {}))
                for name, o in variants:
                    r = time_to_one_degree(held, fastea, metrics, **dict(o))
                    solve["variants"].setdefault(name, []).append(r)
                    log(f"[bench] solve {held.name} {name}: {r}")
            if k == 0 and not args.no_translation:
                log("[bench] stages before the adjustment on the first held-out scene ...")
                translation = translation_stages(held, fastea, synth, args.candidates, not args.no_cpu,
                                                 args.search_cap_px, args.search_cpu_pairs)
                translation["scene"] = held.name
                rt, al = translation["relative_translations"], translation["alignment"]
                ro, fv = translation["rotation"], translation["focal_vote"]
                log(f"[bench] rotation: {ro['ms']:.1f} ms, error {ro['error_init_deg']:.3f} -> "
                    f"{ro['error_deg']:.3f} deg; focal vote: {fv['kernel_ms']:.3f} ms, {fv['within_5pct']:.2f} "
                    f"within 5%; search: k_rt_score {rt['kernel_ms']:.3f} ms, median direction error "
                    f"{rt['direction_error_deg_median']:.2f} deg; alignment {al['ms']:.2f} ms")
            del held
        if solve is not None:
            summary = {}
            for name, rs in solve["variants"].items():
                w = [r["wall_to_1deg_s"] for r in rs]
                summary[name] = {"wall_to_1deg_s": w, "reached_1deg": int(sum(x is not None for x in w)),
                                 "total_s_if_all_reached": (round(sum(w), 4) if all(x is not None for x in w)
                                                            else None)}
            solve["summary"] = summary

    batch = None
    if not args.no_batch:
        t0 = time.perf_counter()
        scenes = synth.config4()
        log(f"[bench] batch: {len(scenes)} scenes, {sum(s.n_matches for s in scenes)} matches "
            f"({time.perf_counter() - t0:.1f} s)")
        from paper_2605_18052_amd import learned
        mlp = learned.load_weights()
        batch = {"early_exit_deg": BATCH_CONVERGE_DEG}
        for name, o, seq in (("per_match", {}, True), ("quadratic_form", {"inner_loop": 1}, True),
                             ("learned_quadratic_form", {"inner_loop": 1, "weight_mode": 1, "mlp": mlp}, False)):
            batch[name] = batched_vs_sequential(scenes, fastea, metrics, synth, sequential=seq,
                                                converge_deg=BATCH_CONVERGE_DEG, **o)
            log(f"[bench] batch {name}: batched {batch[name]['batched_s']} s, sequential "
                f"{batch[name]['sequential_s']} s, {batch[name]['scenes_converged']} scenes converged, "
                f"{batch[name]['scenes_at_or_below_1deg']} scenes <= 1 deg")
        del scenes

    traffic = measured_traffic(tile, Z)
    out = {
        "metric": METRIC, "value": value, "unit": "matches/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}",
                   "matches_loaded": info["n_matches"], "matches_per_step": Z,
                   "pairs": info["n_pairs"], "items": info["n_items"], "irls_round": 0,
                   "tau_px": opt.tau_px_init, "segmenting_s": round(seg_s, 3),
                   "step_timing": "runs of 10 steps replayed as HIP graphs, host clock around the K steps",
                   "settle_steps": settle_steps,
                   "settle_note": f"untimed, between the W warm-up steps and the K timed steps: runs of 10 "
                                  f"steps for at least {SETTLE_S} s of device work (sustained clocks; the "
                                  f"step graph captured at the timed steps' parity)",
                   "ms_per_step_issued_one_by_one": eager_ms},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "achieved_on_traffic": None if traffic is None else traffic / k_avg_s / 1e9,
                     "kernel": "k_resgrad", "kernel_ms": 1e3 * k_avg_s,
                     "kernel_ms_p10_p50_p90": [float(np.percentile(k_each, q)) for q in (10, 50, 90)],
                     "bytes_per_launch": BYTES_PER_MATCH * Z,
                     "measured_read_peak": read_peak, "frac_of_measured_read_peak": achieved / read_peak,
                     "tile": f"{info['tile_matches']} matches x {info['tile_threads']} threads"
                             + (", persistent workgroups" if info["tile_persistent"] else ", one workgroup per item"),
                     "autotuner_ms_per_shape": tune_ms,
                     "traffic_source": "rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, calibrated on a 1 GiB "
                                       "copy (null if the kernel changed since they were taken)"},
        "cpu_baseline": cpu,
        "solve": solve,
        "batch": batch,
        "translation": translation,
    }
    if ablation is not None:
        out["ablation"] = ablation
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
