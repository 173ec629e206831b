"""Ablation passes (design choices of the per-match kernel taken back) give
the same per-pair sums as the library's kernel, so their timings compare
like with like."""
import math

import numpy as np
import pytest

from paper_2605_18052_amd import fastea, synth

from gpu_helpers import make_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_ablations_agree_with_library_kernel():
    sc = synth.sphere_scene(n_cams=12, n_pts=9000, p_det=0.7, sigma=1.0, outlier_frac=0.2, seed=23,
                            name="ablation")
    ctx = make_context(sc, gauge=1, tile_matches=2048)
    ctx.init_poses(sc.R_init, sc.t_init)
    ctx.begin_round(64.0)
    ctx.step(7)  # poses away from the snapshot
    ms0, ref = ctx.ablation(0, reps=2)
    scale = np.abs(ref).max(axis=0) + 1e-30
    for v in (1, 2, 3):
        ms, got = ctx.ablation(v, reps=2)
        assert ms > 0
        # fp32 sums in another order (atomics): agreement to fp32 accumulation error
        err = np.abs(got - ref).max(axis=0) / scale
        assert np.all(err < 2e-5), (v, err)
    with pytest.raises(fastea.FeaError):
        ctx.ablation(4)
    ctx.close()
    other = make_context(sc, gauge=1, tile_matches=4096)
    other.init_poses(sc.R_init, sc.t_init)
    other.begin_round(math.inf)
    with pytest.raises(fastea.FeaError):
        other.ablation(1)
    other.close()
