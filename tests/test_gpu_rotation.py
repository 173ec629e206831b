"""GPU parity of the global rotation stage (Method > Global Rotation)
against the numpy oracle, through the C-ABI."""
import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import fastea, metrics, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def _noisy_rel(R, pc, deg, seed):
    rng = np.random.default_rng(seed)
    Q = synth.rotation_from_axis_angle(rng.normal(size=(len(pc), 3)),
                                       np.deg2rad(deg) * np.abs(rng.normal(size=len(pc))))
    return Q @ np.einsum("pab,pcb->pac", R[pc[:, 1]], R[pc[:, 0]])


def _gauge(Ra, Rb):
    """Mean angle (deg) between Ra and Rb after the best common rotation."""
    return metrics.mean_rotation_error_deg(Ra, Rb)


def test_adam_steps_match_oracle_from_the_same_start():
    """Thirty Adam steps from the oracle's initialisation on 120 cameras with
    3 degrees of noise: the same rotations and losses to 1e-9 (fp64 on both
    sides; running products against pow for the schedule)."""
    pc, R, _, _ = synth.object_pair_graph(120, 70.0, 0)
    Rn = _noisy_rel(R, pc, 3.0, 1)
    a6, _ = oracle.ra_init(pc, Rn, len(R))
    ctx = fastea.Context(0)
    got = ctx.rotation_averaging(len(R), pc, Rn, a6_init=a6, options=fastea.ra_default_options(iters=30))
    ctx.close()
    _, Rref, Lref = oracle.ra_solve(pc, Rn, a6, iters=30)
    L0, _ = oracle.ra_loss_grad(pc, Rn, a6)
    assert got["loss_init"] == pytest.approx(L0, rel=1e-9)
    np.testing.assert_allclose(got["R"], Rref, atol=1e-9)
    assert got["loss"] == pytest.approx(Lref, rel=1e-9)


def test_initialisation_recovers_noiseless_rotations_up_to_one_rotation():
    sc = synth.trajectory_scene(n_cams=80, n_pts=5000, target_matches=100_000, seed=4, name="rot80")
    pc = sc.pairs().astype(np.int32)
    Rr = np.einsum("pab,pcb->pac", sc.R_gt[pc[:, 1]], sc.R_gt[pc[:, 0]])
    v0 = np.random.default_rng(5).normal(size=(2, sc.n_cams, 3))
    ctx = fastea.Context(0)
    got = ctx.rotation_averaging(sc.n_cams, pc, Rr, v0=v0, options=fastea.ra_default_options(iters=0))
    ctx.close()
    V = np.einsum("nba,nbc->nac", sc.R_gt, got["R_init"])
    np.testing.assert_allclose(V, np.broadcast_to(V[0], V.shape), atol=1e-6)
    assert got["loss_init"] < 1e-6


def test_full_solve_matches_oracle_up_to_the_gauge():
    """Initialisation (power iterations here, eigh in the oracle: different
    vectors of the same near-null space) and 1,000 Adam steps on 120 cameras
    with 3 degrees of noise: both end at the same rotations up to one global
    rotation, to 0.01 degree."""
    pc, R, _, _ = synth.object_pair_graph(120, 70.0, 0)
    Rn = _noisy_rel(R, pc, 3.0, 2)
    v0 = np.random.default_rng(6).normal(size=(2, len(R), 3))
    ctx = fastea.Context(0)
    got = ctx.rotation_averaging(len(R), pc, Rn, v0=v0)
    ctx.close()
    a6, Ri = oracle.ra_init(pc, Rn, len(R))
    _, Rref, Lref = oracle.ra_solve(pc, Rn, a6, iters=1000)
    assert _gauge(got["R"], Rref) < 0.01
    assert got["loss"] == pytest.approx(Lref, rel=1e-3)
    e_init, e_fin = _gauge(got["R_init"], R), _gauge(got["R"], R)
    print(f"rotation: init {e_init:.3f} deg -> solved {e_fin:.3f} deg, {got['ms']:.1f} ms", flush=True)
    assert e_fin < e_init


def test_rotation_averaging_rejects_bad_input():
    pc, R, _, _ = synth.object_pair_graph(20, 80.0, 3)
    Rr = np.einsum("pab,pcb->pac", R[pc[:, 1]], R[pc[:, 0]])
    ctx = fastea.Context(0)
    with pytest.raises(fastea.FeaError, match="pair"):
        ctx.rotation_averaging(len(R), np.array([[2, 2]]), Rr[:1], v0=np.zeros((2, len(R), 3)))
    with pytest.raises(fastea.FeaError, match="v0"):
        ctx.rotation_averaging(len(R), pc, Rr)
    bad = Rr.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(fastea.FeaError):
        ctx.rotation_averaging(len(R), pc, bad, v0=np.ones((2, len(R), 3)))
    ctx.close()
