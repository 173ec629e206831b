"""Pins of the oracle's global rotation stage (Method > Global Rotation,
Eq. fastmap-rotation-objective and the initialisation after Martinec and
Pajdla): closed forms of the geodesic distance, the loss at the truth and
its gauge, central differences of the gradient, and exact recovery by the
initialisation without noise."""
import numpy as np
import pytest

import oracle
from paper_2605_18052_amd import metrics, synth


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _rel(R, pc):
    return np.einsum("pab,pcb->pac", R[pc[:, 1]], R[pc[:, 0]])


def test_geodesic_distance_is_the_rotation_angle():
    rng = np.random.default_rng(0)
    R = synth.rotation_from_axis_angle(rng.normal(size=(1, 3)), np.array([0.7]))[0]
    for th in (0.0, 0.1, 1.0, 2.0, 3.0):
        Q = synth.rotation_from_axis_angle(rng.normal(size=(1, 3)), np.array([th]))[0]
        assert oracle.geodesic(R, R @ Q) == pytest.approx(th, abs=1e-7)
        assert oracle.geodesic(R @ Q, R) == pytest.approx(th, abs=1e-7)


def test_loss_zero_at_truth_invariant_to_a_global_rotation_and_gradient_by_differences():
    pc, R, _, _ = synth.object_pair_graph(30, 80.0, 1)
    N = len(R)
    Rr = _rel(R, pc)
    a6_true = np.concatenate([R[:, :, 0], R[:, :, 1]], axis=1)
    L0, g0 = oracle.ra_loss_grad(pc, Rr, a6_true)
    assert L0 < 1e-6  # arccos near 1 carries sqrt(eps)
    rng = np.random.default_rng(2)
    a6 = rng.normal(size=(N, 6))
    L, g = oracle.ra_loss_grad(pc, Rr, a6)
    Rs = np.stack([oracle.rot6d_to_R(a6[k]) for k in range(N)])
    Q = synth.rotation_from_axis_angle(np.array([[0.2, 1.0, -0.5]]), np.array([0.9]))[0]
    RQ = Rs @ Q
    a6q = np.concatenate([RQ[:, :, 0], RQ[:, :, 1]], axis=1)
    assert oracle.ra_loss_grad(pc, Rr, a6q)[0] == pytest.approx(L, rel=1e-10)
    h = 1e-6
    fd = np.zeros_like(a6)
    for k in range(N):
        for c in range(6):
            ap, am = a6.copy(), a6.copy()
            ap[k, c] += h
            am[k, c] -= h
            fd[k, c] = (oracle.ra_loss_grad(pc, Rr, ap)[0] - oracle.ra_loss_grad(pc, Rr, am)[0]) / (2 * h)
    # an O(1) loss differenced at h = 1e-6 carries ~1e-10 of rounding
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_initialisation_recovers_noiseless_rotations_up_to_one_rotation():
    """Without noise every column problem has the columns of R_i V (one V
    for all cameras) as its exact solution: the initialisation returns the
    truth up to a single global rotation."""
    sc = synth.trajectory_scene(n_cams=80, n_pts=5000, target_matches=100_000, seed=4, name="rot80")
    pc = sc.pairs().astype(np.int32)
    _, Ri = oracle.ra_init(pc, _rel(sc.R_gt, pc), sc.n_cams)
    V = np.einsum("nba,nbc->nac", sc.R_gt, Ri)  # R_i^T R_i_est, the same for all i
    np.testing.assert_allclose(V, np.broadcast_to(V[0], V.shape), atol=1e-9)
    np.testing.assert_allclose(np.linalg.det(Ri), 1.0, atol=1e-12)


def test_initialisation_with_noise_lands_near_the_truth():
    """With 3 degrees of noise per pair the column-wise initialisation is
    already within a degree.  Without the orthogonality penalty the second
    column problem has the first column's own solution, and Gram-Schmidt
    would leave rounding noise."""
    pc, R, _, _ = synth.object_pair_graph(120, 70.0, 0)
    rng = np.random.default_rng(1)
    Q = synth.rotation_from_axis_angle(rng.normal(size=(len(pc), 3)),
                                       np.deg2rad(3.0) * np.abs(rng.normal(size=len(pc))))
    a6, Ri, raw2 = oracle.ra_init(pc, Q @ _rel(R, pc), len(R), details=True)
    assert metrics.mean_rotation_error_deg(Ri, R) < 1.0
    # the penalty makes the second problem's own solution nearly orthogonal to
    # the first column in every camera, before any Gram-Schmidt step
    cosines = np.abs(np.sum(a6[:, :3] * raw2, axis=1)) / np.linalg.norm(raw2, axis=1)
    assert cosines.max() < 0.05, cosines.max()


def test_optimisation_lowers_loss_and_error_from_the_initialisation():
    pc, R, _, _ = synth.object_pair_graph(120, 70.0, 0)
    rng = np.random.default_rng(1)
    Q = synth.rotation_from_axis_angle(rng.normal(size=(len(pc), 3)),
                                       np.deg2rad(3.0) * np.abs(rng.normal(size=len(pc))))
    Rn = Q @ _rel(R, pc)
    a6, Ri = oracle.ra_init(pc, Rn, len(R))
    L0, _ = oracle.ra_loss_grad(pc, Rn, a6)
    _, Rs, L1 = oracle.ra_solve(pc, Rn, a6, iters=300)
    e0 = metrics.mean_rotation_error_deg(Ri, R)
    e1 = metrics.mean_rotation_error_deg(Rs, R)
    assert L1 < L0 and e1 < 0.7 * e0, (L0, L1, e0, e1)
