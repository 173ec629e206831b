"""Pose-accuracy metrics used to judge convergence (evaluation only).

Rotation error follows the geodesic distance between rotations that FastMap
uses for global rotation alignment (Method > Optimization Formulations,
Global Rotation): d(R, R') = arccos((tr(R^T R') - 1) / 2), with the argument
clamped to [-1, 1].  Estimated poses are defined up to a global similarity,
so they are first aligned to ground truth by the rotation closest (chordal
sense, via SVD) to sum_i R_gt,i^T R_est,i.
"""
from __future__ import annotations

import numpy as np


def geodesic_deg(Ra: np.ndarray, Rb: np.ndarray) -> np.ndarray:
    tr = np.einsum("...ij,...ij->...", Ra, Rb)
    return np.degrees(np.arccos(np.clip((tr - 1.0) / 2.0, -1.0, 1.0)))


def project_so3(M: np.ndarray) -> np.ndarray:
    U, _, Vt = np.linalg.svd(M)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt))])
    return U @ D @ Vt


def rotation_errors_deg(R_est: np.ndarray, R_gt: np.ndarray) -> np.ndarray:
    """Per-camera error after global alignment: R_est,i ~ R_gt,i R_a."""
    Ra = project_so3(np.einsum("nji,njk->ik", R_gt, R_est))
    return geodesic_deg(R_est, R_gt @ Ra)


def mean_rotation_error_deg(R_est: np.ndarray, R_gt: np.ndarray) -> float:
    return float(rotation_errors_deg(R_est, R_gt).mean())


def relative_rotation_error_deg(R_est: np.ndarray, R_gt: np.ndarray, pairs) -> float:
    """Gauge-free cross-check: mean over pairs of d(R_ij, R_ij,gt)."""
    pairs = np.asarray(pairs)
    i, j = pairs[:, 0], pairs[:, 1]
    Rij = R_est[j] @ np.transpose(R_est[i], (0, 2, 1))
    Rij_gt = R_gt[j] @ np.transpose(R_gt[i], (0, 2, 1))
    return float(geodesic_deg(Rij, Rij_gt).mean())
