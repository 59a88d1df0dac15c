"""Small hand-built scenes and cameras for the tests (no method arithmetic)."""
from __future__ import annotations

import math

import numpy as np

from synth import Camera, Scene

Y00 = 0.5 / math.sqrt(math.pi)


def hand_scene(means, scales, quats=None, opac=None, rgb=None, sh_degree=0, sh=None):
    means = np.asarray(means, np.float64).reshape(-1, 3)
    n = means.shape[0]
    scales = np.broadcast_to(np.asarray(scales, np.float64), (n, 3))
    if quats is None:
        quats = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    quats = np.broadcast_to(np.asarray(quats, np.float64), (n, 4))
    opac = np.broadcast_to(np.asarray(0.5 if opac is None else opac, np.float64), (n,))
    K = (sh_degree + 1) ** 2
    if sh is None:
        rgb = np.broadcast_to(np.asarray(0.8 if rgb is None else rgb, np.float64), (n, 3))
        shv = np.zeros((n, K, 3))
        shv[:, 0, :] = (rgb - 0.5) / Y00
    else:
        shv = np.asarray(sh, np.float64).reshape(n, K, 3)
    f32 = np.float32
    return Scene(
        means=np.ascontiguousarray(means.T.astype(f32)),
        scales=np.ascontiguousarray(scales.T.astype(f32)),
        quats=np.ascontiguousarray(quats.T.astype(f32)),
        opacities=np.ascontiguousarray(opac.astype(f32)),
        sh=np.ascontiguousarray(np.transpose(shv, (1, 2, 0)).astype(f32)),
        log_scales=np.ascontiguousarray(np.log(scales.T).astype(f32)),
        logits=np.ascontiguousarray(np.log(opac / (1 - opac)).astype(f32)),
        sh_degree=sh_degree,
    )


def axis_camera(W, H, f=None, R=None, t=None):
    """Camera at the origin looking down +z (identity rotation)."""
    f = float(W) if f is None else float(f)
    return Camera(R=np.eye(3) if R is None else np.asarray(R, np.float64),
                  t=np.zeros(3) if t is None else np.asarray(t, np.float64),
                  fx=f, fy=f, cx=W / 2.0, cy=H / 2.0, width=int(W), height=int(H))


def rot_z(theta):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def quat_z(theta):
    return np.array([math.cos(theta / 2), 0.0, 0.0, math.sin(theta / 2)])


def random_rotation(rng):
    """Random proper rotation (QR of a Gaussian matrix, sign-fixed)."""
    Q, Rr = np.linalg.qr(rng.normal(size=(3, 3)))
    Q = Q * np.sign(np.diag(Rr))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q
