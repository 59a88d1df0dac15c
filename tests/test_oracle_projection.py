"""Pins of the oracle's projection (Listing "Implementation of XPR-3DGS",
project) against closed forms, a library rotation and invariances."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from helpers import axis_camera, hand_scene, quat_z, random_rotation, rot_z


def _cfg(**kw):
    kw.setdefault("sh_degree", 0)
    return oracle.OracleConfig(**kw)


@pytest.mark.parametrize("Z,s,f", [(4.0, 0.05, 300.0), (2.5, 0.01, 500.0), (7.0, 0.2, 128.0)])
def test_isotropic_on_axis_closed_form(Z, s, f):
    # On the optical axis J = diag(f/Z, f/Z) (third column zero), so
    # cov2D = (f s / Z)^2 I + 0.3 I and mean2D = principal point - 1/2.
    W, H = 201, 151
    cam = axis_camera(W, H, f=f)
    cfg = _cfg()
    sc = hand_scene([[0, 0, Z]], [s, s, s], opac=0.6)
    pr = oracle.project(sc, cam, cfg)
    s32 = float(np.float32(s))
    z32 = float(np.float32(Z))
    var = (f * s32 / z32) ** 2 + 0.3
    np.testing.assert_allclose(pr["cov"][0], [var, 0.0, var], rtol=1e-13, atol=1e-15)
    u, v = W / 2 - 0.5, H / 2 - 0.5
    rec = pr["rec"][0]
    np.testing.assert_allclose(rec[:2], [u, v], rtol=0, atol=1e-12)
    np.testing.assert_allclose(rec[2:5], [-0.5 / var, 0.0, -0.5 / var], rtol=1e-13, atol=1e-15)
    assert pr["depth"][0] == pytest.approx(z32, rel=1e-15)
    r = math.ceil(3 * math.sqrt(var))
    assert pr["radius"][0] == r
    tx = (W + 15) // 16
    ty = (H + 15) // 16
    x0 = min(max(math.floor((u - r) / 16), 0), tx)
    x1 = min(max(math.floor((u + r) / 16) + 1, 0), tx)
    y0 = min(max(math.floor((v - r) / 16), 0), ty)
    y1 = min(max(math.floor((v + r) / 16) + 1, 0), ty)
    assert list(pr["rect"][0]) == [x0, y0, x1, y1]
    assert pr["tc"][0] == (x1 - x0) * (y1 - y0)


@pytest.mark.parametrize("theta", [0.3, 1.1, -2.0])
def test_rotated_about_axis(theta):
    # A Gaussian rotated about the optical axis projects to
    # (f/Z)^2 Rz diag(s1^2, s2^2) Rz^T + 0.3 I.
    f, Z = 400.0, 5.0
    s = np.array([0.03, 0.011, 0.02], np.float32).astype(np.float64)
    cam = axis_camera(160, 120, f=f)
    sc = hand_scene([[0, 0, Z]], s, quats=quat_z(theta))
    pr = oracle.project(sc, cam, _cfg())
    q32 = sc.quats[:, 0].astype(np.float64)
    th = 2 * math.atan2(q32[3], q32[0])
    R2 = rot_z(th)[:2, :2]
    cov = (f / Z) ** 2 * R2 @ np.diag(s[:2] ** 2) @ R2.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(pr["cov"][0], [cov[0, 0], cov[0, 1], cov[1, 1]], rtol=1e-12)


def test_quaternion_matches_library_rotation():
    # Sigma = R S^2 R^T with R from scipy's quaternion convention; on the axis
    # the 2D covariance is the upper-left block scaled by (f/Z)^2.
    rng = np.random.default_rng(1)
    f, Z = 350.0, 6.0
    cam = axis_camera(128, 128, f=f)
    for _ in range(5):
        q = rng.normal(size=4)
        s = np.exp(rng.uniform(-4, -2, size=3)).astype(np.float32).astype(np.float64)
        sc = hand_scene([[0, 0, Z]], s, quats=q)
        q32 = sc.quats[:, 0].astype(np.float64)
        Rl = Rotation.from_quat([q32[1], q32[2], q32[3], q32[0]]).as_matrix()
        Sig = Rl @ np.diag(s ** 2) @ Rl.T
        pr = oracle.project(sc, cam, _cfg())
        exp = (f / Z) ** 2 * Sig[:2, :2] + 0.3 * np.eye(2)
        np.testing.assert_allclose(pr["cov"][0], [exp[0, 0], exp[0, 1], exp[1, 1]], rtol=1e-12)


def test_quaternion_scale_invariance():
    rng = np.random.default_rng(2)
    q = rng.normal(size=(8, 4))
    means = rng.uniform(-0.5, 0.5, size=(8, 3)) + [0, 0, 4]
    a = hand_scene(means, [0.02, 0.05, 0.01], quats=q)
    b = hand_scene(means, [0.02, 0.05, 0.01], quats=4.0 * q)
    cam = axis_camera(100, 90, f=120.0)
    pa, pb = oracle.project(a, cam, _cfg()), oracle.project(b, cam, _cfg())
    np.testing.assert_allclose(pa["cov"], pb["cov"], rtol=1e-12)


def test_off_axis_jacobian_closed_form():
    # At (X, 0, Z) with isotropic scale s: J = [[f/Z, 0, -f X/Z^2], [0, f/Z, 0]]
    # so cov2D = s^2 J J^T + 0.3 I = s^2 diag(f^2/Z^2 + f^2 X^2/Z^4, f^2/Z^2) + 0.3 I.
    f, Z, X, s = 300.0, 4.0, 0.8, 0.04
    W, H = 256, 256
    cam = axis_camera(W, H, f=f)
    sc = hand_scene([[X, 0, Z]], [s, s, s])
    pr = oracle.project(sc, cam, _cfg())
    X32, Z32, s32 = (float(np.float32(v)) for v in (X, Z, s))
    a = s32 ** 2 * (f ** 2 / Z32 ** 2 + f ** 2 * X32 ** 2 / Z32 ** 4) + 0.3
    c = s32 ** 2 * f ** 2 / Z32 ** 2 + 0.3
    np.testing.assert_allclose(pr["cov"][0], [a, 0.0, c], rtol=1e-12, atol=1e-14)
    assert pr["rec"][0][0] == pytest.approx(f * X32 / Z32 + W / 2 - 0.5, abs=1e-11)


def test_jacobian_clamp_off_screen():
    # Beyond 1.3 tan(fov/2) the Jacobian uses the clamped direction:
    # X/Z -> lim = 1.3 W / (2 f), the mean2D does not.
    f, Z, s = 100.0, 2.0, 0.3
    W, H = 64, 64
    X = 3.0  # X/Z = 1.5 > lim = 0.416
    cam = axis_camera(W, H, f=f)
    sc = hand_scene([[X, 0, Z]], [s, s, s], opac=0.9)
    pr = oracle.project(sc, cam, _cfg())
    lim = 1.3 * W / (2 * f)
    s32 = float(np.float32(s))
    a = s32 ** 2 * (f ** 2 / Z ** 2 + f ** 2 * lim ** 2 / Z ** 2) + 0.3
    c = s32 ** 2 * f ** 2 / Z ** 2 + 0.3
    np.testing.assert_allclose(pr["cov"][0], [a, 0.0, c], rtol=1e-12)
    assert pr["rec"][0][0] == pytest.approx(f * X / Z + W / 2 - 0.5, abs=1e-10)


def test_rigid_motion_invariance():
    # Moving the scene and the camera by the same rigid motion changes
    # nothing in image space (pins the use of R vs R^T and of t).
    rng = np.random.default_rng(3)
    n = 40
    means = rng.uniform(-1, 1, size=(n, 3))
    q = rng.normal(size=(n, 4))
    s = np.exp(rng.uniform(np.log(0.01), np.log(0.08), size=(n, 3)))
    cfg = _cfg()
    cam = axis_camera(96, 80, f=90.0, t=[0.1, -0.2, 4.0])
    Q = random_rotation(rng)
    d = rng.normal(size=3)
    # world' = Q world + d; camera' : x_cam = R Q^T (x' - d) + t
    means2 = means @ Q.T + d
    Rq = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    q2 = Rotation.from_matrix(Q[None] @ Rq).as_quat()[:, [3, 0, 1, 2]]
    cam2 = axis_camera(96, 80, f=90.0, R=cam.R @ Q.T, t=cam.t - cam.R @ Q.T @ d)
    a = oracle.project(hand_scene(means, s, quats=q), cam, cfg)
    b = oracle.project(hand_scene(means2, s, quats=q2), cam2, cfg)
    # float32 storage of the moved inputs limits agreement
    np.testing.assert_allclose(a["rec"][:, :2], b["rec"][:, :2], rtol=0, atol=2e-4)
    np.testing.assert_allclose(a["cov"], b["cov"], rtol=2e-4, atol=1e-6)
    np.testing.assert_allclose(a["depth"], b["depth"], rtol=1e-6)


def test_visibility_rules():
    cam = axis_camera(64, 64, f=64.0)
    cfg = _cfg()
    sc = hand_scene([[0, 0, 0.1],      # behind z_near = 0.2
                     [0, 0, 3.0],      # visible
                     [0, 0, 3.0],      # opacity below 1/255
                     [50, 0, 3.0],     # rect entirely off screen
                     [0, 0, -3.0]],    # behind the camera
                    [0.05, 0.05, 0.05], opac=[0.5, 0.5, 0.003, 0.5, 0.5])
    pr = oracle.project(sc, cam, cfg)
    assert list(pr["tc"]) [1] > 0
    assert [int(t > 0) for t in pr["tc"]] == [0, 1, 0, 0, 0]
