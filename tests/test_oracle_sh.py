"""Pins of the oracle's spherical-harmonics colour (listing XPR-3DGS,
compute_color): library basis, exact quadrature, finite differences."""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y, roots_legendre

import oracle
from helpers import axis_camera, hand_scene


def _scipy_real_sh(deg, d):
    """Real SH from scipy's complex ones (Condon-Shortley phase included):
    m > 0: sqrt(2) Re Y_l^m, m = 0: Y_l^0, m < 0: sqrt(2) Im Y_l^|m|."""
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    out = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                out.append(math.sqrt(2) * Y.real)
            elif m < 0:
                out.append(math.sqrt(2) * Y.imag)
            else:
                out.append(Y.real)
    return np.array(out)


def test_basis_matches_scipy():
    rng = np.random.default_rng(0)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        np.testing.assert_allclose(oracle.sh_basis(3, d), _scipy_real_sh(3, d), atol=1e-13)


def test_orthonormal_by_exact_quadrature():
    # Gauss-Legendre (6 nodes) in cos(theta) x 12 uniform nodes in phi is exact
    # for the degree <= 6 products of degree <= 3 harmonics.
    xs, ws = roots_legendre(6)
    nphi = 12
    G = np.zeros((16, 16))
    for ct, w in zip(xs, ws):
        st = math.sqrt(1 - ct * ct)
        for k in range(nphi):
            ph = 2 * math.pi * k / nphi
            d = np.array([st * math.cos(ph), st * math.sin(ph), ct])
            Y = oracle.sh_basis(3, d)
            G += w * (2 * math.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-13)


def test_basis_gradient_by_finite_differences():
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(10):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        _, dY = oracle.sh_basis(3, d, grad=True)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fd = (oracle.sh_basis(3, d + e) - oracle.sh_basis(3, d - e)) / (2 * h)
            np.testing.assert_allclose(dY[:, c], fd, atol=1e-8)


def test_degree0_colour_is_constant_and_clamped():
    cam = axis_camera(64, 64, f=64.0)
    cfg = oracle.OracleConfig(sh_degree=0)
    rgb = np.array([[0.2, 0.7, 1.3], [-0.4, 0.5, 0.0]])
    sc = hand_scene([[0.1, 0.0, 3.0], [-0.2, 0.1, 2.0]], 0.05, rgb=rgb)
    pr = oracle.project(sc, cam, cfg)
    np.testing.assert_allclose(pr["rec"][0, 6:], [0.2, 0.7, 1.3], atol=1e-6)
    np.testing.assert_allclose(pr["rec"][1, 6:], [0.0, 0.5, 0.0], atol=1e-6)


def test_sh_gradient_is_basis_value():
    # colour_k = 0.5 + sum_j sh_jk Y_j(dir) is linear in sh: dcolour/dsh = Y.
    rng = np.random.default_rng(2)
    n = 5
    means = rng.uniform(-0.3, 0.3, size=(n, 3)) + [0, 0, 3]
    sh = np.zeros((n, 16, 3))
    sh[:, 0, :] = 1.0
    sh[:, 1:, :] = rng.normal(0, 0.05, size=(n, 15, 3))
    sc = hand_scene(means, 0.05, sh_degree=3, sh=sh)
    cam = axis_camera(64, 64, f=64.0, t=[0.2, 0.1, 0.5])
    cfg = oracle.OracleConfig(sh_degree=3)
    g9 = np.zeros((n, 9))
    g9[:, 6:] = 1.0
    g = oracle.project_bwd(sc, cam, cfg, g9)
    campos = -cam.R.T @ cam.t
    for i in range(n):
        d = sc.means[:, i].astype(np.float64) - campos
        d /= np.linalg.norm(d)
        Y = _scipy_real_sh(3, d)
        for ch in range(3):
            np.testing.assert_allclose(g["sh"][:, ch, i], Y, atol=1e-12)
