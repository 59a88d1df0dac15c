"""Pins of the oracle's LinPrim backward (project and evaluate of Listing
XPR-LinPrim, blended by Algorithm 1, differentiated by hand as the paper's
pipeline is by automatic differentiation, section Key Interfaces): torch
float64 autograd of the independent per-pixel brute force (for the
parameter gradients and for the 16 per-record values), and central finite
differences of the tiled FP64 forward. Decisions (slab miss, gates, stop,
the entry and exit slabs, rect) are piecewise constant."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import oracle.brute as brute
from helpers import axis_camera, hand_scene
from synth import camera_look_at, scene_clusters

FIELDS = ["means", "scales", "quats", "opacities", "sh"]


def _cfg():
    return oracle.OracleConfig(sh_degree=3, tile_w=8, tile_h=8, bg=(0.2, 0.1, 0.05),
                               method="linprim")


def _clamp_scene():
    """An octahedron long along the view axis (alpha passes the 0.99 clamp
    through its centre), one with a negative colour channel, and ordinary
    ones, overlapping."""
    sh = np.zeros((4, 16, 3))
    sh[:, 0, :] = [[1.2, 0.3, 0.6], [0.4, -2.5, 0.8], [0.9, 0.9, 0.1], [0.2, 0.5, 1.1]]
    rng = np.random.default_rng(11)
    sh[:, 1:, :] = rng.normal(0, 0.05, size=(4, 15, 3))
    means = [[0.05, -0.03, 3.0], [0.15, 0.1, 3.5], [-0.3, 0.2, 4.0], [0.02, 0.03, 2.5]]
    scales = [[0.15, 0.1, 0.12], [0.2, 0.15, 0.18], [0.3, 0.2, 0.25], [0.25, 0.3, 0.8]]
    quats = rng.normal(size=(4, 4)) * [1, 0.2, 0.2, 0.2]
    quats[3] = [1.0, 0.02, -0.03, 0.01]
    return hand_scene(means, scales, quats=quats, opac=[0.7, 0.6, 0.5, 0.95], sh_degree=3, sh=sh)


def _scenes():
    yield "clusters", scene_clusters(30, seed=7, lo=0.05, hi=0.3, n_clusters=3, box=0.8), \
        camera_look_at((0.4, 0.3, -4.0), 40, 34)
    yield "clamps", _clamp_scene(), axis_camera(44, 36, f=40.0)


IDS = lambda x: x if isinstance(x, str) else ""


def _f64_scene(sc):
    return dataclasses.replace(sc, **{f: getattr(sc, f).astype(np.float64) for f in FIELDS})


@pytest.mark.parametrize("name,sc,cam", list(_scenes()), ids=IDS)
def test_lin_analytic_matches_autograd_of_brute_force(name, sc, cam):
    cfg = _cfg()
    dimg = np.random.default_rng(0).normal(size=(3, cam.height, cam.width))
    st = oracle.render(sc, cam, cfg)
    assert st["fwd"]["guard"].sum() == 0
    g = oracle.backward(sc, cam, cfg, dimg, state=st)
    ts = brute.scene_tensors(sc, requires_grad=True)
    img, _ = brute.render_lin_torch(*ts, cam, cfg)
    np.testing.assert_allclose(img.detach().numpy(), st["fwd"]["img"], atol=1e-12)
    (img * torch.as_tensor(dimg)).sum().backward()
    ref = {"means": ts[0].grad.numpy().T, "scales": ts[1].grad.numpy().T,
           "quats": ts[2].grad.numpy().T, "opacities": ts[3].grad.numpy(),
           "sh": np.transpose(ts[4].grad.numpy(), (1, 2, 0))}
    for f in FIELDS:
        scale = max(np.abs(ref[f]).max(), 1e-12)
        assert np.abs(g[f] - ref[f]).max() <= 1e-7 * scale, f
        assert np.abs(ref[f]).max() > 0, f


@pytest.mark.parametrize("name,sc,cam", list(_scenes()), ids=IDS)
def test_lin_record_gradient_matches_autograd_of_brute_force(name, sc, cam):
    """The 16 per-record values of orc_render_bwd_lin against autograd of the
    brute force at its own shader data (u, v, sigma, colour, rows of A^-1;
    the 16th is zero)."""
    cfg = _cfg()
    dimg = np.random.default_rng(2).normal(size=(3, cam.height, cam.width))
    st = oracle.render(sc, cam, cfg)
    g16 = oracle.render_bwd_lin(st["proj"]["rec"], st["bins"]["vals"], st["bins"]["ranges"],
                                cam.width, cam.height, cfg, dimg)
    ts = brute.scene_tensors(sc, requires_grad=True)
    keep = {}
    img, _ = brute.render_lin_torch(*ts, cam, cfg, keep=keep)
    (img * torch.as_tensor(dimg)).sum().backward()
    ref = np.concatenate([keep["u"].grad.numpy()[:, None], keep["v"].grad.numpy()[:, None],
                          keep["sigma"].grad.numpy()[:, None], keep["colour"].grad.numpy(),
                          keep["c"].grad.numpy().reshape(-1, 9),
                          np.zeros((sc.n, 1))], axis=1)
    vis = st["proj"]["tc"] > 0
    assert vis.sum() >= 3
    for cols, what in ((slice(0, 2), "mean2D"), (slice(2, 3), "sigma"), (slice(3, 6), "colour"),
                       (slice(6, 15), "c")):
        r, x = ref[vis, cols], g16[vis, cols]
        scale = max(np.abs(r).max(), 1e-12)
        assert np.abs(x - r).max() <= 1e-8 * scale, what
        assert np.abs(r).max() > 0, what
    assert np.all(g16[:, 15] == 0) and np.all(g16[~vis] == 0)


def test_lin_clamp_scene_exercises_clamps():
    cam = axis_camera(44, 36, f=40.0)
    cfg = _cfg()
    st = oracle.render(_clamp_scene(), cam, cfg)
    pr = st["proj"]
    assert (pr["tc"] > 0).all()
    assert pr["rec"][1, 4] == 0.0                 # negative green clamped to 0
    # the long octahedron's alpha passes the 0.99 clamp through its centre
    px = np.array([[x, y] for y in range(cam.height) for x in range(cam.width)], np.int32)
    ch = oracle.lin_chord(np.repeat(pr["rec"][3:4], len(px), 0), px)
    assert (-np.expm1(-pr["rec"][3, 2] * ch)).max() > 0.99


def _loss_and_sig(sc, cam, cfg, dimg):
    st = oracle.render(sc, cam, cfg)
    sig = (st["proj"]["tc"].tobytes(), st["proj"]["rect"].tobytes(), st["bins"]["vals"].tobytes(),
           st["fwd"]["ncontrib"].tobytes(), st["fwd"]["nblend"].tobytes())
    return float((st["fwd"]["img"] * dimg).sum()), sig


@pytest.mark.parametrize("name,sc,cam", list(_scenes()), ids=IDS)
def test_lin_analytic_matches_central_differences(name, sc, cam):
    cfg = _cfg()
    dimg = np.random.default_rng(1).normal(size=(3, cam.height, cam.width))
    sc = _f64_scene(sc)
    g = oracle.backward(sc, cam, cfg, dimg)
    checked = skipped = 0
    for f in FIELDS:
        arr = getattr(sc, f)
        flat_idx = list(np.ndindex(arr.shape))
        if f == "sh":
            flat_idx = flat_idx[: 3 * 4 * sc.n]  # degrees 0-1 are enough here
        for idx in flat_idx[::3] if f != "opacities" else flat_idx:
            x = arr[idx]
            h = 1e-6 * max(1.0, abs(x))
            arr[idx] = x + h
            lp, sp = _loss_and_sig(sc, cam, cfg, dimg)
            arr[idx] = x - h
            lm, sm = _loss_and_sig(sc, cam, cfg, dimg)
            arr[idx] = x
            if sp != sm:
                skipped += 1
                continue
            fd = (lp - lm) / (2 * h)
            an = g[f][idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (f, idx, fd, an)
            checked += 1
    assert checked > 10 * skipped
