"""Pins of the oracle's 3DGUT backward (the unscented-transform project,
pixel_info and evaluate of Listing XPR-3DGUT, blended by Algorithm 1,
differentiated by hand as the paper's pipeline is by automatic
differentiation, section Key Interfaces): torch float64 autograd of the
independent per-pixel brute force (for the parameter gradients and for the
16 per-record shader-data gradients), and central finite differences of
the tiled FP64 forward. Decisions (validity, gates, stop, rect) are piecewise
constant."""
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
                               method="3dgut")


def _clamp_scene():
    """A negative colour channel and an alpha-clamped Gaussian (opacity
    0.998 compensated below 1 only slightly) beside ordinary ones."""
    sh = np.zeros((4, 16, 3))
    sh[:, 0, :] = [[1.2, 0.3, 0.6], [0.4, -2.5, 0.8], [0.9, 0.9, 0.1], [0.2, 0.5, 1.1]]
    rng = np.random.default_rng(11)
    sh[:, 1:, :] = rng.normal(0, 0.05, size=(4, 15, 3))
    means = [[0.05, -0.03, 3.0], [0.15, 0.1, 3.5], [-0.3, 0.2, 4.0], [0.02, 0.03, 2.5]]
    scales = [[0.05, 0.03, 0.04], [0.08, 0.05, 0.06], [0.3, 0.2, 0.1], [0.6, 0.65, 0.6]]
    quats = rng.normal(size=(4, 4))
    return hand_scene(means, scales, quats=quats, opac=[0.7, 0.6, 0.5, 0.998], sh_degree=3, sh=sh)


def _scenes():
    yield "clusters", scene_clusters(40, seed=7, lo=0.03, hi=0.3, n_clusters=3, box=0.8), \
        camera_look_at((0.4, 0.3, -4.0), 40, 34)
    yield "clamps", _clamp_scene(), axis_camera(44, 36, f=40.0)


def _f64_scene(sc):
    return dataclasses.replace(sc, **{f: getattr(sc, f).astype(np.float64) for f in FIELDS})


@pytest.mark.parametrize("name,sc,cam", list(_scenes()), ids=lambda x: x if isinstance(x, str) else "")
def test_gut_analytic_matches_autograd_of_brute_force(name, sc, cam):
    cfg = _cfg()
    dimg = np.random.default_rng(0).normal(size=(3, cam.height, cam.width))
    st = oracle.render(sc, cam, cfg)
    assert st["fwd"]["guard"].sum() == 0
    g = oracle.backward(sc, cam, cfg, dimg, state=st)
    ts = brute.scene_tensors(sc, requires_grad=True)
    img, _ = brute.render_gut_torch(*ts, cam, cfg)
    np.testing.assert_allclose(img.detach().numpy(), st["fwd"]["img"], atol=1e-12)
    (img * torch.as_tensor(dimg)).sum().backward()
    ref = {"means": ts[0].grad.numpy().T, "scales": ts[1].grad.numpy().T,
           "quats": ts[2].grad.numpy().T, "opacities": ts[3].grad.numpy(),
           "sh": np.transpose(ts[4].grad.numpy(), (1, 2, 0))}
    for f in FIELDS:
        scale = max(np.abs(ref[f]).max(), 1e-12)
        assert np.abs(g[f] - ref[f]).max() <= 1e-7 * scale, f
        assert np.abs(ref[f]).max() > 0, f


@pytest.mark.parametrize("name,sc,cam", list(_scenes()), ids=lambda x: x if isinstance(x, str) else "")
def test_gut_record_gradient_matches_autograd_of_brute_force(name, sc, cam):
    """The 16 per-record values of orc_render_bwd_gut against autograd of the
    brute force at its own shader data: dL/do', dL/dcolour, dL/dro (M
    fixed) and dL/dM with the centre fixed -- the brute force forms ro from
    M and the centre, so autograd's dL/dM is that derivative. It differs
    from dL/dM at fixed ro by dL/dro (campos - mu)^T, which must not be
    zero here (the definition is then pinned, not only the sum)."""
    cfg = _cfg()
    dimg = np.random.default_rng(2).normal(size=(3, cam.height, cam.width))
    st = oracle.render(sc, cam, cfg)
    g16 = oracle.render_bwd_gut(st["proj"]["rec"], st["bins"]["vals"], st["bins"]["ranges"], cam,
                                cfg, dimg)
    ts = brute.scene_tensors(sc, requires_grad=True)
    keep = {}
    img, _ = brute.render_gut_torch(*ts, cam, cfg, keep=keep)
    (img * torch.as_tensor(dimg)).sum().backward()
    d = (keep["campos"][None, :] - ts[0]).detach().numpy()
    gro = keep["ro"].grad.numpy()
    gM = keep["M"].grad.numpy()
    ref = np.concatenate([keep["o2"].grad.numpy()[:, None], keep["colour"].grad.numpy(), gro,
                          gM.reshape(-1, 9)], axis=1)
    vis = st["proj"]["tc"] > 0
    assert vis.sum() >= 3
    shift = np.abs(gro[:, :, None] * d[:, None, :])[vis].max()
    assert shift > 0.1 * np.abs(gM[vis]).max()
    for cols, what in ((slice(0, 1), "o'"), (slice(1, 4), "colour"), (slice(4, 7), "ro"),
                       (slice(7, 16), "M")):
        r, x = ref[vis, cols], g16[vis, cols]
        scale = max(np.abs(r).max(), 1e-12)
        assert np.abs(x - r).max() <= 1e-8 * scale, what
        assert np.abs(r).max() > 0, what
    # invisible records receive nothing
    assert np.all(g16[~vis] == 0)


def test_gut_clamp_scene_exercises_clamps():
    cam = axis_camera(44, 36, f=40.0)
    pr = oracle.project(_clamp_scene(), cam, _cfg())
    assert (pr["tc"] > 0).all()
    assert pr["rec"][1, 7] == 0.0                 # negative green clamped to 0
    # the wide, nearly opaque Gaussian's alpha passes the 0.99 clamp near its centre
    px = np.array([[x, y] for y in range(cam.height) for x in range(cam.width)], np.int32)
    resp = oracle.gut_response(np.repeat(pr["rec"][3:4], len(px), 0), px, cam)
    assert (pr["rec"][3, 5] * resp).max() > 0.99


def _loss_and_sig(sc, cam, cfg, dimg):
    st = oracle.render(sc, cam, cfg)
    sig = (st["proj"]["tc"].tobytes(), st["proj"]["rect"].tobytes(), st["bins"]["vals"].tobytes(),
           st["fwd"]["ncontrib"].tobytes(), st["fwd"]["nblend"].tobytes())
    return float((st["fwd"]["img"] * dimg).sum()), sig


@pytest.mark.parametrize("name,sc,cam", list(_scenes()), ids=lambda x: x if isinstance(x, str) else "")
def test_gut_analytic_matches_central_differences(name, sc, cam):
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
