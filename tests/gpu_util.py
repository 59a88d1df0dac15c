"""Helpers for the GPU parity tests: run the HIP path through the C-ABI and
compare each stage with the FP64 oracle on the same inputs (the stage-wise
protocol: each oracle stage is fed the GPU's previous-stage outputs so that
float32 rounding upstream does not leak into the comparison)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_2606_11529_amd import renderer as R

TOL_PIXEL = 1e-5     # max-abs on FP32 pixel colours
TOL_GRAD = 1e-3      # relative on gradients
U32 = 2.0 ** -24     # float32 unit roundoff
T_SAFETY = 2.0      # slack on the first-order T_final rounding bound


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cam32(cam):
    """The camera exactly as the C-ABI receives it (float32 fields), as
    float64 values for the oracle: both sides then start from identical
    inputs."""
    import dataclasses
    f = lambda x: np.asarray(x, np.float32).astype(np.float64)
    return dataclasses.replace(cam, R=f(cam.R), t=f(cam.t), fx=float(f(cam.fx)),
                               fy=float(f(cam.fy)), cx=float(f(cam.cx)), cy=float(f(cam.cy)))


def ocfg_of(cfg: R.Config) -> oracle.OracleConfig:
    """The method constants exactly as the C-ABI receives them (float32)."""
    f = lambda x: float(np.float32(x))
    return oracle.OracleConfig(tile_w=cfg.tile, tile_h=cfg.tile, sh_degree=cfg.sh_degree,
                               lowpass=f(cfg.lowpass), alpha_min=f(cfg.alpha_min),
                               alpha_max=f(cfg.alpha_max), t_min=f(cfg.t_min),
                               z_near=f(cfg.z_near), fov_clip=f(cfg.fov_clip),
                               bg=tuple(f(b) for b in cfg.bg), tile_cull=cfg.tile_cull,
                               opacity_extents=cfg.opacity_extents, method=cfg.method)


def run_gpu(sc, cams, cfg: R.Config, dimgs=None, want_keys=True, want_grad2d=True,
            device="cuda"):
    """One batch (one scene, several cameras). Returns numpy copies of every
    stage's outputs."""
    if not isinstance(cams, (list, tuple)):
        cams = [cams]
    scene = R.Scene.from_host(sc, device)
    views = R.Views([scene], cams, [0] * len(cams), cfg)
    proj = R.xpr_project(views, cfg)
    bins = R.xpr_bin_sort(views, cfg, proj, want_keys=want_keys)
    frame = R.xpr_render_fwd(views, cfg, proj, bins)
    out = dict(views=views, scene=scene)
    if dimgs is not None:
        flat = torch.cat([torch.from_numpy(np.asarray(d, np.float32)).reshape(-1)
                          for d in dimgs]).to(device)
        grads, g2 = R.xpr_render_bwd(views, cfg, proj, bins, frame, flat, want_grad2d=want_grad2d)
        out["grads"] = {k: v.cpu().numpy() for k, v in grads[0].items()}
        out["grad2d"] = g2.cpu().numpy()[:views.records] if g2 is not None else None
    torch.cuda.synchronize()
    n = views.records
    I = int(bins.n_isect.item())
    out.update(
        splat=proj.splat.cpu().numpy()[:n], depth=proj.depth.cpu().numpy()[:n],
        rect=proj.rect.cpu().numpy()[:n].astype(np.int32), tc=proj.tc.cpu().numpy()[:n],
        I=I, vals=bins.vals.cpu().numpy()[:I], ranges=bins.ranges.cpu().numpy()[:views.tiles],
        keys=bins.keys.cpu().numpy()[:I].view(np.uint64) if want_keys else None,
        image=[views.image(frame.image, v).cpu().numpy() for v in range(len(cams))],
        Tfinal=[views.plane(frame.T_final, v).cpu().numpy() for v in range(len(cams))],
        ncontrib=[views.plane(frame.n_contrib, v).cpu().numpy() for v in range(len(cams))])
    return out


def rec9(splat):
    return splat[:, :9].astype(np.float64)


# ---- P1: projection -------------------------------------------------------

def check_projection(sc, cam, cfg, gpu, rec_off=0, idx=None):
    """Floats within the stated bounds; rect/tc bit-exact except guard-band
    Gaussians. Returns (number of guard Gaussians, number checked)."""
    oc = ocfg_of(cfg)
    sub = sc if idx is None else sc.subset(idx)
    ref = oracle.project(sub, cam32(cam), oc)
    n = sub.n
    sel = np.arange(rec_off, rec_off + sc.n) if idx is None else rec_off + np.asarray(idx)
    g_rec = rec9(gpu["splat"][sel])
    g_tc = gpu["tc"][sel]
    g_rect = gpu["rect"][sel]
    g_depth = gpu["depth"][sel].astype(np.float64)
    guard = ref["guard"].astype(bool)
    vis = (ref["tc"] > 0) & (g_tc > 0)
    ok = ~guard
    # integer outputs: bit-exact outside the guard band
    bad_tc = np.nonzero(ok & (g_tc != ref["tc"]))[0]
    assert bad_tc.size == 0, f"tc mismatch at {bad_tc[:10]}: gpu {g_tc[bad_tc[:10]]} ref {ref['tc'][bad_tc[:10]]}"
    vr = ok & (ref["tc"] > 0)
    assert np.array_equal(g_rect[vr], ref["rect"][vr]), "rect mismatch"
    # floats, on Gaussians visible on both sides
    m = vis
    # The projection's geometry is evaluated in float64 and rounded to float32
    # on output, so each float output is within one float32 ulp of the
    # oracle (plus float64 noise amplified by the 2x2 inverse's condition).
    ulp = 2.0 ** -23
    uv_err = np.abs(g_rec[m, :2] - ref["rec"][m, :2]) / np.maximum(1.0, np.abs(ref["rec"][m, :2]))
    assert uv_err.max(initial=0) <= ulp, f"mean2D error {uv_err.max()}"
    d_err = np.abs(g_depth[m] - ref["depth"][m]) / np.maximum(1.0, np.abs(ref["depth"][m]))
    assert d_err.max(initial=0) <= ulp, f"depth err {d_err.max()}"
    # colour: the SH sum is accumulated in float32
    c_err = np.abs(g_rec[m, 6:9] - ref["rec"][m, 6:9])
    assert c_err.max(initial=0) <= 1e-6, f"colour err {c_err.max()}"
    assert np.array_equal(g_rec[m, 5], ref["rec"][m, 5]), "opacity must pass through"
    cov = ref["cov"][m]
    tr = cov[:, 0] + cov[:, 2]
    det = cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2
    disc = np.sqrt(np.maximum(0, 0.25 * tr * tr - det))
    cond = (0.5 * tr + disc) / np.maximum(0.5 * tr - disc, 1e-300)
    con_ref = ref["rec"][m, 2:5]
    scale = np.abs(con_ref).max(axis=1, keepdims=True)
    lim = ulp * np.abs(con_ref) + 2.0 ** -40 * (cond[:, None] + 1.0) * scale
    worst = (np.abs(g_rec[m, 2:5] - con_ref) / lim).max(initial=0)
    assert worst <= 1.0, f"conic error {worst} x bound"
    return int(guard.sum()), int(n)


# ---- P2: binning ----------------------------------------------------------

def check_binning(gpu, tiles_x_total_tiles, rec_sel=None):
    """Oracle binning fed the GPU's depth / rect / tc: offsets, I, keys, vals
    and ranges bit-exact. ``tiles_x_total_tiles`` = (tiles_x, tiles_y) for a
    single view."""
    tx, ty = tiles_x_total_tiles
    ref = oracle.bin_pairs(gpu["depth"].astype(np.float64), gpu["rect"], gpu["tc"], tx, ty)
    assert ref["I"] == gpu["I"], (ref["I"], gpu["I"])
    assert np.array_equal(gpu["vals"], ref["vals"]), "vals differ"
    if gpu["keys"] is not None:
        assert np.array_equal(gpu["keys"], ref["keys"]), "keys differ"
    assert np.array_equal(gpu["ranges"], ref["ranges"]), "ranges differ"
    return ref


def check_binning_cull(gpu, cam, cfg, tiles_x_y):
    """Binning with the per-(Gaussian, tile) cull: the oracle replicates the
    GPU's rects, applies tile_cull to every pair on the GPU's float32 splat
    (as float64) and sorts culled pairs to its sentinel tile; the GPU's lists
    must be the oracle's kept pairs, bit-exact. A pair whose decision is in
    the oracle's guard band may go either way: then every GPU pair must be
    kept or guard, and all kept non-guard pairs must be there."""
    tx, ty = tiles_x_y
    oc = ocfg_of(cfg)
    nrec = {"3dgut": 21, "linprim": 17}.get(cfg.method, 9)
    crec = gpu["splat"][:, :nrec].astype(np.float64)
    ref = oracle.bin_pairs(gpu["depth"].astype(np.float64), gpu["rect"], gpu["tc"], tx, ty,
                           (crec, cam.width, cam.height, oc))
    n = ref["I_kept"]
    if ref["n_guard"] == 0:
        assert gpu["I"] == n, (gpu["I"], n)
        assert np.array_equal(gpu["vals"], ref["vals"][:n]), "vals differ"
        if gpu["keys"] is not None:
            assert np.array_equal(gpu["keys"], ref["keys"][:n]), "keys differ"
        assert np.array_equal(gpu["ranges"], ref["ranges"]), "ranges differ"
        return ref
    lens = gpu["ranges"][:, 1] - gpu["ranges"][:, 0]
    tid = np.repeat(np.arange(tx * ty), lens)
    trec = crec[:, :17] if cfg.method == "linprim" else crec[:, :9]
    keep, _, _, g = oracle.tile_cull(trec[gpu["vals"]], np.stack([tid % tx, tid // tx], 1),
                                     cam.width, cam.height, oc)
    assert np.all(keep | g), "GPU kept a pair the oracle culls"
    assert int((keep & ~g).sum()) == n - int(ref["pair_guard"][:n].sum())
    if gpu["keys"] is not None:
        assert np.all(gpu["keys"][1:] >= gpu["keys"][:-1])
    return ref


# ---- P3: forward compositing -------------------------------------------

def check_forward(gpu, cam, cfg, v=0, ranges=None, pixel_mask=None):
    """Oracle compositing on the GPU's splat records and lists. Returns
    (max error on non-guard pixels, guard pixel count)."""
    oc = ocfg_of(cfg)
    rg = gpu["ranges"] if ranges is None else ranges
    ref = oracle.render_fwd(rec9(gpu["splat"]), gpu["vals"], rg, cam.width, cam.height, oc)
    guard = ref["guard"].astype(bool)
    sel = ~guard if pixel_mask is None else (~guard & pixel_mask)
    img = gpu["image"][v]
    err = np.abs(img - ref["img"])[:, sel]
    emax = float(err.max(initial=0))
    assert emax <= TOL_PIXEL, f"pixel max-abs {emax} > {TOL_PIXEL}"
    assert np.array_equal(gpu["ncontrib"][v][sel], ref["ncontrib"][sel]), "n_contrib differs"
    # T_final relative to the oracle's per-pixel float32 sensitivity (its
    # tsens, in units of 2^-24: the alpha roundings amplified by
    # alpha / (1 - alpha), plus two roundings per update), with a factor
    # T_SAFETY for the rounding of the staged base-2 conic and second-order
    # terms; relative, so a T near t_min is held to the same precision.
    tref = ref["Tfinal"][sel]
    tb = T_SAFETY * ref["tsens"][sel] * U32 * tref
    tr = np.abs(gpu["Tfinal"][v][sel] - tref) / tb
    assert tr.max(initial=0) <= 1.0, f"T_final error {tr.max()} x its rounding bound"
    gsel = guard if pixel_mask is None else (guard & pixel_mask)
    if gsel.any():
        # a guard pixel may take any of its ambiguous decisions either way:
        # its colour and T may move by its ambiguous contribution (summed
        # over single flips) on top of the non-guard tolerance
        gerr = np.abs(img - ref["img"])[:, gsel].max(axis=0)
        gb = ref["amb"][0][gsel] + TOL_PIXEL
        assert np.all(gerr <= gb), f"guard pixel error {(gerr / gb).max()} x its ambiguous bound"
        terr = np.abs(gpu["Tfinal"][v][gsel] - ref["Tfinal"][gsel])
        tgb = ref["amb"][1][gsel] + T_SAFETY * ref["tsens"][gsel] * U32 * ref["Tfinal"][gsel]
        assert np.all(terr <= tgb), f"guard pixel T error {(terr / tgb).max()} x bound"
    return emax, int(gsel.sum()), ref


def guard_records(ref_fwd, gpu_ncontrib, ranges, vals, tile, tiles_x):
    """Records whose gradient a guard-band decision can reach: at each guard
    pixel, the prefix of its tile's list up to one past the later of the two
    last-blended positions (a flip changes T for later entries and the
    colour-behind of earlier ones)."""
    gy, gx = np.nonzero(ref_fwd["guard"])
    if gy.size == 0:
        return np.zeros(0, np.int64)
    t = (gy // tile) * tiles_x + gx // tile
    n = np.maximum(ref_fwd["ncontrib"][gy, gx], gpu_ncontrib[gy, gx]) + 1
    out = [vals[ranges[tt, 0]:min(ranges[tt, 1], ranges[tt, 0] + nn)] for tt, nn in zip(t, n)]
    return np.unique(np.concatenate(out))


def rel_check(got, ref, name, mask=None, tol=TOL_GRAD):
    """abs(g - r) <= tol * max(abs(r), 1e-3 max abs(r)), per column."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    if mask is not None:
        got, ref = got[mask], ref[mask]
    if ref.size == 0:
        return 0.0
    floor = 1e-3 * np.abs(ref).max(axis=0, keepdims=True)
    bound = tol * np.maximum(np.abs(ref), floor)
    ratio = np.abs(got - ref) / np.maximum(bound, 1e-300)
    worst = float(ratio.max())
    assert worst <= 1.0, f"{name}: error {worst:.3g} x bound (tol {tol})"
    return worst
