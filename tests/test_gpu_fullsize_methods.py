"""Parity of the 3DGUT and LinPrim forward paths (LinPrim also with its tile
cull) at the full benchmark size (3M primitives, SH degree 3, 1600x1064,
16x16 tiles), in the launch configuration the bench times, on sampled
outputs the oracle computes one by one: 100k sampled primitives for the
projection, 48 sampled tiles for binning (their complete lists, bit-exact,
the oracle applying its own cull to the GPU's float32 records) and for
compositing (every pixel of those tiles within 1e-5, n_contrib exact), plus
size-independent properties of the whole pair list."""
import functools

import numpy as np
import pytest

import oracle
import test_gpu_gut as GUT
import test_gpu_linprim as LIN
from gpu_util import cam32, log, ocfg_of, run_gpu, TOL_PIXEL
from paper_2606_11529_amd import renderer as R
from synth import random_cameras, scene_clusters

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=1)
def _scene():
    log("[full-m] generating 3M-primitive scene")
    return scene_clusters(3_000_000, seed=0), random_cameras(8, 0, (1600, 1064))[0]


def _sampled_tiles(g, tx, H, W, seed):
    rng = np.random.default_rng(seed)
    nonempty = np.nonzero(g["ranges"][:, 1] > g["ranges"][:, 0])[0]
    tiles = np.sort(rng.choice(nonempty, 48, replace=False))
    mask = np.zeros((H, W), bool)
    for t in tiles:
        y, x = divmod(int(t), tx)
        mask[16 * y:16 * y + 16, 16 * x:16 * x + 16] = True
    return tiles, mask


@pytest.mark.parametrize("method,cull", [("3dgut", False), ("linprim", False), ("linprim", True)])
def test_fullsize_method_sampled(method, cull):
    sc, cam = _scene()
    cfg = R.Config(sh_degree=3, method=method, tile_cull=cull)
    log(f"[full-m] method={method} cull={cull} n={sc.n} {cam.width}x{cam.height}")
    g = run_gpu(sc, cam, cfg)
    oc = ocfg_of(cfg)
    H, W = cam.height, cam.width
    tx, ty = (W + 15) // 16, (H + 15) // 16
    ncol = 21 if method == "3dgut" else 17

    # P1: projection of 100k sampled primitives
    idx = np.sort(np.random.default_rng(4).choice(sc.n, 100_000, replace=False))
    check = GUT._check_projection if method == "3dgut" else LIN._check_projection
    ng = check(sc, cam, cfg, g, idx)

    # whole list: sorted by (tile, depth), ranges delimit the tiles
    keys = g["keys"]
    assert np.all(keys[1:] >= keys[:-1]), "keys not sorted"
    if not cull:
        assert g["I"] == int(g["tc"].astype(np.int64).sum())
    tile_of = (keys >> np.uint64(32)).astype(np.int64)
    starts = np.flatnonzero(np.r_[True, tile_of[1:] != tile_of[:-1]])
    ends = np.r_[starts[1:], keys.size]
    r = g["ranges"]
    assert np.array_equal(r[tile_of[starts], 0], starts)
    assert np.array_equal(r[tile_of[starts], 1], ends)
    assert np.array_equal(keys & np.uint64(0xffffffff),
                          g["depth"][g["vals"]].view(np.uint32).astype(np.uint64))

    # P2: the complete lists of 48 sampled tiles, from the records touching them
    tiles, mask = _sampled_tiles(g, tx, H, W, seed=5)
    rect = g["rect"]
    touch = np.zeros(rect.shape[0], bool)
    for t in tiles:
        y, x = divmod(int(t), tx)
        touch |= ((g["tc"] > 0) & (rect[:, 0] <= x) & (x < rect[:, 2]) & (rect[:, 1] <= y)
                  & (y < rect[:, 3]))
    sub = np.flatnonzero(touch)
    rec = g["splat"][:, :ncol].astype(np.float64)
    cull_arg = (rec[sub], W, H, oc) if cull else None
    ref = oracle.bin_pairs(g["depth"][sub].astype(np.float64), rect[sub], g["tc"][sub], tx, ty,
                           cull_arg)
    assert ref["n_guard"] == 0, f"{ref['n_guard']} guard pairs in the sampled tiles"
    for t in tiles:
        a, b = ref["ranges"][t]
        assert np.array_equal(g["vals"][r[t, 0]:r[t, 1]], sub[ref["vals"][a:b]]), f"tile {t}"

    # P3: compositing of the sampled tiles
    rg = np.zeros_like(r)
    rg[tiles] = r[tiles]
    if method == "3dgut":
        fr = oracle.render_fwd_gut(rec, g["vals"], rg, cam32(cam), oc)
    else:
        fr = oracle.render_fwd_lin(rec, g["vals"], rg, W, H, oc)
    sel = mask & ~fr["guard"].astype(bool)
    emax = float(np.abs(g["image"][0] - fr["img"])[:, sel].max())
    assert emax <= TOL_PIXEL, f"pixel max-abs {emax}"
    assert np.array_equal(g["ncontrib"][0][sel], fr["ncontrib"][sel]), "n_contrib differs"
    terr = float(np.abs(g["Tfinal"][0][sel] - fr["Tfinal"][sel]).max())
    assert terr <= TOL_PIXEL, f"T_final {terr}"
    gsel = mask & fr["guard"].astype(bool)
    if gsel.any():
        assert np.abs(g["image"][0] - fr["img"])[:, gsel].max() <= 1e-2
    log(f"[full-m] {method} cull={cull}: {idx.size} projected ({ng} guard), I={g['I']}, "
        f"{tiles.size} tiles / {sub.size} records bit-exact, max-abs {emax:.2e} over "
        f"{int(sel.sum())} px ({int(gsel.sum())} guard)")
