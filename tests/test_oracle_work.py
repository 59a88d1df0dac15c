"""Pins of the oracle's per-pixel work counts (the entries a pixel evaluates,
``neval``, and blends, ``nblend``) for the three methods, on a stack of K
identical primitives: every entry of a pixel's list then has the same alpha
a, which one copy alone gives as 1 - T_final. The blending of the
Background section with the stop rule of Algorithm 1 blends
k = min(K, floor(ln t_min / ln(1 - a))) entries when a passes the gate (none
otherwise) and evaluates k + 1 entries when it stops, the whole list when
it does not."""
import math

import numpy as np
import pytest

import oracle
from helpers import axis_camera, hand_scene

T_MIN = float(np.float32(1e-4))
A_MIN = float(np.float32(1.0 / 255.0))


def _cfg(method):
    return oracle.OracleConfig(tile_w=8, tile_h=8, sh_degree=0, method=method, t_min=T_MIN,
                               alpha_min=A_MIN, alpha_max=float(np.float32(0.99)))


def _stack(K, o):
    return hand_scene([[0.03, -0.02, 3.0]] * K, [[0.25, 0.14, 0.2]] * K,
                      quats=[[0.9, 0.2, -0.3, 0.25]] * K, opac=o, rgb=[0.6, 0.4, 0.2])


@pytest.mark.parametrize("method", ["3dgs", "3dgut", "linprim"])
@pytest.mark.parametrize("o", [0.35, 0.8])
def test_stack_counts(method, o):
    K = 30
    cam = axis_camera(31, 23, f=40.0)
    cfg = _cfg(method)
    one = oracle.render(_stack(1, o), cam, cfg)["fwd"]
    st = oracle.render(_stack(K, o), cam, cfg)
    f = st["fwd"]
    assert "neval" in f
    a = 1.0 - one["Tfinal"]
    lit = a > 0
    # a list position stops a pixel iff T (1 - a) < t_min; away from the
    # level (guard), k = floor(ln t_min / ln(1 - a)) entries are blended
    q = np.where(lit, math.log(T_MIN) / np.log1p(-np.where(lit, a, 0.5)), 0.5)
    safe = ~lit | (np.abs(q - np.round(q)) > 1e-6)
    k = np.where(lit, np.minimum(K, np.floor(q)), 0).astype(np.int64)
    # the list of the pixel's tile: K entries where the rect covers it
    tx = -(-cam.width // 8)
    ys, xs = np.mgrid[:cam.height, :cam.width]
    rg = st["bins"]["ranges"]
    L = (rg[:, 1] - rg[:, 0])[(ys // 8) * tx + xs // 8]
    assert set(np.unique(L)) <= {0, K}
    m = safe & (L == K)
    assert m.sum() > 50
    assert np.array_equal(f["nblend"][m], k[m])
    stops = k < K
    want = np.where(lit & stops, k + 1, K)
    assert np.array_equal(f["neval"][m], want[m])
    # at least one pixel stops and one does not
    assert (m & lit & stops).any() and (m & ~(lit & stops)).any()
    # pixels of empty tiles evaluate nothing
    assert np.all(f["neval"][L == 0] == 0)
