"""Pins of the oracle's per-pixel work and guard-band outputs of the 3DGS
compositing (Algorithm 1 with the blending of the Background section):
the entries each pixel evaluates (``neval``), the T sensitivity used to
bound float32 transmittance (``tsens``) and the ambiguous contribution of
guard pixels (``amb``), each against a closed form on hand-built records.

Records are the shader data of the listing's project: u, v, A, B, C, o,
r, g, b with power P = A dx^2 + B dx dy + C dy^2."""
import math

import numpy as np
import pytest

import oracle

A_MIN = float(np.float32(1.0 / 255.0))
A_MAX = float(np.float32(0.99))
T_MIN = float(np.float32(1e-4))


def _cfg(**kw):
    return oracle.OracleConfig(alpha_min=A_MIN, alpha_max=A_MAX, t_min=T_MIN, **kw)


def _render(recs, W=16, H=16, **kw):
    recs = np.asarray(recs, np.float64).reshape(-1, 9)
    vals = np.arange(recs.shape[0], dtype=np.int32)
    ranges = np.array([[0, recs.shape[0]]], np.int32)
    return oracle.render_fwd(recs, vals, ranges, W, H, _cfg(**kw))


# Stacked records are centred a quarter pixel off pixel (7, 7) (an exact
# P = 0 would sit on the P > 0 gate's guard band): there dx = dy = -1/4,
# P = -1/16 and the opacity o e^{1/16} gives alpha = o.
P0 = -0.0625


def _stack(o, K, col=(0.7, 0.3, 0.5)):
    return [[7.25, 7.25, -0.5, 0.0, -0.5, o * math.exp(-P0), *col] for _ in range(K)]


@pytest.mark.parametrize("o,blended", [(0.5, 13), (0.3, 25), (0.6, 10), (0.95, 3)])
def test_neval_is_the_stopping_position(o, blended):
    # the centre pixel blends `blended` entries and stops at the next one
    K = 40
    r = _render(_stack(o, K))
    assert r["nblend"][7, 7] == blended
    assert r["neval"][7, 7] == blended + 1
    # far corner: every entry is below the alpha gate, none stops the pixel
    assert r["nblend"][15, 0] == 0 and r["neval"][15, 0] == K


def test_neval_whole_list_when_no_stop():
    r = _render(_stack(0.5, 9))   # 0.5^9 > 1e-4: no stop
    assert r["nblend"][7, 7] == 9 and r["neval"][7, 7] == 9


@pytest.mark.parametrize("o", [0.2, 0.5, 0.85])
def test_tsens_closed_form_on_a_stack(o):
    # the absolute power terms sum to |P| = 1/16: each blended entry adds
    # alpha/(1-alpha) (7/16 + 3) + 2 to the base 1
    r = _render(_stack(o, 40))
    k = int(r["nblend"][7, 7])
    a = o
    want = 1 + k * (a / (1 - a) * (7 * 0.0625 + 3) + 2)
    assert r["tsens"][7, 7] == pytest.approx(want, rel=1e-9)
    assert r["amb"][:, 7, 7].max() == 0.0 and r["guard"][7, 7] == 0


def test_tsens_clamped_alpha_adds_only_the_update():
    # a record with o e^P = 0.995 > alpha_max (alpha is the constant
    # alpha_max), then one with alpha = 0.5
    r = _render(_stack(0.995, 1) + _stack(0.5, 1))
    assert r["nblend"][7, 7] == 2 and r["guard"][7, 7] == 0
    assert r["Tfinal"][7, 7] == pytest.approx((1 - A_MAX) * 0.5, rel=1e-12)
    assert r["tsens"][7, 7] == pytest.approx(1 + 2 + (1.0 * (7 * 0.0625 + 3) + 2), rel=1e-9)


def test_tsens_grows_with_the_power_terms():
    # the same alpha reached from larger power terms is more sensitive:
    # pixel (8, 7) of a record at (7, 7) with A = C = -0.5 has P = -0.5
    base = _render(_stack(0.5, 1))["tsens"][7, 7]
    r = _render([[7.0, 7.0, -0.5, 0.0, -0.5, 0.5 * math.exp(0.5), 0.7, 0.3, 0.5]])
    assert r["nblend"][7, 8] == 1
    assert r["tsens"][7, 8] == pytest.approx(1 + 1.0 * (7 * 0.5 + 3) + 2, rel=1e-9)
    assert r["tsens"][7, 8] > base


def test_amb_alpha_gate_flip():
    # one record whose alpha at pixel (9, 7) is alpha_min: dx = 2, P = -2 c,
    # o = alpha_min e^{2c}; the gate keeps it (alpha >= alpha_min), the flip
    # drops it: the ambiguous contribution is its colour times alpha
    c = 0.25
    o = A_MIN * math.exp(4 * c)
    col = (0.7, 0.3, 0.5)
    r = _render([[7.0, 7.0, -c, 0.0, -c, o, *col]])
    assert r["guard"][7, 9] == 1
    a = o * math.exp(-4 * c)
    assert a == pytest.approx(A_MIN, rel=1e-12)
    assert r["amb"][0, 7, 9] == pytest.approx(max(col) * a, rel=1e-9)
    assert r["amb"][1, 7, 9] == pytest.approx(a, rel=1e-9)
    # pixel (8, 7) (P = -c, alpha = alpha_min e^{3c}) is far from every threshold
    assert r["guard"][7, 8] == 0 and r["amb"][:, 7, 8].max() == 0.0


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.2, 0.2, 0.2)])
def test_amb_stop_rule_flip(bg):
    # a stack whose 13th blend lands T exactly 0.05% above t_min: the pixel
    # blends it (T >= t_min), the flip stops there. The difference of the
    # two outputs C + T bg is o T_12 (c - bg) per channel.
    n = 13
    o = 1.0 - (T_MIN * (1 + 5e-4)) ** (1.0 / n)
    col = (0.7, 0.3, 0.5)
    r = _render(_stack(o, 20, col=col), bg=bg)
    assert r["guard"][7, 7] == 1 and r["nblend"][7, 7] == n
    T12 = (1 - o) ** (n - 1)
    want = o * T12 * max(abs(c - b) for c, b in zip(col, bg))
    assert r["amb"][0, 7, 7] == pytest.approx(want, rel=1e-9)
    assert r["amb"][1, 7, 7] == pytest.approx(o * T12, rel=1e-9)


def test_amb_sums_over_decisions():
    # two records, each at its own alpha gate at pixel (9, 7): two single
    # flips, each dropping one record; the contributions add
    c = 0.25
    o = A_MIN * math.exp(4 * c)
    cols = [(0.7, 0.3, 0.5), (0.2, 0.9, 0.1)]
    r = _render([[7.0, 7.0, -c, 0.0, -c, o, *cols[0]], [7.0, 7.0, -c, 0.0, -c, o, *cols[1]]])
    a = A_MIN
    # dropping the first: C changes by c0 a - c1 a (1 - a) + c1 a ... computed
    # directly from the two-entry blend
    full = np.array(cols[0]) * a + np.array(cols[1]) * a * (1 - a)
    drop0 = np.array(cols[1]) * a
    drop1 = np.array(cols[0]) * a
    want = np.abs(full - drop0).max() + np.abs(full - drop1).max()
    assert r["amb"][0, 7, 9] == pytest.approx(want, rel=1e-6)


@pytest.mark.parametrize("needle,guard", [(True, 1), (False, 0)])
def test_alpha_gate_band_follows_the_power_terms(needle, guard):
    # alpha at pixel (7, 7) sits 5e-4 (relative) below alpha_min. For a
    # needle-like conic whose power terms cancel (|A| = |C| = 500, B just
    # below 1000, S about 2000) the float32 rounding of the power moves alpha
    # by about 2 (7 S + 3) 2^-24 = 1.7e-3 relative: the decision is in the
    # guard band and the ambiguous contribution is the record's colour times
    # alpha. For an isotropic conic reaching the same alpha (S = |P|) it is
    # decided: not a guard pixel, nothing ambiguous.
    o = 0.5
    a = A_MIN * (1 - 5e-4)
    P = math.log(a / o)      # at dx = dy = 1
    if needle:
        A = C = -500.0
        B = P + 1000.0       # -A - C + B = P
    else:
        A = C = P / 2
        B = 0.0
    col = (0.7, 0.3, 0.5)
    r = _render([[6.0, 6.0, A, B, C, o, *col]])
    assert (r["guard"][7, 7], r["nblend"][7, 7]) == (guard, 0)
    if guard:
        assert r["amb"][0, 7, 7] == pytest.approx(max(col) * a, rel=1e-6)
        assert r["amb"][1, 7, 7] == pytest.approx(a, rel=1e-6)
    else:
        assert r["amb"][:, 7, 7].max() == 0.0
