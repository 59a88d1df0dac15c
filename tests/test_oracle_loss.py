"""The oracle's L1 loss against hand values and finite differences."""
import numpy as np

import oracle


def test_l1_hand_values():
    img = np.array([0.5, 0.2, 0.2, 1.0])
    tgt = np.array([0.2, 0.2, 0.5, 0.0])
    loss, g = oracle.l1_loss(img, tgt)
    assert abs(loss - (0.3 + 0.0 + 0.3 + 1.0) / 4) < 1e-15
    assert np.array_equal(g, np.array([1.0, 0.0, -1.0, 1.0]) / 4)


def test_l1_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(3, 7, 5))
    tgt = rng.uniform(size=(3, 7, 5))
    _, g = oracle.l1_loss(img, tgt)
    h = 1e-7   # far below the smallest |img - tgt| of this draw
    assert np.abs(img - tgt).min() > 1e-4
    for idx in [(0, 0, 0), (1, 3, 2), (2, 6, 4)]:
        e = np.zeros_like(img)
        e[idx] = h
        fd = (oracle.l1_loss(img + e, tgt)[0] - oracle.l1_loss(img - e, tgt)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7
