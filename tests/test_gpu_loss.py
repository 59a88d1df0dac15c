"""The fused L1 loss kernel against the oracle's definition: the gradient
bit-exact (sign(image - target) times the float32 1/n), the loss within
1e-5 relative (float32 partial sums); vector and scalar paths, ragged tails,
exact ties, and n = 0."""
import numpy as np
import pytest
import torch

import oracle
from paper_2606_11529_amd import renderer as R

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,offset", [(3 * 1600 * 1064, 0), (3 * 97 * 53, 0), (1001, 1),
                                      (7, 0), (5, 3)])
def test_l1_loss_matches_oracle(n, offset):
    rng = np.random.default_rng(n + offset)
    img = rng.uniform(size=n).astype(np.float32)
    tgt = rng.uniform(size=n).astype(np.float32)
    tie = rng.random(n) < 0.05
    tgt[tie] = img[tie]
    # an offset view of a larger buffer exercises the unaligned (scalar) path
    gi = torch.zeros(n + offset, device="cuda")
    gt = torch.zeros(n + offset, device="cuda")
    gi[offset:] = torch.from_numpy(img).cuda()
    gt[offset:] = torch.from_numpy(tgt).cuda()
    loss, dimg = R.xpr_l1_loss(gi[offset:], gt[offset:])
    torch.cuda.synchronize()
    ref_loss, ref_g = oracle.l1_loss(img, tgt)
    got = dimg.cpu().numpy()
    assert np.array_equal(got, ref_g.astype(np.float32))
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * ref_loss
    assert np.all(got[tie] == 0)


def test_l1_loss_empty():
    loss = torch.full((1,), 7.0, device="cuda")
    e = torch.empty(0, device="cuda")
    R.xpr_l1_loss(e, e, loss=loss, dimage=torch.empty(0, device="cuda"))
    torch.cuda.synchronize()
    assert float(loss.item()) == 0.0
