"""bdg_net_forward_noalloc (the start-field network's forward pass on the
library's own device scratch) against bdg_net_forward with a caller
workspace: the same kernels, so the outputs must agree bit for bit.  Two
calls in a row, the second on a smaller input, so that the second call runs
on scratch the first one left behind; a shape beyond the scratch capacity is
refused on the host before anything is launched."""
import numpy as np
import pytest

from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _inputs(dev, C, ny, nx, B, seed):
    import torch
    from paper_2310_03341_amd import api
    rng = np.random.default_rng(seed)
    sn = api.StartNet(C, ny, nx, B, dev)
    sn.params.copy_(torch.from_numpy((rng.standard_normal(sn.nparams) * 0.2).astype(np.float32)))
    Vext = torch.from_numpy(rng.uniform(0.0, 2.0, (B, ny * nx))).to(dev)
    theta = torch.from_numpy(rng.uniform(-np.pi, np.pi, (B, ny * nx))).to(dev)
    return sn, Vext, theta


def test_noalloc_forward_matches_workspace_forward(dev):
    import torch
    C = 16
    for ny, nx, B, seed in [(24, 20, 3, 5), (12, 12, 1, 6)]:  # second call: smaller input
        print("noalloc forward C=%d %dx%d batch %d" % (C, ny, nx, B), flush=True)
        sn, Vext, theta = _inputs(dev, C, ny, nx, B, seed)
        ref = sn.forward(Vext, theta, 1.0)
        y = torch.full((B, 2, ny * nx), float("nan"), dtype=torch.float32, device=dev)
        sn.forward_noalloc(Vext, theta, 1.0, y)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), y.cpu().numpy()
        assert np.all(np.isfinite(g))
        assert np.array_equal(r, g), np.abs(r - g).max()


def test_noalloc_forward_refuses_shapes_beyond_scratch(dev):
    import torch
    from paper_2310_03341_amd import api
    # C = 64 on 64 x 64 at batch 16: 2 * 16 * 4096 * 195 bytes of layer inputs (24 MiB)
    # plus the weights fit; batch 32 (49 MiB) does not
    for B, ok in [(16, True), (32, False)]:
        sn = api.StartNet(64, 64, 64, 1, dev)
        sn.shape.batch = B
        Vext = torch.zeros((B, 64 * 64), dtype=torch.float64, device=dev)
        theta = torch.zeros_like(Vext)
        y = torch.zeros((B, 2, 64 * 64), dtype=torch.float32, device=dev)
        if ok:
            sn.forward_noalloc(Vext, theta, 1.0, y)
            torch.cuda.synchronize()
            assert torch.isfinite(y).all()
        else:
            with pytest.raises(api.BdgError) as e:
                sn.forward_noalloc(Vext, theta, 1.0, y)
            assert e.value.code == 4  # BDG_ERR_WORKSPACE
