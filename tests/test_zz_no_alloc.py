"""The allocation-free gradient entry point against the allocating one.

lbmz_net_gradients_noalloc runs the gradient kernels of lbmz_net_gradients
with their per-workgroup partial sums in the library's fixed per-GPU array.
Both are called through the C ABI on the same network and the same seeded
batch; the gradients and the loss must agree bit for bit (same kernels, same
fixed-order reductions).  Two calls in a row, the second with a smaller
batch, check that the shared array carries nothing from one call to the
next; a batch above the array's limit is rejected with a message.
"""
import sys

import numpy as np
import pytest

from gpu_helpers import require_gpu, torch  # noqa: F401

pytestmark = pytest.mark.gpu


def _say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def _batch(b, k, seed):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((b, 36, 8, 8)) * 10.0 ** rng.uniform(-6, -1, (b, 36, 8, 8))).astype(np.float32)
    x[rng.random(x.shape) < 0.3] = 0
    x[:, 9:] = x[:, 9:] ** 2          # the level energies are sums of squares
    t = rng.uniform(-12.0, -4.0, (b, k)).astype(np.float32)
    return x, t


def test_gradients_noalloc_equal_the_allocating_entry_point():
    require_gpu()
    from paper_2302_09883_amd import Net
    from paper_2302_09883_amd.learned import init_params
    from paper_2302_09883_amd.lbmz import LBMZ_EINVAL, LbmzError

    k = 12
    net = Net(k)
    net.set_params(init_params(k, seed=3))
    dev = torch.device("cuda", 0)
    for b, seed in ((300, 11), (77, 12)):
        _say("gradients noalloc, batch", b)
        x, t = _batch(b, k, seed)
        g_ref, loss_ref = net.gradients(x, t)
        xd = torch.from_numpy(x).to(dev)
        td = torch.from_numpy(t).to(dev)
        gd = torch.full((net.nparams,), float("nan"), dtype=torch.float32, device=dev)
        ld = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
        net.gradients_noalloc(xd, td, gd, ld)
        torch.cuda.synchronize()
        g = gd.cpu().numpy()
        loss = float(ld.cpu().numpy()[0])
        assert np.all(np.isfinite(g)) and np.isfinite(loss)
        assert np.array_equal(g, g_ref), float(np.max(np.abs(g - g_ref)))
        assert loss == loss_ref
    # above the fixed workspace: a clear error, nothing launched.  The limit:
    # ceil(B / 16) workgroups of 4 * nparams bytes (rounded up to 256) plus 4 bytes each
    blocks = (16 << 20) // (4 * net.nparams)
    while blocks > 0 and ((blocks * 4 * net.nparams + 255) // 256 * 256 + 4 * blocks) > (16 << 20):
        blocks -= 1
    limit = 16 * blocks
    big = limit + 16
    x, t = _batch(big, k, 13)
    xd = torch.from_numpy(x).to(dev)
    td = torch.from_numpy(t).to(dev)
    gd = torch.zeros(net.nparams, dtype=torch.float32, device=dev)
    ld = torch.zeros(1, dtype=torch.float32, device=dev)
    with pytest.raises(LbmzError) as err:
        net.gradients_noalloc(xd, td, gd, ld)
    assert err.value.code == LBMZ_EINVAL and f"batch <= {limit}" in str(err.value)
    net.close()
