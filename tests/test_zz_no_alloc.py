"""zh_hash_noalloc (scratch in a fixed device array of the library, for
callers that cannot allocate) against zh_hash through the C-ABI: codes and
keys bitwise, on two calls in a row, the second with fewer rows; a size
beyond the array's limit is refused."""
import numpy as np
import pytest

import synthdata

pytestmark = pytest.mark.gpu


def _max_rows(k):
    f = (k + 2 + 3) & ~3
    return ((8 * 1024 * 1024 - 512) // (9 + 4 * f)) & ~15


def test_hash_noalloc_equals_hash_on_two_calls():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    from paper_1004_3980_amd import zoomhash as zb
    from paper_1004_3980_amd.pipeline import GpuWorkload
    # the 1024^2 workload's parameters (L = 24, k = 20) over a smaller dictionary
    wl = synthdata.scaled(synthdata.WORKLOADS["precision"], n_dict=100_000, dict_images=8, test_h=0, test_w=0)
    g = GpuWorkload(wl)
    ctx = g.ctx
    rng = np.random.default_rng(11)
    nmax = _max_rows(wl.k)
    assert nmax == 79872
    for n in (nmax, 37_003):
        rows = torch.from_numpy(rng.choice(g.n, n, replace=False).astype(np.int64)).cuda()
        # dictionary rows plus noise: many codes close to a bin edge are fixed in FP64
        feat = (g.feat[rows] + 1e-4 * torch.randn((n, wl.D), device="cuda")).contiguous()
        c1 = torch.full((n, wl.L * wl.k), -7, dtype=torch.int32, device="cuda")
        k1 = torch.zeros((n, wl.L), dtype=torch.int64, device="cuda")
        c2 = torch.full_like(c1, -9)
        k2 = torch.ones_like(k1)
        ctx.hash(wl.scale, feat, n, c1, k1)
        ctx.hash_noalloc(wl.scale, feat, n, c2, k2)
        ctx.sync()
        assert torch.equal(c1, c2) and torch.equal(k1, k2), n
        k3 = torch.zeros_like(k1)
        ctx.hash_noalloc(wl.scale, feat, n, None, k3)       # keys alone
        ctx.sync()
        assert torch.equal(k1, k3)
    big = torch.zeros((nmax + 16, wl.D), device="cuda")
    kb = torch.zeros((nmax + 16, wl.L), dtype=torch.int64, device="cuda")
    with pytest.raises(zb.ZHError) as e:
        ctx.hash_noalloc(wl.scale, big, nmax + 16, None, kb)
    assert e.value.status == zb.ZH_EINVAL
    with pytest.raises(zb.ZHError) as e:
        ctx.hash_noalloc(wl.scale, big, 16, None, None)     # keys are required
    assert e.value.status == zb.ZH_EINVAL
