"""Dictionary-construction tools through the C-ABI against the oracle:
training-crop corners and crops bit-exact (integer weights and cumulative
sums, so no rounding order enters), bucket entropies within 1e-12 relative
(FP64 sums in another order, device log2)."""
import numpy as np
import pytest

import synthdata
from oracle import pipeline, training

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


@pytest.fixture(scope="module")
def ctx():
    _torch()
    from paper_1004_3980_amd import zoomhash as zb
    return zb.Context(0)


def _crops(ctx, stack, draws, side, with_crops=True):
    torch = _torch()
    n, H, W = stack.shape
    m = draws.shape[1]
    imgs = torch.from_numpy(np.ascontiguousarray(stack, dtype=np.float32)).cuda()
    dr = torch.from_numpy(np.ascontiguousarray(draws).view(np.int64)).cuda()
    corners = torch.full((n, m, 2), -7, dtype=torch.int32, device="cuda")
    crops = torch.empty((n, m, side, side), dtype=torch.float32, device="cuda") if with_crops else None
    ctx.sample_crops(imgs, n, H, W, dr, m, side, corners, crops)
    torch.cuda.synchronize()
    return corners.cpu().numpy(), (crops.cpu().numpy() if with_crops else None)


@pytest.mark.parametrize("n,H,W,m,side", [(3, 300, 257, 500, 100), (2, 41, 33, 200, 33), (1, 5, 7, 50, 1)])
def test_crops_bit_exact(ctx, n, H, W, m, side):
    stack = synthdata.image_stack(synthdata.SEED_BASE + 8000 + H, n, H, W)
    draws = synthdata.crop_draws(synthdata.SEED_BASE + 8100 + H, n, m)
    c_ref, x_ref = training.sample_crops(stack, draws, side)
    c, x = _crops(ctx, stack, draws, side)
    assert np.array_equal(c, c_ref)
    assert np.array_equal(x, x_ref)


def test_crops_of_flat_edge_and_bright_images(ctx):
    H, W = 64, 80
    stack = np.zeros((3, H, W), np.float32)
    stack[0] = 0.25                         # no gradient: uniform centres
    stack[1, :, 50:] = 1.0                  # one vertical edge
    stack[2] = synthdata.fractal_voronoi_image(synthdata.SEED_BASE + 8200, H, W)
    stack[2, 10, 10] = 3e38                 # saturated weights around one pixel
    draws = synthdata.crop_draws(synthdata.SEED_BASE + 8201, 3, 300)
    c_ref, x_ref = training.sample_crops(stack, draws, 16)
    c, x = _crops(ctx, stack, draws, 16)
    assert np.array_equal(c, c_ref) and np.array_equal(x, x_ref)


def test_crops_of_a_large_image(ctx):
    # 2048^2: 4096 blocks of cumulative weights, the block scan in 16 passes
    img = synthdata.fractal_voronoi_image(synthdata.SEED_BASE + 8300, 2048, 2048)[None]
    draws = synthdata.crop_draws(synthdata.SEED_BASE + 8301, 1, 4000)
    cen = training.sample_centres(img[0], draws[0])
    c_ref = training.crop_corners(cen, 2048, 2048, 100)[None]
    c, _ = _crops(ctx, img, draws, 100, with_crops=False)
    assert np.array_equal(c, c_ref)


def test_crop_argument_errors(ctx):
    torch = _torch()
    from paper_1004_3980_amd import zoomhash as zb
    imgs = torch.zeros((1, 20, 30), device="cuda")
    dr = torch.zeros((1, 4), dtype=torch.int64, device="cuda")
    cor = torch.zeros((1, 4, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(zb.ZHError):
        ctx.sample_crops(imgs, 1, 20, 30, dr, 4, 21, cor)      # crop taller than the image
    with pytest.raises(zb.ZHError):
        ctx.sample_crops(imgs, 1, 20, 30, dr, 4, 0, cor)


@pytest.mark.parametrize("name,kw", [("tiny", {}), ("tiny", {"scale": 3, "n_dict": 10000}),
                                     ("mid", {"n_dict": 60000, "dict_images": 16})])
def test_table_entropy(name, kw):
    _torch()
    from paper_1004_3980_amd.pipeline import GpuWorkload
    wl = synthdata.scaled(synthdata.WORKLOADS[name], **kw)
    g = GpuWorkload(wl)
    got = g.ctx.table_entropy(wl.scale, wl.L)
    pre = pipeline.prepare(wl.dictionary_images(), wl.positions(), wl.scale, wl.feat_mode, wl.L, wl.k, wl.w,
                           wl.hash_seed)
    keys = np.stack(pre.tables.sorted_keys, axis=1)
    ref = training.bucket_entropy(keys)
    assert np.all(np.abs(got - ref) <= 1e-12 * ref), (got, ref)
    from paper_1004_3980_amd import zoomhash as zb
    with pytest.raises(zb.ZHError):
        g.ctx.table_entropy(wl.scale, wl.L - 1)                # no room for L values
