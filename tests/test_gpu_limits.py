"""The largest sizes the boundary accepts.  Per axis (H, W <= 2^20; the C ABI
rejects more): parity with the oracle on a 3 x 2^20 and a 2^20 x 3 image for
the integer, float and four-sector paths, and rejection one past the limit.
In pixel count (46272^2, the most 64 x 64 tiles whose pixel count stays
below 2^31): hysteresis with a known answer at the largest component names,
and the integer and float operators against the oracle on sampled windows."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from helpers import unpack_classes

pytestmark = pytest.mark.gpu
MAXD = 1 << 20


@pytest.fixture(scope="module")
def canny():
    import paper_1710_07745_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


@pytest.mark.parametrize("shape", [(3, MAXD), (MAXD, 3)])
def test_max_extent_u8(canny, shape):
    img = workloads.natural_u8(*shape, seed=77)
    e, cls = canny.canny_u8(torch.from_numpy(img).cuda(), 40, 100, return_classes=True)
    oe, oc = oracle.canny_u8(img, 40, 100)
    assert np.array_equal(unpack_classes(cls.cpu().numpy(), *shape), oc)
    assert np.array_equal(e.cpu().numpy(), oe)


@pytest.mark.parametrize("shape", [(3, MAXD), (MAXD, 3)])
def test_max_extent_f32(canny, shape):
    X = workloads.natural_u8(*shape, seed=78).astype(np.float32)
    dev = torch.from_numpy(X).cuda()
    e, cls = canny.canny_f32(dev, return_classes=True)
    oc, _, amb, _ = oracle.classify_f32(X)
    c = unpack_classes(cls.cpu().numpy(), *shape)
    assert ((c != oc) & ((amb & 3) == 0)).sum() == 0
    assert np.array_equal(e.cpu().numpy(), oracle.hysteresis(c)[0])
    _, _, _, mx = oracle.classify_f32(X)
    e2, cls2 = canny.canny_f32_sector(dev, 1.4, 3, 0.05 * mx, 0.15 * mx, return_classes=True)
    oc2, _, amb2, _ = oracle.classify_f32_sector(X, 1.4, 3, 0.05 * mx, 0.15 * mx)
    c2 = unpack_classes(cls2.cpu().numpy(), *shape)
    assert ((c2 != oc2) & ((amb2 & 11) == 0)).sum() == 0
    assert np.array_equal(e2.cpu().numpy(), oracle.hysteresis(c2)[0])


def test_one_past_the_limit_is_rejected(canny):
    x = torch.zeros((2, MAXD + 1), dtype=torch.uint8, device="cuda")
    with pytest.raises(canny.CannyError):
        canny.canny_u8(x)
    y = torch.zeros((2, MAXD + 1), dtype=torch.float32, device="cuda")
    with pytest.raises(canny.CannyError):
        canny.canny_f32(y)


def test_hysteresis_largest_names(canny):
    """Step 4 at the largest pixel count the boundary accepts (46272^2:
    522,729 tiles, so component names reach 1.34e8, just under 2^27): weak
    lines across the whole image whose one strong pixel lies in the last tile
    column, the last tile row or the bottom-right tile (the largest names),
    and one with no strong pixel.  The class map is built on the GPU and the
    exact edge map is known: every pixel of a seeded line is an edge, nothing
    else is."""
    H = W = 46272
    assert (H // 64) * (W // 64) * 4096 < (1 << 31)
    print(f"[largest names] {H}x{W}", flush=True)
    P = canny.class_pitch(W)
    cm = torch.zeros((H, P), dtype=torch.uint8, device="cuda")
    want = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    nb = W // 4
    cm[100, :nb] = 0x55               # weak row, seeded at its right end
    cm[100, nb - 1] = 0x95            # pixel W - 1: code 2
    want[100, :] = 255
    cm[300, :nb] = 0x55               # weak row, no strong pixel
    ys = torch.arange(1000, H, device="cuda")
    cm[ys, 37 // 4] = 1 << (2 * (37 % 4))  # weak column x = 37 from y = 1000, seeded at the bottom
    cm[H - 1, 37 // 4] = 2 << (2 * (37 % 4))
    want[1000:, 37] = 255
    xs = ys                           # weak diagonal (y, y) from y = 1000, seeded at its end
    cm[ys, xs // 4] = (1 << (2 * (xs % 4))).to(torch.uint8)
    cm[H - 1, (W - 1) // 4] = 2 << (2 * ((W - 1) % 4))
    want[ys, xs] = 255
    e = canny.hysteresis(cm, H, W)
    torch.cuda.synchronize()
    assert int(e[300].max()) == 0
    assert torch.equal(e, want)


def _largest_pattern(H, W, dtype, px=37, py=53):
    """A checkerboard of px x py rectangles (levels 60 and 160) built on the
    GPU without wide temporaries."""
    xr = ((torch.arange(W, device="cuda") // px) % 2).to(torch.uint8)
    yc = ((torch.arange(H, device="cuda") // py) % 2).to(torch.uint8)
    img = (xr[None, :] ^ yc[:, None]).mul_(100).add_(60)
    return img if dtype == torch.uint8 else img.to(dtype)


@pytest.mark.parametrize("path", ["u8", "f32"])
def test_operator_largest_pixel_count(canny, path):
    """The whole operator at the largest pixel count the boundary accepts
    (46272^2).  Classes on sampled 64 x 64 windows (the corners and seeded
    random ones) equal the oracle's on crops with a halo wider than the
    operator's reach; the edge map equals Step 4 run by the standalone
    hysteresis entry point on the returned class map (the float path with
    absolute thresholds, so that a crop sees the thresholds of the image)."""
    H = W = 46272
    print(f"[largest {path}] {H}x{W}", flush=True)
    if path == "u8":
        img = _largest_pattern(H, W, torch.uint8)
        e, cls = canny.canny_u8(img, 40, 100, return_classes=True)
        halo = 6
    else:
        img = _largest_pattern(H, W, torch.float32)
        e, cls = canny.canny_f32(img, 1.4, 3, 20.0, 60.0, False, return_classes=True)
        halo = 8
    torch.cuda.synchronize()
    assert torch.equal(e, canny.hysteresis(cls, H, W))
    rng = np.random.default_rng(5)
    wins = [(0, 0), (H - 64, W - 64), (0, W - 64), (H - 64, 0)]
    wins += [(int(rng.integers(0, H - 64)), int(rng.integers(0, (W - 64) // 4)) * 4) for _ in range(8)]
    for y0, x0 in wins:
        a, b = max(0, y0 - halo), min(H, y0 + 64 + halo)
        c, d = max(0, x0 - halo), min(W, x0 + 64 + halo)
        crop = img[a:b, c:d].cpu().numpy()
        if path == "u8":
            oc = oracle.classify_u8(crop, 40, 100)[0]
            amb = np.zeros_like(oc)
        else:
            oc, _, amb, _ = oracle.classify_f32(crop, 1.4, 3, 20.0, 60.0, False)
        oc = oc[y0 - a:y0 - a + 64, x0 - c:x0 - c + 64]
        amb = amb[y0 - a:y0 - a + 64, x0 - c:x0 - c + 64]
        gc = unpack_classes(cls[y0:y0 + 64, x0 // 4:x0 // 4 + 16].cpu().numpy(), 64, 64)
        bad = (gc != oc) & ((amb & 3) == 0)
        assert not bad.any(), f"window ({y0}, {x0}): {int(bad.sum())} class mismatches"
    if path == "f32":
        # the benchmark's path at this size: relative thresholds, edges only
        # (the largest strength from the walk's per-wave slots or, past 4,096
        # waves, from one atomic word) against the class-map path, and the
        # largest strength against the oracle's on an interior crop (the
        # pattern is periodic, so a crop holds the image's largest strength)
        del e, cls
        e_rel, mx = canny.canny_f32(img, return_max=True)
        e_cls, _ = canny.canny_f32(img, return_classes=True)
        torch.cuda.synchronize()
        assert torch.equal(e_rel, e_cls)
        omx = oracle.classify_f32(img[20000:20400, 20000:20400].cpu().numpy())[3]
        assert abs(float(mx) - omx) <= 1e-5 * omx, (float(mx), omx)


def test_batch_largest_images(canny):
    """One batch plan over two images at (and near) the largest accepted size
    and a small one: every image's edges equal canny_u8 on that image alone
    (per-image tile, merge and name offsets at their largest)."""
    shapes = [(46272, 46272), (1000, 1500), (46208, 46080)]
    print(f"[largest batch] {shapes}", flush=True)
    imgs = [_largest_pattern(h, w, torch.uint8, 37 + 4 * i, 53 - 6 * i) for i, (h, w) in enumerate(shapes)]
    outs = [torch.empty((h, w), dtype=torch.uint8, device="cuda") for h, w in shapes]
    plan = canny.BatchPlan(shapes, 40, 100, autotune=False)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.run(imgs, outs, ws)
    torch.cuda.synchronize()
    for x, o in zip(imgs, outs):
        assert torch.equal(o, canny.canny_u8(x, 40, 100))
    plan.close()
