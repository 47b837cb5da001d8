"""GPU parity of the Laplacian zero-crossing detector (canny_log_u8) with the
oracle, bit for bit (integer path): the Laplacian L and the edge map, on
shapes from 1x1 to several strips and row blocks with ragged tails, unaligned
rows, the largest accepted extents, thresholds from 0 to past the largest
slope, and the closed-form inputs the oracle is pinned on (constant, ramp,
quadratic, step)."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def canny():
    import paper_1710_07745_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


def check(canny, img, t, label=""):
    H, W = img.shape
    print(f"[log] {label} {H}x{W} t={t}", flush=True)
    dev = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    e, L = canny.canny_log_u8(dev, t, return_laplacian=True)
    torch.cuda.synchronize()
    oe, oL = oracle.log_u8(img, t)
    assert np.array_equal(L.cpu().numpy().astype(np.int32), oL), "Laplacian differs"
    ge = e.cpu().numpy()
    diff = np.argwhere(ge != oe)
    assert len(diff) == 0, f"{len(diff)} edge pixels differ, first {diff[:5].tolist()}"
    return ge


@pytest.mark.parametrize("H,W", [(1, 1), (1, 7), (5, 3), (2, 250), (9, 249), (31, 248), (33, 497),
                                 (40, 40), (70, 500), (64, 745), (129, 1000), (300, 17)])
def test_log_small_and_ragged(canny, H, W):
    img = workloads.natural_u8(H, W, seed=H * 7 + W)
    check(canny, img, 10, "ragged")


@pytest.mark.parametrize("t", [0, 1, 4, 10, 40, 2040, 2041, 5000])
def test_log_thresholds(canny, t):
    check(canny, workloads.natural_u8(300, 517, seed=t % 97), t, "threshold")


def test_log_512_and_4096(canny):
    e = check(canny, workloads.natural_u8(512, 512, seed=0), 10, "config-0 scene")
    assert 0.005 < (e > 0).mean() < 0.1
    check(canny, workloads.natural_u8(4096, 4096, seed=10), 10, "4096^2 benchmark image")


def test_log_7680x4320_and_odd(canny):
    check(canny, workloads.natural_u8(4320, 7680, seed=2), 10, "8K")
    check(canny, workloads.natural_u8(1001, 2049, seed=3), 6, "odd")


@pytest.mark.parametrize("H,W", [(7, 9), (129, 1000), (512, 512), (1001, 2049), (4096, 4096)])
def test_log_edges_only(canny, H, W):
    """Edges without the Laplacian output (the launch variant the benchmark
    runs: 4-byte stores into an aligned edge buffer, no Laplacian stores):
    equal to the oracle and to the run that also writes the Laplacian."""
    img = workloads.natural_u8(H, W, seed=H + 7 * W)
    print(f"[log] edges only {H}x{W}", flush=True)
    dev = torch.from_numpy(img).cuda()
    e = canny.canny_log_u8(dev, 10)
    e2, _ = canny.canny_log_u8(dev, 10, return_laplacian=True)
    torch.cuda.synchronize()
    oe, _ = oracle.log_u8(img, 10)
    assert np.array_equal(e.cpu().numpy(), oe)
    assert torch.equal(e, e2)


def test_log_unaligned(canny):
    """Rows whose start is not 4-byte aligned and odd pitches for the input,
    an odd-pitch edge buffer (byte stores)."""
    img = workloads.natural_u8(203, 611, seed=9)
    H, W = img.shape
    big = torch.zeros((H, W + 5), dtype=torch.uint8, device="cuda")
    big[:, 3:W + 3] = torch.from_numpy(img).cuda()
    eb = torch.zeros((H, W + 3), dtype=torch.uint8, device="cuda")
    canny.canny_log_u8(big[:, 3:W + 3], 8, edges=eb[:, 1:W + 1])
    torch.cuda.synchronize()
    oe, _ = oracle.log_u8(img, 8)
    assert np.array_equal(eb[:, 1:W + 1].cpu().numpy(), oe)
    assert not eb[:, 0].any() and not eb[:, W + 1:].any()


def test_log_closed_forms(canny):
    check(canny, np.full((77, 300), 131, np.uint8), 0, "constant")
    y, x = np.mgrid[0:90, 0:520]
    check(canny, ((x // 3 + y) % 256).astype(np.uint8), 1, "ramp")
    y, x = np.mgrid[0:15, 0:15]
    check(canny, ((x - 7) ** 2 + (y - 7) ** 2 + 5).astype(np.uint8), 1, "quadratic")
    img = np.zeros((50, 600), np.uint8)
    img[:, 300:] = 160
    e = check(canny, img, 40, "step")
    assert np.flatnonzero(e.any(axis=0)).tolist() == [299]


@pytest.mark.parametrize("H,W", [(3, 1 << 20), (1 << 20, 3)])
def test_log_largest_extents(canny, H, W):
    check(canny, workloads.natural_u8(H, W, seed=11), 10, "largest extent")
