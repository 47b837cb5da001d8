"""The allocation-free entry point canny_u8_noalloc (static device scratch)
against canny_u8 (caller workspace) through the C ABI: two calls in a row,
the second on a smaller image, so that the second runs on scratch the first
left behind; class maps and edge maps must be equal bit for bit.  The smaller
image is also checked against the oracle."""
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


def one_call(canny, H, W, seed, low=40, high=100):
    print(f"[noalloc] {H}x{W} seed {seed}", flush=True)
    img = workloads.natural_u8(H, W, seed=seed)
    dev = torch.from_numpy(img).cuda()
    assert canny.u8_workspace_bytes(H, W) <= canny._lib.CANNY_NOALLOC_SCRATCH_BYTES
    e_ref, c_ref = canny.canny_u8(dev, low, high, return_classes=True)
    e = torch.full((H, W), 7, dtype=torch.uint8, device="cuda")
    c = torch.full_like(c_ref, 7)
    canny.canny_u8_noalloc(dev, low, high, edges=e, class_map=c)
    torch.cuda.synchronize()
    nb = (W + 3) // 4  # class bytes of a row (padding past them is unspecified)
    assert torch.equal(e, e_ref)
    assert torch.equal(c[:, :nb], c_ref[:, :nb])
    return img, e.cpu().numpy()


def test_noalloc_two_calls_second_smaller(canny):
    one_call(canny, 1500, 2000, seed=61)
    img, e = one_call(canny, 333, 517, seed=62)
    oe, _ = oracle.canny_u8(img, 40, 100)
    assert np.array_equal(e, oe)


def test_noalloc_rejects_too_large(canny):
    H = W = 8192
    assert canny.u8_workspace_bytes(H, W) > canny._lib.CANNY_NOALLOC_SCRATCH_BYTES
    dev = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    e = torch.empty_like(dev)
    with pytest.raises(canny.CannyError) as ex:
        canny.canny_u8_noalloc(dev, 40, 100, edges=e)
    assert ex.value.status == canny._lib.CANNY_ERR_TOO_LARGE


def test_noalloc_at_the_scratch_limit(canny):
    """The largest square (a multiple of 64) whose workspace fits the scratch
    runs and matches canny_u8; the next one up is rejected."""
    lim = canny._lib.CANNY_NOALLOC_SCRATCH_BYTES
    S = 64
    while canny.u8_workspace_bytes(S + 64, S + 64) <= lim:
        S += 64
    one_call(canny, S, S, seed=63)
    big = torch.zeros((S + 64, S + 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(canny.CannyError) as ex:
        canny.canny_u8_noalloc(big, 40, 100, edges=torch.empty_like(big))
    assert ex.value.status == canny._lib.CANNY_ERR_TOO_LARGE
