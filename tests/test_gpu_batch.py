"""GPU parity for the batched uneven-size path: every image's edge map must be
bit-identical to the single-image path and to the oracle (paper Section 2.2.1,
Steps 1-4 per image), through one plan replayed several times with new buffers."""
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


def step(msg):
    print(f"[batch test] {msg}", flush=True)


def make_images(shapes, seed0):
    return [workloads.natural_u8(h, w, seed=seed0 + i) for i, (h, w) in enumerate(shapes)]


def test_batch_matches_single_and_oracle(canny):
    rng = np.random.default_rng(21)
    shapes = [(1, 1), (1, 700), (500, 1), (3, 5)] + [
        (int(rng.integers(2, 700)), int(rng.integers(2, 900))) for _ in range(24)]
    imgs = make_images(shapes, 100)
    step("create plan (28 images)")
    plan = canny.BatchPlan(shapes, 40, 100)
    dev = [torch.from_numpy(im).cuda() for im in imgs]
    step("first replay")
    out = plan.run(dev)
    torch.cuda.synchronize()
    step("compare")
    for k, (im, e) in enumerate(zip(imgs, out)):
        single = canny.canny_u8(dev[k], 40, 100)
        torch.cuda.synchronize()
        assert torch.equal(e, single), k
        oe, _ = oracle.canny_u8(im, 40, 100)
        assert np.array_equal(e.cpu().numpy(), oe), k
    # replay with other images in other buffers (same plan, no new recording)
    imgs2 = make_images(shapes, 900)
    dev2 = [torch.from_numpy(im).cuda() for im in imgs2]
    for rep in range(3):
        out2 = plan.run(dev2)
        torch.cuda.synchronize()
        for k, (im, e) in enumerate(zip(imgs2, out2)):
            assert np.array_equal(e.cpu().numpy(), oracle.canny_u8(im, 40, 100)[0]), (rep, k)
    plan.close()


def test_batch_pitched_inputs(canny):
    shapes = [(123, 301), (64, 64), (70, 1000)]
    imgs = make_images(shapes, 7)
    views = []
    for im in imgs:
        h, w = im.shape
        buf = torch.zeros((h, w + 13), dtype=torch.uint8, device="cuda")
        buf[:, :w] = torch.from_numpy(im)
        views.append(buf[:, :w])
    plan = canny.BatchPlan(shapes, 40, 100)
    out = plan.run(views)
    torch.cuda.synchronize()
    for im, e in zip(imgs, out):
        assert np.array_equal(e.cpu().numpy(), oracle.canny_u8(im, 40, 100)[0])


def test_batch_autotuned(canny):
    rng = np.random.default_rng(3)
    shapes = [(int(rng.integers(240, 900)), int(rng.integers(320, 1200))) for _ in range(12)]
    step("create autotuned plan")
    plan = canny.BatchPlan(shapes, 40, 100, autotune=True)
    step(f"tuned {plan.info()}")
    info = plan.info()
    assert info["fwd_rows"] in (32, 48, 64, 96, 128) and info["hyst_rows"] == 64
    imgs = make_images(shapes, 55)
    out = plan.run([torch.from_numpy(im).cuda() for im in imgs])
    torch.cuda.synchronize()
    for im, e in zip(imgs, out):
        assert np.array_equal(e.cpu().numpy(), oracle.canny_u8(im, 40, 100)[0])


def test_batch_full_256_uneven(canny):
    """The batched workload: 256 images, H ~ U{240..2160}, W ~ U{320..3840};
    every image against the single-image path, three against the oracle."""
    shapes = workloads.batch_shapes(256, seed=3)
    step("create plan (256 images)")
    plan = canny.BatchPlan(shapes, 40, 100)
    dev = [torch.from_numpy(workloads.natural_u8(h, w, seed=1000 + i)).cuda()
           for i, (h, w) in enumerate(shapes)]
    out = plan.run(dev)
    torch.cuda.synchronize()
    for k in range(len(shapes)):
        single = canny.canny_u8(dev[k], 40, 100)
        torch.cuda.synchronize()
        assert torch.equal(out[k], single), k
    for k in (0, 100, 255):
        oe, _ = oracle.canny_u8(dev[k].cpu().numpy(), 40, 100)
        assert np.array_equal(out[k].cpu().numpy(), oe), k


def test_batch_invalid(canny):
    with pytest.raises(canny.CannyError):
        canny.BatchPlan([(10, 10)], 50, 10)
    with pytest.raises(canny.CannyError):
        canny.BatchPlan([(0, 10)], 10, 50)
    plan = canny.BatchPlan([(10, 10)], 10, 50)
    with pytest.raises(ValueError):
        plan.run([torch.zeros((10, 11), dtype=torch.uint8, device="cuda")])
