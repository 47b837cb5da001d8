"""GPU checks of the streaming integer path (canny_video_*): every frame's
edge map equals the oracle's (Section 2.2.1, Steps 1-4 per frame) bit for bit,
across slot reuse, ring depths 1-4 and pinned or pageable host buffers."""
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


def run_frames(canny, vs, frames, pinned):
    ins = [torch.from_numpy(f) for f in frames]
    outs = [torch.full(f.shape, 7, dtype=torch.uint8) for f in frames]
    if pinned:
        ins = [t.pin_memory() for t in ins]
        outs = [t.pin_memory() for t in outs]
    for a, b in zip(ins, outs):
        vs.push(a, b)
    vs.sync()
    for f, o in zip(frames, outs):
        assert np.array_equal(o.numpy(), oracle.canny_u8(f, 40, 100)[0])


@pytest.mark.parametrize("depth", [1, 2, 3, 4])
def test_video_frames_match_oracle(canny, depth):
    H, W = 301, 517
    vs = canny.VideoStream(H, W, 40, 100, depth=depth)
    frames = [workloads.natural_u8(H, W, seed=600 + 10 * depth + i) for i in range(7)]
    run_frames(canny, vs, frames, pinned=True)
    # a second batch reuses every slot after its earlier download
    run_frames(canny, vs, [workloads.natural_u8(H, W, seed=700 + i) for i in range(5)], pinned=True)
    vs.close()


def test_video_pageable_buffers_and_large_frames(canny):
    H, W = 2160, 3840
    vs = canny.VideoStream(H, W, 40, 100, depth=3)
    run_frames(canny, vs, [workloads.natural_u8(H, W, seed=800 + i) for i in range(4)], pinned=False)
    vs.close()


def test_video_rejects_bad_buffers(canny):
    vs = canny.VideoStream(16, 16)
    with pytest.raises(ValueError):
        vs.push(torch.zeros((16, 15), dtype=torch.uint8), torch.zeros((16, 16), dtype=torch.uint8))
    with pytest.raises(ValueError):
        vs.push(torch.zeros((16, 16), dtype=torch.uint8, device="cuda"),
                torch.zeros((16, 16), dtype=torch.uint8))
    vs.close()
    with pytest.raises(ValueError):
        vs.push(torch.zeros((16, 16), dtype=torch.uint8), torch.zeros((16, 16), dtype=torch.uint8))
