"""Capture of the single-image paths into a HIP graph (torch.cuda.graph): no
call of the library allocates, synchronises or records a memset, so a
captured call replays.  Each replay reads the input buffer afresh: the test
rewrites it eagerly between replays and compares every replay with an eager
call on the same image."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def canny():
    import paper_1710_07745_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


def capture(fn):
    fn()  # outside capture first: the runtime loads the code objects
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


def replay_and_compare(g, x, out, images, eager):
    for X in images:
        x.copy_(torch.from_numpy(X))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = eager(torch.from_numpy(X).cuda())
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_graph_f32_relative(canny):
    H, W = 700, 1100
    imgs = [workloads.natural_u8(H, W, seed=900 + i).astype(np.float32) for i in range(3)]
    x = torch.from_numpy(imgs[0]).cuda()
    e = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    ws = torch.empty(canny.f32_workspace_bytes(H, W), dtype=torch.uint8, device="cuda")
    g = capture(lambda: canny.canny_f32(x, edges=e, workspace=ws))
    replay_and_compare(g, x, e, [imgs[1], imgs[0], imgs[2], imgs[1]], lambda t: canny.canny_f32(t))


def test_graph_f32_sector_and_u8(canny):
    H, W = 500, 900
    fimgs = [workloads.natural_u8(H, W, seed=950 + i).astype(np.float32) for i in range(2)]
    x = torch.from_numpy(fimgs[0]).cuda()
    e = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    ws = torch.empty(canny.f32_workspace_bytes(H, W), dtype=torch.uint8, device="cuda")
    g = capture(lambda: canny.canny_f32_sector(x, 1.4, 3, 16.0, 48.0, edges=e, workspace=ws))
    replay_and_compare(g, x, e, [fimgs[1], fimgs[0], fimgs[1]],
                       lambda t: canny.canny_f32_sector(t, 1.4, 3, 16.0, 48.0))
    uimgs = [workloads.natural_u8(H, W, seed=960 + i) for i in range(2)]
    xu = torch.from_numpy(uimgs[0]).cuda()
    eu = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    wsu = torch.empty(canny.u8_workspace_bytes(H, W), dtype=torch.uint8, device="cuda")
    gu = capture(lambda: canny.canny_u8(xu, 40, 100, edges=eu, workspace=wsu))
    replay_and_compare(gu, xu, eu, [uimgs[1], uimgs[0], uimgs[1]], lambda t: canny.canny_u8(t, 40, 100))
