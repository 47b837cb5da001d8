"""Out-of-bounds write canaries for every entry point of the C ABI.

Each output and each workspace is placed inside a larger device buffer with
4 KiB guard bands of 0xA5 on both sides; an edge map also gets a row pitch
wider than the image whose padding bytes are 0xA5.  After each call the
guards and the padding must be unchanged, and the results must equal those
of a call on plain buffers.  Calls with an invalid argument must return
their error code and write nothing: the whole output (and workspace) still
holds 0xA5 afterwards.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu
G = 4096
CANARY = 0xA5


@pytest.fixture(scope="module")
def canny():
    import paper_1710_07745_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


@pytest.fixture(scope="module")
def L(canny):
    return canny._lib.lib()


class Guarded:
    """nbytes of device memory at a 256-byte aligned address inside a buffer
    whose first and last G bytes (and, until written, the region itself) hold
    0xA5."""

    def __init__(self, nbytes):
        self.n = int(nbytes)
        self.buf = torch.full((G + self.n + G,), CANARY, dtype=torch.uint8, device="cuda")
        assert self.buf.data_ptr() % 256 == 0
        self.ptr = self.buf.data_ptr() + G

    def inner(self):
        return self.buf[G:G + self.n]

    def guards_ok(self):
        torch.cuda.synchronize()
        head = self.buf[:G]
        tail = self.buf[G + self.n:]
        return bool((head == CANARY).all()) and bool((tail == CANARY).all())

    def untouched(self):
        torch.cuda.synchronize()
        return bool((self.buf == CANARY).all())


def stream():
    return torch.cuda.current_stream().cuda_stream


def edge_map(H, W, pad):
    """Guarded H x (W + pad) edge buffer; returns (guarded, pitch)."""
    pitch = W + pad
    return Guarded(H * pitch), pitch


def edges_of(g, H, W, pitch):
    rows = g.inner().view(H, pitch)
    return rows[:, :W].cpu().numpy(), rows[:, W:]


def padding_ok(g, H, W, pitch):
    _, pad = edges_of(g, H, W, pitch)
    return bool((pad == CANARY).all())


@pytest.mark.parametrize("H,W,pad", [(300, 517, 13), (257, 1000, 24), (64, 64, 0), (5, 3, 1)])
def test_u8_canaries(canny, L, H, W, pad):
    img = torch.from_numpy(workloads.natural_u8(H, W, seed=H + W)).cuda()
    ref_e, ref_c = canny.canny_u8(img, 40, 100, return_classes=True)
    e, pitch = edge_map(H, W, pad)
    cp = canny.class_pitch(W)
    cls = Guarded(H * cp)
    ws = Guarded(canny.u8_workspace_bytes(H, W))
    st = L.canny_u8(img.data_ptr(), W, H, W, 40, 100, e.ptr, pitch, cls.ptr, ws.ptr, ws.n, stream())
    assert st == 0
    assert e.guards_ok() and cls.guards_ok() and ws.guards_ok()
    assert padding_ok(e, H, W, pitch)
    got, _ = edges_of(e, H, W, pitch)
    assert np.array_equal(got, ref_e.cpu().numpy())
    nb = (W + 3) // 4
    assert torch.equal(cls.inner().view(H, cp)[:, :nb], ref_c[:, :nb])


@pytest.mark.parametrize("H,W,pad", [(200, 333, 5), (130, 1000, 24)])
@pytest.mark.parametrize("mode", ["relative", "absolute", "edges_only", "sector"])
def test_f32_canaries(canny, L, H, W, pad, mode):
    X = torch.from_numpy(workloads.natural_u8(H, W, seed=7 * H + W).astype(np.float32)).cuda()
    rel = mode in ("relative", "edges_only")
    lo, hi = (0.05, 0.15) if rel else (16.0, 48.0)
    e, pitch = edge_map(H, W, pad)
    ws = Guarded(canny.f32_workspace_bytes(H, W))
    cp = canny.class_pitch(W)
    if mode == "sector":
        ref = canny.canny_f32_sector(X, 1.4, 3, lo, hi)
        cls, mag = Guarded(H * cp), Guarded(H * W * 4)
        st = L.canny_f32_sector(X.data_ptr(), W, H, W, 1.4, 3, lo, hi, e.ptr, pitch, cls.ptr,
                                mag.ptr, ws.ptr, ws.n, stream())
        outs = [cls, mag]
    elif mode == "edges_only":
        ref = canny.canny_f32(X, 1.4, 3, lo, hi, True)
        mx = Guarded(4)
        st = L.canny_f32(X.data_ptr(), W, H, W, 1.4, 3, lo, hi, 1, e.ptr, pitch, None, None,
                         mx.ptr, ws.ptr, ws.n, stream())
        outs = [mx]
    else:
        ref = canny.canny_f32(X, 1.4, 3, lo, hi, rel)
        cls, mag, mx = Guarded(H * cp), Guarded(H * W * 4), Guarded(4)
        st = L.canny_f32(X.data_ptr(), W, H, W, 1.4, 3, lo, hi, int(rel), e.ptr, pitch, cls.ptr,
                         mag.ptr, mx.ptr if rel else None, ws.ptr, ws.n, stream())
        outs = [cls, mag] + ([mx] if rel else [])
    assert st == 0
    assert e.guards_ok() and ws.guards_ok() and all(o.guards_ok() for o in outs)
    assert padding_ok(e, H, W, pitch)
    got, _ = edges_of(e, H, W, pitch)
    assert np.array_equal(got, ref.cpu().numpy())


def test_hysteresis_canaries(canny, L):
    H, W, pad = 190, 700, 12
    cls = workloads.random_classes(H, W, seed=3, p_weak=0.4, p_strong=0.01)
    from helpers import pack_classes
    packed = torch.from_numpy(pack_classes(cls)).cuda()
    ref = canny.hysteresis(packed, H, W)
    e, pitch = edge_map(H, W, pad)
    ws = Guarded(int(L.canny_hysteresis_workspace_bytes(H, W)))
    assert L.canny_hysteresis(packed.data_ptr(), H, W, e.ptr, pitch, ws.ptr, ws.n, stream()) == 0
    assert e.guards_ok() and ws.guards_ok() and padding_ok(e, H, W, pitch)
    assert np.array_equal(edges_of(e, H, W, pitch)[0], ref.cpu().numpy())


def test_mag_canaries(canny, L):
    N, H, W, R = 2, 37, 91, 9
    I = torch.from_numpy(np.stack([workloads.natural_unit_f32(H, W, seed=50 + i)
                                   for i in range(N)])).cuda()
    sig = torch.tensor([1.3, 2.2], device="cuda")
    refM = canny.mag_forward(I, sig, R)
    dM = torch.randn(N, H, W, device="cuda")
    ref_dI, ref_ds = canny.mag_backward(I, sig, dM, R)
    M = Guarded(N * H * W * 4)
    assert L.canny_mag_forward(I.data_ptr(), sig.data_ptr(), N, H, W, R, M.ptr, stream()) == 0
    assert M.guards_ok()
    assert torch.equal(M.inner().view(torch.float32).view(N, H, W), refM)
    dI, ds = Guarded(N * H * W * 4), Guarded(N * 4)
    ws = Guarded(int(L.canny_mag_backward_workspace_bytes(N, H, W, R)))
    assert L.canny_mag_backward(I.data_ptr(), sig.data_ptr(), dM.data_ptr(), N, H, W, R, dI.ptr,
                                ds.ptr, ws.ptr, ws.n, stream()) == 0
    assert dI.guards_ok() and ds.guards_ok() and ws.guards_ok()
    assert torch.equal(dI.inner().view(torch.float32).view(N, H, W), ref_dI)
    assert torch.equal(ds.inner().view(torch.float32), ref_ds)


def test_batch_canaries(canny, L):
    shapes = [(61, 130), (300, 517), (1, 1), (77, 1000)]
    imgs = [torch.from_numpy(workloads.natural_u8(h, w, seed=i)).cuda() for i, (h, w) in enumerate(shapes)]
    plan = canny.BatchPlan(shapes, 40, 100)
    ref = plan.run(imgs)
    pads = [3, 24, 0, 8]
    outs = [edge_map(h, w, p) for (h, w), p in zip(shapes, pads)]
    ws = Guarded(plan.workspace_bytes)
    n = len(shapes)
    ip = (C.c_void_p * n)(*[t.data_ptr() for t in imgs])
    ipt = (C.c_int64 * n)(*[t.stride(0) for t in imgs])
    ep = (C.c_void_p * n)(*[g.ptr for g, _ in outs])
    ept = (C.c_int64 * n)(*[p for _, p in outs])
    st = L.canny_batch(plan._h, C.cast(ip, C.c_void_p), C.cast(ipt, C.c_void_p),
                       C.cast(ep, C.c_void_p), C.cast(ept, C.c_void_p), ws.ptr, ws.n, stream())
    assert st == 0
    assert ws.guards_ok()
    for (g, p), (h, w), r in zip(outs, shapes, ref):
        assert g.guards_ok() and padding_ok(g, h, w, p)
        assert np.array_equal(edges_of(g, h, w, p)[0], r.cpu().numpy())
    plan.close()


def test_video_host_canaries(canny, L):
    H, W = 70, 133
    frames = [torch.from_numpy(workloads.natural_u8(H, W, seed=900 + i)) for i in range(3)]
    ref = [canny.canny_u8(f.cuda(), 40, 100).cpu().numpy() for f in frames]
    vs = canny.VideoStream(H, W, 40, 100, depth=2)
    bufs = [np.full(G + H * W + G, CANARY, np.uint8) for _ in frames]
    for f, b in zip(frames, bufs):
        st = L.canny_video_push(vs._h, f.data_ptr(), b.ctypes.data + G)
        assert st == 0
    vs.sync()
    vs.close()
    for b, r in zip(bufs, ref):
        assert (b[:G] == CANARY).all() and (b[G + H * W:] == CANARY).all()
        assert np.array_equal(b[G:G + H * W].reshape(H, W), r)


# ------------------------------------------------------- invalid arguments

def test_invalid_calls_write_nothing(canny, L):
    H, W = 100, 200
    img = torch.from_numpy(workloads.natural_u8(H, W, seed=1)).cuda()
    X = img.float()
    e, pitch = edge_map(H, W, 8)
    cls = Guarded(H * canny.class_pitch(W))
    mag, mx = Guarded(H * W * 4), Guarded(4)
    ws_u8 = Guarded(canny.u8_workspace_bytes(H, W))
    ws_f32 = Guarded(canny.f32_workspace_bytes(H, W))
    s = stream()
    calls = [
        # low > high, negative low, pitch < W, workspace too small
        (1, lambda: L.canny_u8(img.data_ptr(), W, H, W, 100, 40, e.ptr, pitch, cls.ptr, ws_u8.ptr, ws_u8.n, s)),
        (1, lambda: L.canny_u8(img.data_ptr(), W, H, W, -1, 40, e.ptr, pitch, cls.ptr, ws_u8.ptr, ws_u8.n, s)),
        (1, lambda: L.canny_u8(img.data_ptr(), W - 1, H, W, 40, 100, e.ptr, pitch, cls.ptr, ws_u8.ptr, ws_u8.n, s)),
        (2, lambda: L.canny_u8(img.data_ptr(), W, H, W, 40, 100, e.ptr, pitch, cls.ptr, ws_u8.ptr, ws_u8.n - 1, s)),
        (1, lambda: L.canny_f32(X.data_ptr(), W, H, W, 1.4, 3, 0.2, 0.1, 1, e.ptr, pitch, cls.ptr,
                                mag.ptr, mx.ptr, ws_f32.ptr, ws_f32.n, s)),
        (1, lambda: L.canny_f32(X.data_ptr(), W, H, W, -1.0, 3, 0.05, 0.15, 1, e.ptr, pitch, cls.ptr,
                                mag.ptr, mx.ptr, ws_f32.ptr, ws_f32.n, s)),
        (1, lambda: L.canny_f32(X.data_ptr(), W, H, W, 1.4, 9, 0.05, 0.15, 1, e.ptr, pitch, cls.ptr,
                                mag.ptr, mx.ptr, ws_f32.ptr, ws_f32.n, s)),
        (2, lambda: L.canny_f32(X.data_ptr(), W, H, W, 1.4, 3, 0.05, 0.15, 1, e.ptr, pitch, cls.ptr,
                                mag.ptr, mx.ptr, ws_f32.ptr, 1024, s)),
        (1, lambda: L.canny_f32_sector(X.data_ptr(), W, H, W, 1.4, 3, 60.0, 20.0, e.ptr, pitch,
                                       cls.ptr, mag.ptr, ws_f32.ptr, ws_f32.n, s)),
        (1, lambda: L.canny_hysteresis(cls.ptr, H, W, e.ptr, W - 1, ws_u8.ptr, ws_u8.n, s)),
        (1, lambda: L.canny_mag_forward(X.data_ptr(), mx.ptr, 1, H, W, 13, mag.ptr, s)),
        (1, lambda: L.canny_mag_backward(X.data_ptr(), mx.ptr, X.data_ptr(), 1, H, W, 0, mag.ptr,
                                         mx.ptr, ws_f32.ptr, ws_f32.n, s)),
    ]
    for k, (code, fn) in enumerate(calls):
        assert fn() == code, k
        for g in (e, cls, mag, mx, ws_u8, ws_f32):
            assert g.untouched(), k
