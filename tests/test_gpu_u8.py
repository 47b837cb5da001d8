"""GPU parity for the integer path: class maps and edge maps bit-exact against
the CPU oracle (paper Section 2.2.1, Steps 1-4), through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from helpers import pack_classes, unpack_classes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def canny():
    import paper_1710_07745_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


def run_u8(canny, img, low=40, high=100, pitch_pad=0, offset=0):
    H, W = img.shape
    if pitch_pad or offset:
        buf = torch.zeros(H * (W + pitch_pad) + offset + 64, dtype=torch.uint8, device="cuda")
        view = buf[offset:offset + H * (W + pitch_pad)].view(H, W + pitch_pad)[:, :W]
        view.copy_(torch.from_numpy(img))
        dev = view
    else:
        dev = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    edges, cls = canny.canny_u8(dev, low, high, return_classes=True)
    torch.cuda.synchronize()
    return edges.cpu().numpy(), unpack_classes(cls.cpu().numpy(), H, W)


def check_exact(canny, img, low=40, high=100, **kw):
    e, c = run_u8(canny, img, low, high, **kw)
    oe, oc = oracle.canny_u8(img, low, high)
    H, W = img.shape
    bad = np.argwhere(c != oc)
    assert bad.size == 0, f"class mismatch at {bad[:5].tolist()} (H={H}, W={W}) gpu={c[tuple(bad[0])]} oracle={oc[tuple(bad[0])]}"
    if not np.array_equal(e, oe):
        d = np.argwhere(e != oe)
        info = [(int(y), int(x), int(y) % 64, int(x) % 64, int(e[y, x]), int(oe[y, x]), int(oc[y, x]))
                for y, x in d[:12]]
        raise AssertionError(f"edge mismatch (H={H}, W={W}): {len(d)} px, gpu-only "
                             f"{int(((e > 0) & (oe == 0)).sum())}, oracle-only "
                             f"{int(((e == 0) & (oe > 0)).sum())}; (y, x, y%64, x%64, gpu, oracle, class) {info}")
    return oc


def test_config0_512(canny):
    """512x512 natural image, low 40 / high 100."""
    oc = check_exact(canny, workloads.natural_u8(512, 512, seed=0))
    assert (oc == 2).sum() > 100 and (oc == 1).sum() > 100


@pytest.mark.parametrize("H", [1, 2, 3, 4, 5, 7, 8, 9, 13, 31, 32, 33, 36, 37, 40, 41])
def test_small_sizes(canny, H):
    for W in [1, 2, 3, 4, 5, 6, 7, 8, 9, 11, 16, 17, 31, 33, 40]:
        img = workloads.natural_u8(H, W, seed=H * 64 + W)
        check_exact(canny, img, 10, 40)


@pytest.mark.parametrize("H,W", [(300, 517), (257, 249), (250, 251), (1000, 1001), (64, 1000), (1000, 3)])
def test_ragged_multi_tile(canny, H, W):
    check_exact(canny, workloads.natural_u8(H, W, seed=H + 7 * W))


@pytest.mark.parametrize("pad,offset", [(3, 0), (1, 1), (64, 3), (4, 4)])
def test_unaligned_pitch(canny, pad, offset):
    check_exact(canny, workloads.natural_u8(123, 301, seed=5), pitch_pad=pad, offset=offset)


# Shapes for the balanced forward launch (interior blocks of 40 rows, border
# blocks of 20): images under 20 rows, exactly 40 rows (no interior block),
# 55 rows (two bottom border blocks), three border strips (the right halo of
# the second-to-last strip leaves the image), and every strip bordered (rows
# not 4-byte aligned).
@pytest.mark.parametrize("H,W", [(19, 253952), (40, 130000), (55, 90000), (3000, 4218)])
def test_balanced_split_shapes(canny, H, W):
    check_exact(canny, workloads.natural_u8(H, W, seed=H + W))


def test_balanced_split_unaligned(canny):
    check_exact(canny, workloads.natural_u8(2048, 4096, seed=44), pitch_pad=3, offset=1)


def test_step_edge_golden(canny):
    for D, expect_line in [(15, False), (16, False), (40, False), (41, False), (42, True), (120, True)]:
        for transpose in (False, True):
            img = np.full((24, 24), 100, np.uint8)
            img[:, 12:] = 100 + D
            if transpose:
                img = img.T.copy()
            e, _ = run_u8(canny, img)
            exp = np.zeros((24, 24), np.uint8)
            if expect_line:
                if transpose:
                    exp[11, :] = 255
                else:
                    exp[:, 11] = 255
            assert np.array_equal(e, exp), (D, transpose)


def test_degenerate(canny):
    flat = np.full((70, 300), 9, np.uint8)
    e, c = run_u8(canny, flat, 0, 0)
    assert not e.any() and not c.any()
    img = workloads.natural_u8(200, 260, seed=4)
    for lo, hi in [(0, 0), (0, 2040), (40, 40), (2040, 2040), (3000, 5000), (0, 1)]:
        check_exact(canny, img, lo, hi)


def test_noise_only(canny):
    rng = np.random.default_rng(1)
    check_exact(canny, rng.integers(0, 256, (333, 444), dtype=np.uint8), 100, 400)


def test_full_4096(canny):
    """The 4096x4096 benchmark image, checked whole against the oracle."""
    check_exact(canny, workloads.natural_u8(4096, 4096, seed=10))


def test_invalid_arguments(canny):
    img = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(canny.CannyError):
        canny.canny_u8(img, 50, 10)  # low > high
    with pytest.raises(canny.CannyError):
        canny.canny_u8(img, -1, 10)
    with pytest.raises(ValueError):
        canny.canny_u8(img, 10, 20, workspace=torch.empty(3, dtype=torch.uint8, device="cuda"))


# ---------------------------------------------------------------- hysteresis alone

def run_hyst(canny, cls):
    H, W = cls.shape
    packed = torch.from_numpy(pack_classes(cls)).cuda()
    e = canny.hysteresis(packed, H, W)
    torch.cuda.synchronize()
    return e.cpu().numpy()


@pytest.mark.parametrize("h,w", [(3, 3), (3, 4)])
def test_hysteresis_exhaustive_small(canny, h, w):
    import itertools
    maps = np.array(list(itertools.product((0, 1, 2), repeat=h * w)), np.uint8)
    cols = int(np.ceil(np.sqrt(len(maps))))
    rows = -(-len(maps) // cols)
    big = np.zeros((rows * (h + 1), cols * (w + 1)), np.uint8)
    for k, m in enumerate(maps):
        r, c = divmod(k, cols)
        big[r * (h + 1):r * (h + 1) + h, c * (w + 1):c * (w + 1) + w] = m.reshape(h, w)
    assert np.array_equal(run_hyst(canny, big), oracle.hysteresis(big)[0])


@pytest.mark.parametrize("H,W,p", [(1, 1, 0.5), (1, 300, 0.6), (300, 1, 0.6), (65, 65, 0.45),
                                   (128, 64, 0.41), (1000, 1000, 0.41), (777, 1333, 0.5),
                                   (2048, 2048, 0.38), (4096, 4096, 0.42)])
def test_hysteresis_random(canny, H, W, p):
    cls = workloads.random_classes(H, W, seed=H + W, p_weak=p, p_strong=0.002)
    assert np.array_equal(run_hyst(canny, cls), oracle.hysteresis(cls)[0])


def test_hysteresis_long_chain(canny):
    """One weak spiral seeded at its outer end: the whole chain must be found."""
    N = 2048
    ys, xs = workloads.spiral_path(N, spacing=4)
    cls = np.zeros((N, N), np.uint8)
    cls[ys, xs] = 1
    cls[ys[0], xs[0]] = 2
    e = run_hyst(canny, cls)
    oe, depth = oracle.hysteresis(cls)
    assert depth > 100000
    assert np.array_equal(e, oe)


def _line_classes(N, kind, seed_at):
    """A one-pixel weak line across the whole image (16 tiles of 64 pixels),
    strong at one position of it (or nowhere)."""
    cls = np.zeros((N, N), np.uint8)
    t = np.arange(N)
    if kind == "row":
        ys, xs = np.full(N, 100), t
    elif kind == "col":
        ys, xs = t, np.full(N, 37)
    elif kind == "diag":  # crosses every tile corner diagonally: (63, 63) -> (64, 64)
        ys, xs = t, t
    else:  # anti-diagonal: (63, 64) -> (64, 63) corners
        ys, xs = t, N - 1 - t
    cls[ys, xs] = 1
    if seed_at is not None:
        k = {"first": 0, "middle": N // 2, "last": N - 1}[seed_at]
        cls[ys[k], xs[k]] = 2
    return cls


def _comb_classes(N):
    cls = np.zeros((N, N), np.uint8)
    for r, seed in ((100, "all"), (300, "end"), (500, None)):
        cls[r, :] = 2 if seed == "all" else 1
        if seed == "end":
            cls[r, N - 1] = 2
        # teeth of uneven length, down at x = 5 mod 7 and up at x = 1 mod 7,
        # so teeth of different combs are never 8-neighbours
        for x in range(5, N - 3, 7):
            ln = 20 + (x * 37) % 90
            cls[r + 1:r + 1 + ln, x] = 1
            cls[r - ln:r, x + 3] = 1
    return cls


@pytest.mark.parametrize("kind", ["row", "col", "diag", "anti"])
@pytest.mark.parametrize("seed_at", ["first", "middle", "last", None])
def test_hysteresis_strong_anywhere_on_chain(canny, kind, seed_at):
    """One weak component spread over 16 tiles: its edge pixels appear iff a
    strong pixel lies anywhere on it, whichever tile holds that pixel (the
    strong tile's component name may be larger or smaller than those of the
    weak tiles it is joined to)."""
    N = 1024
    cls = _line_classes(N, kind, seed_at)
    e = run_hyst(canny, cls)
    oe = oracle.hysteresis(cls)[0]
    assert np.array_equal(e, oe)
    assert int((e == 255).sum()) == (0 if seed_at is None else int((cls > 0).sum()))


def test_hysteresis_combs(canny):
    """Weak teeth hanging off spines that cross tile borders: a strong spine,
    a weak spine seeded only at its far end, and a weak spine with no seed;
    teeth cross the horizontal tile borders and touch each other only
    through the spine."""
    cls = _comb_classes(768)
    e = run_hyst(canny, cls)
    oe = oracle.hysteresis(cls)[0]
    assert np.array_equal(e, oe)
    assert e[300, :].min() == 255 and e[500, :].max() == 0


def _oracle_classes_chunked(img, low, high, rows=1024, threads=16):
    """The oracle's class map of a large image, in row bands with a 4-row
    overlap (the integer pipeline reaches 4 rows: blur 2, Sobel 1,
    suppression 1), computed by a thread pool (the oracle's ctypes calls run
    without the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    H, W = img.shape
    out = np.empty((H, W), np.uint8)

    def band(y0):
        y1 = min(H, y0 + rows)
        a, b = max(0, y0 - 4), min(H, y1 + 4)
        oc, _, _ = oracle.classify_u8(img[a:b], low, high)
        out[y0:y1] = oc[y0 - a:y0 - a + (y1 - y0)]

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(band, range(0, H, rows)))
    return out


@pytest.mark.parametrize("noise", [workloads.NOISE_SIGMA, 0.0], ids=["noisy", "clean"])
def test_spiral_stress_16384(canny, noise):
    """Hysteresis stress image, 16384x16384: a one-pixel weak spiral seeded by a
    short strong segment, plus the Gaussian noise of the natural scenes
    (sigma 8, as the workload is named) or without noise (one chain of about
    3.4e7 pixels).  The whole class map is compared with the oracle's and the
    edges with breadth-first search on the oracle's class map, bit for bit;
    the search depth and the number of candidate components are printed."""
    import scipy.ndimage as ndi
    import time
    N = 16384
    t0 = time.time()
    img = workloads.spiral_u8(N, seed=5, noise_sigma=noise)
    dev = torch.from_numpy(img).cuda()
    edges, cls = canny.canny_u8(dev, 40, 100, return_classes=True)
    torch.cuda.synchronize()
    c = unpack_classes(cls.cpu().numpy(), N, N)
    e = edges.cpu().numpy()
    del edges, cls, dev
    print(f"[spiral {noise}] gpu done {time.time() - t0:.1f} s", flush=True)
    oc = _oracle_classes_chunked(img, 40, 100)
    bad = np.argwhere(c != oc)
    assert bad.size == 0, f"class mismatch at {bad[:5].tolist()}"
    print(f"[spiral {noise}] class map equal {time.time() - t0:.1f} s", flush=True)
    oe, depth = oracle.hysteresis(oc)
    assert np.array_equal(e, oe)
    lab, ncomp = ndi.label(oc >= 1, structure=np.ones((3, 3), int))
    nstrong = len(np.unique(lab[oc == 2]))
    print(f"[spiral {noise}] edges equal; BFS depth {depth}, candidate components {ncomp}, "
          f"with a strong pixel {nstrong}, edge px {int((oe > 0).sum())}, "
          f"{time.time() - t0:.1f} s", flush=True)
    if noise == 0.0:
        assert depth > 1000000 and nstrong == 1


@pytest.mark.parametrize("off", [1, 2, 3, 5])
def test_edges_into_misaligned_rows(canny, off):
    """Edge rows that start at every alignment (a row view at a byte offset
    into a buffer with an odd pitch): the hysteresis writes and rereads
    16-pixel segments at any alignment, touching no byte outside the image
    (guard bytes 0xA5 around every row stay as they were)."""
    H, W = 203, 1001
    img = workloads.natural_u8(H, W, seed=70 + off)
    big = torch.full((H, W + 9), 0xA5, dtype=torch.uint8, device="cuda")
    view = big[:, off:off + W]
    canny.canny_u8(torch.from_numpy(img).cuda(), 40, 100, edges=view)
    torch.cuda.synchronize()
    oe, _ = oracle.canny_u8(img, 40, 100)
    b = big.cpu().numpy()
    assert np.array_equal(b[:, off:off + W], oe)
    assert (b[:, :off] == 0xA5).all() and (b[:, off + W:] == 0xA5).all()
