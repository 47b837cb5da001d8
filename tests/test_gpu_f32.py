"""GPU parity for the float path against the fp64 oracle (paper Section 2.2.1,
Steps 1-4; Gaussian sigma=1.4, 7 taps, L2 strength, continuous-direction
suppression, thresholds 0.05 / 0.15 of the largest strength).

Tolerance: |M_gpu - M_64| <= 1e-5 * max(M_64, 0.05 * max M) per pixel (relative,
floored at the low threshold: fp32 cannot hold a purely relative 1e-5 near
M = 0).  Class codes must equal the oracle's on every pixel the oracle does not
flag as within 1e-5 of a threshold or of a suppression tie; the edge map must
equal breadth-first search run on the GPU's own class map, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from helpers import unpack_classes

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def canny():
    import paper_1710_07745_amd as m
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


def run_f32(canny, X, with_max=True, **kw):
    """Requesting the largest strength (or relative thresholds) selects the
    signed-strength path; absolute thresholds without it select the one-launch
    path that classifies inside the walk."""
    H, W = X.shape
    dev = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    out = canny.canny_f32(dev, return_classes=True, return_magnitude=True, return_max=with_max,
                          **kw)
    e, cls, mag = out[:3]
    mx = float(out[3].cpu()[0]) if with_max else None
    torch.cuda.synchronize()
    return e.cpu().numpy(), unpack_classes(cls.cpu().numpy(), H, W), mag.cpu().numpy(), mx


def check_float(canny, X, sigma=1.4, R=3, low=0.05, high=0.15, relative=True, max_unamb_diff=0,
                tol=TOL, with_max=True, excuse_tol=None, label=""):
    """Strength within ``tol`` (relative, floored at 0.05 max M); classes equal
    the oracle's wherever it flags no decision within ``excuse_tol`` (default
    ``tol``) of a threshold or a suppression tie; edges equal BFS on the GPU's
    classes.  Prints the achieved strength error and the number of excused
    pixels that differ."""
    excuse_tol = tol if excuse_tol is None else excuse_tol
    e, c, m, mx = run_f32(canny, X, with_max=with_max, sigma=sigma, radius=R, low=low, high=high,
                          relative=relative)
    oc, oM, amb, omx = oracle.classify_f32(X, sigma, R, low, high, relative, excuse_tol)
    floor = 0.05 * omx
    err = np.abs(m - oM) / np.maximum(np.maximum(oM, floor), 1e-30)
    unamb = (amb & 3) == 0
    diff = (c != oc) & unamb
    print(f"[float {label} {X.shape[0]}x{X.shape[1]} R={R}] strength error {err.max():.3g} "
          f"(bound {tol:.3g}); excused pixels {int((~unamb).sum())}, of which differ "
          f"{int(((c != oc) & ~unamb).sum())}", flush=True)
    assert err.max() <= tol or omx == 0.0, f"strength error {err.max():.3g}"
    if with_max:
        assert abs(mx - omx) <= tol * omx
    assert diff.sum() <= max_unamb_diff, f"{diff.sum()} class mismatches at {np.argwhere(diff)[:5].tolist()}"
    be, _ = oracle.hysteresis(c)
    assert np.array_equal(e, be)
    return oc, amb


def test_float_512(canny):
    X = workloads.natural_u8(512, 512, seed=0).astype(np.float32)
    oc, amb = check_float(canny, X)
    assert (oc == 2).sum() > 100


@pytest.mark.parametrize("R", [1, 2, 3, 4, 5, 6, 7, 8])
def test_float_radii(canny, R):
    """Wider kernels smooth more, so the largest strength (and the floor 0.05*max
    of the error measure) shrinks while the fp32 rounding of the blur stays at
    about eps*255 per tap; the bound used here, 16*eps*255*(2R+1)/floor with
    eps = 2^-24, is that rounding summed over the 2R+1 taps of each pass and
    amplified by Sobel's 8, and never tighter than 1e-5.  That bound applies
    to the strength only: the set of excused pixels (decisions within the
    tolerance of a threshold or a suppression tie) stays at 1e-5."""
    X = workloads.natural_u8(97, 301, seed=R).astype(np.float32)
    sigma = 0.5 + 0.4 * R
    _, _, _, omx = oracle.classify_f32(X, sigma, R)
    tol = max(TOL, 16 * 2.0 ** -24 * 255 * (2 * R + 1) / (0.05 * omx))
    check_float(canny, X, sigma=sigma, R=R, tol=tol, excuse_tol=TOL, label=f"radius {R}")


@pytest.mark.parametrize("H", [1, 2, 3, 5, 8, 13, 33, 40])
def test_float_small_sizes(canny, H):
    for W in [1, 2, 3, 4, 5, 7, 9, 16, 17, 33, 40, 247, 248]:
        X = workloads.natural_u8(H, W, seed=100 + H * 64 + W).astype(np.float32)
        check_float(canny, X)


@pytest.mark.parametrize("with_max", [True, False])
def test_float_absolute_thresholds(canny, with_max):
    X = workloads.natural_u8(200, 333, seed=3).astype(np.float32)
    check_float(canny, X, low=20.0, high=60.0, relative=False, with_max=with_max)


def absolute_like_relative(X, sigma=1.4, R=3):
    """Absolute thresholds equal to 0.05 / 0.15 of the oracle's largest strength."""
    _, _, _, omx = oracle.classify_f32(X, sigma, R)
    return 0.05 * omx, 0.15 * omx


@pytest.mark.parametrize("H", [1, 2, 5, 13, 33, 40])
def test_float_one_launch_small_sizes(canny, H):
    for W in [1, 3, 4, 5, 17, 40, 247, 248, 249]:
        X = workloads.natural_u8(H, W, seed=300 + H * 64 + W).astype(np.float32)
        lo, hi = absolute_like_relative(X)
        check_float(canny, X, low=lo, high=hi, relative=False, with_max=False)


def test_float_one_launch_ragged(canny):
    X = workloads.natural_u8(1001, 2049, seed=13).astype(np.float32)
    lo, hi = absolute_like_relative(X)
    check_float(canny, X, low=lo, high=hi, relative=False, with_max=False)


def test_float_one_launch_4096(canny):
    """The launch the bench times for the classification walk alone."""
    X = workloads.natural_u8(4096, 4096, seed=1).astype(np.float32)
    lo, hi = absolute_like_relative(X)
    check_float(canny, X, low=lo, high=hi, relative=False, with_max=False)


def test_float_unaligned_pitch(canny):
    """Row pitch not a multiple of 4 floats: scalar loads in every pass."""
    X = workloads.natural_u8(77, 301, seed=21).astype(np.float32)
    H, W = X.shape
    big = torch.zeros((H, W + 3), dtype=torch.float32, device="cuda")
    big[:, 1:W + 1] = torch.from_numpy(X).cuda()
    view = big[:, 1:W + 1]
    for rel, lo, hi in [(True, 0.05, 0.15), (False,) + absolute_like_relative(X)]:
        e, cls = canny.canny_f32(view, 1.4, 3, lo, hi, rel, return_classes=True)
        c = unpack_classes(cls.cpu().numpy(), H, W)
        oc, _, amb, _ = oracle.classify_f32(X, 1.4, 3, lo, hi, rel, TOL)
        assert ((c != oc) & ((amb & 3) == 0)).sum() == 0
        be, _ = oracle.hysteresis(c)
        assert np.array_equal(e.cpu().numpy(), be)


@pytest.mark.parametrize("kind", ["dc_offset", "low_contrast_dc", "hdr", "tiny", "mixed_range", "ramp"])
def test_float_value_ranges(canny, kind):
    """The strength bound on content away from 0..255: a DC offset of 1000,
    low contrast on that offset (values 1000..1002.55), a high dynamic range
    (x1000), tiny values (x1e-3), a left half at 1 % contrast beside a
    full-contrast right half, and the scene on a ramp rising by 5000 across
    the image."""
    X = workloads.natural_u8(512, 768, seed=5).astype(np.float32)
    if kind == "dc_offset":
        X = X + np.float32(1000.0)
    elif kind == "low_contrast_dc":
        X = X * np.float32(0.01) + np.float32(1000.0)
    elif kind == "hdr":
        X = X * np.float32(1000.0)
    elif kind == "tiny":
        X = X * np.float32(1e-3)
    elif kind == "mixed_range":
        X[:, :384] *= np.float32(0.01)
    else:
        X = X + np.linspace(0.0, 5000.0, X.shape[1], dtype=np.float32)[None, :]
    check_float(canny, X, label=kind)


def test_float_constant(canny):
    e, c, m, mx = run_f32(canny, np.full((100, 300), 7.25, np.float32))
    assert not e.any() and not c.any() and not m.any() and mx == 0.0


def test_float_ragged(canny):
    X = workloads.natural_u8(1001, 2049, seed=12).astype(np.float32)
    check_float(canny, X)


def test_float_4096(canny):
    X = workloads.natural_u8(4096, 4096, seed=1).astype(np.float32)
    check_float(canny, X)


def test_float_7680x4320(canny):
    X = workloads.natural_u8(4320, 7680, seed=2).astype(np.float32)
    check_float(canny, X)


# Shapes for the balanced walk launch (interior blocks of 40 rows, border
# blocks of 23): images under 23 rows (one border block per strip), exactly
# 46 rows (no interior block), 60 rows (no interior block, two bottom border
# blocks), three border strips (right halo of the second-to-last strip leaves
# the image), and every strip bordered (rows not 16-byte aligned).
@pytest.mark.parametrize("shape", [(22, 245760), (46, 123000), (60, 82000), (3000, 4084)])
@pytest.mark.parametrize("relative", [True, False])
def test_float_balanced_split(canny, shape, relative):
    X = workloads.natural_u8(*shape, seed=shape[0] + shape[1]).astype(np.float32)
    if relative:
        check_float(canny, X)
    else:
        lo, hi = absolute_like_relative(X)
        check_float(canny, X, low=lo, high=hi, relative=False, with_max=False)


def test_float_balanced_split_unaligned(canny):
    X = workloads.natural_u8(2048, 4096, seed=41).astype(np.float32)
    H, W = X.shape
    big = torch.zeros((H, W + 3), dtype=torch.float32, device="cuda")
    big[:, 1:W + 1] = torch.from_numpy(X).cuda()
    e, cls, mag = canny.canny_f32(big[:, 1:W + 1], 1.4, 3, 0.05, 0.15, True, return_classes=True,
                                  return_magnitude=True)
    c = unpack_classes(cls.cpu().numpy(), H, W)
    oc, oM, amb, omx = oracle.classify_f32(X, 1.4, 3, 0.05, 0.15, True, TOL)
    err = np.abs(mag.cpu().numpy() - oM) / np.maximum(oM, 0.05 * omx)
    assert err.max() <= TOL
    assert ((c != oc) & ((amb & 3) == 0)).sum() == 0
    be, _ = oracle.hysteresis(c)
    assert np.array_equal(e.cpu().numpy(), be)


def test_float_stage_timing(canny):
    """Stage timing records one event pair per stage and call and leaves the
    results unchanged."""
    X = workloads.natural_u8(300, 500, seed=31).astype(np.float32)
    dev = torch.from_numpy(X).cuda()
    ref_e, ref_c = canny.canny_f32(dev, return_classes=True)
    with canny.StageTiming(8) as t:
        for _ in range(3):
            e, c = canny.canny_f32(dev, return_classes=True)
        torch.cuda.synchronize()
        for stage in ("f32_clear", "f32_walk", "f32_classify", "hysteresis"):
            ms, n = t.read(stage)
            assert n == 3 and ms > 0.0, stage
        assert t.read("u8_forward") == (0.0, 0)
    nb = (X.shape[1] + 3) // 4  # class bytes of a row (padding past them is unspecified)
    assert torch.equal(e, ref_e) and torch.equal(c[:, :nb], ref_c[:, :nb])


@pytest.mark.parametrize("shape,seed", [((1, 1), 78), ((5, 7), 82), ((63, 65), 140), ((200, 333), 277),
                                        ((1001, 2049), 1078), ((4096, 4096), 1), ((4320, 7680), 2),
                                        ((33000, 1024), 3)])
def test_float_edges_only_path(canny, shape, seed):
    """Edges alone (no class map or strength requested) take the path where
    the hysteresis pass classifies from the signed strength map.  Its edges
    must equal, bit for bit, those of the path through an explicit class map
    and BFS on that class map; that class map must equal the oracle's on
    every pixel the oracle does not flag.  Seeds 1 (4096^2) and 2
    (7680x4320) are the benchmark's own images.  Up to 4096 walk waves the
    largest strength comes from per-wave slots that the hysteresis pass
    reduces; 33000x1024 (about 4,100 waves) takes the shared word instead.  The number of final edge
    pixels that differ from the pure oracle (its classes, its BFS) is
    printed; they can differ only through components joined or split at
    flagged pixels, and are bounded here at 1e-4 of the image."""
    H, W = shape
    X = workloads.natural_u8(H, W, seed=seed).astype(np.float32)
    dev = torch.from_numpy(X).cuda()
    e_fused, mx = canny.canny_f32(dev, return_max=True)
    e_cls, cls = canny.canny_f32(dev, return_classes=True)
    torch.cuda.synchronize()
    assert torch.equal(e_fused, e_cls)
    c = unpack_classes(cls.cpu().numpy(), H, W)
    e = e_fused.cpu().numpy()
    be, _ = oracle.hysteresis(c)
    assert np.array_equal(e, be)
    oc, _, amb, omx = oracle.classify_f32(X, 1.4, 3, 0.05, 0.15, True, TOL)
    assert abs(float(mx.cpu()[0]) - omx) <= TOL * omx
    unamb = (amb & 3) == 0
    assert ((c != oc) & unamb).sum() == 0
    oe, _ = oracle.hysteresis(oc)
    ndiff = int((e != oe).sum())
    print(f"[edges-only {H}x{W} seed {seed}] class differences at flagged pixels "
          f"{int(((c != oc) & ~unamb).sum())} of {int((~unamb).sum())}; final edge pixels "
          f"differing from the pure oracle {ndiff} of {int((oe > 0).sum())} edge pixels", flush=True)
    assert ndiff <= max(1, 1e-4 * H * W)


def test_float_edges_only_absolute_with_max(canny):
    """Absolute thresholds with the maximum requested also take the signed
    path; with edges alone the hysteresis pass classifies with the absolute
    thresholds (and writes the maximum)."""
    X = workloads.natural_u8(300, 517, seed=91).astype(np.float32)
    dev = torch.from_numpy(X).cuda()
    e_fused, mx = canny.canny_f32(dev, 1.4, 3, 20.0, 60.0, False, return_max=True)
    e_cls, cls = canny.canny_f32(dev, 1.4, 3, 20.0, 60.0, False, return_classes=True)
    torch.cuda.synchronize()
    assert torch.equal(e_fused, e_cls)
    oc, _, amb, omx = oracle.classify_f32(X, 1.4, 3, 20.0, 60.0, False, TOL)
    c = unpack_classes(cls.cpu().numpy(), *X.shape)
    assert ((c != oc) & ((amb & 3) == 0)).sum() == 0
    assert abs(float(mx.cpu()[0]) - omx) <= TOL * omx


# ---- four-sector variant (absolute thresholds, one launch) -------------------

def check_sector(canny, X, sigma=1.4, R=3, low=None, high=None, tol=TOL, label=""):
    """Classes equal the four-sector oracle's on every pixel it does not flag
    (threshold, suppression near-tie, sector boundary); strength within the
    float tolerance; edges = breadth-first search on the GPU's classes.
    Prints the achieved strength error, the excused pixels, how many of them
    differ, and how many would be excused at 1e-5."""
    H, W = X.shape
    if low is None:
        lo, hi = absolute_like_relative(X, sigma, R)
    else:
        lo, hi = low, high
    dev = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    e, cls, mag = canny.canny_f32_sector(dev, sigma, R, lo, hi, return_classes=True,
                                         return_magnitude=True)
    torch.cuda.synchronize()
    c = unpack_classes(cls.cpu().numpy(), H, W)
    oc, oM, amb, omx = oracle.classify_f32_sector(X, sigma, R, lo, hi, False, tol)
    err = np.abs(mag.cpu().numpy() - oM) / np.maximum(np.maximum(oM, 0.05 * omx), 1e-30)
    unamb = (amb & 11) == 0
    diff = (c != oc) & unamb
    narrow = int(((oracle.classify_f32_sector(X, sigma, R, lo, hi, False, TOL)[2] & 11) != 0).sum()) \
        if tol != TOL else int((~unamb).sum())
    print(f"[sector {label} {H}x{W} R={R}] strength error {err.max():.3g} (bound {tol:.3g}); "
          f"excused pixels {int((~unamb).sum())} ({narrow} at 1e-5), of which differ "
          f"{int(((c != oc) & ~unamb).sum())}", flush=True)
    assert err.max() <= tol or omx == 0.0, f"strength error {err.max():.3g}"
    assert diff.sum() == 0, f"{diff.sum()} class mismatches at {np.argwhere(diff)[:5].tolist()}"
    be, _ = oracle.hysteresis(c)
    assert np.array_equal(e.cpu().numpy(), be)
    return oc, c


def test_sector_512(canny):
    X = workloads.natural_u8(512, 512, seed=0).astype(np.float32)
    oc, c = check_sector(canny, X)
    assert (oc == 2).sum() > 100
    # the four-sector rule is a different suppression: it keeps other pixels
    ic, _, _, _ = oracle.classify_f32(X, 1.4, 3, *absolute_like_relative(X), False)
    assert (ic != oc).sum() > 0


@pytest.mark.parametrize("H", [1, 2, 5, 13, 33, 40])
def test_sector_small_sizes(canny, H):
    for W in [1, 3, 4, 5, 17, 40, 247, 248, 249]:
        X = workloads.natural_u8(H, W, seed=500 + H * 64 + W).astype(np.float32)
        check_sector(canny, X)


@pytest.mark.parametrize("R", [1, 2, 3, 4, 5, 6, 7, 8])
def test_sector_radii(canny, R):
    X = workloads.natural_u8(97, 301, seed=40 + R).astype(np.float32)
    sigma = 0.5 + 0.4 * R
    _, _, _, omx = oracle.classify_f32(X, sigma, R)
    tol = max(TOL, 16 * 2.0 ** -24 * 255 * (2 * R + 1) / (0.05 * omx))
    check_sector(canny, X, sigma=sigma, R=R, tol=tol, label=f"radius {R}")


def test_sector_ragged_and_4096(canny):
    check_sector(canny, workloads.natural_u8(1001, 2049, seed=14).astype(np.float32))
    check_sector(canny, workloads.natural_u8(4096, 4096, seed=1).astype(np.float32))


def test_sector_balanced_split_shapes(canny):
    for shape in [(22, 245760), (60, 82000), (3000, 4084)]:
        check_sector(canny, workloads.natural_u8(*shape, seed=7 + shape[0]).astype(np.float32))


def test_sector_axis_and_diagonal_steps_match_interpolated(canny):
    """Where the gradient lies on an axis or the (1, 1) diagonal the two
    suppression rules coincide (see the oracle pins); the GPU variants must
    agree with each other there too."""
    X = np.full((300, 400), 40.0, np.float32)
    X[:, 150] = 90.0
    X[:, 151:] = 170.0
    dev = torch.from_numpy(X).cuda()
    a = canny.canny_f32(dev, 1.4, 3, 5.0, 20.0, False)
    b = canny.canny_f32_sector(dev, 1.4, 3, 5.0, 20.0)
    assert torch.equal(a, b) and int((a > 0).sum()) == 300


def test_sector_unaligned_pitch(canny):
    X = workloads.natural_u8(77, 301, seed=22).astype(np.float32)
    H, W = X.shape
    big = torch.zeros((H, W + 3), dtype=torch.float32, device="cuda")
    big[:, 1:W + 1] = torch.from_numpy(X).cuda()
    lo, hi = absolute_like_relative(X)
    e, cls = canny.canny_f32_sector(big[:, 1:W + 1], 1.4, 3, lo, hi, return_classes=True)
    c = unpack_classes(cls.cpu().numpy(), H, W)
    oc, _, amb, _ = oracle.classify_f32_sector(X, 1.4, 3, lo, hi, False, TOL)
    assert ((c != oc) & ((amb & 11) == 0)).sum() == 0
    be, _ = oracle.hysteresis(c)
    assert np.array_equal(e.cpu().numpy(), be)


def test_sector_constant(canny):
    dev = torch.full((100, 300), 7.25, dtype=torch.float32, device="cuda")
    e, cls = canny.canny_f32_sector(dev, 1.4, 3, 0.0, 1.0, return_classes=True)
    assert not e.any() and not unpack_classes(cls.cpu().numpy(), 100, 300).any()

