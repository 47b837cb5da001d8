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


def run_f32(canny, X, **kw):
    H, W = X.shape
    dev = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    e, cls, mag, mx = canny.canny_f32(dev, return_classes=True, return_magnitude=True,
                                      return_max=True, **kw)
    torch.cuda.synchronize()
    return (e.cpu().numpy(), unpack_classes(cls.cpu().numpy(), H, W), mag.cpu().numpy(),
            float(mx.cpu()[0]))


def check_float(canny, X, sigma=1.4, R=3, low=0.05, high=0.15, relative=True, max_unamb_diff=0,
                tol=TOL):
    e, c, m, mx = run_f32(canny, X, sigma=sigma, radius=R, low=low, high=high, relative=relative)
    oc, oM, amb, omx = oracle.classify_f32(X, sigma, R, low, high, relative, tol)
    floor = 0.05 * omx
    err = np.abs(m - oM) / np.maximum(np.maximum(oM, floor), 1e-30)
    assert err.max() <= tol or omx == 0.0, f"strength error {err.max():.3g}"
    if relative:
        assert abs(mx - omx) <= tol * omx
    unamb = (amb & 3) == 0
    diff = (c != oc) & unamb
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
    amplified by Sobel's 8, and never tighter than 1e-5."""
    X = workloads.natural_u8(97, 301, seed=R).astype(np.float32)
    sigma = 0.5 + 0.4 * R
    _, _, _, omx = oracle.classify_f32(X, sigma, R)
    tol = max(TOL, 16 * 2.0 ** -24 * 255 * (2 * R + 1) / (0.05 * omx))
    check_float(canny, X, sigma=sigma, R=R, tol=tol)


@pytest.mark.parametrize("H", [1, 2, 3, 5, 8, 13, 33, 40])
def test_float_small_sizes(canny, H):
    for W in [1, 2, 3, 4, 5, 7, 9, 16, 17, 33, 40, 247, 248]:
        X = workloads.natural_u8(H, W, seed=100 + H * 64 + W).astype(np.float32)
        check_float(canny, X)


def test_float_absolute_thresholds(canny):
    X = workloads.natural_u8(200, 333, seed=3).astype(np.float32)
    check_float(canny, X, low=20.0, high=60.0, relative=False)


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
