"""Pins for the oracle of the Laplacian zero-crossing detector (the
comparator the paper's introduction names, Laplace(f) = f_xx + f_yy), each
against something other than the oracle's own code: a library Laplacian,
closed forms (quadratic surfaces, ramps, constants, step edges), hand-derived
step profiles, hand-made crossing maps, a brute force written per pixel
(gather form, where the oracle visits pairs), and the transpose symmetry of
the tie rule.  CPU only."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import workloads


def rnd_u8(H, W, seed):
    return np.random.default_rng(seed).integers(0, 256, (H, W), dtype=np.uint8)


@pytest.mark.parametrize("H,W", [(1, 1), (1, 9), (7, 1), (2, 3), (5, 5), (13, 40), (37, 29)])
def test_laplace_equals_library(H, W):
    """The 5-point Laplacian with replicate border == scipy.ndimage.laplace
    (second differences per axis) in 'nearest' mode."""
    B = rnd_u8(H, W, 7 * H + W)
    ref = ndi.laplace(B.astype(np.int64), mode="nearest")
    assert np.array_equal(oracle.laplace_i32(B), ref)


@pytest.mark.parametrize("a,b", [(1, 1), (2, 0), (0, 3), (1, 2)])
def test_quadratic_surface_constant_laplacian(a, b):
    """f = a (x-7)^2 + b (y-7)^2 + 5: the binomial (1,4,6,4,1)/16 has variance
    1 per axis, so its blur of a quadratic is f + a + b exactly (an integer,
    no rounding), and Laplace(f) = 2a + 2b everywhere at least 3 pixels from
    the border (2 for the blur, 1 for the stencil)."""
    y, x = np.mgrid[0:15, 0:15]
    f = a * (x - 7) ** 2 + b * (y - 7) ** 2 + 5
    assert f.max() <= 255
    B = oracle.blur_binomial(f.astype(np.uint8))
    assert np.array_equal(B[2:-2, 2:-2], (f + a + b)[2:-2, 2:-2])
    _, L = oracle.log_u8(f.astype(np.uint8), 1)
    assert np.all(L[3:-3, 3:-3] == 2 * a + 2 * b)


def test_constant_has_no_crossings():
    for v in (0, 1, 128, 255):
        e, L = oracle.log_u8(np.full((20, 31), v, np.uint8), 0)
        assert not L.any() and not e.any()


@pytest.mark.parametrize("a,b", [(1, 0), (0, 2), (1, 1), (2, 1)])
def test_ramp_interior_zero_and_no_edges(a, b):
    """A linear ramp is blurred to itself away from the border, so its
    Laplacian is exactly 0 at least 3 pixels in; the clamped border leaves
    |L| <= 2 (a + b) near the edge, so a threshold above 4 (a + b) leaves no
    crossing anywhere."""
    y, x = np.mgrid[0:40, 0:50]
    f = (a * x + b * y + 3).astype(np.uint8)
    e, L = oracle.log_u8(f, 4 * (a + b) + 1)
    assert not L[3:-3, 3:-3].any()
    assert np.abs(L).max() <= 2 * (a + b)
    assert not e.any()


# cumulative sums of the binomial (1,4,6,4,1): the blur of a unit step at
# column c seen at columns c-3 .. c+2 is 0, 1, 5, 11, 15, 16 (/16)
CUM = np.array([0, 1, 5, 11, 15, 16])


def step_image(delta, H=12, W=16, c=8):
    img = np.zeros((H, W), np.uint8)
    img[:, c:] = delta
    return img


@pytest.mark.parametrize("delta", range(1, 256))
def test_step_edge_profile_and_single_line(delta):
    """A vertical step of contrast delta at column c = 8: the blur of every row
    is floor((delta * CUM + 8) / 16) at columns 5..10 (one rounding, half up),
    and the Laplacian is its second difference.  The binomial is symmetric, so
    apart from rounding L(c-1) = -L(c) with L >= 0 left of the step and <= 0
    right of it (the rounding breaks this only for delta in {2, 3, 5, 6},
    where only the profile is checked): the only sign change is the tie at
    (c-1, c), which the earlier pixel wins, so the edge is exactly column
    c - 1 over the full height at any threshold up to that crossing's slope
    (the tails that return to 0 mark nothing); one above the slope removes
    it."""
    img = step_image(delta)
    Bc = (delta * CUM + 8) // 16  # columns 5..10
    B = oracle.blur_binomial(img)
    assert np.array_equal(B[:, 5:11], np.broadcast_to(Bc, (12, 6)))
    prof = np.concatenate([[0, 0], Bc, [delta, delta]])  # columns 3..12
    Lc = prof[:-2] + prof[2:] - 2 * prof[1:-1]           # columns 4..11
    _, L = oracle.log_u8(img, 1)
    assert np.array_equal(L[:, 4:12], np.broadcast_to(Lc, (12, 8)))
    clean = Lc[3] == -Lc[4] and Lc[3] > 0 and (Lc[:3] >= 0).all() and (Lc[5:] <= 0).all()
    assert clean == (delta not in (2, 3, 5, 6))
    if not clean:
        return
    slope = int(L[0, 7]) - int(L[0, 8])
    for t in (0, 1, slope):
        e, _ = oracle.log_u8(img, t)
        assert np.flatnonzero(e.any(axis=0)).tolist() == [7], (delta, t, L[0, 3:13].tolist())
        assert e[:, 7].all()
    e2, _ = oracle.log_u8(img, slope + 1)
    assert not e2.any()


def test_step_edge_worked_examples():
    """Hand-derived rows (columns 4..11) for three contrasts; the edge column
    is 7 in all three (a tie |L(7)| = |L(8)|, the earlier pixel wins)."""
    worked = {
        7: [0, 0, 2, 1, -1, -2, 0, 0],        # B = 0 0 0 2 5 7 7 7 at columns 4..11
        100: [0, 6, 19, 13, -13, -19, -6, 0],  # B = 0 6 31 69 94 100 at 5..10
        160: [0, 10, 30, 20, -20, -30, -10, 0],
    }
    for delta, row in worked.items():
        e, L = oracle.log_u8(step_image(delta), 1)
        assert L[5, 4:12].tolist() == row, delta
        assert np.flatnonzero(e[5]).tolist() == [7]


def test_crossing_rule_hand_maps():
    zc = oracle.zero_crossings
    # right neighbour: the smaller |L| is marked; a tie marks the left pixel
    assert np.flatnonzero(zc(np.array([[5, -3]]), 1)).tolist() == [1]
    assert np.flatnonzero(zc(np.array([[-3, 5]]), 1)).tolist() == [0]
    assert np.flatnonzero(zc(np.array([[3, -3]]), 1)).tolist() == [0]
    assert np.flatnonzero(zc(np.array([[-3, 3]]), 1)).tolist() == [0]
    # a zero never pairs: (0, -1) and (4, 0) do not cross
    assert not zc(np.array([[0, -1]]), 0).any()
    assert not zc(np.array([[4, 0]]), 0).any()
    assert not zc(np.array([[0, 0]]), 0).any()
    # a zero between strictly opposite neighbours is the crossing itself
    assert zc(np.array([[5, 0, -5]]), 10).tolist() == [[0, 255, 0]]
    assert not zc(np.array([[5, 0, -5]]), 11).any()
    assert zc(np.array([[-1], [0], [2]]), 3).tolist() == [[0], [255], [0]]
    assert not zc(np.array([[5, 0, 0, -5]]), 1).any()  # a zero run marks nothing
    assert not zc(np.array([[0, 5, 0], [0, 0, 0]]), 1).any()
    # the slope threshold is on |L(p) - L(q)|, inclusive
    assert not zc(np.array([[2, -1]]), 4).any()
    assert np.flatnonzero(zc(np.array([[2, -2]]), 4)).tolist() == [0]
    # lower neighbour: same rule, the upper pixel wins a tie
    assert np.flatnonzero(zc(np.array([[4], [-4]]), 1)).tolist() == [0]
    assert np.flatnonzero(zc(np.array([[4], [-2]]), 1)).tolist() == [1]
    # diagonal neighbours are not paired
    assert not zc(np.array([[5, 1], [1, -5]]) * np.array([[1, 1], [1, 1]]) + np.array([[0, 0], [0, 6]]), 1).any()
    m = np.array([[5, 7], [9, 2]])
    m[1, 1] = -4
    # (1,1) = -4 pairs with (0,1) = 7 and (1,0) = 9: marked itself (smaller |L|)
    assert zc(m, 1).tolist() == [[0, 0], [0, 255]]


def brute_force(L, t):
    """Per pixel (gather form): p is marked iff some 4-neighbour q inside the
    image has the strictly opposite sign with slope >= t and p is the pair's
    chosen pixel (smaller |L|; on a tie, the earlier of the two in raster
    order), or L(p) = 0 and the products of its opposite neighbours' values
    (left * right or up * down, inside the image) are negative with slope
    >= t."""
    H, W = L.shape
    e = np.zeros((H, W), np.uint8)
    for y in range(H):
        for x in range(W):
            lp = int(L[y, x])
            for dy, dx in ((0, 1), (1, 0), (0, -1), (-1, 0)):
                yy, xx = y + dy, x + dx
                if not (0 <= yy < H and 0 <= xx < W):
                    continue
                lq = int(L[yy, xx])
                if lp * lq >= 0 or abs(lp - lq) < t:
                    continue
                earlier = (y, x) < (yy, xx)
                if abs(lp) < abs(lq) or (abs(lp) == abs(lq) and earlier):
                    e[y, x] = 255
            if lp == 0:
                for (y1, x1), (y2, x2) in (((y, x - 1), (y, x + 1)), ((y - 1, x), (y + 1, x))):
                    if min(y1, y2, x1, x2) < 0 or max(y1, y2) >= H or max(x1, x2) >= W:
                        continue
                    a, b = int(L[y1, x1]), int(L[y2, x2])
                    if a * b < 0 and abs(a - b) >= t:
                        e[y, x] = 255
    return e


@pytest.mark.parametrize("seed", range(6))
def test_crossings_equal_brute_force(seed):
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(1, 14)), int(rng.integers(1, 14))
    L = rng.integers(-3, 4, (H, W)).astype(np.int32)  # many zeros and ties
    for t in (0, 1, 3, 7):
        assert np.array_equal(oracle.zero_crossings(L, t), brute_force(L, t)), (seed, t)


def test_transpose_symmetry():
    """The blur and the Laplacian are symmetric in x and y, and the tie rule
    picks the earlier pixel of a horizontal and of a vertical pair alike, so
    transposing the image transposes the edges."""
    img = workloads.natural_u8(97, 131, seed=3)
    for t in (1, 8, 20):
        e, _ = oracle.log_u8(img, t)
        eT, _ = oracle.log_u8(np.ascontiguousarray(img.T), t)
        assert np.array_equal(e.T, eT)
