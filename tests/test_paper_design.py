"""CPU checks of the paper-design baseline (row-parallel Steps 1-3, serial
hysteresis; Section 2.2.1 and Section 2.2.2): it runs the oracle's per-pixel
arithmetic in parallel loops, so its edge map must equal the oracle's bit for
bit at any thread count, and it reports the time of its two parts."""
import numpy as np
import pytest

import oracle
import workloads


@pytest.mark.parametrize("shape,threads", [((1, 1), 2), ((3, 7), 3), ((97, 301), 1), ((517, 733), 4),
                                           ((256, 1000), 8)])
def test_equals_oracle(shape, threads):
    X = workloads.natural_u8(*shape, seed=shape[0] + 3 * shape[1]).astype(np.float32)
    e, _ = oracle.canny_f32(X)
    e2, tp, ts = oracle.paper_design_canny_f32(X, threads)
    assert np.array_equal(e, e2)
    assert tp >= 0.0 and ts >= 0.0


def test_equals_oracle_absolute_and_radius():
    X = workloads.natural_u8(200, 333, seed=3).astype(np.float32)
    for R, sigma in ((1, 0.8), (5, 2.2)):
        e, _ = oracle.canny_f32(X, sigma, R, 20.0, 60.0, False)
        e2, _, _ = oracle.paper_design_canny_f32(X, 4, sigma, R, 20.0, 60.0, False)
        assert np.array_equal(e, e2)


def test_constant_image_has_no_edges():
    e, _, _ = oracle.paper_design_canny_f32(np.full((50, 70), 3.5, np.float32), 4)
    assert not e.any()
