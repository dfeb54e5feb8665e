"""Pins of the oracle's wire form (one byte per AO value, Section 3.2; one
visibility bit per light, Section 3.1 and Fig. 1)."""
import numpy as np

import oracle as orc


def test_quantize_round_trips_every_code():
    # k / 255 (rounded to fp32) is the centre of code k: every code comes back
    k = np.arange(256)
    x = (k / 255.0).astype(np.float32)
    assert np.array_equal(orc.quantize_u8(x), k.astype(np.uint8))


def test_quantize_error_bound_and_monotone():
    rng = np.random.default_rng(0)
    x = np.sort(rng.random(200_000).astype(np.float32))
    q = orc.quantize_u8(x).astype(np.int64)
    # nearest code: |q/255 - x| <= 1/510 (+ fp32 rounding of 255 x)
    assert np.abs(q / 255.0 - x.astype(np.float64)).max() <= 0.5 / 255 + 1e-6
    assert (np.diff(q) >= 0).all()


def test_quantize_clamps_and_nan():
    x = np.array([-1.0, -0.0, np.nan, 1.0, 1.5, np.inf, -np.inf, 0.5 / 255 * 0.999, 0.5 / 255 * 1.001],
                 np.float32)
    assert orc.quantize_u8(x).tolist() == [0, 0, 0, 255, 255, 255, 0, 0, 1]


def test_light_mask_figure1_and_majority():
    # Fig. 1: with one ray per light, lights (0, 1, 2) -> bits 2..0 read as a
    # string: hard shadows 110 = light 1 and 2 visible; soft shadows 010
    hard = np.array([[0], [1], [1]], np.uint8)
    soft = np.array([[0], [1], [0]], np.uint8)
    assert orc.light_mask(hard, 1)[0] == 0b110
    assert orc.light_mask(soft, 1)[0] == 0b010
    # several rays per light: visible from half of them on
    counts = np.array([[0, 1, 2, 3, 4]], np.uint8)
    assert orc.light_mask(counts, 4).tolist() == [0, 0, 1, 1, 1]
    counts = np.array([[0, 1, 2, 3]], np.uint8)
    assert orc.light_mask(counts, 3).tolist() == [0, 0, 1, 1]
