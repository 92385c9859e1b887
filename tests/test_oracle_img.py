"""Pins for the oracle's integer image filters (Section 1: image filters are stencils).

* Rounding rule: over every reachable window sum S in [0, 6375] the exact
  rational S/25 is never a tie, and floor((S + 12) / 25) is the nearest
  integer, so "round half down" and any round-to-nearest agree.
* Special images: constant (box = value, lap = 0), impulse (box = 10 on the
  5x5 footprint, lap = -1020 / 255), ramp (box = ramp in the interior).
* Independent evaluator: numpy.pad(mode='edge') is clamp-to-edge; sums of
  shifted slices give both filters.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1207_1746_amd import workloads as W


def test_division_rule_exhaustive():
    for S in range(0, 25 * 255 + 1):
        q = Fraction(S, 25)
        lo = q.numerator // q.denominator
        frac = q - lo
        assert frac != Fraction(1, 2)
        nearest = lo + (1 if frac > Fraction(1, 2) else 0)
        assert (S + 12) // 25 == nearest


def _independent(img, lap_kind):
    p = np.pad(img.astype(np.int64), ((0, 0), (2, 2), (2, 2)), mode="edge")
    nl, ny, nx = img.shape
    S = np.zeros(img.shape, np.int64)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            S += p[:, 2 + dy:2 + dy + ny, 2 + dx:2 + dx + nx]
    box = (S + 12) // 25
    sh = lambda dx, dy: p[:, 2 + dy:2 + dy + ny, 2 + dx:2 + dx + nx]
    if lap_kind == 4:
        lap = sh(0, -1) + sh(0, 1) + sh(-1, 0) + sh(1, 0) - 4 * sh(0, 0)
    else:
        lap = sum(sh(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1)) - 9 * sh(0, 0)
    return box.astype(np.uint8), lap.astype(np.int16)


@pytest.mark.parametrize("lap_kind", [4, 8])
@pytest.mark.parametrize("shape", [(2, 37, 53), (1, 1, 1), (1, 3, 2), (3, 8, 5)])
def test_matches_padded_evaluator(shape, lap_kind):
    img = W.rng(3, 9).integers(0, 256, size=shape, dtype=np.uint8)
    box, lap = oracle.img(img, lap_kind)
    eb, el = _independent(img, lap_kind)
    assert np.array_equal(box, eb) and np.array_equal(lap, el)


def test_constant_image():
    img = np.full((1, 9, 11), 173, np.uint8)
    box, lap = oracle.img(img)
    assert np.all(box == 173) and np.all(lap == 0)


def test_impulse():
    img = np.zeros((1, 11, 13), np.uint8)
    img[0, 5, 6] = 255
    box, lap = oracle.img(img)
    assert np.all(box[0, 3:8, 4:9] == 10) and box.sum() == 250
    assert lap[0, 5, 6] == -1020
    for y, x in [(4, 6), (6, 6), (5, 5), (5, 7)]:
        assert lap[0, y, x] == 255
    assert np.count_nonzero(lap) == 5
    _, lap8 = oracle.img(img, 8)
    assert lap8[0, 5, 6] == -2040 and np.count_nonzero(lap8) == 9


def test_ramp_is_reproduced_in_interior():
    x = np.arange(40)
    img = np.broadcast_to((3 * x + 7).astype(np.uint8), (1, 12, 40)).copy()
    box, lap = oracle.img(img)
    assert np.array_equal(box[0, :, 2:-2], img[0, :, 2:-2])
    assert np.all(lap[0, :, 1:-1] == 0)
