"""Pins of the 16-bit storage rounding used to form the oracle's inputs."""
import numpy as np

from storage16 import stored


def test_bf16_ties_to_even_and_truncation():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5 - 2.0 ** -9, 3.0 + 2.0 ** -7])
    assert np.array_equal(stored(x, 3).real, [1.0, 1.0, 1.0 + 2.0 ** -6, -2.5, 3.0])


def test_fp16_ties_to_even():
    x = np.array([1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 65504.0])
    assert np.array_equal(stored(x, 2).real, [1.0, 1.0 + 2.0 ** -9, 65504.0])


def test_imaginary_parts_round_alone():
    z = np.array([(1.0 + 2.0 ** -8) + 1j * (1.0 + 3 * 2.0 ** -8)])
    assert stored(z, 3)[0] == 1.0 + 1j * (1.0 + 2.0 ** -6)


def test_fp16_links_round_once_from_fp64():
    """a value just above an FP16 tie: FP64 -> FP16 rounds up, FP64 -> FP32 -> FP16 lands on the
    tie and rounds to even (down)"""
    x = np.array([1.0 + 2.0 ** -11 + 2.0 ** -30])
    assert stored(x, 2, links=True).real[0] == 1.0 + 2.0 ** -10
    assert stored(x, 2).real[0] == 1.0
