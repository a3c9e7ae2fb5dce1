"""Philox4x32-10 against the known-answer vectors published with Random123 (Salmon et al. 2011)."""
import numpy as np
import pytest

from oracle.philox import philox4x32_10, white_noise

KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    out = philox4x32_10(np.array([ctr], dtype=np.uint64), np.array([key], dtype=np.uint64))[0]
    assert [int(v) for v in out] == list(expect)


def test_white_noise_moments_and_counter_slicing():
    w = white_noise(7, 64)
    assert w.shape == (64**3,)
    assert abs(w.mean()) < 5.0 / np.sqrt(w.size)
    assert abs(w.var() - 1.0) < 5.0 * np.sqrt(2.0 / w.size)
    # kurtosis of a Gaussian is 3
    assert abs((w**4).mean() / w.var() ** 2 - 3.0) < 0.05
    # counter based: a slice equals the matching part of the full stream
    part = white_noise(7, 64, start=1000, count=500)
    assert np.array_equal(part, w[1000:1500])
    assert not np.array_equal(white_noise(8, 8), white_noise(7, 8))
