"""The seeded generator shared by the tests and the library's own starting
vectors: Philox4x32-10 against the known-answer vectors published with the
generator's reference implementation (Random123), and the Gaussian mapping's
moments."""
import numpy as np

import synth


def test_philox4x32_10_known_answers():
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = synth.philox4x32_10(np.array([ctr], dtype=np.uint64), key)[0]
        assert [int(x) for x in got] == list(want)


def test_philox_gaussian_moments_and_offsets():
    g = synth.philox_gaussian(400000, 12345)
    for part in (g.real, g.imag):
        assert abs(part.mean()) < 5e-3 and abs(part.std() - 1.0) < 5e-3
        assert abs(np.mean(part ** 4) - 3.0) < 0.05  # Gaussian kurtosis
    assert abs(np.mean(g.real * g.imag)) < 5e-3
    # counters are absolute: a window equals the same range of a longer draw
    assert np.array_equal(synth.philox_gaussian(100, 12345, offset=1000), g[1000:1100])
    assert not np.array_equal(synth.philox_gaussian(100, 12346), g[:100])
