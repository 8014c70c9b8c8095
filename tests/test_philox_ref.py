"""Known-answer vectors of Philox4x32-10 (the generator authors' published
test vectors) for the test-side reference, and the moments of its normals."""
import numpy as np

from tests.philox_ref import galaxy_normals, philox4x32_10

KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_philox_known_answers():
    for ctr, key, want in KAT:
        got = philox4x32_10(np.array([ctr], np.uint64), key)[0]
        assert tuple(int(v) for v in got) == want


def test_normals_are_standard():
    z = np.concatenate([galaxy_normals(7, g, 4096) for g in range(16)])
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02
    # tails of a normal: P(|z| > 3) = 0.0027
    assert 0.0015 < np.mean(np.abs(z) > 3) < 0.004
