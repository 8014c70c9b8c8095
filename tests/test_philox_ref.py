"""Known-answer vectors of Philox4x32-10 (the generator authors' published
test vectors) for the test-side reference, and the moments of its normals."""
import numpy as np

from tests import philox_ref
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


def test_poisson1_thresholds_against_exact_cdf():
    # exact CDF of Poisson(1) with 60-digit decimals: the FP64 table may differ
    # from floor(2^32 F) by at most one unit where 2^32 F is within rounding of
    # an integer
    from decimal import Decimal, getcontext

    getcontext().prec = 60
    e1 = Decimal(-1).exp()
    term, cdf, exact = e1, e1, []
    for k in range(12):
        if k:
            term = term / k
            cdf = cdf + term
        exact.append(int((cdf * (2 ** 32)).to_integral_value(rounding="ROUND_FLOOR")))
    t = philox_ref.poisson1_thresholds()
    assert np.all(np.abs(t.astype(np.int64) - np.array(exact, np.int64)) <= 1)
    assert np.all(np.diff(t.astype(np.int64)) > 0) and int(t[-1]) < 2 ** 32


def test_poisson1_distribution():
    rng = np.random.default_rng(0)
    x = rng.integers(0, 2 ** 32, size=2_000_000, dtype=np.uint64)
    k = philox_ref.poisson1(x)
    # probabilities of 0, 1, 2, 3: e^-1 (1, 1, 1/2, 1/6)
    p = np.exp(-1.0) * np.array([1.0, 1.0, 0.5, 1.0 / 6.0])
    f = np.bincount(k, minlength=13)[:4] / k.size
    assert np.all(np.abs(f - p) < 5 * np.sqrt(p * (1 - p) / k.size))
    assert abs(k.mean() - 1.0) < 5e-3 and abs(k.var() - 1.0) < 1e-2
    # the inversion at the table's edges
    t = philox_ref.poisson1_thresholds()
    assert philox_ref.poisson1(np.array([0, int(t[0]) - 1, int(t[0]), int(t[1]), 2 ** 32 - 1])).tolist() == [0, 0, 1, 2, 12]


def test_replica_weights_layout():
    w = philox_ref.replica_weights(seed=7, galaxy=3, replica=2, npix=10)
    r = philox_ref.philox4x32_10(np.array([[2, 3, 2, 1]], np.uint64), (7, 0))[0]
    assert w.shape == (10,) and w[8] == philox_ref.poisson1(r[0]) and w[9] == philox_ref.poisson1(r[1])
