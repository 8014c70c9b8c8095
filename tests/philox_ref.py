"""Test-side Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
published definition, and the Box-Muller map the library documents for its
training-image noise."""
import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)


def philox4x32_10(ctr, key):
    """ctr: uint32-valued array [..., 4]; key: (k0, k1).  Returns [..., 4]."""
    c = np.asarray(ctr, dtype=np.uint64)
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0 = np.uint64(key[0]) & _MASK
    k1 = np.uint64(key[1]) & _MASK
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK, lo1, (hi0 ^ c3 ^ k1) & _MASK, lo0
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return np.stack([c0, c1, c2, c3], axis=-1)


def box_muller(a, b):
    """Two standard normals from two uint32 words: u1 = (a + 1) / 2^32 in
    (0, 1], u2 = b / 2^32; r = sqrt(-2 ln u1); (r cos 2 pi u2, r sin 2 pi u2)."""
    u1 = (np.asarray(a, np.float64) + 1.0) * 2.0 ** -32
    u2 = np.asarray(b, np.float64) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def galaxy_normals(seed: int, galaxy_index: int, npix: int):
    """The npix standard normals of one galaxy: counter {pixel // 4, index low
    word, index high word, 0}, key (seed low word, seed high word)."""
    nq = (npix + 3) // 4
    ctr = np.zeros((nq, 4), np.uint64)
    ctr[:, 0] = np.arange(nq)
    ctr[:, 1] = galaxy_index & 0xFFFFFFFF
    ctr[:, 2] = galaxy_index >> 32
    r = philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
    z0, z1 = box_muller(r[:, 0], r[:, 1])
    z2, z3 = box_muller(r[:, 2], r[:, 3])
    return np.stack([z0, z1, z2, z3], axis=1).ravel()[:npix]


def poisson1_thresholds():
    """T_k = floor(2^32 F(k)), k = 0..11, F(k) = e^-1 sum_{j<=k} 1/j! summed in
    that order in FP64 (the library's documented inversion table)."""
    term = np.float64(0.36787944117144233)
    cdf = term
    out = [int(np.floor(cdf * np.float64(4294967296.0)))]
    for k in range(1, 12):
        term = term / np.float64(k)
        cdf = cdf + term
        out.append(int(np.floor(cdf * np.float64(4294967296.0))))
    return np.array(out, np.uint64)


def poisson1(x):
    """Poisson(1) deviates from uint32 words: the number of thresholds <= x."""
    t = poisson1_thresholds()
    x = np.asarray(x, np.uint64)
    return (x[..., None] >= t).sum(axis=-1)


def replica_weights(seed: int, galaxy: int, replica: int, npix: int):
    """Poisson(1) pixel multipliers of bootstrap replica `replica` of galaxy
    `galaxy`: counter {pixel // 4, galaxy, replica, 1}, word pixel mod 4, key
    (seed low word, seed high word)."""
    nq = (npix + 3) // 4
    ctr = np.zeros((nq, 4), np.uint64)
    ctr[:, 0] = np.arange(nq)
    ctr[:, 1] = galaxy
    ctr[:, 2] = replica
    ctr[:, 3] = 1
    r = philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
    return poisson1(r.reshape(-1)[:npix])
