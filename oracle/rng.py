"""Counter-based normal variates for the oracle (test infrastructure only).

The paper needs independent unit-variance Gaussians for the dry noise
(Sec. II.D, eq step2) and for the stochastic stress (Sec. II.D, stage 3); it does
not fix a generator.  Both implementations use Philox4x32-10 from its published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key, ten rounds of two
32x32->64 multiplies, with the key bumped by the Weyl constants between rounds.

Counter layout shared with the GPU library (stated, not derived from the paper):
  counter = (index, step mod 2^32, tag, pair), key = (seed mod 2^32, seed >> 32)
where index is the stable ion id or the linear cell index, tag names the noise
stream and pair selects one of several draws.  One Philox call yields four
words (o0, o1, o2, o3); u1 is built from (o0, o1), u2 from (o2, o3) as
u = ((a >> 5) * 2^26 + (b >> 6) + 0.5) * 2^-53, which lies in (0, 1), and the
Box-Muller pair is (sqrt(-2 ln u1) cos(2 pi u2), sqrt(-2 ln u1) sin(2 pi u2)).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)

TAG_DRY = 1          # dry Brownian increment of each ion
TAG_STRESS_DIAG = 2  # diagonal stochastic stress at cell centres
TAG_STRESS_EDGE = 3  # off-diagonal stochastic stress at cell edges
TAG_RFD = 4          # random finite difference direction of each ion


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds; all arguments are arrays (or scalars) of uint32 values."""
    c = [np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return [v.astype(np.uint32) for v in c]


def _uniform(a, b):
    a = np.asarray(a, dtype=np.uint64) >> np.uint64(5)
    b = np.asarray(b, dtype=np.uint64) >> np.uint64(6)
    return (a.astype(np.float64) * 67108864.0 + b.astype(np.float64) + 0.5) * 2.0**-53


def normal_pair(seed, step, tag, pair, index):
    """Two independent N(0,1) arrays for the counters (index, step, tag, pair)."""
    index = np.asarray(index, dtype=np.uint64)
    seed = int(seed)
    o = philox4x32_10(index, np.uint64(int(step) & 0xFFFFFFFF), np.uint64(tag),
                      np.uint64(pair), np.uint64(seed & 0xFFFFFFFF),
                      np.uint64((seed >> 32) & 0xFFFFFFFF))
    u1 = _uniform(o[0], o[1])
    u2 = _uniform(o[2], o[3])
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def ion_normals(seed, step, tag, ids):
    """W [3, N]: x and y from pair 0, z from the first normal of pair 1."""
    wx, wy = normal_pair(seed, step, tag, 0, ids)
    wz, _ = normal_pair(seed, step, tag, 1, ids)
    return np.stack([wx, wy, wz])
