"""Width-generic Philox reference (Salmon, Moraes, Dror, Shaw, SC'11) in pure Python.

The 4x64 instance is checked against numpy's Philox bit generator, which pins the
round and key-schedule structure; the 4x32 instance then differs only in the
published multiplier and Weyl constants, and is compared with the oracle's and
the GPU's Philox4x32-10.  Pure test helper: holds no rendering arithmetic.
"""

PARAMS = {
    32: dict(M=(0xD2511F53, 0xCD9E8D57), W=(0x9E3779B9, 0xBB67AE85)),
    64: dict(M=(0xD2E7470EE14C6C93, 0xCA5A826395121157), W=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)),
}


def philox(ctr, key, width=32, rounds=10):
    mask = (1 << width) - 1
    M0, M1 = PARAMS[width]["M"]
    W0, W1 = PARAMS[width]["W"]
    c = [int(x) & mask for x in ctr]
    k0, k1 = int(key[0]) & mask, int(key[1]) & mask
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & mask
            k1 = (k1 + W1) & mask
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> width, p0 & mask
        hi1, lo1 = p1 >> width, p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def uniform24(r):
    """The 24-bit uniform of the stream specification: (r >> 8) * 2^-24."""
    return (int(r) >> 8) * (1.0 / 16777216.0)


def draw4(c0, c1, c2, c3, seed, scene_id):
    return [uniform24(x) for x in philox((c0, c1, c2, c3), (seed, scene_id))]
