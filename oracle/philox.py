"""Philox4x32-10 counter-based generator, written from its published
definition (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11).  Test infrastructure only.

One round maps counter (c0, c1, c2, c3) and key (k0, k1) to
  (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
with 32x32->64-bit products; the key is bumped by the Weyl constants
(W0, W1) between rounds; ten rounds are applied.

Site-proposal uniforms (the counter layout is part of the library's
interface): counter = (site, slice, sweep, pass), key = (seed & 0xffffffff,
seed >> 32); u = (w0 * 2^21 + (w1 >> 11)) * 2^-53, a double in [0, 1) with
53 random bits.
"""
M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK, p1 & MASK, ((p0 >> 32) ^ c3 ^ k1) & MASK, p0 & MASK
    return (c0, c1, c2, c3)


def u53(w0, w1):
    return ((w0 << 21) + (w1 >> 11)) * (1.0 / 9007199254740992.0)


def uniform_site(seed, sweep, pas, l, i):
    seed = int(seed)
    w = philox4x32_10((i, l, sweep, pas), (seed & MASK, (seed >> 32) & MASK))
    return u53(w[0], w[1])
