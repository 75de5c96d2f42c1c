"""Oracle: Philox4x32-10 and Z(4) noise (test infrastructure only).

The Hutchinson estimator samples eta^dagger A eta with eta a vector of Z(4)
noise, entries in {1, i, -1, -i} (Sec. 1).  The paper does not fix a
generator; both sides of this project implement the same published
counter-based generator independently:

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11): a 4x32-bit counter and a 2x32-bit key, ten rounds of

    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)

with the key bumped by the Weyl constants (W0, W1) between rounds.

Z(4) convention (a reading; the paper only says "Z(4) noise"):
  key     = (seed mod 2^32, seed >> 32)
  counter = (c // 64, noise index, stream, 0)      c = (site*4 + spin)*3 + colour
  k       = (word[(c % 64) // 16] >> 2*(c % 16)) & 3
  eta_c   = i**k

Pins: the generator is checked against the published known-answer vectors of
the Philox paper's reference distribution (tests/golden/philox_kat.txt); the
symbol statistics are checked against their exact expectations.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function.

    ctr: array (..., 4) of uint32-valued integers; key: array (..., 2).
    Returns an array (..., 4) of uint32 output words.
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i] & MASK for i in range(4))
    k0 = key[..., 0] & MASK
    k1 = key[..., 1] & MASK
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0          # both factors < 2^32, so the product is exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> S32, p0 & MASK
        hi1, lo1 = p1 >> S32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def z4_symbols(seed, stream, index, n):
    """Integer symbols k in {0,1,2,3} for components c = 0..n-1 of one noise vector."""
    seed = int(seed)
    nblk = (n + 63) // 64
    ctr = np.zeros((nblk, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nblk, dtype=np.uint64)
    ctr[:, 1] = np.uint64(int(index) & 0xFFFFFFFF)
    ctr[:, 2] = np.uint64(int(stream) & 0xFFFFFFFF)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    words = philox4x32_10(ctr, np.broadcast_to(key, (nblk, 2)))   # (nblk, 4)
    c = np.arange(n)
    w = words[c // 64, (c % 64) // 16].astype(np.uint64)
    return ((w >> (2 * (c % 16)).astype(np.uint64)) & np.uint64(3)).astype(np.int64)


_I_POW = np.array([1.0 + 0j, 1j, -1.0 + 0j, -1j])


def z4_noise(seed, stream, index, n):
    """One Z(4) noise vector eta (complex128, length n) in canonical component order."""
    return _I_POW[z4_symbols(seed, stream, index, n)]


def z4_noise_batch(seed, stream, first, nrhs, n):
    """Noise vectors with indices first .. first+nrhs-1, shape (nrhs, n)."""
    return np.stack([z4_noise(seed, stream, first + r, n) for r in range(nrhs)])
