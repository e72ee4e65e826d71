"""Philox4x32-10 counter-based generator (test infrastructure only).

Written from the published definition (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11): a 4x32-bit counter and a
2x32-bit key; each of the 10 rounds multiplies counter words 0 and 2 by
0xD2511F53 and 0xCD9E8D57, mixes the high halves with words 1 and 3 and the
key, and the key is bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85
between rounds.

Also the mapping of generator words to the numbers a Metropolis step uses:
two words -> a double uniform in [0, 1) with 53 random bits; two uniforms ->
a normal pair by the Box-Muller transform.
"""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: uint array [..., 4], key: uint array [..., 2] -> uint64 array [..., 4] of 32-bit words."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & MASK for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = c[0] * np.uint64(M0)
        p1 = c[2] * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [(hi1 ^ c[1] ^ k0) & MASK, lo1, (hi0 ^ c[3] ^ k1) & MASK, lo0]
    return np.stack(c, axis=-1)


def words_to_uniform(hi, lo):
    """Two 32-bit words -> double in [0, 1): the top 53 bits of (hi << 32 | lo) times 2^-53."""
    v = ((np.asarray(hi, np.uint64) << np.uint64(32)) | np.asarray(lo, np.uint64)) >> np.uint64(11)
    return v.astype(np.float64) * (2.0 ** -53)


def metropolis_draws(seed, member, walkers, step, sigma):
    """Displacements [Wk, 3] (N(0, sigma^2)) and uniforms [Wk] for one step.

    Counter = (step low, step high, walker, member << 16 | block) with blocks
    0, 1, 2; key = (seed low, seed high).  Block 0 gives two uniforms u1, u2 ->
    z0 = sqrt(-2 ln(1 - u1)) cos(2 pi u2), z1 = ... sin(...); block 1 gives z2
    the same way (cos branch); block 2 words 0, 1 give the acceptance uniform.
    """
    walkers = np.asarray(walkers, dtype=np.uint64)
    n = walkers.shape[0]
    key = np.zeros((n, 2), np.uint64)
    key[:, 0] = seed & MASK
    key[:, 1] = (seed >> 32) & MASK
    out = []
    for blk in range(3):
        ctr = np.zeros((n, 4), np.uint64)
        ctr[:, 0] = step & MASK
        ctr[:, 1] = (step >> 32) & MASK
        ctr[:, 2] = walkers
        ctr[:, 3] = (member << 16) | blk
        out.append(philox4x32_10(ctr, key))
    u = [words_to_uniform(out[b][:, 0], out[b][:, 1]) for b in range(3)]
    v = [words_to_uniform(out[b][:, 2], out[b][:, 3]) for b in range(2)]
    r0 = np.sqrt(-2.0 * np.log1p(-u[0]))
    r1 = np.sqrt(-2.0 * np.log1p(-u[1]))
    z0 = r0 * np.cos(2.0 * np.pi * v[0])
    z1 = r0 * np.sin(2.0 * np.pi * v[0])
    z2 = r1 * np.cos(2.0 * np.pi * v[1])
    disp = sigma * np.stack([z0, z1, z2], axis=-1)
    return disp, u[2]
