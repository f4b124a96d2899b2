"""Philox-4x32-10 counter-based generator and Box-Muller normals (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Philox-4x32 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11).  A 128-bit counter
(four 32-bit words) and a 64-bit key (two words) pass through 10 rounds.  In
one round, the first and third counter words are multiplied by two fixed odd
constants; the high halves of those products are xor-ed with the other two
counter words and the two key words; and the words are permuted.  The key is
advanced by two Weyl constants (golden-ratio and sqrt(3)-1 derived) between
rounds.  Written here from that definition with numpy uint64 arithmetic.

Normals come from the Box-Muller transform (Box & Muller, 1958): for two
independent uniforms u1, u2 in (0, 1), r = sqrt(-2 ln u1) and theta = 2 pi u2
give the independent standard normals r cos(theta) and r sin(theta).  A
32-bit word x maps to the uniform (x + 1/2) / 2^32, which is never 0 or 1.

The starts of the solver draw their Gaussian test matrices from this
generator (the device draws the same numbers from its own implementation).
Element e (column-major index) of the matrix drawn for stream `stream` of
restart `restart` under seed `seed` is normal e mod 4 of the Philox block
with counter (e div 4 low word, e div 4 high word, restart, stream) and key
(seed low word, seed high word); the block's words (x0, x1) give normals 0
and 1, (x2, x3) give normals 2 and 3.
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)

# stream ids of the draws made by the solver's starts
STREAM_GAUSS_A0 = 1     # n x r Gaussian start
STREAM_RRF_OMEGA = 2    # p x r Gaussian test matrix of the randomized range finder


def philox4x32_10(ctr, key):
    """Philox-4x32-10 of counters `ctr` (..., 4) under keys `key` (..., 2); uint32 words."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64)
    k1 = np.asarray(key[..., 1], dtype=np.uint64)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1).astype(np.uint32)


def uniform_from_word(x):
    """(x + 1/2) / 2^32 in fp64."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


def normals(count: int, seed: int, restart: int, stream: int) -> np.ndarray:
    """The first `count` standard normals of (seed, restart, stream), fp64."""
    nblk = (count + 3) // 4
    b = np.arange(nblk, dtype=np.uint64)
    ctr = np.stack([b & MASK, b >> np.uint64(32),
                    np.full(nblk, restart, dtype=np.uint64), np.full(nblk, stream, dtype=np.uint64)], axis=-1)
    s = np.uint64(seed)
    key = np.broadcast_to(np.array([s & MASK, s >> np.uint64(32)], dtype=np.uint64), (nblk, 2))
    w = philox4x32_10(ctr, key)
    out = np.empty((nblk, 4))
    for pair in (0, 1):
        u1 = uniform_from_word(w[:, 2 * pair])
        u2 = uniform_from_word(w[:, 2 * pair + 1])
        rad = np.sqrt(-2.0 * np.log(u1))
        th = 2.0 * np.pi * u2
        out[:, 2 * pair] = rad * np.cos(th)
        out[:, 2 * pair + 1] = rad * np.sin(th)
    return out.reshape(-1)[:count]


def gaussian_matrix(rows: int, cols: int, seed: int, restart: int, stream: int) -> np.ndarray:
    """rows x cols matrix of normals, element e = i + rows*j (column-major numbering)."""
    z = normals(rows * cols, seed, restart, stream)
    return z.reshape(cols, rows).T.copy()
