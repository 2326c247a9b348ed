"""Counter-based uniform random numbers: Philox4x32-10.

Test infrastructure only (see the package docstring).

The generator is the one published by Salmon, Moraes, Dror and Shaw
("Parallel random numbers: as easy as 1, 2, 3", SC'11): a 128-bit counter
and a 64-bit key, ten rounds of two 32x32->64 multiplications with the
multipliers 0xD2511F53 and 0xCD9E8D57, and a Weyl key schedule with
increments 0x9E3779B9 and 0xBB67AE85.  Written here in Python integers.

The hop decision of Sec. II.B needs one uniform number per trajectory and
step.  Counter = (step low 32 bits, step high 32 bits, trajectory, stream),
key = (seed low 32 bits, seed high 32 bits); the uniform is built from the
first two output words as ((w1 << 32 | w0) >> 11) * 2^-53, in [0, 1).
Stream 0 is the hop decision; stream 1 draws the Fermi occupations of the
initial state.
"""
from __future__ import annotations

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = (int(c) & MASK for c in ctr)
    k0, k1 = (int(k) & MASK for k in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return c0, c1, c2, c3


def uniform(seed: int, traj: int, counter: int, stream: int = 0) -> float:
    """Uniform in [0, 1) for (seed, trajectory, counter, stream)."""
    w = philox4x32_10((counter & MASK, (counter >> 32) & MASK, traj, stream),
                      (seed & MASK, (seed >> 32) & MASK))
    u64 = (w[1] << 32) | w[0]
    return (u64 >> 11) * (1.0 / 9007199254740992.0)
