"""SplitMix64, from its published definition (oracle side; test infrastructure).

SplitMix64 (Steele, Lea and Flood, OOPSLA 2014; the reference generator of
Vigna's xoshiro family) keeps a 64-bit state x.  Each step adds the odd
constant gamma = 0x9E3779B97F4A7C15 to x and returns the state passed through
a 64-bit finalizer (two xor-shift-multiply rounds and a final xor-shift).

Because the state is a plain counter, output number i (i >= 1) of the stream
seeded with s is mix(s + i * gamma): a counter-based generator.  The k-means++
seeding consumes output number  r * 2**32 + t + 1  for restart r and draw t,
turned into a double in [0, 1) from its top 53 bits.

The GPU library implements the same generator independently from the same
definition; the two share no code.
"""

from __future__ import annotations

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _mix(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64_outputs(seed: int, count: int, start: int = 1):
    """Outputs number start, start+1, ... of the stream seeded with `seed`."""
    return [_mix((seed + (start + i) * GAMMA) & MASK) for i in range(count)]


def splitmix64_uniform(seed: int, restart: int, draw: int) -> float:
    """Uniform double in [0, 1) for (seed, restart, draw)."""
    z = _mix((seed + ((restart << 32) + draw + 1) * GAMMA) & MASK)
    return (z >> 11) * (1.0 / 9007199254740992.0)
