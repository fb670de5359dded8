"""Counter-based random start vectors (oracle; test infrastructure).

The power method starts from a random vector at the first Newton step
(Sec. 2, smoothers).  Both implementations draw it from SplitMix64
(Steele, Lea and Flood, OOPSLA 2014), used as a counter-based generator:
the value at flat index i of level l is the (i+1)-th output of the
SplitMix64 sequence whose state starts at seed + l * 2^32, i.e.

    z = s0 + (i + 1) * 0x9E3779B97F4A7C15             (mod 2^64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

mapped to [-1, 1) as (z >> 11) * 2^-52 - 1.  Pinned against the
generator's known first outputs from state 0 (tests/test_oracle_rng.py);
the GPU side implements the same definition independently and tests
compare the two.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix_uniform(seed, level, count):
    """count values in [-1, 1) for flat indices 0..count-1."""
    s0 = np.uint64((int(seed) + int(level) * (1 << 32)) % (1 << 64))
    with np.errstate(over='ignore'):
        z = s0 + (np.arange(count, dtype=np.uint64) + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0
