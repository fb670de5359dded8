"""Pin of the oracle's SplitMix64 start vectors against the generator's
known first outputs from state 0 (tests/golden/splitmix64_state0.txt), and
of the map to [-1, 1)."""
import os

import numpy as np

from oracle.rng import splitmix_uniform

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden', 'splitmix64_state0.txt')


def test_first_outputs_of_state_zero():
    ref = [int(l, 16) for l in open(GOLDEN) if l.strip() and not l.startswith('#')]
    got = splitmix_uniform(0, 0, len(ref))
    # the map keeps the top 53 bits: (z >> 11) 2^-52 - 1
    want = np.array([(z >> 11) * 2.0 ** -52 - 1.0 for z in ref])
    assert np.array_equal(got, want)
    assert np.all(got >= -1.0) and np.all(got < 1.0)


def test_level_offsets_the_state():
    # level l starts at state seed + l 2^32, so level 1 of seed 5 is level 0
    # of seed 5 + 2^32, and its values differ from level 0's
    a = splitmix_uniform(5, 0, 64)
    b = splitmix_uniform(5, 1, 64)
    c = splitmix_uniform(5 + (1 << 32), 0, 64)
    assert np.array_equal(b, c)
    assert not np.any(np.isin(a, b))
