"""Pins of the oracle's reading S5 (Section 2.1 replaces bases other than A, C, G, T by random
ones): the replacement draws come from SplitMix64 (Steele, Lea and Flood, 2014), output i for
reference position i, seeded with the build's rng_seed.

* the oracle's SplitMix64 reproduces the published sequence for state 1234567;
* A, C, G, T map to 0..3 in either case, and every other byte takes the low two bits of the draw
  at its own position (not of a running count of ambiguous bases).
"""
import numpy as np

import oracle

PUBLISHED_1234567 = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                     4593380528125082431, 16408922859458223821]


def test_splitmix64_published_sequence():
    assert list(map(int, oracle.splitmix64(1234567, 5))) == PUBLISHED_1234567


def test_codes_from_ascii():
    assert oracle.codes_from_ascii(b"ACGTacgt").tolist() == [0, 1, 2, 3, 0, 1, 2, 3]
    ref = b"NxACnRY-g"
    got = oracle.codes_from_ascii(ref, 1234567)
    draws = [v & 3 for v in PUBLISHED_1234567] + [None] * 4
    want = []
    for i, ch in enumerate(ref):
        if chr(ch).upper() in "ACGT":
            want.append("ACGT".index(chr(ch).upper()))
        else:
            want.append(draws[i] if draws[i] is not None else int(oracle.splitmix64(1234567, i + 1)[i] & np.uint64(3)))
    assert got.tolist() == want
    # a position's draw does not depend on the other ambiguous bases
    a = oracle.codes_from_ascii(b"AAAAN", 77)
    b = oracle.codes_from_ascii(b"NNNNN", 77)
    assert a[4] == b[4]
