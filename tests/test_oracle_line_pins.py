"""Pins of the oracle's access counter (O2's line_ctr), the numerator of the SMEM roofline.

The counter counts, for a given occurrence-line layout of B rows per line: per extension step
(Algorithm 1 call) the lines holding rows x1 and x2 = x1 + s that its two rank queries read (1
when x1 // B == x2 // B, else 2); one line per k-mer table lookup; per LF step of LocateSlow
(Algorithm 2) one line; per SA-sample read one sample.  These tests fix those numbers on reads
whose Algorithm-3 path is known in advance (an exact substring of the text: stage 1 extends
backwards from l - 1 to 0 without failing, stage 2 forwards to the end), from quantities computed
by brute force (no oracle code):
  * the extension step count is |P| (|P| - K with a K-mer lookup replacing the first K steps);
  * the rows ranked by each step follow from the definitions: a backward step from P[j+1, l)
    reads rows lo(P[j+1, l)) and that + occ; a forward step from P[0, j) reads
    lo(revcomp P[0, j)) and that + occ;
  * an LF walk from the row of text position p takes t steps, the smallest t >= 0 with
    ISA[p - t] a multiple of r (positions wrap through n - 1 after 0).
"""
import bisect

import numpy as np
import pytest

import brute
import oracle

ACGT = "ACGT"


def codes_of(s):
    return np.array([ACGT.index(ch) for ch in s], dtype=np.uint8)


class Brute:
    """Sorted suffixes of a small text, for lo / occ / ISA by definition."""

    def __init__(self, R: str):
        self.T = brute.text_of(R)
        self.n = len(self.T)
        self.SA = brute.suffix_array(self.T)
        self.sufs = [self.T[i:] for i in self.SA]
        self.ISA = [0] * self.n
        for x, p in enumerate(self.SA):
            self.ISA[p] = x

    def lo(self, P: str) -> int:
        return bisect.bisect_left(self.sufs, P)

    def occ(self, P: str) -> int:
        return bisect.bisect_left(self.sufs, P + "~") - self.lo(P)

    def walk(self, p: int, r: int) -> int:
        t = 0
        while self.ISA[(p - t) % self.n] % r != 0:
            t += 1
        return t


def expected(bf: Brute, P: str, l: int, K: int, B: int, r: int):
    """(steps, extension lines, k-mer lookups, LF steps, SA reads) of one exact-substring read."""
    m = len(P)
    steps = lines = 0
    first = K if K > 0 else 0           # a K-mer lookup replaces the backward steps that add P[l-K, l)
    # stage 1: backward from P[l-1] down to P[0]; the step adding P[j] starts from P[j+1, l)
    for j in range(l - 1 - first, -1, -1):
        cur = P[j + 1:l]
        x1 = bf.lo(cur) if cur else 0
        s = bf.occ(cur) if cur else bf.n
        steps += 1
        lines += 1 if x1 // B == (x1 + s) // B else 2
    # stage 2: forward from P[0, j) for j = l .. m-1 (the step adding P[j])
    for j in range(l, m):
        cur = P[:j]
        x1 = bf.lo(brute.revcomp(cur))
        s = bf.occ(cur)
        steps += 1
        lines += 1 if x1 // B == (x1 + s) // B else 2
    pos = [i for i in range(bf.n - m + 1) if bf.T[i:i + m] == P]
    lf = sum(bf.walk(p, r) for p in pos)
    return steps, lines, (1 if K > 0 else 0), lf, len(pos)


REF = "".join(ACGT[int(x)] for x in np.random.default_rng(7).integers(0, 4, 1500))
# a 60-base unit present three times (plus its mirror on the other strand)
UNIT = REF[200:260]
REF_REP = REF[:700] + UNIT + REF[700:1100] + UNIT + REF[1100:]


@pytest.mark.parametrize("B", [1, 2, 7, 384, 10 ** 9])
@pytest.mark.parametrize("r", [1, 3, 8, 10 ** 9])
@pytest.mark.parametrize("K", [0, 4])
def test_line_counter_exact_substrings(B, r, K):
    """Unique reads (s = 1 throughout stage 2) and a read inside a three-copy repeat (s = 3): the
    oracle's counts equal the brute-force ones for every line size B (1: every row its own line;
    10^9: the whole index one line), sampling rate r (10^9: only row 0 sampled, so a walk from
    position p takes p + 1 steps) and with or without a K-mer lookup."""
    for R, reads in ((REF, [REF[100:180], REF[900:1050], brute.revcomp(REF[300:340])]),
                     (REF_REP, [UNIT[5:55]])):
        bf = Brute(R)
        ox = oracle.OracleIndex(codes_of(R), sa_rate=r)
        for P in reads:
            seq = np.frombuffer(P.encode(), np.uint8).copy()
            offs = np.array([0, len(P)], np.uint64)
            res = ox.seed(seq, offs, min_len=19, reseed=False, max_occ=10 ** 6, method=1, kmer_k=K, bases_per_line=B)
            assert len(res) == 1 and int(res.qbeg[0]) == 0 and int(res.qend[0]) == len(P)
            steps, lines, kmer, lf, sa = expected(bf, P, 19, K, B, r)
            got = res.lines
            assert got["steps"] == steps, (P[:10], got, steps)
            assert got["kmer_lookups"] == kmer
            assert got["sa_reads"] == sa == int(res.s[0])
            assert got["lf_steps"] == lf
            assert got["lines"] == lines + lf, (got, lines, lf)


def test_line_counter_closed_forms():
    """Numbers that need no computation at all: a unique 100-base read with one line per row
    (B = 1: every step reads two lines) and one line for the whole index (one line per step) takes
    100 steps; with only row 0 sampled its one position p costs p + 1 LF steps; with r = 1 none."""
    ox1 = oracle.OracleIndex(codes_of(REF), sa_rate=1)
    oxn = oracle.OracleIndex(codes_of(REF), sa_rate=10 ** 9)
    P = REF[500:600]
    seq = np.frombuffer(P.encode(), np.uint8).copy()
    offs = np.array([0, 100], np.uint64)
    a = ox1.seed(seq, offs, reseed=False, method=1, bases_per_line=1).lines
    assert (a["steps"], a["lines"], a["lf_steps"], a["sa_reads"], a["kmer_lookups"]) == (100, 200, 0, 1, 0)
    b = ox1.seed(seq, offs, reseed=False, method=1, bases_per_line=10 ** 9).lines
    assert (b["steps"], b["lines"]) == (100, 100)
    c = oxn.seed(seq, offs, reseed=False, method=1, bases_per_line=1).lines
    assert (c["lf_steps"], c["lines"], c["sa_reads"]) == (501, 200 + 501, 1)
    d = ox1.seed(seq, offs, reseed=False, method=1, kmer_k=10, bases_per_line=1).lines
    assert (d["steps"], d["lines"], d["kmer_lookups"]) == (90, 180, 1)


def test_line_counter_is_off_without_a_layout():
    """bases_per_line = 0 counts steps and LF steps but no lines."""
    ox = oracle.OracleIndex(codes_of(REF), sa_rate=8)
    P = REF[500:600]
    res = ox.seed(np.frombuffer(P.encode(), np.uint8).copy(), np.array([0, 100], np.uint64), reseed=False, method=1)
    assert res.lines["lines"] == 0 and res.lines["steps"] == 100
