"""Pins of the mate-rescue prefilter oracle (Section 2.7) against what the definition fixes.

M_t = #{(i, j): P[i, i+q) = W[j, j+q), j - i = t}.  The oracle counts it pair by pair; these tests
hold it to values computed another way:
  * closed forms: periodic read and window (M_t is the overlap length on every period-aligned
    diagonal, zero elsewhere); an exact copy (M = |P|-q+1 on its diagonal); one substitution or one
    N inside the copy (the q q-mers covering it drop out: |P|-2q+1);
  * a library routine: for q = 1 (and q = 2 on dinucleotide codes) M is the sum over symbols of
    numpy's full cross-correlation of the indicator sequences;
  * an invariant: sum_t M_t = sum over q-mers x of (#x in P)(#x in W);
  * brute force over explicit (i, j) pair sets on tiny random strings with N bases;
  * the candidate plumbing (windows in T coordinates, both strands, bisulfite text, read
    conversion by role, best_t = smallest maximising t) against those pair sets.
"""
from collections import Counter

import numpy as np
import pytest

import oracle
import synth

COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def revcomp(s):
    return "".join(COMP[c] for c in reversed(s))


def pairs_brute(p, w, q):
    """M as a dict t -> count from the explicit set of matching (i, j) pairs."""
    good = set("ACGT")
    m = Counter()
    for i in range(len(p) - q + 1):
        a = p[i:i + q]
        if not set(a) <= good:
            continue
        for j in range(len(w) - q + 1):
            if w[j:j + q] == a:
                m[j - i] += 1
    return m


def as_vector(m, np_, nw, q):
    nd = np_ + nw - 2 * q + 1 if np_ >= q and nw >= q else 0
    v = np.zeros(nd, np.int64)
    for t, c in m.items():
        v[t + np_ - q] = c
    return v


def rand_seq(rng, n, alphabet="ACGT"):
    return "".join(rng.choice(list(alphabet), n))


@pytest.mark.parametrize("a,b,q", [(10, 40, 7), (37, 37, 7), (5, 3, 3), (12, 50, 1), (30, 31, 15)])
def test_periodic_closed_form(a, b, q):
    p, w = "ACGT" * a, "ACGT" * b
    P, W = len(p), len(w)
    M = oracle.rescue_diagonals(p, w, q)
    assert M.size == P + W - 2 * q + 1
    for t in range(-(P - q), W - q + 1):
        lo, hi = max(0, -t), min(P - q, W - q - t)
        exp = hi - lo + 1 if (t % 4 == 0 and hi >= lo) else 0
        assert M[t + P - q] == exp, t


def test_phase_shift_picks_smallest_t():
    # P[i] = W[i + 1]: every diagonal t = 1 (mod 4) matches; the longest overlaps are t in [1, |W|-|P|]
    p, w = "CGTA" * 10, "ACGT" * 30
    M = oracle.rescue_diagonals(p, w, 7)
    P = len(p)
    t_best = int(np.argmax(M)) - (P - 7)
    assert M.max() == P - 7 + 1 and t_best == 1


@pytest.mark.parametrize("q", [1, 2])
def test_correlation_library_routine(q):
    rng = np.random.default_rng(5 + q)
    for _ in range(20):
        p = rand_seq(rng, int(rng.integers(q, 60)))
        w = rand_seq(rng, int(rng.integers(q, 200)))
        M = oracle.rescue_diagonals(p, w, q)
        pc = [p[i:i + q] for i in range(len(p) - q + 1)]
        wc = [w[j:j + q] for j in range(len(w) - q + 1)]
        exp = np.zeros(len(pc) + len(wc) - 1, np.int64)
        for x in set(pc):
            exp += np.correlate(np.array([c == x for c in wc], np.int64), np.array([c == x for c in pc], np.int64), "full")
        assert np.array_equal(M.astype(np.int64), exp)


@pytest.mark.parametrize("q", [5, 7, 11])
def test_copy_substitution_and_n_closed_form(q):
    rng = np.random.default_rng(100 + q)
    w = rand_seq(rng, 600)
    L, a = 150, 217
    copy = w[a:a + L]
    M = oracle.rescue_diagonals(copy, w, q)
    assert M[a + L - q] == L - q + 1
    s = 60
    for sub in ("N", {"A": "C", "C": "G", "G": "T", "T": "A"}[copy[s]]):
        p = copy[:s] + sub + copy[s + 1:]
        M = oracle.rescue_diagonals(p, w, q)
        assert M[a + L - q] == L - 2 * q + 1, sub


def test_sum_invariant_and_n():
    rng = np.random.default_rng(9)
    for q in (3, 4, 7):
        for _ in range(10):
            p = rand_seq(rng, int(rng.integers(1, 90)), "ACGTN")
            w = rand_seq(rng, int(rng.integers(1, 300)), "ACGT") if q > 3 else rand_seq(rng, 40)
            M = oracle.rescue_diagonals(p, w, q)
            cp = Counter(p[i:i + q] for i in range(len(p) - q + 1) if "N" not in p[i:i + q])
            cw = Counter(w[j:j + q] for j in range(len(w) - q + 1))
            assert int(M.sum()) == sum(c * cw[x] for x, c in cp.items())


def test_brute_pairs_tiny():
    rng = np.random.default_rng(11)
    for _ in range(60):
        q = int(rng.integers(1, 6))
        p = rand_seq(rng, int(rng.integers(0, 25)), "ACGTN" if rng.random() < 0.5 else "AC")
        w = rand_seq(rng, int(rng.integers(0, 40)), "ACGT" if rng.random() < 0.5 else "AC")
        M = oracle.rescue_diagonals(p, w, q)
        assert np.array_equal(M.astype(np.int64), as_vector(pairs_brute(p, w, q), len(p), len(w), q))


def test_role_conversion():
    rng = np.random.default_rng(13)
    p = rand_seq(rng, 80)
    w = rand_seq(rng, 200, "AGT")
    assert np.array_equal(oracle.rescue_diagonals(p, w, 7, role=1), oracle.rescue_diagonals(p.replace("C", "T"), w, 7))
    w2 = rand_seq(rng, 200, "ACT")
    assert np.array_equal(oracle.rescue_diagonals(p, w2, 7, role=2), oracle.rescue_diagonals(p.replace("G", "A"), w2, 7))


def _best(m, np_, q):
    if not m or max(m.values()) == 0:
        return 0, 0
    mx = max(m.values())
    return mx, min(t for t, c in m.items() if c == mx)


@pytest.mark.parametrize("bis", [False, True])
def test_candidates_against_pair_sets(bis):
    rng = np.random.default_rng(21 + bis)
    R = rand_seq(rng, 3000)
    codes = np.array(["ACGT".index(c) for c in R], np.uint8)
    if bis:
        half = R.replace("C", "T") + R.replace("G", "A")
        T = half + revcomp(half)
    else:
        T = R + revcomp(R)
    reads, rid, beg, wl, role = [], [], [], [], 1 if bis else 0
    for c in range(40):
        L = int(rng.integers(0, 160))
        x = int(rng.integers(0, len(T) - L))
        r = T[x:x + L]
        if bis and L:
            r = "".join(("C" if (ch == "T" and rng.random() < 0.5) else ch) for ch in r)
        if L > 20:
            r = r[:10] + "N" + r[11:]
        reads.append(r)
        w = int(rng.integers(0, 700))
        b = int(rng.integers(0, len(T) - w + 1))
        if c % 2 == 0:   # a window around the read's source
            b = max(0, min(len(T) - w, x - int(rng.integers(0, 200))))
        rid.append(c)
        beg.append(b)
        wl.append(w)
    # one window ending exactly at the sentinel, one empty window
    rid += [0, 1]
    beg += [len(T) - 300, 17]
    wl += [300, 0]
    seq = np.frombuffer("".join(reads).encode(), np.uint8)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reads])
    mh, bt = oracle.rescue(codes, seq, offs, rid, beg, wl, q=7, role=role, bisulfite=bis)
    for c in range(len(rid)):
        p = reads[rid[c]]
        if role == 1:
            p = p.replace("C", "T")
        m = pairs_brute(p, T[beg[c]:beg[c] + wl[c]], 7)
        assert (int(mh[c]), int(bt[c])) == _best(m, len(p), 7), c
    with pytest.raises(ValueError):
        oracle.rescue(codes, seq, offs, [0], [len(T) - 10], [11], q=7, bisulfite=bis)


def test_workload_candidates_find_true_mates():
    """The paired workload's rescue candidates: the window built around the known mate holds the
    other mate (max_t M_t close to |P|-q+1 at low error), a random window almost never passes."""
    ref = synth.workload_reference("small_1mbp")
    reads = synth.reads_fixed(ref, 300, 150, True, p_sub=0.005, p_indel=0.0005, seed=4)
    cand, decoy = synth.rescue_candidates(reads, len(ref), decoys=True, seed=7)
    mh, bt = oracle.rescue(ref.codes, reads.seq, reads.offsets, cand["read_id"], cand["win_beg"], cand["win_len"], q=7)
    true = decoy == 0
    assert true.sum() == 300 and (~true).sum() == 300
    assert np.mean(mh[true] >= 10) > 0.98 and np.median(mh[true]) > 100
    assert np.mean(mh[~true] >= 10) < 0.05
