"""Pins of the chaining oracle (Section 2.6: minimap2's chaining recurrence, adapted to
variable-length seeds, up to 50 chains per read) against statements that share nothing with it:

* the recurrence's value f(i) equals the best score over every chain ending at anchor i,
  enumerated subset by subset (a chain = anchors j1 < ... < jk = i in chaining order, each
  consecutive pair allowed, at most h apart; its score w_j1 + sum of alpha - beta);
* hand-computed values: collinear seeds add their lengths, overlapping ones their union, a gap of
  l costs floor(l * wbar / 100) + floor(floor(log2 l) / 2);
* the constraints: no chaining across copies, backwards on the read, beyond the maximum gap, or
  beyond h predecessors;
* chain extraction: chains are disjoint, increase in x and y, score as the sum along them, cover
  every anchor when nothing is filtered, and the top-50 rule keeps the 50 best.
"""
import itertools

import numpy as np
import pytest

import brute
import oracle
import synth


def gamma(l, wbar):
    l = abs(l)
    if l == 0:
        return 0
    return l * wbar // 100 + (l.bit_length() - 1) // 2


def allowed(a, b, G):
    """b may follow a in a chain (a earlier in chaining order)."""
    return a[3] == b[3] and a[0] < b[0] and a[1] < b[1] and b[0] - a[0] <= G and b[1] - a[1] <= G


def step(a, b, wbar):
    dx, dy = b[0] - a[0], b[1] - a[1]
    return min(dx, dy, b[2]) - gamma(dy - dx, wbar)


def brute_f(anchors, G, h):
    """Best chain score ending at each anchor, by enumerating every subset that ends there."""
    n = len(anchors)
    wbar = sum(a[2] for a in anchors) // n
    f = []
    for i in range(n):
        best = anchors[i][2]
        for k in range(1, i + 1):
            for sub in itertools.combinations(range(i), k):
                idx = list(sub) + [i]
                if any(idx[t + 1] - idx[t] > h for t in range(len(idx) - 1)):
                    continue
                if not all(allowed(anchors[idx[t]], anchors[idx[t + 1]], G) for t in range(len(idx) - 1)):
                    continue
                sc = anchors[idx[0]][2] + sum(step(anchors[idx[t]], anchors[idx[t + 1]], wbar)
                                              for t in range(len(idx) - 1))
                best = max(best, sc)
        f.append(best)
    return f


def as_arrays(anchors):
    A = sorted(anchors, key=lambda a: (a[0], a[1], a[2]))
    x = np.array([a[0] for a in A], np.uint64)
    y = np.array([a[1] for a in A], np.uint32)
    w = np.array([a[2] for a in A], np.uint32)
    g = np.array([a[3] for a in A], np.uint32)
    return A, x, y, w, g


def random_anchors(rng, n):
    out = set()
    while len(out) < n:
        w = int(rng.integers(5, 40))
        y = int(rng.integers(w - 1, 200))
        x = int(rng.integers(w - 1, 260))
        out.add((x, y, w, int(rng.integers(0, 2)) if rng.random() < 0.2 else 0))
    return list(out)


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("G,h", [(10 ** 6, 50), (60, 50), (10 ** 6, 2), (40, 1)])
def test_dp_equals_enumeration_of_all_chains(seed, G, h):
    rng = np.random.default_rng(seed)
    A, x, y, w, g = as_arrays(random_anchors(rng, 8))
    f, p = oracle.chain_dp(x, y, w, g, max_gap=G, max_pred=h)
    assert list(f) == brute_f(A, G, h)
    # predecessor: the largest allowed j within h reaching f(i) when that exceeds w_i, else -1
    wbar = int(w.sum()) // len(A)
    for i in range(len(A)):
        cands = [j for j in range(max(0, i - h), i) if allowed(A[j], A[i], G) and
                 f[j] + step(A[j], A[i], wbar) == f[i]]
        want = max(cands) if f[i] > A[i][2] and cands else -1
        assert p[i] == want, (i, p[i], want)


def test_closed_forms():
    # three collinear seeds of 20, 15 and 30 bases with no gaps: 65
    A, x, y, w, g = as_arrays([(119, 19, 20, 0), (134, 34, 15, 0), (164, 64, 30, 0)])
    f, p = oracle.chain_dp(x, y, w, g)
    assert list(f) == [20, 35, 65] and list(p) == [-1, 0, 1]
    # overlapping collinear seeds [0,30) and [10,50) on the same diagonal: the union, 50
    A, x, y, w, g = as_arrays([(1029, 29, 30, 0), (1049, 49, 40, 0)])
    f, _ = oracle.chain_dp(x, y, w, g)
    assert list(f) == [30, 50]
    # two 30-base seeds with one extra text base between them (dx = 31, dy = 30, l = 1): wbar = 30,
    # gamma(1) = 0 + 0 -> 60; with twelve (dx = 42, l = 12): gamma(12) = 12*30//100 + 3//2 = 3 + 1 = 4 -> 56
    A, x, y, w, g = as_arrays([(29, 29, 30, 0), (60, 59, 30, 0)])
    f, _ = oracle.chain_dp(x, y, w, g)
    assert list(f) == [30, 60]
    A, x, y, w, g = as_arrays([(29, 29, 30, 0), (71, 59, 30, 0)])
    f, _ = oracle.chain_dp(x, y, w, g)
    assert list(f) == [30, 56]
    # a gap cost larger than the second seed's contribution: starting afresh is better
    A, x, y, w, g = as_arrays([(29, 29, 30, 0), (1529, 49, 20, 0)])
    f, p = oracle.chain_dp(x, y, w, g, max_gap=5000)
    # dx = 1500, dy = 20: alpha = 20, gamma(1480) = 1480*25//100 + 10//2 = 370 + 5
    assert list(f) == [30, 20] and list(p) == [-1, -1]


def test_constraints():
    base = (29, 29, 30, 0)
    # other copy, read going backwards, equal x, gap beyond G: never a predecessor
    for other in [(60, 59, 30, 1), (60, 20, 10, 0), (29, 50, 20, 0)]:
        A, x, y, w, g = as_arrays([base, other])
        f, p = oracle.chain_dp(x, y, w, g)
        assert p[1] == -1 and f[1] == A[1][2], other
    A, x, y, w, g = as_arrays([base, (29 + 101, 29 + 100, 30, 0)])
    assert oracle.chain_dp(x, y, w, g, max_gap=100)[1][1] == -1
    assert oracle.chain_dp(x, y, w, g, max_gap=101)[1][1] == 0
    # h = 1: only the anchor right before may be a predecessor
    A, x, y, w, g = as_arrays([(29, 29, 30, 0), (40, 200, 5, 1), (70, 69, 30, 0)])
    assert oracle.chain_dp(x, y, w, g, max_pred=1)[1][2] == -1
    assert oracle.chain_dp(x, y, w, g, max_pred=2)[1][2] == 0


def seeds_of(rows):
    """A seeding result holding rows (read, qbeg, qend, [positions]) sorted by read."""
    read_id = np.array([r[0] for r in rows], np.uint32)
    npos = np.array([len(r[3]) for r in rows], np.uint32)
    pos_off = np.concatenate([[0], np.cumsum(npos)[:-1]]).astype(np.uint64) if rows else np.zeros(0, np.uint64)
    pos = np.array([p for r in rows for p in r[3]], np.uint64)
    z = np.zeros(len(rows), np.uint64)
    return oracle.SeedResult(read_id=read_id, qbeg=np.array([r[1] for r in rows], np.uint32),
                             qend=np.array([r[2] for r in rows], np.uint32), k=z, kr=z, s=npos.astype(np.uint64),
                             npos=npos, flags=np.zeros(len(rows), np.uint32), pos_off=pos_off, pos=pos)


def test_two_loci_give_two_chains_in_score_order():
    """A read whose three seeds sit collinear at one locus and whose first two also occur at a second
    locus: the first chain holds all three (score 90), the second the two (60), ordered by score."""
    rows = [(0, 0, 30, [1000, 50000]), (0, 30, 60, [1030, 50030]), (0, 60, 90, [1060])]
    chains, anchors = oracle.chain(seeds_of(rows), seg_len=10 ** 6, min_score=19)
    assert list(chains["score"]) == [90, 60] and list(chains["n_anchors"]) == [3, 2]
    assert list(anchors["pos"]) == [1000, 1030, 1060, 50000, 50030]
    assert list(anchors["qbeg"]) == [0, 30, 60, 0, 30]


def test_used_anchor_stops_a_chain():
    """Two chains share a prefix: the second, found later, stops where the first already took its
    anchors, and scores f(end) - f(stop)."""
    # anchors a(0..30 @100) b(30..60 @130) c(60..90 @160) d(60..80 @175): d chains onto b with a small gap
    rows = [(0, 0, 30, [100]), (0, 30, 60, [130]), (0, 60, 80, [175]), (0, 60, 90, [160])]
    chains, anchors = oracle.chain(seeds_of(rows), seg_len=10 ** 6, min_score=0)
    # ends (x, y): a (129, 29), b (159, 59), c (189, 89), d (194, 79); wbar = 110 // 4 = 27
    # f: a 30, b 60, c 90; d from b: dx = 35, dy = 20, alpha = 20, l = 15,
    # gamma(15) = 15 * 27 // 100 + 3 // 2 = 5 -> f(d) = 75 (from a: 30 + 20 - 5 = 45; c lies after it on the read)
    assert list(chains["score"]) == [90, 75 - 60]
    assert list(chains["n_anchors"]) == [3, 1]


def test_top_fifty():
    """60 seeds of one read at 60 unrelated loci (different scores 20..79): exactly the 50 best
    chains, in score order; min_score drops the rest."""
    rows = [(0, i, i + 20 + (i % 60), [10 ** 6 * (i + 1)]) for i in range(60)]
    rows.sort(key=lambda r: (r[1], r[2]))
    res = seeds_of(rows)
    chains, _ = oracle.chain(res, seg_len=10 ** 9, max_gap=5000)
    scores = sorted((r[2] - r[1] for r in rows), reverse=True)
    assert list(chains["score"]) == scores[:50]
    chains, _ = oracle.chain(res, seg_len=10 ** 9, min_score=70)
    assert list(chains["score"]) == [s for s in scores if s >= 70]


def test_workload_invariants():
    """On seeds of the 1 Mbp workload (repeats included): chains are disjoint and strictly
    increasing in x and y; with nothing filtered every anchor lies in exactly one chain; a chain
    that starts at an anchor without predecessor scores w_first + sum(alpha - beta); at most 50
    chains per read with the default filter, in score order."""
    ref = synth.workload_reference("small_1mbp")
    reads = synth.workload_reads("small_1mbp", ref, 600)
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    res = ox.seed(reads.seq, reads.offsets, min_len=19, max_occ=500)
    L = len(ref)
    chains, anchors = oracle.chain(res, seg_len=L, max_chains=10 ** 6, min_score=0)
    assert chains.size > 600
    total = int(res.npos.sum())
    assert anchors.size == total
    keys = set()
    for c in chains:
        a = anchors[int(c["anchor_off"]):int(c["anchor_off"]) + int(c["n_anchors"])]
        x = a["pos"].astype(np.int64) + (a["qend"] - a["qbeg"]).astype(np.int64) - 1
        y = a["qend"].astype(np.int64) - 1
        assert np.all(np.diff(x) > 0) and np.all(np.diff(y) > 0)
        assert np.all(x // L == int(c["copy"]))
        for t in a:
            k = (int(c["read_id"]), int(t["qbeg"]), int(t["qend"]), int(t["pos"]))
            assert k not in keys
            keys.add(k)
    assert len(keys) == total
    # score as a sum along chains whose first anchor has no predecessor (recomputed per read)
    by_read = {}
    for t in range(len(res)):
        by_read.setdefault(int(res.read_id[t]), []).append(t)
    checked = 0
    for c in chains[:400]:
        r = int(c["read_id"])
        A = []
        for t in by_read[r]:
            for q in range(int(res.npos[t])):
                p = int(res.pos[int(res.pos_off[t]) + q])
                w = int(res.qend[t] - res.qbeg[t])
                A.append((p + w - 1, int(res.qend[t]) - 1, w, (p + w - 1) // L))
        A, x, y, w, g = as_arrays(A)
        f, pr = oracle.chain_dp(x, y, w, g)
        wbar = int(w.sum()) // len(A)
        a = anchors[int(c["anchor_off"]):int(c["anchor_off"]) + int(c["n_anchors"])]
        idx = [A.index((int(t["pos"]) + int(t["qend"] - t["qbeg"]) - 1, int(t["qend"]) - 1, int(t["qend"] - t["qbeg"]),
                        (int(t["pos"]) + int(t["qend"] - t["qbeg"]) - 1) // L)) for t in a]
        if pr[idx[0]] == -1:
            assert int(c["score"]) == A[idx[0]][2] + sum(step(A[idx[t]], A[idx[t + 1]], wbar) for t in range(len(idx) - 1))
            checked += 1
    assert checked > 300
    # default filter: at most 50 per read, in score order
    chains, _ = oracle.chain(res, seg_len=L)
    assert np.all(chains["score"] >= 19)
    for r in np.unique(chains["read_id"]):
        s = chains["score"][chains["read_id"] == r]
        assert s.size <= 50 and np.all(np.diff(s) <= 0)
    assert brute.revcomp("ACGT") == "ACGT"
