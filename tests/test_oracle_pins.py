"""Pins of the CPU oracle against things other than itself (CPU only).

* brute force on tiny texts (every substring counted by scanning, every suffix compared directly),
* textbook invariants of the BWT / LF-mapping,
* closed forms (homopolymer counts, a unique error-free read, mirrored strands),
* the paper's algorithms (Algorithm 1/2/3 in oracle O2) against the definitions (oracle O1).
"""
import json
import os

import numpy as np
import pytest

import brute
import oracle
import synth

ACGT = "ACGT"


def to_str(codes):
    return "".join(ACGT[int(x)] for x in codes)


def to_codes(s):
    return np.frombuffer(s.encode(), dtype=np.uint8).copy()


def ref_codes(s):
    return np.array(["ACGT".index(ch) for ch in s], dtype=np.uint8)


def csr(reads):
    seq = np.frombuffer("".join(reads).encode(), dtype=np.uint8).copy()
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum([len(r) for r in reads])
    return seq, offs


def seeds_of(res, r):
    return [(int(a), int(b), (int(k), int(kr), int(s)))
            for a, b, k, kr, s, rid in zip(res.qbeg, res.qend, res.k, res.kr, res.s, res.read_id) if rid == r]


TINY_REFS = {
    "random60": to_str(np.random.default_rng(1).integers(0, 4, 60)),
    "random200": to_str(np.random.default_rng(2).integers(0, 4, 200)),
    "homopolymer": "A" * 30,
    "period2": "AC" * 20,
    "palindrome": "ACGGTCA" + brute.revcomp("ACGGTCA"),
    "len1": "G",
    "len2": "CA",
    "len4": "ACGT",
    "repeats": "ACGTTGCA" * 3 + "GGATCCAT" + "ACGTTGCA" * 2,
}


@pytest.mark.parametrize("name", sorted(TINY_REFS))
def test_text_sa_bwt_brute(name):
    R = TINY_REFS[name]
    ix = oracle.OracleIndex(ref_codes(R), sa_rate=3)
    T = brute.text_of(R)
    assert "".join("$ACGT"[x] for x in ix.text()) == T
    SA = brute.suffix_array(T)
    assert list(ix.sa()) == SA
    B = brute.bwt(T, SA)
    assert "".join("$ACGT"[x] for x in ix.bwt()) == B
    assert ix.primary == SA.index(0)
    Cc = ix.C()
    for a, ch in enumerate("$ACGT"):
        assert int(Cc[a]) == sum(1 for x in B if x < ch)


@pytest.mark.parametrize("name", sorted(TINY_REFS))
def test_interval_brute(name):
    R = TINY_REFS[name]
    ix = oracle.OracleIndex(ref_codes(R), sa_rate=2)
    T = brute.text_of(R)
    rng = np.random.default_rng(7)
    pats = ["A", "C", "G", "T", "AC", "TT", "ACGT", "GATTACA"]
    for _ in range(30):
        i = int(rng.integers(0, len(R)))
        j = int(rng.integers(i + 1, min(len(R), i + 12) + 1))
        pats.append(R[i:j])
        pats.append(brute.revcomp(R[i:j]))
        pats.append(R[i:j] + ACGT[int(rng.integers(0, 4))])
    for P in pats:
        assert ix.interval(P) == brute.ds_interval(T, P), P


def test_lf_invariants():
    R = TINY_REFS["random200"]
    ix = oracle.OracleIndex(ref_codes(R), sa_rate=5)
    B = ix.bwt()
    n = ix.n
    # LF(x) = pi(B[x], x) is a permutation of the rows, and following it from the primary row
    # spells T backwards (BWT inversion)
    lf = [0 if x == ix.primary else ix.pi(int(B[x]), x) for x in range(n)]
    assert sorted(lf) == list(range(n))
    T = ix.text()
    x, out = 0, []
    for _ in range(n - 1):
        out.append(int(B[x]))
        x = lf[x]
    assert out[::-1] == [int(v) for v in T[: n - 1]]
    # SA(LF(x)) = SA(x) - 1 mod n
    SA = ix.sa()
    for xx in range(n):
        assert int(SA[lf[xx]]) == (int(SA[xx]) - 1) % n


@pytest.mark.parametrize("name", ["random60", "repeats", "palindrome", "homopolymer", "period2"])
def test_algorithm1_properties(name):
    """BackwardExt / ForwardExt give ds(aP) / ds(Pa); the $ term matters for patterns that start
    the text.  Also s(P) = s(revcomp P) and the counts of all one-symbol extensions sum to s(P)
    minus the occurrence preceded by $ (the suffix T itself)."""
    R = TINY_REFS[name]
    ix = oracle.OracleIndex(ref_codes(R), sa_rate=4)
    T = brute.text_of(R)
    rng = np.random.default_rng(3)
    pats = [R[:k] for k in range(1, min(len(R), 8) + 1)]
    for _ in range(25):
        i = int(rng.integers(0, len(R)))
        pats.append(R[i:i + int(rng.integers(1, 7))])
    for P in pats:
        iv = ix.interval(P)
        assert iv[2] == brute.occ(T, brute.revcomp(P))
        tot = 0
        for a in range(4):
            b = ix.backward(iv, a + 1)
            assert b == brute.ds_interval(T, ACGT[a] + P)
            f = ix.forward(iv, a + 1)
            assert f == brute.ds_interval(T, P + ACGT[a])
            tot += b[2]
        assert tot == iv[2] - (1 if T.startswith(P) else 0)


@pytest.mark.parametrize("name", sorted(TINY_REFS))
@pytest.mark.parametrize("method", [0, 1])
def test_smems_brute(name, method):
    R = TINY_REFS[name]
    ix = oracle.OracleIndex(ref_codes(R), sa_rate=3)
    T = brute.text_of(R)
    rng = np.random.default_rng(11)
    reads = []
    for _ in range(6):
        if len(R) < 3:
            break
        i = int(rng.integers(0, len(R) - 2))
        j = int(rng.integers(i + 2, min(len(R), i + 30) + 1))
        s = list(R[i:j])
        for t in range(len(s)):
            if rng.random() < 0.08:
                s[t] = ACGT[int(rng.integers(0, 4))]
        s = "".join(s)
        reads.append(s if rng.random() < 0.5 else brute.revcomp(s))
    reads += ["ACGTACGTAC", "GGGGGGGG", "TAGCTAGNNACGT", "A", ""]
    seq, offs = csr(reads)
    for (l, c) in [(1, 1), (3, 1), (4, 2), (6, 1), (2, 3), (5, 4)]:
        for kmer in ([0] if method == 0 else [0, 2, 3]):
            if kmer > l:
                continue
            res = ix.seed(seq, offs, min_len=l, min_occ=c, reseed=False, method=method, kmer_k=kmer,
                          max_occ=10 ** 6)
            for r, P in enumerate(reads):
                assert seeds_of(res, r) == brute.smems(T, P, l, c), (l, c, kmer, P)
            for t in range(len(res)):
                P = reads[res.read_id[t]][res.qbeg[t]:res.qend[t]]
                got = [int(x) for x in res.pos[res.pos_off[t]:res.pos_off[t] + res.npos[t]]]
                assert got == brute.positions(T, P)


@pytest.mark.parametrize("method", [0, 1])
def test_two_round_seeding_brute(method):
    """Second round: long, rare round-1 SMEMs are re-seeded with (floor(len/2), s+1)."""
    rng = np.random.default_rng(5)
    unit = to_str(rng.integers(0, 4, 24))
    R = to_str(rng.integers(0, 4, 40)) + unit + to_str(rng.integers(0, 4, 30)) + unit[:14] + \
        to_str(rng.integers(0, 4, 30)) + unit[10:] + to_str(rng.integers(0, 4, 20))
    ix = oracle.OracleIndex(ref_codes(R), sa_rate=4)
    T = brute.text_of(R)
    reads = [R[30:80], R[35:70], brute.revcomp(R[38:72]), unit + "AC"]
    seq, offs = csr(reads)
    for (l, c, rl, ro) in [(6, 1, 12, 2), (5, 1, 10, 3), (8, 1, 16, 1)]:
        res = ix.seed(seq, offs, min_len=l, min_occ=c, reseed=True, reseed_len=rl, reseed_occ=ro,
                      method=method, max_occ=10 ** 6)
        for r, P in enumerate(reads):
            assert seeds_of(res, r) == brute.seeds_two_rounds(T, P, l, c, rl, ro), (l, c, P)


@pytest.mark.parametrize("rate", [1, 2, 3, 8, 32])
def test_locate_slow_equals_full_sa(rate):
    R = TINY_REFS["random200"]
    ix = oracle.OracleIndex(ref_codes(R), sa_rate=rate)
    SA = ix.sa()
    for x in range(ix.n):
        assert ix.locate_slow(x) == int(SA[x])


def test_homopolymer_closed_form():
    """T = A^L T^L $: occ(A^m) = L - m + 1, lo(A^m) = 1 (only the $ suffix is smaller)."""
    L = 40
    ix = oracle.OracleIndex(np.zeros(L, np.uint8), sa_rate=4)
    for m in range(1, L + 1):
        k, kr, s = ix.interval("A" * m)
        assert s == L - m + 1
        assert k == 1
        assert kr == ix.interval("T" * m)[0]
    assert ix.interval("A" * (L + 1))[2] == 0


def test_unique_read_closed_form():
    """An error-free read from unique sequence has exactly one SMEM, the whole read, with s = 1;
    its reverse complement gives the mirrored interval."""
    ref = synth.random_reference(20_000, 9).codes
    R = to_str(ref)
    ix = oracle.OracleIndex(ref, sa_rate=8)
    reads = [R[1000:1150], brute.revcomp(R[5000:5150]), R[:150]]
    seq, offs = csr(reads)
    for method in (0, 1):
        res = ix.seed(seq, offs, method=method)
        for r in range(3):
            sd = seeds_of(res, r)
            assert len(sd) == 1 and sd[0][0] == 0 and sd[0][1] == 150 and sd[0][2][2] == 1
        assert [int(p) for p in res.pos[:1]] == [1000]
    # mirrored strands: SMEMs of revcomp(P) = mirrored SMEMs of P with (k, k') swapped
    rng = np.random.default_rng(4)
    for _ in range(5):
        i = int(rng.integers(0, 19000))
        s = list(R[i:i + 120])
        for t in rng.integers(0, 120, 3):
            s[t] = ACGT[(ACGT.index(s[t]) + 1) % 4]
        P = "".join(s)
        seq, offs = csr([P, brute.revcomp(P)])
        res = ix.seed(seq, offs, min_len=12, reseed=False)
        a = seeds_of(res, 0)
        b = seeds_of(res, 1)
        mir = sorted((120 - j, 120 - i_, (kr, k, s_)) for (i_, j, (k, kr, s_)) in a)
        assert b == mir


def test_min_occ_above_copy_number():
    ref = synth.random_reference(5_000, 10).codes
    R = to_str(ref)
    ix = oracle.OracleIndex(ref, sa_rate=8)
    seq, offs = csr([R[100:250], R[2000:2150]])
    res = ix.seed(seq, offs, min_occ=3, reseed=False)
    assert len(res) == 0


def test_bisulfite_brute():
    """Bisulfite index (Section 2.9): T over C->T(R) . G->A(R) and its reverse complement; read-1
    converted C->T keeps positions in segments 0 and 2, read-2 converted G->A in segments 1, 3."""
    R = to_str(np.random.default_rng(12).integers(0, 4, 50))
    ix = oracle.OracleIndex(ref_codes(R), bisulfite=True, sa_rate=3)
    T = brute.bs_text_of(R)
    assert "".join("$ACGT"[x] for x in ix.text()) == T
    reads = [R[5:30], brute.revcomp(R[12:40]), R[20:45]]
    seq, offs = csr(reads)
    for role in (1, 2):
        res = ix.seed(seq, offs, min_len=6, reseed=False, bs_role=role, max_occ=10 ** 6)
        for r, P in enumerate(reads):
            Pc = P.replace("C", "T") if role == 1 else P.replace("G", "A")
            exp = brute.smems(T, Pc, 6, 1)
            assert seeds_of(res, r) == exp
        keep = {1: (0, 2), 2: (1, 3)}[role]
        for t in range(len(res)):
            P = reads[res.read_id[t]]
            Pc = P.replace("C", "T") if role == 1 else P.replace("G", "A")
            sub = Pc[res.qbeg[t]:res.qend[t]]
            exp = [p for p in brute.positions(T, sub) if p // len(R) in keep]
            got = [int(x) for x in res.pos[res.pos_off[t]:res.pos_off[t] + res.npos[t]]]
            assert got == exp


def test_max_occ_rule():
    """Seeds with s > max_occ are reported with their interval but not located (flag bit 0)."""
    R = "ACGTTGCAAT" * 12 + to_str(np.random.default_rng(2).integers(0, 4, 100))
    ix = oracle.OracleIndex(ref_codes(R), sa_rate=4)
    seq, offs = csr(["ACGTTGCAATACGTTGCAAT", R[130:170]])
    res = ix.seed(seq, offs, min_len=10, reseed=False, max_occ=5)
    assert len(res) >= 2
    for t in range(len(res)):
        if int(res.s[t]) > 5:
            assert res.flags[t] == 1 and res.npos[t] == 0
        else:
            assert res.flags[t] == 0 and res.npos[t] == res.s[t]


def test_algorithm3_equals_definition_small_workload():
    """O2 (Algorithm 3 + LocateSlow, with and without the k-mer shortcut) reproduces O1 on a
    slice of the 1 Mbp workload (all fields, all positions)."""
    ref = synth.workload_reference("small_1mbp")
    reads = synth.workload_reads("small_1mbp", ref, n=2000)
    ix = oracle.OracleIndex(ref.codes, sa_rate=8)
    a = ix.seed(reads.seq, reads.offsets, method=0)
    for kw in (dict(method=1), dict(method=1, kmer_k=10)):
        b = ix.seed(reads.seq, reads.offsets, **kw)
        for f in ("read_id", "qbeg", "qend", "k", "kr", "s", "npos", "flags", "pos_off", "pos"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), (kw, f)
    assert len(a) > 2000


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_worked_aca.json")


def test_hand_worked_example():
    """The hand-derived example (R = ACA, T = ACATGT$): suffix array, BWT, C, ds-intervals,
    positions, LocateSlow through the $ row and SMEM sets, for both oracles."""
    g = json.load(open(GOLDEN))
    ox = oracle.OracleIndex(ref_codes(g["R"]), sa_rate=2)
    assert "".join("$ACGT"[int(x)] for x in ox.text()) == g["T"]
    assert [int(x) for x in ox.sa()] == g["SA"]
    assert "".join("$ACGT"[int(x)] for x in ox.bwt()) == g["BWT"]
    assert ox.primary == g["primary"]
    C = ox.C()
    assert [int(C[oracle.SYM[a]]) for a in "ACGT"] == [g["C"][a] for a in "ACGT"]
    for p, iv in g["intervals"].items():
        assert ox.interval(p) == tuple(iv), p
        a = oracle.SYM[p[0]]
        assert ox.backward(ox.interval(p[1:]), a) == tuple(iv) if len(p) > 1 else True
    for row, v in g["locate_r2"].items():
        if not row.startswith("_"):
            assert ox.locate_slow(int(row)) == v[1]
    for case in g["smems"]:
        seq, offs = csr([case["read"]])
        for method in (0, 1):
            res = ox.seed(seq, offs, min_len=case["l"], min_occ=case["c"], method=method)
            got = [[int(res.qbeg[t]), int(res.qend[t]), int(res.k[t]), int(res.kr[t]), int(res.s[t])]
                   for t in range(len(res))]
            assert got == case["out"], (case, method)
            for t in range(len(res)):
                sub = case["read"][got[t][0]:got[t][1]]
                if sub in g["positions"]:
                    ps = res.pos[int(res.pos_off[t]):int(res.pos_off[t]) + int(res.npos[t])]
                    assert [int(x) for x in ps] == g["positions"][sub]


def _same_except_bounds(a, b):
    """Equal seed sets, occurrence counts, flags and positions (the scan oracle has no lo bounds)."""
    assert len(a) == len(b)
    for f in ("read_id", "qbeg", "qend", "s", "npos", "flags", "pos_off"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.array_equal(a.pos, b.pos)
    assert np.all(a.k == np.uint64(2 ** 64 - 1)) and np.all(a.kr == np.uint64(2 ** 64 - 1))


@pytest.mark.parametrize("name", ["random200", "period2", "palindrome", "repeats", "homopolymer", "len2"])
def test_scan_oracle_equals_definition_tiny(name):
    """O3 (one scan of T per q-mer set) reproduces O1 on tiny references: c in {1,2,3}, with and
    without re-seeding, reads with N bases, reads shorter than l."""
    R = TINY_REFS[name]
    ox = oracle.OracleIndex(ref_codes(R), sa_rate=3)
    rng = np.random.default_rng(11)
    reads = []
    for _ in range(30):
        if len(R) < 3:
            break
        i = int(rng.integers(0, len(R) - 2))
        j = int(rng.integers(i + 2, min(len(R), i + 40) + 1))
        s = list(R[i:j])
        for t in range(len(s)):
            if rng.random() < 0.05:
                s[t] = "ACGTN"[int(rng.integers(0, 5))]
        s = "".join(s)
        reads.append(s if rng.random() < 0.5 else brute.revcomp(s.replace("N", "A")))
    reads += ["ACGTAC", "NNACGN", "A", "", "GATTACAGATTACA"]
    seq, offs = csr(reads)
    for l, c in [(3, 1), (4, 2), (2, 3), (5, 1)]:
        for reseed in (False, True):
            kw = dict(min_len=l, min_occ=c, max_occ=10 ** 6, reseed=reseed, reseed_len=2 * l, reseed_occ=3)
            exp = ox.seed(seq, offs, **kw)
            got = oracle.scan_seed(ref_codes(R), seq, offs, **kw)
            _same_except_bounds(got, exp)


def test_scan_oracle_equals_definition_workload_slice():
    """O3 reproduces O1 on 150 bp reads over a 300 kbp slice of the 1 Mbp workload (l = 19,
    re-seeding on, max_occ 500 and a small max_occ) and on bisulfite reads of both roles."""
    ref = synth.workload_reference("small_1mbp")
    sub = np.ascontiguousarray(ref.codes[:300_000])
    ox = oracle.OracleIndex(sub, sa_rate=8)
    sref = synth.Reference(sub, np.zeros((0, 2), np.uint64), 0, 0)
    rs = synth.reads_fixed(sref, 400, 150, True, p_sub=0.01, p_indel=0.001, seed=9)
    for mo in (500, 2):
        exp = ox.seed(rs.seq, rs.offsets, max_occ=mo)
        got = oracle.scan_seed(sub, rs.seq, rs.offsets, max_occ=mo)
        _same_except_bounds(got, exp)
    bref = synth.reference(0, 60_000, 31)
    obs = oracle.OracleIndex(bref.codes, bisulfite=True, sa_rate=8)
    brs = synth.reads_bisulfite(bref, 300, seed=5)
    for role in (1, 2):
        exp = obs.seed(brs.seq, brs.offsets, bs_role=role)
        got = oracle.scan_seed(bref.codes, brs.seq, brs.offsets, bisulfite=True, bs_role=role)
        _same_except_bounds(got, exp)


def _bs_convert(s, frm, to, rng, p=1.0):
    return "".join(to if (ch == frm and rng.random() < p) else ch for ch in s)


@pytest.mark.parametrize("strand,role", [("fwd", 1), ("rev", 1), ("fwd", 2)])
def test_bs_refine_truth(strand, role):
    """Bisulfite refinement (Section 2.9) against simulation truth.  A read 1 is the C->T image of
    the forward (or reverse) strand at offset o with 70% of its C's converted; a read 2 the G->A
    image of the forward strand.  At its true text position (forward C->T copy: o; reverse: the
    reverse G->A copy at 3|R| - o - m; forward G->A copy: |R| + o) the seed stays whole, and a
    planted read C over reference T (read 2: G over A) at base q splits it into [0, q) and [q+1, m)
    (pieces shorter than 19 dropped), the second piece at text position + q + 1."""
    rng = np.random.default_rng(7)
    L = 20_000
    R = to_str(rng.integers(0, 4, L))
    ox = oracle.OracleIndex(ref_codes(R), bisulfite=True, sa_rate=4)
    m = 120
    for trial in range(12):
        o = int(rng.integers(0, L - m))
        src = R[o:o + m] if strand == "fwd" else brute.revcomp(R[o:o + m])
        if role == 1:
            clean = _bs_convert(src, "C", "T", rng, 0.7)
            bad, over = "C", "T"
        else:
            clean = _bs_convert(src, "G", "A", rng, 0.7)
            bad, over = "G", "A"
        truth = o if (strand == "fwd" and role == 1) else (L + o if role == 2 else 3 * L - o - m)
        cand = [q for q in range(5, m - 5) if src[q] == over]
        q = cand[int(rng.integers(0, len(cand)))]
        planted = clean[:q] + bad + clean[q + 1:]
        for read, cut in ((clean, None), (planted, q)):
            seq, offs = csr([read])
            res = ox.seed(seq, offs, min_len=19, bs_role=role, reseed=False)
            pieces = oracle.bs_refine(ref_codes(R), seq, offs, res, role, min_len=19)
            at = [(int(p["qbeg"]), int(p["qend"]), int(p["pos"])) for p in pieces
                  if int(p["pos"]) - int(p["qbeg"]) == truth]
            if cut is None:
                assert at == [(0, m, truth)], (trial, at)
            else:
                exp = [(a, b, truth + a) for a, b in ((0, cut), (cut + 1, m)) if b - a >= 19]
                assert at == exp, (trial, cut, at, exp)


def test_bs_refine_pieces_are_maximal_and_clean():
    """On a bisulfite workload: pieces lie inside their seeds, are at least 19 long, sorted, and
    two pieces of one (seed, position) are separated by exactly the excluded base(s)."""
    ref = synth.reference(0, 100_000, 31)
    ox = oracle.OracleIndex(ref.codes, bisulfite=True, sa_rate=8)
    rs = synth.reads_bisulfite(ref, 400, seed=5)
    res = ox.seed(rs.seq, rs.offsets, bs_role=1)
    pieces = oracle.bs_refine(ref.codes, rs.seq, rs.offsets, res, 1, min_len=19)
    assert len(pieces) > 200
    for p in pieces:
        t = int(p["seed"])
        assert res.read_id[t] == p["read_id"] and res.qbeg[t] <= p["qbeg"] < p["qend"] <= res.qend[t]
        assert p["qend"] - p["qbeg"] >= 19
    key = np.lexsort((pieces["pos"], pieces["qend"], pieces["qbeg"], pieces["read_id"]))
    assert np.array_equal(key, np.arange(len(pieces)))
