"""GPU parity: the HIP library against the CPU oracle, element by element, through the C-ABI.

Integer results must be bit-exact: same seeds (read, qbeg, qend), same ds-intervals (k, k', s),
same position sets (canonical order: seeds by (read, qbeg, qend), positions ascending).
"""
import os
import tempfile

import numpy as np
import pytest

import brute
import oracle
import synth
from mbw_helpers import compare_with_oracle, decode_bwt, gpu_seed, read_index_file, unpack_kmer

mbw = pytest.importorskip("paper_2606_15357_amd")

pytestmark = pytest.mark.gpu

ACGT = "ACGT"


def ref_codes(s):
    return np.array(["ACGT".index(ch) for ch in s], dtype=np.uint8)


def to_str(codes):
    return "".join(ACGT[int(x)] for x in codes)


def readset(reads):
    lens = np.array([len(r) for r in reads], dtype=np.uint32)
    offs = np.zeros(len(reads) + 1, np.uint64)
    offs[1:] = np.cumsum(lens)
    seq = np.frombuffer("".join(reads).encode(), dtype=np.uint8).copy()
    return synth.ReadSet(seq, lens, offs, np.zeros(len(reads), np.uint64), np.zeros(len(reads), np.uint8))


TINY = {
    "random300": to_str(np.random.default_rng(1).integers(0, 4, 300)),
    "homopolymer": "A" * 50,
    "period2": "AC" * 40,
    "palindrome": "ACGGTCAT" + brute.revcomp("ACGGTCAT"),
    "len1": "G",
    "repeats": "ACGTTGCAAG" * 5 + "GGATCCATTA" + "ACGTTGCAAG" * 4,
}


@pytest.mark.parametrize("name", sorted(TINY))
@pytest.mark.parametrize("r,K,ri", [(1, 0, 1), (3, 2, 3), (8, 3, 4), (8, 0, 0)])
def test_index_structure(name, r, K, ri):
    """BWT, C, primary row, SA samples, k-mer intervals, packed text and inverse-SA samples of the
    GPU index equal the oracle's."""
    R = TINY[name]
    idx = mbw.Index.build(ref_codes(R), sa_sample=r, kmer_k=K, isa_sample=ri)
    info = idx.info()
    ox = oracle.OracleIndex(ref_codes(R), sa_rate=r)
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "ix.mbw")
        idx.save(p)
        f = read_index_file(p)
    assert f["n"] == ox.n and info["n"] == ox.n
    assert info["primary"] == ox.primary
    B = ox.bwt().astype(np.int64) - 1
    B[ox.primary] = 0
    assert np.array_equal(decode_bwt(f), B.astype(np.uint8))
    assert [int(x) for x in info["C"]] == [int(x) for x in ox.C()[:5]]
    SA = ox.sa()
    assert np.array_equal(f["ssa"], SA[::r])
    assert f["isa_sample"] == ri and info["isa_sample"] == ri
    if ri:
        T = ox.text().astype(np.int64)                  # oracle codes: $ = 0, A..T = 1..4
        m = ox.n - 1
        sh = np.arange(32, dtype=np.uint64) * 2
        tsyms = ((f["text"][:, None] >> sh) & 3).reshape(-1).astype(np.int64)
        assert np.array_equal(tsyms[:m], T[:m] - 1)
        assert not np.any(tsyms[m:])                     # padding after the last symbol
        ISA = np.empty(ox.n, np.int64)
        ISA[SA.astype(np.int64)] = np.arange(ox.n)
        assert np.array_equal(f["isa"].astype(np.int64), ISA[::ri])
    else:
        assert f["text"].size == 0 and f["isa"].size == 0
    # line headers: superblock base + u32 count = count of A, C, G before the line ($ row as A);
    # sub-checkpoint b (1..5): counts of A, C, G in the line's first 64 b rows, 9 bits each
    Braw = B.astype(np.int64)
    w32 = f["lines"].view(np.uint32).reshape(f["n_lines"], 32)
    for L in range(f["n_lines"]):
        lo = L * 384
        for a in range(3):
            assert int(f["sb"][L >> f["sb_shift"]][a]) + int(w32[L, a]) == int(np.sum(Braw[:lo] == a))
        for b in range(1, 6):
            if lo + 64 * b > f["n"]:
                continue
            blk = Braw[lo:lo + 64 * b]
            sub = int(w32[L, 3 if b == 1 else 4 + (b - 2)])
            assert [(sub >> (9 * a)) & 511 for a in range(3)] == [int(np.sum(blk == a)) for a in range(3)]
    if K:
        T = brute.text_of(R)
        for code in range(4 ** K):
            kmer = "".join(ACGT[(code >> (2 * q)) & 3] for q in range(K))
            exp = ox.interval(kmer)
            got = unpack_kmer(f["kmer"][code])
            if exp[2] == 0:
                assert got[2] == 0
            else:
                assert got == exp, (kmer, got, exp)
        assert T


@pytest.mark.parametrize("name", sorted(TINY))
@pytest.mark.parametrize("kernel,variant", [(0, "default"), (1, "default"), (0, "segmented")])
def test_tiny_seeding(name, kernel, variant):
    """Tiny references, reads up to 60 bases, (l, c) in {(3,1), (5,1), (4,2), (2,3)}, both rounds;
    'segmented' runs every read unstaged in 32-base segments."""
    R = TINY[name]
    rng = np.random.default_rng(3)
    reads = []
    for _ in range(40):
        if len(R) < 4:
            break
        i = int(rng.integers(0, len(R) - 3))
        j = int(rng.integers(i + 3, min(len(R), i + 60) + 1))
        s = list(R[i:j])
        for t in range(len(s)):
            if rng.random() < 0.05:
                s[t] = ACGT[int(rng.integers(0, 4))]
        s = "".join(s)
        reads.append(s if rng.random() < 0.5 else brute.revcomp(s))
    reads += ["ACGTACGTACGTAGCT", "NNNNACGTNN", "A", "", "GATTACAGATTACA"]
    rs = readset(reads)
    ox = oracle.OracleIndex(ref_codes(R), sa_rate=3)
    for K in (0, 3):
        idx = mbw.Index.build(ref_codes(R), sa_sample=3, kmer_k=K)
        for (l, c) in [(3, 1), (5, 1), (4, 2), (2, 3)]:
            for reseed in (False, True):
                exp = ox.seed(rs.seq, rs.offsets, min_len=l, min_occ=c, max_occ=10 ** 6, reseed=reseed,
                              reseed_len=2 * l, reseed_occ=3)
                extra = dict(stage=False, seg_len=32) if variant == "segmented" else {}
                out, seeds, pos = gpu_seed(idx, rs, min_seed_len=l, min_occ=c, max_occ=10 ** 6, reseed=reseed,
                                           reseed_len=2 * l, reseed_occ=3, kernel=kernel, **extra)
                compare_with_oracle(seeds, pos, exp)
        idx.free()


@pytest.fixture(scope="module")
def cfg0():
    ref = synth.workload_reference("small_1mbp")
    reads = synth.workload_reads("small_1mbp", ref)
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    exp = ox.seed(reads.seq, reads.offsets, min_len=19, max_occ=500)
    return ref, reads, ox, exp


@pytest.mark.parametrize("kernel,K,ri,uniq,defer", [(0, 10, 4, True, 0), (0, 10, 4, False, 0), (0, 0, 1, True, 0),
                                                    (1, 0, 4, True, 0), (0, 12, 8, True, 0), (0, 12, 0, True, 0),
                                                    (0, 14, 4, True, 0), (1, 14, 4, True, 0), (0, 15, 4, True, 0),
                                                    (0, 10, 4, True, 1), (0, 0, 1, True, 1), (0, 12, 8, True, 1),
                                                    (0, 15, 1, True, 1)])
def test_small_workload_parity(cfg0, kernel, K, ri, uniq, defer):
    """1 Mbp + repeat family reference, 10,000 x 150 bp reads, (19,1)-SMEMs with re-seeding,
    max_occ 500: every seed, interval and position equals the oracle's, with and without the
    direct extension of unique matches (inverse-SA samples every ri text positions), and with the
    unique matches finished in the lane (defer 0) or by the continuation kernel in alternating
    passes (defer 1)."""
    ref, reads, ox, exp = cfg0
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=K, isa_sample=ri)
    out, seeds, pos = gpu_seed(idx, reads, min_seed_len=19, max_occ=500, kernel=kernel, unique_ext=uniq,
                               unique_defer=defer)
    compare_with_oracle(seeds, pos, exp)
    assert out.n_seeds == len(exp)
    idx.free()


def test_automatic_kmer_size(cfg0):
    """kmer_k = -1 picks floor(log4 n) - 1 (n = 2,080,001 here: 9) and seeds bit-exactly."""
    ref, reads, ox, exp = cfg0
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=-1)
    n = idx.info()["n"]
    assert idx.info()["kmer_k"] == max(1, min(15, int(np.floor(np.log(n) / np.log(4))) - 1)) == 9
    out, seeds, pos = gpu_seed(idx, reads, min_seed_len=19, max_occ=500)
    compare_with_oracle(seeds, pos, exp)
    idx.free()


def test_line_count_matches_oracle(cfg0):
    """The kernel's algorithmic line counter equals the oracle's count for the same layout."""
    ref, reads, ox, _ = cfg0
    for K in (0, 10):
        idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=K)
        out, seeds, pos = gpu_seed(idx, reads, min_seed_len=19, max_occ=500, kernel=0, unique_ext=False)
        o2 = ox.seed(reads.seq, reads.offsets, method=1, kmer_k=K, bases_per_line=384)
        assert out.steps == o2.lines["steps"]
        assert out.lines_smem == o2.lines["lines"] - o2.lines["lf_steps"] + o2.lines["kmer_lookups"]
        assert out.lf_steps == o2.lines["lf_steps"]
        assert out.lines_locate == o2.lines["lf_steps"] + o2.lines["sa_reads"]
        idx.free()


def test_edge_cases(cfg0):
    ref, _, ox, _ = cfg0
    R = to_str(ref.codes[:5000])
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    ctx = mbw.Context(idx)
    # empty batch
    out = ctx.seed(np.zeros(0, np.uint8), np.zeros(0, np.uint32))
    assert out.n_seeds == 0 and out.n_pos == 0
    # reads shorter than l, empty reads, N runs, lower case, ragged lengths
    reads = ["", "A", R[:18], R[:19], R[100:400].lower(), R[500:600] + "N" * 30 + R[700:800],
             R[1000:1001 + 250], "N" * 40, R[2000:2150]]
    rs = readset(reads)
    for kernel in (0, 1):
        out, seeds, pos = gpu_seed(idx, rs, kernel=kernel)
        exp = ox.seed(rs.seq, rs.offsets)
        compare_with_oracle(seeds, pos, exp)
    # a single maximal-length read (65535) and an over-long one
    long = to_str(ref.codes[10000:10000 + 65535])
    rs = readset([long])
    out, seeds, pos = gpu_seed(idx, rs, kernel=0)
    exp = ox.seed(rs.seq, rs.offsets)
    compare_with_oracle(seeds, pos, exp)
    with pytest.raises(mbw.MbwError):
        ctx.seed(np.frombuffer((long + "A").encode(), np.uint8).copy(), np.array([65536], np.uint32))
    with pytest.raises(mbw.MbwError):
        ctx.seed(rs.seq, rs.lengths, min_seed_len=0)
    ctx.free()
    idx.free()


def test_ragged_lengths_and_occ(cfg0):
    """Ragged read lengths 1..600 (staged and unstaged length bins, long reads in segments of 256,
    64 and 32 bases), c in {1,2,3}, max_occ small enough to skip repeats."""
    ref, _, ox, _ = cfg0
    rs = synth.reads_uniform_len(ref, 3000, 1, 600, seed=77)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    for c, mo in [(1, 3), (2, 500), (3, 20)]:
        exp = ox.seed(rs.seq, rs.offsets, min_occ=c, max_occ=mo)
        for kernel, seg in ((0, 0), (1, 0), (0, 64), (0, 32)):
            out, seeds, pos = gpu_seed(idx, rs, min_occ=c, max_occ=mo, kernel=kernel, seg_len=seg)
            compare_with_oracle(seeds, pos, exp)
    idx.free()


def test_bisulfite_parity():
    ref = synth.reference(0, 200_000, 31)
    ox = oracle.OracleIndex(ref.codes, bisulfite=True, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10, bisulfite=True)
    rs = synth.reads_bisulfite(ref, 2000, seed=5)
    for role in (1, 2):
        for kernel in (0, 1):
            out, seeds, pos = gpu_seed(idx, rs, bs_role=role, kernel=kernel)
            exp = ox.seed(rs.seq, rs.offsets, bs_role=role)
            compare_with_oracle(seeds, pos, exp)
    idx.free()


def test_index_save_load_roundtrip(cfg0):
    ref, reads, ox, exp = cfg0
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "cfg0.mbw")
        idx.save(p)
        idx2 = mbw.Index.load(p)
        out, seeds, pos = gpu_seed(idx2, reads)
        compare_with_oracle(seeds, pos, exp)
        # corrupt one byte in the middle: the checksum must catch it
        with open(p, "r+b") as f:
            f.seek(4096)
            b = f.read(1)
            f.seek(4096)
            f.write(bytes([b[0] ^ 0xFF]))
        with pytest.raises(mbw.MbwError) as e:
            mbw.Index.load(p)
        assert e.value.code == mbw.MBW_E_FORMAT
        idx2.free()
    idx.free()


def test_index_file_streams_in_chunks(cfg0):
    """Save and load move arrays through 64 MiB host chunks: a 12-mer table (256 MiB) spans
    four; the reloaded index seeds bit-exact, its file is byte-identical when
    saved again, and a file cut short, one with bytes appended, or one with a byte flipped in its
    last chunk is refused."""
    ref, reads, ox, exp = cfg0
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=12, isa_sample=4)
    with tempfile.TemporaryDirectory() as d:
        p, q = os.path.join(d, "a.mbw"), os.path.join(d, "b.mbw")
        idx.save(p)
        idx.free()
        size = os.path.getsize(p)
        assert size > 4 * (64 << 20)
        idx2 = mbw.Index.load(p)
        out, seeds, pos = gpu_seed(idx2, reads)
        compare_with_oracle(seeds, pos, exp)
        idx2.save(q)
        idx2.free()
        with open(p, "rb") as fa, open(q, "rb") as fb:
            while True:
                a, b = fa.read(1 << 24), fb.read(1 << 24)
                assert a == b
                if not a:
                    break
        os.truncate(q, size - 8)
        with pytest.raises(mbw.MbwError) as e:
            mbw.Index.load(q)
        assert e.value.code == mbw.MBW_E_FORMAT and "truncated" in str(e.value)
        with open(p, "ab") as f:
            f.write(b"\0" * 8)
        with pytest.raises(mbw.MbwError) as e:
            mbw.Index.load(p)
        assert e.value.code == mbw.MBW_E_FORMAT
        os.truncate(p, size)
        with open(p, "r+b") as f:
            f.seek(size - 12)
            b = f.read(1)
            f.seek(size - 12)
            f.write(bytes([b[0] ^ 0x10]))
        with pytest.raises(mbw.MbwError) as e:
            mbw.Index.load(p)
        assert e.value.code == mbw.MBW_E_FORMAT and "checksum" in str(e.value)


def test_hand_worked_example():
    """The hand-derived example (R = ACA, T = ACATGT$) straight from the GPU index and kernels."""
    import json
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_worked_aca.json")))
    for K in (0, 1, 2):
        idx = mbw.Index.build(ref_codes(g["R"]), sa_sample=2, kmer_k=K)
        info = idx.info()
        assert info["n"] == len(g["T"]) and info["primary"] == g["primary"]
        assert [int(x) for x in info["C"]] == [0] + [g["C"][a] for a in "ACGT"]
        with tempfile.TemporaryDirectory() as d:
            p = os.path.join(d, "aca.mbw")
            idx.save(p)
            f = read_index_file(p)
        B = "".join("ACGT"[int(x)] for x in decode_bwt(f))
        assert B[:g["primary"]] + "$" + B[g["primary"] + 1:] == g["BWT"]
        assert [int(x) for x in f["ssa"]] == g["SA"][::2]
        for case in g["smems"]:
            rs = readset([case["read"]])
            for kernel in (0, 1):
                out, seeds, pos = gpu_seed(idx, rs, min_seed_len=case["l"], min_occ=case["c"], kernel=kernel)
                s, flat = mbw.canonical(seeds, pos)
                got = [[int(s["qbeg"][t]), int(s["qend"][t]), int(s["k"][t]), int(s["kr"][t]), int(s["s"][t])]
                       for t in range(len(s))]
                assert got == case["out"], (case, kernel, K)
                off = 0
                for t in range(len(s)):
                    sub = case["read"][got[t][0]:got[t][1]]
                    n = int(s["npos"][t])
                    if sub in g["positions"]:
                        assert sorted(int(x) for x in flat[off:off + n]) == g["positions"][sub]
                    off += n
        idx.free()


def test_bisulfite_refinement():
    """Refined bisulfite seed matches (Section 2.9) equal the oracle's, piece for piece, for read 1
    (C->T) and read 2 (G->A) reads, with SNP-like planted mismatches; the index's stored original
    reference decodes to R."""
    ref = synth.reference(0, 200_000, 31)
    ox = oracle.OracleIndex(ref.codes, bisulfite=True, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10, bisulfite=True)
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "bs.mbw")
        idx.save(p)
        f = read_index_file(p)
    sh = np.arange(32, dtype=np.uint64) * 2
    orig = ((f["orig"][:, None] >> sh) & 3).reshape(-1)[: len(ref)].astype(np.uint8)
    assert np.array_equal(orig, ref.codes)
    rs = synth.reads_bisulfite(ref, 2000, seed=5)
    # read 2 form: the G->A image of the same fragments (complement strand view)
    seq2 = rs.seq.copy()
    comp = bytes.maketrans(b"ACGT", b"TGCA")
    for r in range(len(rs)):
        a, b = int(rs.offsets[r]), int(rs.offsets[r + 1])
        seq2[a:b] = np.frombuffer(rs.seq[a:b].tobytes().translate(comp)[::-1], np.uint8)
    rng = np.random.default_rng(4)
    for s_ in (rs.seq, seq2):                                   # a few planted C/G changes
        hit = rng.integers(0, s_.size, s_.size // 200)
        s_[hit] = np.where(rng.random(hit.size) < 0.5, ord("C"), ord("G"))
    for role, seq in ((1, rs.seq), (2, seq2)):
        exp_seeds = ox.seed(seq, rs.offsets, bs_role=role)
        exp = oracle.bs_refine(ref.codes, seq, rs.offsets, exp_seeds, role, min_len=19)
        assert len(exp) > 500
        for kernel in (0, 1):
            ctx = mbw.Context(idx)
            out = ctx.seed(seq, rs.lengths, bs_role=role, kernel=kernel, bs_refine=True)
            seeds, pos = out.download()
            compare_with_oracle(seeds, pos, exp_seeds)
            got = out.download_pieces()
            order = np.lexsort((got["pos"], got["qend"], got["qbeg"], got["read_id"]))
            got = got[order]
            for fld in ("read_id", "qbeg", "qend", "pos"):
                assert np.array_equal(got[fld], exp[fld]), fld
            # the source seed: same (read, interval) family
            assert np.all(seeds["read_id"][got["seed"]] == got["read_id"])
            ctx.free()
    idx.free()


# ---------------------------------------------------------------------------------------------
# several superblocks on small references: the row arithmetic past the first superblock (counts
# relative to a superblock, the superblock table, lines on both sides of a boundary) that the
# 3.1 Gbp indexes need, checked against the definition oracle with every field compared

@pytest.mark.parametrize("kernel,K,ri,uniq,defer", [(0, 10, 4, True, 0), (0, 10, 4, False, 0), (0, 0, 1, True, 0),
                                                    (1, 10, 4, True, 0), (0, 15, 4, True, 0), (1, 0, 0, True, 0),
                                                    (0, 15, 1, True, 1), (0, 10, 4, True, 1)])
def test_multi_superblock_parity(cfg0, kernel, K, ri, uniq, defer):
    """The 1 Mbp workload on an index with 2^10 lines (393,216 rows) per superblock, so that its
    2,080,001 rows span 6 superblocks: every seed, ds-interval (k, k', s) and position of all
    10,000 reads equals O1's, with and without the unique-match path."""
    ref, reads, ox, exp = cfg0
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=K, isa_sample=ri, sb_lines_log2=10)
    info = idx.info()
    assert info["sb_lines_log2"] == 10 and info["n_superblocks"] == 6
    out, seeds, pos = gpu_seed(idx, reads, min_seed_len=19, max_occ=500, kernel=kernel, unique_ext=uniq,
                               unique_defer=defer)
    compare_with_oracle(seeds, pos, exp)
    # seeds whose intervals lie wholly past the first superblock (k and k + s above 393,216)
    assert np.sum(seeds["k"] > 393_216 * 2) > 1000
    idx.free()


def test_multi_superblock_structure_and_tiny_seeding():
    """A 60 kbp reference (random with repeats) indexed with 2^6 lines (24,576 rows) per superblock
    (5 superblocks): the stored superblock table and every line header equal prefix counts of the
    oracle's BWT, the 6-mer table equals the oracle's intervals, the file round trip keeps the
    superblock size, and seeding with (l, c) in {(12,1), (15,2), (10,3)} equals O1 for both kernels,
    segmented and not."""
    ref = synth.reference(0, 20_000, 41)
    R = ref.codes
    ox = oracle.OracleIndex(R, sa_rate=4)
    idx = mbw.Index.build(R, sa_sample=4, kmer_k=6, isa_sample=2, sb_lines_log2=6)
    info = idx.info()
    assert info["n_superblocks"] == ((info["n_lines"] - 1) >> 6) + 1 >= 3
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "sb.mbw")
        idx.save(p)
        f = read_index_file(p)
        idx2 = mbw.Index.load(p)
        assert idx2.info()["sb_lines_log2"] == 6 and idx2.info()["n_superblocks"] == info["n_superblocks"]
    assert f["sb_shift"] == 6
    B = ox.bwt().astype(np.int64) - 1
    B[ox.primary] = 0
    assert np.array_equal(decode_bwt(f), B.astype(np.uint8))
    cum = np.zeros((4, B.size + 1), np.int64)
    for a in range(4):
        cum[a, 1:] = np.cumsum(B == a)
    for sb in range(info["n_superblocks"]):
        row = min(sb * 64 * 384, B.size)
        assert [int(f["sb"][sb][a]) for a in range(4)] == [int(cum[a, row]) for a in range(4)]
        assert [int(f["sb"][sb][4 + c]) for c in range(4)] == [int(sum(cum[d, row] for d in range(c + 1, 4)))
                                                               for c in range(4)]
    w32 = f["lines"].view(np.uint32).reshape(f["n_lines"], 32)
    for L in range(f["n_lines"]):
        lo = L * 384
        for a in range(3):
            assert int(f["sb"][L >> 6][a]) + int(w32[L, a]) == int(cum[a, lo])
    for code in range(4 ** 6):
        kmer = "".join(ACGT[(code >> (2 * q)) & 3] for q in range(6))
        exp = ox.interval(kmer)
        got = unpack_kmer(f["kmer"][code])
        assert got[2] == exp[2] and (exp[2] == 0 or got == exp), (kmer, got, exp)
    rs = synth.reads_uniform_len(ref, 400, 1, 200, seed=42)
    for ix_ in (idx, idx2):
        for (l, c) in [(12, 1), (15, 2), (10, 3)]:
            exp = ox.seed(rs.seq, rs.offsets, min_len=l, min_occ=c, max_occ=10 ** 6, reseed=True, reseed_len=2 * l,
                          reseed_occ=3)
            for kernel, extra in ((0, {}), (1, {}), (0, dict(stage=False, seg_len=32))):
                out, seeds, pos = gpu_seed(ix_, rs, min_seed_len=l, min_occ=c, max_occ=10 ** 6, reseed=True,
                                           reseed_len=2 * l, reseed_occ=3, kernel=kernel, **extra)
                compare_with_oracle(seeds, pos, exp)
    idx2.free()
    idx.free()


def test_multi_superblock_bisulfite():
    """A bisulfite (four-copy) index of 200 kbp with 2^8 lines per superblock (800,001 rows in 9
    superblocks would exceed the table, so 2^9: 5 superblocks): both read roles, both kernels,
    with refinement, equal the oracle; an index that would need more than 8 superblocks is
    refused."""
    ref = synth.reference(0, 200_000, 31)
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10, bisulfite=True, sb_lines_log2=8)
    assert e.value.code == mbw.MBW_E_INVAL and "superblock" in str(e.value)
    ox = oracle.OracleIndex(ref.codes, bisulfite=True, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10, bisulfite=True, sb_lines_log2=9)
    assert idx.info()["n_superblocks"] == 5
    rs = synth.reads_bisulfite(ref, 2000, seed=5)
    for role in (1, 2):
        exp = ox.seed(rs.seq, rs.offsets, bs_role=role)
        pieces = oracle.bs_refine(ref.codes, rs.seq, rs.offsets, exp, role, min_len=19)
        for kernel in (0, 1):
            ctx = mbw.Context(idx)
            out = ctx.seed(rs.seq, rs.lengths, bs_role=role, kernel=kernel, bs_refine=True)
            seeds, pos = out.download()
            compare_with_oracle(seeds, pos, exp)
            got = out.download_pieces()
            got = got[np.lexsort((got["pos"], got["qend"], got["qbeg"], got["read_id"]))]
            for fld in ("read_id", "qbeg", "qend", "pos"):
                assert np.array_equal(got[fld], pieces[fld]), fld
            ctx.free()
    idx.free()
