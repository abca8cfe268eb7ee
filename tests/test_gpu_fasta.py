"""Index build from a FASTA file (mbw_index_build_fasta) and the record table.

* A multi-record FASTA (wrapped lines, CRLF line ends, blank lines, lower case, ambiguous bases,
  headers with descriptions) builds the same occurrence lines, sampled SA and k-mer table as
  mbw_index_build on the records' sequences back to back; the record table holds each record's
  name (header up to the first blank), start and length; positions map back to records; the
  table survives save / load; seeding on it equals the oracle's on the concatenated reference.
* Malformed files are refused: a missing file (MBW_E_IO), no record, sequence before the first
  header, a record without sequence (MBW_E_FORMAT).
"""
import os

import numpy as np
import pytest

import oracle
import synth
from mbw_helpers import compare_with_oracle, gpu_seed, read_index_file

mbw = pytest.importorskip("paper_2606_15357_amd")

pytestmark = pytest.mark.gpu

ACGT = np.frombuffer(b"ACGT", np.uint8)


def _records(seed=3):
    rng = np.random.default_rng(seed)
    recs = []
    for name, desc, ln in (("chr1", " the first one", 70_003), ("chrM", "", 16_569), ("scaffold_7", "\tx=1", 40_000)):
        recs.append((name, desc, ACGT[rng.integers(0, 4, ln)].tobytes()))
    return recs


def _as_written(recs, ambiguous):
    """Each record's sequence as the file holds it: the third in lower case, and six ambiguous
    bases at 100..105 when asked."""
    out = []
    for i, (_, _, seq) in enumerate(recs):
        s = seq.lower() if i == 2 else seq
        if ambiguous:
            s = s[:100] + b"NNNNRY" + s[106:]
        out.append(s)
    return out


def _write_fasta(path, recs, width=61, crlf_record=1, ambiguous=False):
    with open(path, "wb") as f:
        f.write(b"\n")
        for i, ((name, desc, _), s) in enumerate(zip(recs, _as_written(recs, ambiguous))):
            eol = b"\r\n" if i == crlf_record else b"\n"
            f.write(b">" + name.encode() + desc.encode() + eol)
            for a in range(0, len(s), width):
                f.write(s[a:a + width] + eol)
            f.write(eol)


def test_fasta_build_equals_memory_build(tmp_path):
    recs = _records()
    fa = str(tmp_path / "ref.fa")
    _write_fasta(fa, recs, ambiguous=True)
    seq = b"".join(_as_written(recs, True))
    a = mbw.Index.build_fasta(fa, sa_sample=8, kmer_k=10, rng_seed=9)
    b = mbw.Index.build(seq, sa_sample=8, kmer_k=10, rng_seed=9)
    starts = np.cumsum([0] + [len(s) for _, _, s in recs])
    want = [(name, int(starts[i]), len(s)) for i, (name, _, s) in enumerate(recs)]
    assert a.contigs() == want
    assert b.contigs() == [("", 0, len(seq))]
    for i, (name, st, ln) in enumerate(want):
        for off in (0, ln // 2, ln - 1):
            assert a.ref_to_contig(st + off) == (i, off)
    with pytest.raises(mbw.MbwError):
        a.ref_to_contig(int(starts[-1]))
    pa, pb = str(tmp_path / "a.mbw"), str(tmp_path / "b.mbw")
    a.save(pa)
    b.save(pb)
    fa_, fb_ = read_index_file(pa), read_index_file(pb)
    for k in ("n", "len_r", "primary", "C"):
        assert fa_[k] == fb_[k], k
    for k in ("lines", "ssa", "kmer", "text", "isa"):
        assert np.array_equal(fa_[k], fb_[k]), k
    assert fa_["contigs"] == want and fa_["end"] == fa_["size"]
    c = mbw.Index.load(pa)
    assert c.contigs() == want
    # seeding against the records back to back (no ambiguous bases here, so the oracle sees the
    # same reference)
    _write_fasta(fa, recs)
    d = mbw.Index.build_fasta(fa, sa_sample=8, kmer_k=10)
    codes = np.frombuffer(b"".join(s for _, _, s in recs).upper(), np.uint8)
    ref = synth.Reference(np.searchsorted(ACGT, codes).astype(np.uint8), np.zeros((0, 2), np.uint64), 0, 0)
    reads = synth.reads_fixed(ref, 2000, 150, False, p_sub=0.01, p_indel=0.001, seed=4)
    out, seeds, pos = gpu_seed(d, reads)
    compare_with_oracle(seeds, pos, oracle.OracleIndex(ref.codes, sa_rate=8).seed(reads.seq, reads.offsets))
    for x in (a, b, c, d):
        x.free()


@pytest.mark.parametrize("content,code", [
    (None, "MBW_E_IO"), (b"", "MBW_E_FORMAT"), (b"\n\n", "MBW_E_FORMAT"), (b"ACGT\n>r1\nACGT\n", "MBW_E_FORMAT"),
    (b">r1\nACGT\n>r2\n>r3\nACGT\n", "MBW_E_FORMAT"), (b">r1\nACGT\n>r2\n", "MBW_E_FORMAT")])
def test_fasta_refusals(tmp_path, content, code):
    p = str(tmp_path / "bad.fa")
    if content is not None:
        with open(p, "wb") as f:
            f.write(content)
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.build_fasta(p, sa_sample=8, kmer_k=4)
    assert e.value.code == getattr(mbw, code)


def test_ambiguous_reference_bases_follow_the_oracle(tmp_path):
    """Reading S5: bases other than A, C, G, T (N runs, IUPAC codes, one in a hundred) become the
    low two bits of SplitMix64 output i at reference position i, seeded with rng_seed; the GPU
    index (from memory and from FASTA) has the oracle's BWT, C and primary row for the converted
    reference, and seeding on it equals the oracle's."""
    import tempfile
    from mbw_helpers import decode_bwt
    rng = np.random.default_rng(17)
    n = 60_000
    ascii_ = ACGT[rng.integers(0, 4, n)].copy()
    amb = rng.choice(n, n // 100, replace=False)
    ascii_[amb] = np.frombuffer(b"NRYKMSWBDHV", np.uint8)[rng.integers(0, 11, amb.size)]
    ascii_[1000:1040] = ord("N")
    seed = 1234567
    codes = oracle.codes_from_ascii(ascii_.tobytes(), seed)
    ox = oracle.OracleIndex(codes, sa_rate=8)
    fa = str(tmp_path / "amb.fa")
    with open(fa, "wb") as f:
        f.write(b">amb\n")
        for a in range(0, n, 70):
            f.write(ascii_[a:a + 70].tobytes() + b"\n")
    for idx in (mbw.Index.build(ascii_.tobytes(), sa_sample=8, kmer_k=8, rng_seed=seed),
                mbw.Index.build_fasta(fa, sa_sample=8, kmer_k=8, rng_seed=seed)):
        info = idx.info()
        assert info["n"] == ox.n and info["primary"] == ox.primary
        assert [int(x) for x in info["C"]] == [int(x) for x in ox.C()[:5]]
        with tempfile.TemporaryDirectory() as d:
            p = os.path.join(d, "amb.mbw")
            idx.save(p)
            fidx = read_index_file(p)
        B = ox.bwt().astype(np.int64) - 1
        B[ox.primary] = 0
        assert np.array_equal(decode_bwt(fidx), B.astype(np.uint8))
        ref = synth.Reference(codes, np.zeros((0, 2), np.uint64), 0, 0)
        reads = synth.reads_fixed(ref, 1500, 150, False, p_sub=0.01, p_indel=0.001, seed=18)
        out, s, p = gpu_seed(idx, reads)
        compare_with_oracle(s, p, ox.seed(reads.seq, reads.offsets))
        idx.free()
