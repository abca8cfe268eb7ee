"""Captured graphs (mbw_graph_*): the seeding path recorded once as a HIP graph and replayed.

Every replay must give exactly the seeds and positions of an eager mbw_seed call with the same
options (and so the oracle's): the whole 1 Mbp workload, then one graph replayed on batches of
other sizes, lengths (1-160 bases, N runs) and an empty one, each twice with eager calls and
synchronisations in between (a replayed graph must not depend on state the first replay left
behind), from host and from device memory; plans too small and inputs outside the plan are
refused with the documented codes and leave the graph usable.
"""
import numpy as np
import pytest

import oracle
import synth
from mbw_helpers import compare_with_oracle

mbw = pytest.importorskip("paper_2606_15357_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def same(a, b):
    sa, pa = a.download()
    sb, pb = b.download()
    assert sa.size == sb.size and pa.size == pb.size
    for f in sa.dtype.names:
        if f != "reserved":
            assert np.array_equal(sa[f], sb[f]), f
    assert np.array_equal(pa, pb)
    return sa, pa


def subset(reads, ids):
    ids = np.asarray(ids, dtype=np.int64)
    lens = reads.lengths[ids]
    offs = np.zeros(len(ids) + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    seq = np.concatenate([reads.seq[int(reads.offsets[r]):int(reads.offsets[r + 1])] for r in ids]) if len(ids) else \
        np.zeros(0, np.uint8)
    return synth.ReadSet(seq, lens.astype(np.uint32), offs, reads.tpos[ids], reads.tstrand[ids])


@pytest.fixture(scope="module")
def small():
    ref = synth.workload_reference("small_1mbp")
    reads = synth.workload_reads("small_1mbp", ref)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    yield ref, reads, idx
    idx.free()


@pytest.mark.parametrize("kw", [{}, dict(unique_ext=False), dict(reseed=False), dict(use_kmer=False),
                                dict(blocks_per_cu=-1, wave_chunk=64)])
def test_graph_equals_seed_and_oracle(small, kw):
    """10,000 x 150 bp reads of the 1 Mbp workload: a graph's replay equals mbw_seed array for array
    and the oracle, under several seeding options."""
    ref, reads, idx = small
    ctx = mbw.Context(idx)
    base = ctx.seed(reads.seq, reads.lengths, **kw)
    g = ctx.graph(len(reads), **kw)
    out = g.seed(reads.seq, reads.lengths)
    s, p = same(out, base)
    if kw.get("reseed", True):
        ox = oracle.OracleIndex(ref.codes, sa_rate=8)
        compare_with_oracle(s, p, ox.seed(reads.seq, reads.offsets, min_len=19, max_occ=500))
    assert out.ms_total > 0 and out.n_smem_launches == (1 if kw.get("reseed") is False else 2)
    g.free()
    ctx.free()


def test_graph_replays(small):
    """One graph (plan: 4,000 reads) replayed on batches of different sizes and lengths, host and
    device inputs, each twice with eager calls in between; every replay equals the eager result."""
    ref, reads, idx = small
    rag = synth.reads_uniform_len(ref, 3000, 1, 160, seed=91)
    seq = rag.seq.copy()
    rng = np.random.default_rng(92)
    for r in range(0, len(rag), 7):
        a, n = int(rag.offsets[r]), int(rag.lengths[r])
        if n > 40:
            seq[a + 20:a + 20 + int(rng.integers(1, 6))] = ord("N")
    rag = synth.ReadSet(seq, rag.lengths, rag.offsets, rag.tpos, rag.tstrand)
    batches = [subset(reads, range(4000)), subset(reads, range(4000, 4001)), subset(reads, []),
               subset(reads, rng.permutation(10000)[:2500]), rag, subset(reads, range(9000, 10000))]
    ctx = mbw.Context(idx)
    g = ctx.graph(4000)
    plan = g.plan()
    assert plan["max_reads"] == 4000 and plan["max_bases"] == 4000 * 160
    for b in batches:
        for rep in range(2):
            eager = ctx.seed(b.seq, b.lengths)
            ref_s, ref_p = eager.download()
            torch.cuda.synchronize()
            if rep == 0:
                out = g.seed(b.seq, b.lengths)
            else:
                dseq = torch.from_numpy(b.seq.copy() if b.seq.size else np.zeros(1, np.uint8)).to(DEV)
                dlen = torch.from_numpy(b.lengths.view(np.int32).copy()).to(DEV)
                out = g.seed(dseq, dlen)
            s, p = out.download()
            assert s.size == ref_s.size and p.size == ref_p.size
            for f in s.dtype.names:
                if f != "reserved":
                    assert np.array_equal(s[f], ref_s[f]), f
            assert np.array_equal(p, ref_p)
    g.free()
    ctx.free()


def test_graph_refusals(small):
    ref, reads, idx = small
    ctx = mbw.Context(idx)
    g = ctx.graph(100, max_positions=50)
    with pytest.raises(mbw.MbwError) as e:          # more reads than the plan
        g.seed(reads.seq[: int(reads.offsets[101])], reads.lengths[:101])
    assert e.value.code == mbw.MBW_E_INVAL
    long_read = np.frombuffer(b"ACGT" * 50, dtype=np.uint8)
    with pytest.raises(mbw.MbwError) as e:          # a read of 200 bases
        g.seed(long_read, np.array([200], np.uint32))
    assert e.value.code == mbw.MBW_E_INVAL
    with pytest.raises(mbw.MbwError) as e:          # positions beyond the plan
        g.seed(reads.seq[: int(reads.offsets[100])], reads.lengths[:100])
    assert e.value.code == mbw.MBW_E_CAPACITY and "positions" in str(e.value)
    one = subset(reads, [0])                        # the graph still serves a batch that fits
    out = g.seed(one.seq, one.lengths)
    base = ctx.seed(one.seq, one.lengths)
    if base.n_pos <= 50:
        same(out, base)
    g.free()
    for kw in (dict(kernel=mbw.KERNEL_PLAIN), dict(stage=False), dict(unique_defer=1)):
        with pytest.raises(mbw.MbwError) as e:
            ctx.graph(10, **kw)
        assert e.value.code == mbw.MBW_E_INVAL
    with pytest.raises(mbw.MbwError):
        ctx.graph(0)
    ctx.free()


@pytest.fixture(scope="module")
def ragged(small):
    """3,000 reads of 20-700 bases with N runs (both length bins, segments) and the oracle's result."""
    ref, _, idx = small
    rs = synth.reads_uniform_len(ref, 3000, 20, 700, seed=61)
    seq = rs.seq.copy()
    rng = np.random.default_rng(62)
    for r in range(0, len(rs), 9):
        a, n = int(rs.offsets[r]), int(rs.lengths[r])
        if n > 60:
            seq[a + 30:a + 30 + int(rng.integers(1, 8))] = ord("N")
    rs = synth.ReadSet(seq, rs.lengths, rs.offsets, rs.tpos, rs.tstrand)
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    return rs, ox.seed(rs.seq, rs.offsets, min_len=19, max_occ=500)


@pytest.mark.parametrize("kw", [{}, dict(seg_len=32), dict(unique_ext=False, seg_len=100)])
def test_graph_length_bins(small, ragged, kw):
    """Reads of 20-700 bases: a plan with max_read_len 700 runs the staged bin and the long reads in
    segments (both rounds) inside the graph; equal to mbw_seed and the oracle."""
    ref, _, idx = small
    rs, exp = ragged
    ctx = mbw.Context(idx)
    g = ctx.graph(len(rs), max_read_len=700, **kw)
    plan = g.plan()
    assert plan["max_read_len"] == 700 and plan["max_bases"] == len(rs) * 700
    out = g.seed(rs.seq, rs.lengths)
    s, p = same(out, ctx.seed(rs.seq, rs.lengths, **kw))
    compare_with_oracle(s, p, exp)
    assert out.n_smem_launches == 4
    g.free()
    ctx.free()


def test_graph_length_bins_replays(small, ragged):
    """One binned graph (above a million seed slots) replayed on batches of only short reads, only
    long reads, a mix and an empty batch, twice each with eager calls in between; every replay
    equals mbw_seed.  A read longer than
    the plan's max_read_len is refused."""
    ref, reads, idx = small
    rs, _ = ragged
    longs = np.flatnonzero(rs.lengths > 160)
    shorts = np.flatnonzero(rs.lengths <= 160)
    batches = [subset(rs, longs[:800]), subset(rs, shorts), subset(rs, np.sort(np.concatenate([longs[800:1200],
               shorts[:300]]))), subset(rs, []), subset(reads, range(2000))]
    ctx = mbw.Context(idx)
    g = ctx.graph(2000, max_read_len=700)
    # more seed slots than rocPRIM's merge-sort limit (2^20): the graph's sorts must still avoid the
    # onesweep path, whose resets are memsets, on every replay
    assert g.plan()["max_seeds"] > 1 << 20
    for b in batches:
        for rep in range(2):
            eager = ctx.seed(b.seq, b.lengths)
            torch.cuda.synchronize()
            out = g.seed(b.seq, b.lengths)
            same(out, eager)
    too_long = np.frombuffer(b"ACGT" * 200, dtype=np.uint8)
    with pytest.raises(mbw.MbwError) as e:
        g.seed(too_long, np.array([800], np.uint32))
    assert e.value.code == mbw.MBW_E_INVAL
    g.free()
    ctx.free()


def test_graph_bisulfite_filter_and_refinement():
    """A 200 kbp four-copy bisulfite index, 2,000 directional reads in read-1 form and their read-2
    image with planted C/G changes: for both roles, a graph with the strand filter and the seed
    refinement gives the seeds, kept positions and pieces of mbw_seed (and the oracle's), replayed
    twice on different batches with eager calls in between."""
    ref = synth.reference(0, 200_000, 31)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10, bisulfite=True)
    ox = oracle.OracleIndex(ref.codes, bisulfite=True, sa_rate=8)
    rs = synth.reads_bisulfite(ref, 2000, seed=5)
    seq2 = rs.seq.copy()
    comp = bytes.maketrans(b"ACGT", b"TGCA")
    for r in range(len(rs)):
        a, b = int(rs.offsets[r]), int(rs.offsets[r + 1])
        seq2[a:b] = np.frombuffer(rs.seq[a:b].tobytes().translate(comp)[::-1], np.uint8)
    rng = np.random.default_rng(4)
    for s_ in (rs.seq, seq2):
        hit = rng.integers(0, s_.size, s_.size // 200)
        s_[hit] = np.where(rng.random(hit.size) < 0.5, ord("C"), ord("G"))
    ctx = mbw.Context(idx)
    for role, seq in ((1, rs.seq), (2, seq2)):
        full = synth.ReadSet(seq, rs.lengths, rs.offsets, rs.tpos, rs.tstrand)
        for refine in (False, True):
            g = ctx.graph(len(rs), bs_role=role, bs_refine=refine)
            for b in (full, subset(full, range(0, 2000, 3))):
                for rep in range(2):
                    eager = ctx.seed(b.seq, b.lengths, bs_role=role, bs_refine=refine)
                    e_p = eager.download_pieces() if refine else None
                    torch.cuda.synchronize()
                    out = g.seed(b.seq, b.lengths)
                    s, p = same(out, eager)
                    if refine:
                        got = out.download_pieces()
                        assert got.size == e_p.size > 0
                        for f in got.dtype.names:
                            assert np.array_equal(got[f], e_p[f]), f
                    if b is full and rep == 0 and not refine:
                        compare_with_oracle(s, p, ox.seed(b.seq, b.offsets, bs_role=role))
            g.free()
    ctx.free()
    idx.free()
