"""GPU parity of chaining (Section 2.6) against the chaining oracle, through the C-ABI.

The oracle chains the oracle's own seeds (O1, or O3 at full size: no input comes from the GPU);
the GPU chains the seeds it found itself.  Both results must be identical: the same chains per
read in the same rank order (score, anchor count, copy) and the same anchors (seed interval and
text position) in the same order.
"""
import numpy as np
import pytest

import oracle
import synth
from mbw_helpers import compare_with_oracle

mbw = pytest.importorskip("paper_2606_15357_amd")

pytestmark = pytest.mark.gpu


def compare_chains(gpu, exp):
    gc, ga = gpu
    ec, ea = exp
    assert gc.size == ec.size, (gc.size, ec.size)
    for f in ("read_id", "score", "n_anchors", "copy"):
        if not np.array_equal(gc[f].astype(np.int64), ec[f].astype(np.int64)):
            bad = np.nonzero(gc[f].astype(np.int64) != ec[f].astype(np.int64))[0][:5]
            raise AssertionError(f"chain field {f} differs at {bad}: gpu {gc[f][bad]} oracle {ec[f][bad]} "
                                 f"(reads {gc['read_id'][bad]})")
    assert ga.size == ea.size
    # anchors chain by chain (both are laid out chain after chain)
    assert np.array_equal(gc["anchor_off"], ec["anchor_off"])
    for f in ("qbeg", "qend", "pos"):
        assert np.array_equal(ga[f].astype(np.uint64), ea[f].astype(np.uint64)), f


@pytest.fixture(scope="module")
def small():
    ref = synth.workload_reference("small_1mbp")
    reads = synth.workload_reads("small_1mbp", ref)
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    yield ref, reads, ox, idx
    idx.free()


@pytest.mark.parametrize("G,h,maxc,minsc", [(5000, 50, 50, 19), (200, 5, 3, 0), (100000, 64, 64, 30), (50, 1, 1, 19),
                                            (5000, 50, 50, 0)])
def test_chain_small_workload(small, G, h, maxc, minsc):
    """10,000 reads of the 1 Mbp workload (repeat family copies included)."""
    ref, reads, ox, idx = small
    exp_seeds = ox.seed(reads.seq, reads.offsets, min_len=19, max_occ=500)
    exp = oracle.chain(exp_seeds, seg_len=len(ref), max_gap=G, max_pred=h, max_chains=maxc, min_score=minsc)
    ctx = mbw.Context(idx)
    out = ctx.seed(reads.seq, reads.lengths, min_seed_len=19, max_occ=500)
    seeds, pos = out.download()
    compare_with_oracle(seeds, pos, exp_seeds)
    ch = ctx.chain(out, len(reads), max_gap=G, max_pred=h, max_chains=maxc, min_score=minsc)
    assert ch.n_input_anchors == pos.size
    compare_chains(ch.download(), exp)
    ctx.free()


def repeat_reference(seed=17):
    """200 kbp of random sequence with 150 copies of one 300 bp unit at 1% divergence inserted."""
    rng = np.random.default_rng(seed)
    unit = rng.integers(0, 4, 300, dtype=np.uint8)
    parts, start = [], 0
    cuts = np.sort(rng.choice(200_000, 150, replace=False))
    bg = rng.integers(0, 4, 200_000, dtype=np.uint8)
    for c in cuts:
        parts.append(bg[start:c])
        cp = unit.copy()
        m = rng.random(300) < 0.01
        cp[m] = (cp[m] + rng.integers(1, 4, int(m.sum()), dtype=np.uint8)) % 4
        parts.append(cp)
        start = c
    parts.append(bg[start:])
    return synth.Reference(np.concatenate(parts), np.zeros((0, 2), np.uint64), -1, seed)


def test_chain_many_anchors_per_read():
    """A reference with 150 copies of a 300 bp unit, reads of 150-1000 bp with max_occ 5000: reads
    over copies have hundreds of anchors (more than the 64 lanes of a wave and more than h), with
    many equal scores among the chains."""
    ref = repeat_reference()
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    rep = synth.reads_uniform_len(ref, 600, 150, 1000, p_sub=0.002, p_indel=0.0002, seed=91)
    exp_seeds = ox.seed(rep.seq, rep.offsets, min_len=19, max_occ=5000)
    counts = np.bincount(exp_seeds.read_id, weights=exp_seeds.npos, minlength=len(rep))
    assert counts.max() > 200 and np.sum(counts > 64) > 20
    ctx = mbw.Context(idx)
    out = ctx.seed(rep.seq, rep.lengths, min_seed_len=19, max_occ=5000)
    for G, h, maxc, minsc in ((5000, 50, 50, 19), (300, 10, 64, 0), (5000, 64, 1, 19)):
        exp = oracle.chain(exp_seeds, seg_len=len(ref), max_gap=G, max_pred=h, max_chains=maxc, min_score=minsc)
        ch = ctx.chain(out, len(rep), max_gap=G, max_pred=h, max_chains=maxc, min_score=minsc)
        compare_chains(ch.download(), exp)
    ctx.free()
    idx.free()


def test_chain_bisulfite():
    """Four-copy bisulfite index, read 1: chains never mix copies and equal the oracle's."""
    ref = synth.reference(0, 200_000, 31)
    ox = oracle.OracleIndex(ref.codes, bisulfite=True, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10, bisulfite=True)
    rs = synth.reads_bisulfite(ref, 2000, seed=5)
    exp_seeds = ox.seed(rs.seq, rs.offsets, bs_role=1)
    exp = oracle.chain(exp_seeds, seg_len=len(ref))
    ctx = mbw.Context(idx)
    out = ctx.seed(rs.seq, rs.lengths, bs_role=1)
    ch = ctx.chain(out, len(rs))
    gc, ga = ch.download()
    compare_chains((gc, ga), exp)
    assert set(np.unique(gc["copy"])) <= {0, 2}
    ctx.free()
    idx.free()


def test_chain_edges_and_errors(small):
    """An empty batch, reads without seeds between others, one anchor; bad options and a read count
    below the seeds' read ids are refused."""
    ref, reads, ox, idx = small
    ctx = mbw.Context(idx)
    out = ctx.seed(np.zeros(0, np.uint8), np.zeros(0, np.uint32))
    ch = ctx.chain(out, 0)
    assert ch.n_chains == 0 and ch.n_anchors == 0
    R = "".join("ACGT"[int(x)] for x in ref.codes[:3000])
    rl = ["", "ACGTTGCA", R[100:250], "N" * 50, R[1000:1019], R[2000:2100]]
    seq = np.frombuffer("".join(rl).encode(), np.uint8).copy()
    lens = np.array([len(x) for x in rl], np.uint32)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    exp_seeds = ox.seed(seq, offs, min_len=19, max_occ=500)
    exp = oracle.chain(exp_seeds, seg_len=len(ref))
    out = ctx.seed(seq, lens, min_seed_len=19, max_occ=500)
    compare_chains(ctx.chain(out, len(rl)).download(), exp)
    assert set(exp[0]["read_id"]) == {2, 4, 5}
    with pytest.raises(mbw.MbwError) as e:
        ctx.chain(out, 3)
    assert e.value.code == mbw.MBW_E_INVAL
    for bad in (dict(max_pred=0), dict(max_pred=65), dict(max_chains=0), dict(max_chains=65), dict(max_gap=0)):
        with pytest.raises(mbw.MbwError):
            ctx.chain(out, len(rl), **bad)
    ctx.free()
