"""Schedule invariance: every launch schedule, batch split and read order gives the same seeds.

The SMEM set, each interval and each position set are fixed by the reads and the index, so the
result must not depend on how the work is scheduled.  On ragged reads (20-700 bases, N runs) over
the 1 Mbp genome, bit-exact in canonical order:
  * length binning on / off x persistent blocks per CU (sized by the work, occupancy limit, 2,
    1) x segment length (32, default) x unique-match path on / off, against the oracle; the unique
    matches of staged reads finished in alternating continuation passes, under several grids and
    work chunks;
  * the same call twice (determinism, byte for byte);
  * the batch split at arbitrary points (read ids offset), against the whole batch;
  * the reads in shuffled order (seeds mapped back through the permutation).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from mbw_helpers import compare_with_oracle

mbw = pytest.importorskip("paper_2606_15357_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    ref = synth.workload_reference("small_1mbp")
    reads = synth.reads_uniform_len(ref, 3000, 20, 700, seed=61)
    seq = reads.seq.copy()
    rng = np.random.default_rng(62)
    for r in range(0, len(reads), 9):
        a, n = int(reads.offsets[r]), int(reads.lengths[r])
        if n > 60:
            seq[a + 30:a + 30 + int(rng.integers(1, 8))] = ord("N")
    reads = synth.ReadSet(seq, reads.lengths, reads.offsets, reads.tpos, reads.tstrand)
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    exp = ox.seed(reads.seq, reads.offsets, min_len=19, max_occ=500)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    yield reads, exp, idx
    idx.free()


def canon(out):
    s, p = out.download()
    a, f = mbw.canonical(s, p)
    return a, f


def test_every_schedule_matches_the_oracle(setup):
    reads, exp, idx = setup
    ctx = mbw.Context(idx)
    for stage, bpc, seg, uniq in itertools.product((True, False), (0, -1, 2, 1), (32, 0), (True, False)):
        out = ctx.seed(reads.seq, reads.lengths, stage=stage, blocks_per_cu=bpc, seg_len=seg, unique_ext=uniq)
        s, p = out.download()
        compare_with_oracle(s, p, exp)
    for bpc in (4, 8):   # locate's automatic cap, and its occupancy limit (the SMEM kernel stops at 4)
        out = ctx.seed(reads.seq, reads.lengths, blocks_per_cu=bpc)
        s, p = out.download()
        compare_with_oracle(s, p, exp)
    for chunk in (1, 7, 64, 256):
        out = ctx.seed(reads.seq, reads.lengths, wave_chunk=chunk)
        s, p = out.download()
        compare_with_oracle(s, p, exp)
    for bpc, chunk, seg in itertools.product((0, -1, 1), (0, 1, 64), (32, 0)):
        out = ctx.seed(reads.seq, reads.lengths, unique_defer=1, blocks_per_cu=bpc, wave_chunk=chunk, seg_len=seg)
        s, p = out.download()
        compare_with_oracle(s, p, exp)
    for bad in (-1, 2):
        with pytest.raises(mbw.MbwError):
            ctx.seed(reads.seq, reads.lengths, unique_defer=bad)
    with pytest.raises(mbw.MbwError):
        ctx.seed(reads.seq, reads.lengths, wave_chunk=257)
    ctx.free()


def test_deterministic_bytes(setup):
    reads, exp, idx = setup
    ctx = mbw.Context(idx)
    a1, f1 = canon(ctx.seed(reads.seq, reads.lengths))
    a2, f2 = canon(ctx.seed(reads.seq, reads.lengths))
    assert a1.tobytes() == a2.tobytes() and f1.tobytes() == f2.tobytes()
    ctx.free()


def test_batch_split_points(setup):
    reads, exp, idx = setup
    ctx = mbw.Context(idx)
    whole, wpos = canon(ctx.seed(reads.seq, reads.lengths))
    parts, pparts = [], []
    cuts = [0, 1, 777, 778, 2000, len(reads)]
    for a, b in zip(cuts[:-1], cuts[1:]):
        sub = reads.subset(np.arange(a, b))
        s, p = canon(ctx.seed(sub.seq, sub.lengths))
        s = s.copy()
        s["read_id"] += a
        parts.append(s)
        pparts.append(p)
    joined = np.concatenate(parts)
    for f in ("read_id", "qbeg", "qend", "k", "kr", "s", "npos"):
        assert np.array_equal(joined[f], whole[f]), f
    assert np.array_equal(np.concatenate(pparts), wpos)
    ctx.free()


def test_read_order_shuffle(setup):
    reads, exp, idx = setup
    perm = np.random.default_rng(63).permutation(len(reads))
    sh = reads.subset(perm)
    ctx = mbw.Context(idx)
    s, p = canon(ctx.seed(sh.seq, sh.lengths))
    s = s.copy()
    s["read_id"] = perm[s["read_id"]].astype(np.uint32)      # back to the original read ids
    off = np.concatenate([[0], np.cumsum(s["npos"].astype(np.int64))])
    order = np.lexsort((s["qend"], s["qbeg"], s["read_id"]))
    flat = np.concatenate([p[off[t]:off[t + 1]] for t in order]) if len(order) else p
    s = s[order]
    for f in ("read_id", "qbeg", "qend", "k", "kr", "s", "npos"):
        assert np.array_equal(s[f].astype(np.uint64), getattr(exp, f).astype(np.uint64)), f
    assert np.array_equal(flat, exp.pos)
    ctx.free()
