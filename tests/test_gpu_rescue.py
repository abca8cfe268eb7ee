"""Mate-rescue prefilter (Section 2.7) through the C-ABI, element by element against the oracle.

Every candidate's (max_t M_t, smallest maximising t) must equal the oracle's exactly, and the pass
list must be exactly the candidates with max_t M_t >= min_hits, ascending.  Cases: the paired
workload's true-mate and decoy windows on a 1 Mbp genome, q = 1 / 7 / 15, thresholds 0 and 10,
ragged reads (0-700 bases, N runs) against ragged windows (0-3000 bases) that start at text
position 0, end at the sentinel or straddle the forward / reverse-complement boundary, more
candidates than the persistent grid holds, candidates already in device memory, the bisulfite
text with both read roles, and the errors (a read id or window out of range, q outside 1..15).
"""
import numpy as np
import pytest

import oracle
import synth

mbw = pytest.importorskip("paper_2606_15357_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    ref = synth.workload_reference("small_1mbp")
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    yield ref, idx
    idx.free()


def as_cands(rid, beg, wl):
    c = np.zeros(len(rid), dtype=mbw.RESCUE_CAND_DTYPE)
    c["read_id"], c["win_beg"], c["win_len"] = rid, beg, wl
    return c


def check(ctx, ref, reads, cands, q=7, min_hits=10, role=0, bisulfite=False, **kw):
    out = ctx.rescue(reads.seq, reads.lengths, cands, q=q, min_hits=min_hits, bs_role=role, **kw)
    hits, passed = out.download()
    mh, bt = oracle.rescue(ref.codes, reads.seq, reads.offsets, cands["read_id"], cands["win_beg"], cands["win_len"],
                           q=q, role=role, bisulfite=bisulfite)
    bad = np.nonzero((hits["max_hits"] != mh) | (hits["best_t"] != bt))[0]
    assert bad.size == 0, (bad[:5], hits[bad[:5]], mh[bad[:5]], bt[bad[:5]], cands[bad[:5]])
    assert np.array_equal(passed, np.flatnonzero(mh >= min_hits).astype(np.uint32))
    assert out.n_pass == passed.size and out.n_cands == len(cands)
    return mh, bt


def ragged(ref, n_text, seed):
    """Reads of 0-700 bases (some with N runs) and windows of 0-3000 bases placed anywhere in the
    text, a third of them around the read's own source."""
    rng = np.random.default_rng(seed)
    reads = synth.reads_uniform_len(ref, 600, 1, 700, seed=seed)
    seq = reads.seq.copy()
    for r in range(0, len(reads), 7):
        a = int(reads.offsets[r])
        n = int(reads.lengths[r])
        if n > 30:
            seq[a + 5:a + 5 + int(rng.integers(1, 20))] = ord("N")
    lens = reads.lengths.copy()
    lens[::50] = 0                                   # empty reads
    lens[1::50] = np.minimum(lens[1::50], 5)         # reads shorter than q
    offs = np.zeros(len(lens) + 1, np.uint64)
    offs[1:] = np.cumsum(lens)
    seq2 = np.concatenate([seq[int(reads.offsets[r]):int(reads.offsets[r]) + int(lens[r])] for r in range(len(lens))])
    reads = synth.ReadSet(seq2, lens.astype(np.uint32), offs, reads.tpos, reads.tstrand)
    nc = 3000
    rid = rng.integers(0, len(reads), nc)
    wl = rng.integers(0, 3001, nc)
    wl[::97] = rng.integers(0, 7, wl[::97].size)     # windows shorter than q
    beg = (rng.random(nc) * (n_text - wl + 1)).astype(np.int64)
    own = np.arange(nc) % 3 == 0
    src = np.where(reads.tstrand[rid] == 0, reads.tpos[rid].astype(np.int64),
                   n_text - reads.tpos[rid].astype(np.int64) - lens[rid].astype(np.int64))
    beg[own] = np.clip(src[own] - rng.integers(0, 1000, own.sum()), 0, n_text - wl[own])
    beg[0], wl[0] = 0, 2000                         # from text position 0
    beg[1], wl[1] = n_text - 2500, 2500             # up to the sentinel
    beg[2], wl[2] = n_text // 2 - 1000, 2000        # across the forward / reverse-complement boundary
    return reads, as_cands(rid, beg, wl)


def test_workload_candidates(small):
    ref, idx = small
    reads = synth.reads_fixed(ref, 4000, 150, True, p_sub=0.005, p_indel=0.0005, seed=31)
    cands, decoy = synth.rescue_candidates(reads, len(ref), decoys=True, seed=32)
    ctx = mbw.Context(idx)
    mh, _ = check(ctx, ref, reads, cands)
    assert np.mean(mh[decoy == 0] >= 10) > 0.98 and np.mean(mh[decoy == 1] >= 10) < 0.05
    ctx.free()


@pytest.mark.parametrize("q,min_hits", [(7, 10), (1, 0), (15, 3), (4, 25)])
def test_ragged_reads_and_windows(small, q, min_hits):
    ref, idx = small
    n_text = 2 * len(ref)
    reads, cands = ragged(ref, n_text, seed=40 + q)
    ctx = mbw.Context(idx)
    check(ctx, ref, reads, cands, q=q, min_hits=min_hits)
    ctx.free()


def test_device_inputs_and_many_candidates(small):
    ref, idx = small
    reads = synth.reads_fixed(ref, 30000, 150, True, p_sub=0.005, p_indel=0.0005, seed=33)
    cands, _ = synth.rescue_candidates(reads, len(ref), decoys=True, seed=34)   # 60,000 > the grid
    dev = torch.device("cuda:0")
    dseq = torch.from_numpy(reads.seq).to(dev)
    dlen = torch.from_numpy(reads.lengths.view(np.int32)).to(dev)
    dc = torch.from_numpy(cands.view(np.uint8)).to(dev)
    ctx = mbw.Context(idx)
    out = ctx.rescue(dseq, dlen, dc, stream=torch.cuda.current_stream())
    hits, passed = out.download()
    sub = np.random.default_rng(35).choice(len(cands), 3000, replace=False)
    mh, bt = oracle.rescue(ref.codes, reads.seq, reads.offsets, cands["read_id"][sub], cands["win_beg"][sub],
                           cands["win_len"][sub], q=7)
    assert np.array_equal(hits["max_hits"][sub], mh) and np.array_equal(hits["best_t"][sub], bt)
    assert np.array_equal(passed, np.flatnonzero(hits["max_hits"] >= 10).astype(np.uint32))
    ctx.free()


def test_seeding_result_survives_rescue(small):
    ref, idx = small
    reads = synth.reads_fixed(ref, 500, 150, True, p_sub=0.005, p_indel=0.0005, seed=36)
    ctx = mbw.Context(idx)
    s_out = ctx.seed(reads.seq, reads.lengths)
    s1, p1 = s_out.download()
    cands, _ = synth.rescue_candidates(reads, len(ref), decoys=True, seed=37)
    check(ctx, ref, reads, cands)
    s2, p2 = s_out.download()
    assert s1.tobytes() == s2.tobytes() and p1.tobytes() == p2.tobytes()
    ctx.free()


@pytest.mark.parametrize("role", [1, 2])
def test_bisulfite_text(role):
    ref = synth.random_reference(200_000, seed=77)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10, bisulfite=True)
    reads = synth.reads_bisulfite(ref, 1500, 150, seed=78)
    n_text = 4 * len(ref)
    rng = np.random.default_rng(79)
    rid = np.arange(len(reads))
    wl = rng.integers(100, 900, len(reads))
    beg = (rng.random(len(reads)) * (n_text - wl + 1)).astype(np.int64)
    # half the windows around the read's source: a forward read in the C->T copy at its start, a
    # reverse one in the reverse G->A copy at 3|R| - start - length
    L, st = len(ref), reads.tpos.astype(np.int64)
    src = np.where(reads.tstrand == 0, st, 3 * L - st - reads.lengths.astype(np.int64) - 32)
    own = rid % 2 == 0
    wl[own] = 900
    beg[own] = np.clip(src[own] - 400, 0, n_text - 900)
    cands = as_cands(rid, beg, wl)
    ctx = mbw.Context(idx)
    mh, _ = check(ctx, ref, reads, cands, role=role, bisulfite=True)
    if role == 1:
        assert np.mean(mh[own] >= 10) > 0.9
    ctx.free()
    idx.free()


def test_errors(small):
    ref, idx = small
    reads = synth.reads_fixed(ref, 10, 150, False, seed=38)
    ctx = mbw.Context(idx)
    n_text = 2 * len(ref)
    for c in (as_cands([10], [0], [100]), as_cands([0], [n_text - 99], [100]), as_cands([0], [n_text + 1], [0])):
        with pytest.raises(mbw.MbwError) as e:
            ctx.rescue(reads.seq, reads.lengths, c)
        assert e.value.code == mbw.MBW_E_INVAL
    for q in (0, 16):
        with pytest.raises(mbw.MbwError):
            ctx.rescue(reads.seq, reads.lengths, as_cands([0], [0], [100]), q=q)
    out = ctx.rescue(reads.seq, reads.lengths, as_cands([], [], []))
    assert out.n_cands == 0 and out.n_pass == 0
    # the context still works after the errors
    check(ctx, ref, reads, as_cands([0, 1], [0, n_text - 400], [400, 400]))
    ctx.free()
