"""mbw_seed_into: the seeding path with caller-owned device memory (torch tensors) through the C-ABI.

Its result must equal mbw_seed's array for array (and so the oracle's); too small buffers must give
MBW_E_CAPACITY with the sizes needed written back, and growing them to those sizes must converge to
the same result; the context's own result buffers stay untouched.
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


def buffers(ws_bytes, seeds_cap, pos_cap, pieces_cap=0):
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=DEV)
    seeds = torch.empty(max(seeds_cap, 1) * mbw.SEED_DTYPE.itemsize, dtype=torch.uint8, device=DEV)
    pos = torch.empty(max(pos_cap, 1), dtype=torch.int64, device=DEV)
    pieces = torch.empty(max(pieces_cap, 1) * mbw.PIECE_DTYPE.itemsize, dtype=torch.uint8, device=DEV) \
        if pieces_cap else None
    return ws, seeds, pos, pieces


def seed_into_converging(ctx, reads, lengths, start=(1 << 20, 16, 16, 0), **kw):
    """Start from small buffers, grow them to the reported needs until the call succeeds."""
    ws_b, sc, pc, qc = start
    tries = 0
    while True:
        tries += 1
        assert tries <= 8, "capacity retries did not converge"
        ws, seeds, pos, pieces = buffers(ws_b, sc, pc, qc)
        try:
            out, b = ctx.seed_into(reads, lengths, ws, seeds, pos, pieces, **kw)
            return out, b, tries, (ws, seeds, pos, pieces)
        except mbw.MbwError as e:
            assert e.code == mbw.MBW_E_CAPACITY, e
            b = e.buffers
            grew = False
            if b.workspace_needed > ws_b:
                ws_b = int(b.workspace_needed)
                grew = True
            if b.seeds_needed > sc:
                sc = int(b.seeds_needed)
                grew = True
            if b.pos_needed > pc:
                pc = int(b.pos_needed)
                grew = True
            if b.pieces_needed > qc:
                qc = int(b.pieces_needed)
                grew = True
            assert grew, "MBW_E_CAPACITY without a larger size reported"


def same(a_seeds, a_pos, b_seeds, b_pos):
    assert a_seeds.size == b_seeds.size and a_pos.size == b_pos.size
    for f in a_seeds.dtype.names:
        if f != "reserved":
            assert np.array_equal(a_seeds[f], b_seeds[f]), f
    assert np.array_equal(a_pos, b_pos)


@pytest.fixture(scope="module")
def small():
    ref = synth.workload_reference("small_1mbp")
    reads = synth.workload_reads("small_1mbp", ref)
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    exp = ox.seed(reads.seq, reads.offsets, min_len=19, max_occ=500)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    yield ref, reads, exp, idx
    idx.free()


@pytest.mark.parametrize("where", ["host", "device"])
def test_seed_into_equals_seed(small, where):
    ref, reads, exp, idx = small
    ctx = mbw.Context(idx)
    base = ctx.seed(reads.seq, reads.lengths, min_seed_len=19, max_occ=500)
    s0, p0 = base.download()
    if where == "device":
        rd = torch.from_numpy(reads.seq).to(DEV)
        ld = torch.from_numpy(reads.lengths.view(np.int32)).to(DEV)
    else:
        rd, ld = reads.seq, reads.lengths
    ws, seeds, pos, _ = buffers(512 << 20, s0.size + 10, p0.size + 10)
    out, b = ctx.seed_into(rd, ld, ws, seeds, pos, min_seed_len=19, max_occ=500)
    assert (b.seeds_needed, b.pos_needed) == (s0.size, p0.size) and 0 < b.workspace_needed <= (512 << 20)
    assert out.seeds_ptr == seeds.data_ptr() and out.pos_ptr == pos.data_ptr()
    s1, p1 = out.download()
    same(s1, p1, s0, p0)
    compare_with_oracle(s1, p1, exp)
    # the context's own result of the earlier call is untouched
    s2, p2 = base.download()
    same(s2, p2, s0, p0)
    ctx.free()


def test_seed_into_capacity_recovery(small):
    """From a 1 MiB work space and 16-record buffers: MBW_E_CAPACITY with larger needs each time
    (the first one an estimate of the whole call), then after a few enlargements to exactly the
    reported sizes the same result as mbw_seed; a work space of exactly the size used is enough and
    one 4 KiB smaller is not."""
    ref, reads, exp, idx = small
    ctx = mbw.Context(idx)
    s0, p0 = ctx.seed(reads.seq, reads.lengths).download()
    out, b, tries, keep = seed_into_converging(ctx, reads.seq, reads.lengths)
    assert 2 <= tries <= 4
    s1, p1 = out.download()
    same(s1, p1, s0, p0)
    need = int(b.workspace_needed)
    ws, seeds, pos, _ = buffers(need, s1.size, p1.size)
    out2, b2 = ctx.seed_into(reads.seq, reads.lengths, ws, seeds, pos)
    same(*out2.download(), s0, p0)
    with pytest.raises(mbw.MbwError) as e:
        ws, seeds, pos, _ = buffers(need - 4096, s1.size, p1.size)
        ctx.seed_into(reads.seq, reads.lengths, ws, seeds, pos)
    assert e.value.code == mbw.MBW_E_CAPACITY and e.value.buffers.workspace_needed > need - 4096
    ctx.free()


def test_seed_into_ragged_and_plain_kernel(small):
    """Ragged lengths (unstaged bins, segments) and the plain kernel through the caller's buffers."""
    ref, _, _, idx = small
    rs = synth.reads_uniform_len(ref, 2000, 1, 600, seed=77)
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    exp = ox.seed(rs.seq, rs.offsets, min_occ=2, max_occ=20)
    ctx = mbw.Context(idx)
    for kernel, seg in ((mbw.KERNEL_COOP, 64), (mbw.KERNEL_PLAIN, 0)):
        out, b, _, keep = seed_into_converging(ctx, rs.seq, rs.lengths, min_occ=2, max_occ=20, kernel=kernel, seg_len=seg)
        compare_with_oracle(*out.download(), exp)
    ctx.free()


def test_seed_into_bisulfite_pieces():
    """Bisulfite read 1 with refinement: positions after the strand filter and the refined pieces
    land in the caller's buffers and equal mbw_seed's."""
    ref = synth.reference(0, 200_000, 31)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10, bisulfite=True)
    rs = synth.reads_bisulfite(ref, 2000, seed=5)
    ctx = mbw.Context(idx)
    base = ctx.seed(rs.seq, rs.lengths, bs_role=1, bs_refine=True)
    s0, p0 = base.download()
    q0 = base.download_pieces()
    out, b, tries, keep = seed_into_converging(ctx, rs.seq, rs.lengths, bs_role=1, bs_refine=True)
    same(*out.download(), s0, p0)
    assert b.pieces_needed == q0.size
    q1 = out.download_pieces()
    for f in q0.dtype.names:
        assert np.array_equal(q0[f], q1[f]), f
    ctx.free()
    idx.free()
