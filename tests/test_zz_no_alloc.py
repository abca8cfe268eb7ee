"""The allocation-free entry point (mbw_seed_static) against mbw_seed_into, the entry point whose work
space it replaces with the library's static device array: the same arrays, bit for bit, on two
calls in a row (the second on a smaller batch, over the first one's leftovers in the array), the
same work space size, the oracle's seeds; a batch too large for the array and host inputs are
refused with clear errors."""
import numpy as np
import pytest

import oracle
import synth
from mbw_helpers import compare_with_oracle

mbw = pytest.importorskip("paper_2606_15357_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SCRATCH = 128 << 20


def out_buffers(seeds_cap, pos_cap):
    seeds = torch.empty(max(seeds_cap, 1) * mbw.SEED_DTYPE.itemsize, dtype=torch.uint8, device=DEV)
    pos = torch.empty(max(pos_cap, 1), dtype=torch.int64, device=DEV)
    return seeds, pos


def test_static_entry_matches_seed_into_twice():
    ref = synth.workload_reference("small_1mbp")
    reads = synth.workload_reads("small_1mbp", ref, 6000)
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    ctx = mbw.Context(idx)
    for n in (6000, 1500):
        sub = reads.subset(np.arange(n))
        rd = torch.from_numpy(sub.seq).to(DEV)
        ld = torch.from_numpy(sub.lengths.view(np.int32)).to(DEV)
        ws = torch.empty(512 << 20, dtype=torch.uint8, device=DEV)
        s_in, p_in = out_buffers(20 * n, 200 * n)
        out_i, b_i = ctx.seed_into(rd, ld, ws, s_in, p_in)
        si, pi = out_i.download()
        s_st, p_st = out_buffers(si.size, pi.size)
        out_s, b_s = ctx.seed_static(rd, ld, s_st, p_st)
        ss, ps = out_s.download()
        assert out_s.seeds_ptr == s_st.data_ptr() and out_s.pos_ptr == p_st.data_ptr()
        assert ss.size == si.size and ps.size == pi.size
        for f in ss.dtype.names:
            if f != "reserved":
                assert np.array_equal(ss[f], si[f]), f
        assert np.array_equal(ps, pi)
        assert b_s.workspace_needed == b_i.workspace_needed <= SCRATCH
        assert (b_s.seeds_needed, b_s.pos_needed) == (si.size, pi.size)
        compare_with_oracle(ss, ps, ox.seed(sub.seq, sub.offsets, min_len=19, max_occ=500))
    ctx.free()
    idx.free()


def test_static_entry_refusals():
    ref = synth.workload_reference("small_1mbp")
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    ctx = mbw.Context(idx)
    big = synth.workload_reads("small_1mbp", ref, 200_000)
    rd = torch.from_numpy(big.seq).to(DEV)
    ld = torch.from_numpy(big.lengths.view(np.int32)).to(DEV)
    s, p = out_buffers(16, 16)
    with pytest.raises(mbw.MbwError) as e:
        ctx.seed_static(rd, ld, s, p)
    assert e.value.code == mbw.MBW_E_CAPACITY and "allocation-free" in str(e.value)
    assert e.value.buffers.workspace_needed > SCRATCH
    small = big.subset(np.arange(10))
    with pytest.raises(mbw.MbwError) as e:
        ctx.seed_static(small.seq, small.lengths, s, p)    # host arrays
    assert e.value.code == mbw.MBW_E_INVAL and "device memory" in str(e.value)
    # the context still seeds normally afterwards
    out = ctx.seed(small.seq, small.lengths)
    assert out.n_seeds > 0
    ctx.free()
    idx.free()
