"""Parity at full workload sizes, in the launch configuration the benchmark times.

The GPU seeds the whole batch (reads resident in device memory, one ``mbw_seed`` call); the
oracle recomputes a seeded sample of the reads one by one and every seed, occurrence count and
position of the sampled reads must agree exactly:

* 100 Mbp mixed genome, 1,000,000 read pairs of 150 bp: oracle O1 (full suffix array,
  definitions) on 20,000 sampled reads, all fields including the ds-interval bounds; the whole
  results of the wave kernels (with and without length binning) and the plain kernel are
  identical array for array;
* the same genome, 500,000 reads of 100-5000 bp (lognormal, median 300): O1 on 3,000 reads; wave
  and plain kernels identical over the whole batch;
* 3.1 Gbp mixed genome, 10,000,000 read pairs: the wave and plain kernels identical over the
  whole batch; oracle O3 (one scan of T per q-mer set, no index) on 100 uniformly drawn reads
  plus 20 reads from satellite arrays; the bounds k' of the sampled seeds are checked through the
  strand mirror (seeding revcomp(P) gives (k', k, s) and the mirrored positions).  The whole batch
  is chained (Section 2.6) and the chains of the sampled reads equal the chaining oracle's on the
  scan oracle's seeds.  The mate-rescue prefilter runs over 20,000,000 candidates of the same
  batch; 1,200 sampled candidates must match the oracle exactly.  The resident line table of the
  index passes a CPU check from its definitions (check_line_table);
* the same genome's four-copy bisulfite index: the line table check, wave and plain kernels
  identical for read 1 and read 2 over 1,000,000 reads, and O3 on 60 sampled reads per role
  (with the refined pieces of read 1).
"""
import time

import numpy as np
import pytest

import oracle
import synth
from mbw_helpers import check_line_table, compare_with_oracle

mbw = pytest.importorskip("paper_2606_15357_amd")
torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

COMP = bytes.maketrans(b"ACGTNacgtn", b"TGCANtgcan")


def log(*a):
    print(*a, flush=True)


def device_batch(reads):
    dev = torch.device("cuda:0")
    return torch.from_numpy(reads.seq).to(dev), torch.from_numpy(reads.lengths.view(np.int32)).to(dev)


def gpu_seed_batch(ctx, reads, **kw):
    dseq, dlen = device_batch(reads)
    out = ctx.seed(dseq, dlen, stream=torch.cuda.current_stream(), **kw)
    torch.cuda.synchronize()
    seeds, pos = out.download()
    del dseq, dlen
    return out, seeds, pos


def sample_of(seeds, pos, ids):
    """The seeds of reads `ids` (sorted), renumbered 0..len(ids)-1, with their own position array."""
    m = np.isin(seeds["read_id"], ids)
    sel = seeds[m].copy()
    sel["read_id"] = np.searchsorted(ids, sel["read_id"]).astype(np.uint32)
    chunks, off = [], 0
    for t in range(sel.size):
        o, c = int(sel["pos_off"][t]), int(sel["npos"][t])
        chunks.append(pos[o:o + c])
        sel["pos_off"][t] = off
        off += c
    p = np.concatenate(chunks) if chunks else np.zeros(0, np.uint64)
    return sel, p


def chains_of(chains, anchors, ids):
    """The chains of reads `ids` (sorted), renumbered 0..len(ids)-1, with their own anchor array."""
    m = np.isin(chains["read_id"], ids)
    sel = chains[m].copy()
    sel["read_id"] = np.searchsorted(ids, sel["read_id"]).astype(np.uint32)
    parts, off = [], 0
    for t in range(sel.size):
        o, c = int(sel["anchor_off"][t]), int(sel["n_anchors"][t])
        parts.append(anchors[o:o + c])
        sel["anchor_off"][t] = off
        off += c
    a = np.concatenate(parts) if parts else anchors[:0]
    return sel, a


def same_arrays(seeds, pos, seeds0, pos0):
    """Two whole results are identical (every field of every seed, every position)."""
    if len(seeds) != len(seeds0) or len(pos) != len(pos0):
        log(f"sizes differ: {len(seeds)} / {len(seeds0)} seeds, {len(pos)} / {len(pos0)} positions")
        return False
    for f in seeds.dtype.names:
        if f != "reserved" and not np.array_equal(seeds[f], seeds0[f]):
            bad = np.nonzero(seeds[f] != seeds0[f])[0][:5]
            log(f"field {f} differs at {bad}")
            return False
    return bool(np.array_equal(pos, pos0))


def compare_without_bounds(seeds, pos, exp):
    s, flat = mbw.canonical(seeds, pos)
    assert len(s) == len(exp), (len(s), len(exp))
    for f in ("read_id", "qbeg", "qend", "s", "npos"):
        a, b = s[f].astype(np.uint64), getattr(exp, f).astype(np.uint64)
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0][:5]
            raise AssertionError(f"{f} differs at {bad}: gpu {a[bad]} oracle {b[bad]}")
    assert np.array_equal((s["flags"] & 1).astype(np.uint32), exp.flags & 1)
    assert np.array_equal(flat, exp.pos)
    return s, flat


# ---------------------------------------------------------------------------------------------
# 100 Mbp

@pytest.fixture(scope="module")
def genome100():
    t = time.time()
    ref = synth.workload_reference("paired_100mbp")
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=15)
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    log(f"100 Mbp: GPU index + oracle index in {time.time() - t:.1f} s")
    yield ref, idx, ox
    idx.free()


def test_paired_100mbp_sampled_parity(genome100):
    ref, idx, ox = genome100
    reads = synth.workload_reads("paired_100mbp", ref)
    ids = np.sort(np.random.default_rng(101).choice(len(reads), 20_000, replace=False))
    sub = reads.subset(ids)
    exp = ox.seed(sub.seq, sub.offsets, min_len=19, max_occ=500)
    assert len(exp) > 20_000
    ctx = mbw.Context(idx)
    first = None
    for kernel, stage in ((mbw.KERNEL_COOP, True), (mbw.KERNEL_COOP, False), (mbw.KERNEL_PLAIN, True)):
        out, seeds, pos = gpu_seed_batch(ctx, reads, min_seed_len=19, max_occ=500, kernel=kernel, stage=stage)
        log(f"kernel {kernel} stage {stage}: {out.n_seeds} seeds, {out.n_pos} positions")
        if first is None:
            first = (seeds.copy(), pos.copy())
        else:   # every schedule returns the same arrays: seeds sorted by read, positions in SA-row order
            assert same_arrays(seeds, pos, *first)
        s, p = sample_of(seeds, pos, ids)
        compare_with_oracle(s, p, exp)
    ctx.free()


def test_lognormal_100mbp_sampled_parity(genome100):
    ref, idx, ox = genome100
    reads = synth.workload_reads("lognormal_100mbp", ref)
    assert reads.lengths.max() > 160 and reads.lengths.min() >= 100
    ids = np.sort(np.random.default_rng(102).choice(len(reads), 3_000, replace=False))
    sub = reads.subset(ids)
    exp = ox.seed(sub.seq, sub.offsets, min_len=19, max_occ=500)
    ctx = mbw.Context(idx)
    first = None
    for kernel in (mbw.KERNEL_COOP, mbw.KERNEL_PLAIN):
        out, seeds, pos = gpu_seed_batch(ctx, reads, min_seed_len=19, max_occ=500, kernel=kernel)
        log(f"kernel {kernel}: {out.n_seeds} seeds, {out.n_pos} positions")
        if first is None:
            first = (seeds.copy(), pos.copy())
        else:
            assert same_arrays(seeds, pos, *first)
        s, p = sample_of(seeds, pos, ids)
        compare_with_oracle(s, p, exp)
    ctx.free()


# ---------------------------------------------------------------------------------------------
# 3.1 Gbp

def test_human_3gbp_sampled_parity():
    t0 = time.time()
    ref = synth.workload_reference("human_3gbp")
    log(f"3.1 Gbp reference in {time.time() - t0:.1f} s")
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=15)
    info = idx.info()
    log(f"GPU index in {time.time() - t0:.1f} s, n = {info['n']}")
    assert info["n_superblocks"] == 2
    check_line_table(idx, log)
    reads = synth.workload_reads("human_3gbp", ref)
    ctx = mbw.Context(idx)
    out, seeds, pos = gpu_seed_batch(ctx, reads, min_seed_len=19, max_occ=500)
    log(f"{len(reads)} reads: {out.n_seeds} seeds, {out.n_pos} positions ({time.time() - t0:.1f} s)")
    # chaining of the whole batch (Section 2.6); the sampled reads are compared with the chaining
    # oracle run on the scan oracle's seeds below
    ch = ctx.chain(out, len(reads))
    gchains, ganchors = ch.download()
    log(f"chaining: {ch.n_input_anchors} anchors -> {ch.n_chains} chains ({ch.n_anchors} anchors), kernel "
        f"{ch.ms_kernel:.1f} ms, call {ch.ms_total:.1f} ms ({time.time() - t0:.1f} s)")
    # the plain one-read-per-thread kernel returns the same arrays for the whole batch
    _, seeds_p, pos_p = gpu_seed_batch(ctx, reads, min_seed_len=19, max_occ=500, kernel=mbw.KERNEL_PLAIN)
    assert same_arrays(seeds_p, pos_p, seeds, pos)
    del seeds_p, pos_p
    log(f"plain kernel: same {out.n_seeds} seeds and {out.n_pos} positions ({time.time() - t0:.1f} s)")
    # a captured graph planned for 20,000 reads returns the eager call's arrays on the first 20,000,
    # replayed twice
    sub20 = reads.subset(np.arange(20_000))
    e20 = ctx.seed(sub20.seq, sub20.lengths, min_seed_len=19, max_occ=500)
    es, ep = e20.download()
    g20 = ctx.graph(20_000, min_seed_len=19, max_occ=500)
    for _ in range(2):
        gs, gp = g20.seed(sub20.seq, sub20.lengths).download()
        assert same_arrays(gs, gp, es, ep)
    g20.free()
    del sub20, es, ep, gs, gp
    log(f"captured graph: same arrays on 20,000 reads ({time.time() - t0:.1f} s)")
    # mate-rescue prefilter over the whole batch (a true-mate and a decoy window per pair, device
    # inputs, as the benchmark runs it); the oracle recomputes 1,200 sampled candidates
    cands, decoy = synth.rescue_candidates(reads, len(ref), decoys=True, seed=104)
    dseq, dlen = device_batch(reads)
    dc = torch.from_numpy(cands.view(np.uint8)).to(torch.device("cuda:0"))
    rout = ctx.rescue(dseq, dlen, dc, stream=torch.cuda.current_stream())
    hits, passed = rout.download()
    del dseq, dlen, dc
    assert np.array_equal(passed, np.flatnonzero(hits["max_hits"] >= 10).astype(np.uint32))
    csub = np.sort(np.random.default_rng(105).choice(len(cands), 1200, replace=False))
    rids, inv = np.unique(cands["read_id"][csub], return_inverse=True)
    rsub = reads.subset(rids)
    mh, bt = oracle.rescue(ref.codes, rsub.seq, rsub.offsets, inv.astype(np.uint32), cands["win_beg"][csub],
                           cands["win_len"][csub], q=7)
    assert np.array_equal(hits["max_hits"][csub], mh) and np.array_equal(hits["best_t"][csub], bt)
    assert np.mean(hits["max_hits"][decoy == 0] >= 10) > 0.95 and np.mean(hits["max_hits"][decoy == 1] >= 10) < 0.05
    log(f"rescue prefilter: {len(cands)} candidates, {rout.n_pass} pass, kernel {rout.ms_kernel:.1f} ms "
        f"({time.time() - t0:.1f} s)")
    del cands, decoy, hits, passed
    # 100 uniform reads and 20 whose fragment starts inside a satellite array
    rng = np.random.default_rng(103)
    uni = rng.choice(len(reads), 100, replace=False)
    sats = ref.sats[np.argsort(ref.sats[:, 0])]
    j = np.searchsorted(sats[:, 0], reads.tpos, side="right") - 1
    in_sat = np.nonzero((j >= 0) & (reads.tpos < sats[np.maximum(j, 0), 1]))[0]
    sat = rng.choice(in_sat, 20, replace=False)
    ids = np.unique(np.concatenate([uni, sat]))
    sub = reads.subset(ids)
    del reads
    s_gpu, p_gpu = sample_of(seeds, pos, ids)
    del seeds, pos
    gc, ga = chains_of(gchains, ganchors, ids)
    del gchains, ganchors
    exp = oracle.scan_seed(ref.codes, sub.seq, sub.offsets, min_len=19, max_occ=500)
    log(f"scan oracle: {len(exp)} seeds, {exp.pos.size} positions, {int((exp.flags & 1).sum())} over max_occ "
        f"({time.time() - t0:.1f} s)")
    assert len(exp) > 200 and (exp.flags & 1).sum() > 0
    s, flat = compare_without_bounds(s_gpu, p_gpu, exp)
    ec, ea = oracle.chain(exp, seg_len=len(ref))
    assert gc.size == ec.size and gc.size > 100
    for f in ("read_id", "score", "n_anchors", "copy", "anchor_off"):
        assert np.array_equal(gc[f].astype(np.int64), ec[f].astype(np.int64)), f
    for f in ("qbeg", "qend", "pos"):
        assert np.array_equal(ga[f].astype(np.uint64), ea[f].astype(np.uint64)), f
    log(f"chains of the sample equal the chaining oracle's ({gc.size} chains)")
    # k' through the strand mirror: seeding revcomp(P[i,j)) gives one SMEM (k', k, s) whose positions
    # are 2|R| - p - (j - i)
    loc = np.nonzero((s["npos"] > 0))[0]
    rc = []
    for t in loc:
        r = int(s["read_id"][t])
        a = int(sub.offsets[r]) + int(s["qbeg"][t])
        b = int(sub.offsets[r]) + int(s["qend"][t])
        rc.append(sub.seq[a:b].tobytes().translate(COMP)[::-1])
    lens = np.array([len(x) for x in rc], np.uint32)
    rseq = np.frombuffer(b"".join(rc), np.uint8).copy()
    out2 = ctx.seed(rseq, lens, min_seed_len=19, max_occ=500, reseed=False)
    s2, p2 = out2.download()
    s2, flat2 = mbw.canonical(s2, p2)
    assert len(s2) == len(loc)
    assert np.all(s2["qbeg"] == 0) and np.array_equal(s2["qend"], lens)
    assert np.array_equal(s2["k"], s["kr"][loc]) and np.array_equal(s2["kr"], s["k"][loc])
    assert np.array_equal(s2["s"], s["s"][loc])
    two_r = 2 * len(ref)
    off = np.concatenate([[0], np.cumsum(s["npos"].astype(np.int64))])
    off2 = np.concatenate([[0], np.cumsum(s2["npos"].astype(np.int64))])
    for q, t in enumerate(loc):
        mine = flat[off[t]:off[t + 1]].astype(np.int64)
        mirrored = np.sort(two_r - mine - int(lens[q]))
        assert np.array_equal(mirrored, flat2[off2[q]:off2[q + 1]].astype(np.int64))
    ctx.free()
    idx.free()
    log(f"done in {time.time() - t0:.1f} s")


# ---------------------------------------------------------------------------------------------
# 3.1 Gbp, bisulfite four-copy index

def test_bisulfite_3gbp_sampled_parity():
    """The four-copy bisulfite index of the 3.1 Gbp genome (n = 12.4 G + 1, four superblocks of
    2^23 lines, so superblocks 2 and 3 and the copy-2/3 strand filter are used): the line table
    passes the CPU check; 1,000,000 directional reads are seeded as read 1 (with the seed
    refinement) and, reverse-complemented, as read 2; the wave and plain kernels give the same
    arrays for the whole batch; on 60 sampled reads per role the seeds, occurrence counts and
    positions equal the scan oracle's on the four-copy text, and for read 1 the refined pieces
    equal the refinement oracle's on those seeds."""
    t0 = time.time()
    ref = synth.workload_reference("serve_bs_3gbp")
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=15, bisulfite=True, isa_sample=8)
    info = idx.info()
    log(f"bisulfite index in {time.time() - t0:.1f} s, n = {info['n']}, {info['n_superblocks']} superblocks")
    assert info["n"] == 4 * len(ref) + 1 and info["n_superblocks"] == 4
    check_line_table(idx, log)
    log(f"line table checked ({time.time() - t0:.1f} s)")
    r1 = synth.reads_bisulfite(ref, 1_000_000, seed=synth.READ_SEED + 40)
    # read 2 of a directional library: the reverse complement of a read-1-form read
    seq2 = np.frombuffer(r1.seq.tobytes().translate(COMP)[::-1], np.uint8).copy()
    len2 = r1.lengths[::-1].copy()
    off2 = np.concatenate([[0], np.cumsum(len2, dtype=np.uint64)]).astype(np.uint64)
    r2 = synth.ReadSet(seq2, len2, off2, r1.tpos[::-1].copy(), r1.tstrand[::-1].copy())
    ctx = mbw.Context(idx)
    rng = np.random.default_rng(106)
    for role, reads in ((1, r1), (2, r2)):
        out, seeds, pos = gpu_seed_batch(ctx, reads, min_seed_len=19, max_occ=500, bs_role=role, bs_refine=role == 1)
        pieces = out.download_pieces() if role == 1 else None
        log(f"role {role}: {out.n_seeds} seeds, {out.n_pos} positions, {0 if pieces is None else len(pieces)} pieces "
            f"({time.time() - t0:.1f} s)")
        _, seeds_p, pos_p = gpu_seed_batch(ctx, reads, min_seed_len=19, max_occ=500, bs_role=role,
                                           kernel=mbw.KERNEL_PLAIN)
        assert same_arrays(seeds_p, pos_p, seeds, pos)
        del seeds_p, pos_p
        ids = np.sort(rng.choice(len(reads), 60, replace=False))
        sub = reads.subset(ids)
        s_gpu, p_gpu = sample_of(seeds, pos, ids)
        exp = oracle.scan_seed(ref.codes, sub.seq, sub.offsets, bisulfite=True, bs_role=role, min_len=19, max_occ=500)
        log(f"role {role} scan oracle: {len(exp)} seeds, {exp.pos.size} positions ({time.time() - t0:.1f} s)")
        assert len(exp) > 60 and exp.pos.size > 60
        compare_without_bounds(s_gpu, p_gpu, exp)
        if role == 1:
            m = np.isin(pieces["read_id"], ids)
            got = pieces[m].copy()
            got["read_id"] = np.searchsorted(ids, got["read_id"]).astype(np.uint32)
            got = got[np.lexsort((got["pos"], got["qend"], got["qbeg"], got["read_id"]))]
            want = oracle.bs_refine(ref.codes, sub.seq, sub.offsets, exp, 1, min_len=19)
            assert len(got) == len(want) and len(want) > 0
            for f in ("read_id", "qbeg", "qend", "pos"):
                assert np.array_equal(got[f].astype(np.uint64), want[f].astype(np.uint64)), f
        del seeds, pos, pieces
    ctx.free()
    idx.free()
    log(f"done in {time.time() - t0:.1f} s")
