"""The autotuner and the serving runtime, through the C-ABI.

* mbw_tune picks one of its candidate schedules; seeding with it is bit-exact against the oracle.
* mbw_serve: every request's result equals the oracle's for that request alone, both when it is
  served alone and when it is batched with many others submitted concurrently (tolerance 0);
  batches really merge requests; submissions are refused when the queue is full and when a
  request can never fit a worker's device arena; a batch that runs short of its arena is split and
  retried so that no request fails because of another; requests queued without a host copy and
  results read in place; the device-side split of a batch handles empty and seedless requests.
"""
import threading

import numpy as np
import pytest

import oracle
import synth
from mbw_helpers import compare_with_oracle, gpu_seed

mbw = pytest.importorskip("paper_2606_15357_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    ref = synth.workload_reference("small_1mbp")
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    yield ref, ox, idx
    idx.free()


def _requests(ref, n, seed):
    """n requests of mixed sizes (1..2500 reads) and read lengths (20..700, some with N runs)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        m = int(rng.integers(1, 2500))
        if q % 3 == 0:
            rs = synth.reads_uniform_len(ref, m, 20, 700, seed=seed * 1000 + q)
        else:
            rs = synth.reads_fixed(ref, m, 150, False, p_sub=0.01, p_indel=0.001, seed=seed * 1000 + q)
        seq = rs.seq.copy()
        if q % 5 == 1 and seq.size > 40:
            seq[10:25] = ord("N")
        out.append(synth.ReadSet(seq, rs.lengths, rs.offsets, rs.tpos, rs.tstrand))
    return out


def test_tune_picks_a_valid_schedule(small):
    ref, ox, idx = small
    reads = synth.reads_uniform_len(ref, 4000, 50, 900, seed=12)
    ctx = mbw.Context(idx)
    best = ctx.tune(reads.seq, reads.lengths)
    assert best["seg_len"] in (128, 256, 1024) and best["blocks_per_cu"] in (0, -1, 2) and best["ms"] > 0
    assert best["wave_chunk"] in (0, 16, 64, 256)
    ms = best.pop("ms")
    assert best.pop("cached") is False
    out = ctx.seed(reads.seq, reads.lengths, **best)
    seeds, pos = out.download()
    compare_with_oracle(seeds, pos, ox.seed(reads.seq, reads.offsets))
    ctx.free()
    assert ms < 1e5


def test_tune_cache(small, tmp_path):
    """A stored pick is returned for the same index, parameters and read-length profile without
    timing; another length profile is tuned and stored beside it."""
    ref, ox, idx = small
    short = synth.reads_fixed(ref, 3000, 150, False, seed=13)
    long_ = synth.reads_uniform_len(ref, 2000, 400, 2000, seed=14)
    path = str(tmp_path / "tune.json")
    ctx = mbw.Context(idx)
    a = ctx.tune(short.seq, short.lengths, cache=path)
    b = ctx.tune(short.seq, short.lengths, cache=path)
    assert a["cached"] is False and b["cached"] is True
    assert {k: a[k] for k in a if k != "cached"} == {k: b[k] for k in b if k != "cached"}
    c = ctx.tune(long_.seq, long_.lengths, cache=path)
    assert c["cached"] is False
    import json
    assert len(json.load(open(path))) == 2
    ctx.free()


def test_serve_alone_and_in_a_mix(small):
    ref, ox, idx = small
    reqs = _requests(ref, 40, seed=5)
    exp = [ox.seed(r.seq, r.offsets) for r in reqs]
    srv = mbw.Server(idx, n_workers=2, max_batch_reads=6000)
    # request 7 alone
    t = srv.submit(reqs[7].seq, reqs[7].lengths)
    s_alone, p_alone, info_alone = srv.wait(t)
    compare_with_oracle(s_alone, p_alone, exp[7])
    # all requests from two threads at once
    tickets = [None] * len(reqs)

    def submit(lo):
        for q in range(lo, len(reqs), 2):
            while True:
                tk = srv.submit(reqs[q].seq, reqs[q].lengths)
                if tk is not None:
                    tickets[q] = tk
                    break

    th = [threading.Thread(target=submit, args=(lo,)) for lo in (0, 1)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    merged = 0
    for q in range(len(reqs)):
        s, p, info = srv.wait(tickets[q])
        compare_with_oracle(s, p, exp[q])
        merged += info["batch_reads"] > len(reqs[q])
        if q == 7:
            a, fa = mbw.canonical(s, p)
            b, fb = mbw.canonical(s_alone, p_alone)
            assert a.tobytes() == b.tobytes() and fa.tobytes() == fb.tobytes()
        assert info["t_submit"] <= info["t_start"] <= info["t_done"]
    st = srv.stats()
    assert merged > 0 and st["batches"] < len(reqs) + 1
    srv.close()


def test_serve_admission_by_queued_bases(small):
    ref, ox, idx = small
    reqs = _requests(ref, 12, seed=9)
    srv = mbw.Server(idx, n_workers=1, max_batch_reads=3000, max_batch_bases=2_000_000, max_queued_bases=2000)
    accepted, refused = [], 0
    for q, r in enumerate(reqs):
        t = srv.submit(r.seq, r.lengths)
        if t is None:
            refused += 1
        else:
            accepted.append((q, t))
    assert refused > 0 and accepted
    for q, t in accepted:
        s, p, _ = srv.wait(t)
        compare_with_oracle(s, p, ox.seed(reqs[q].seq, reqs[q].offsets))
    srv.close()


def test_serve_empty_request_and_close_with_queue(small):
    ref, ox, idx = small
    srv = mbw.Server(idx, n_workers=1)
    t0 = srv.submit(np.zeros(0, np.uint8), np.zeros(0, np.uint32))
    reqs = _requests(ref, 3, seed=3)
    ts = [srv.submit(r.seq, r.lengths) for r in reqs]
    s, p, _ = srv.wait(t0)
    assert len(s) == 0 and len(p) == 0
    for q, t in enumerate(ts):
        s, p, _ = srv.wait(t)
        compare_with_oracle(s, p, ox.seed(reqs[q].seq, reqs[q].offsets))
    srv.close()


def test_serve_bisulfite_refined_pieces():
    """A bisulfite server (read 1, strand filter, refinement): every request's seeds, positions and
    refined pieces equal the oracle's for that request alone, with piece read ids and seed indexes
    counted within the request, also when requests share a device batch."""
    ref = synth.reference(0, 200_000, 31)
    ox = oracle.OracleIndex(ref.codes, bisulfite=True, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10, bisulfite=True)
    rs = synth.reads_bisulfite(ref, 1500, seed=6)
    seq = rs.seq.copy()
    rng = np.random.default_rng(7)
    hit = rng.integers(0, seq.size, seq.size // 200)            # a few planted C changes
    seq[hit] = ord("C")
    cuts = np.unique(np.concatenate([[0, len(rs)], rng.integers(1, len(rs), 24)]))
    reqs = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        o0, o1 = int(rs.offsets[a]), int(rs.offsets[b])
        offs = (rs.offsets[a:b + 1] - rs.offsets[a]).astype(np.uint64)
        reqs.append((seq[o0:o1].copy(), rs.lengths[a:b].copy(), offs))
    srv = mbw.Server(idx, n_workers=2, max_batch_reads=1500, bs_role=1, bs_refine=True)
    tickets = [srv.submit(s, l) for s, l, _ in reqs]
    merged = 0
    for (s, l, offs), t in zip(reqs, tickets):
        seeds, pos, info = srv.wait(t)
        exp = ox.seed(s, offs, bs_role=1)
        compare_with_oracle(seeds, pos, exp)
        pieces = info["pieces"]
        want = oracle.bs_refine(ref.codes, s, offs, exp, 1, min_len=19)
        got = pieces[np.lexsort((pieces["pos"], pieces["qend"], pieces["qbeg"], pieces["read_id"]))]
        assert len(got) == len(want)
        for f in ("read_id", "qbeg", "qend", "pos"):
            assert np.array_equal(got[f], want[f]), f
        assert np.all(pieces["seed"] < len(seeds))
        assert np.all(seeds["read_id"][pieces["seed"]] == pieces["read_id"])
        assert np.all((seeds["qbeg"][pieces["seed"]] <= pieces["qbeg"]) & (pieces["qend"] <= seeds["qend"][pieces["seed"]]))
        merged += info["batch_reads"] > len(l)
    assert merged > 0
    srv.close()
    idx.free()


def test_serve_many_tiny_requests_share_a_batch(small):
    """The per-request split of a batch (done on the device) at its edges: empty requests, requests
    whose reads are all shorter than the minimum seed length (no seeds), and one- to three-read
    requests, all queued behind a large request so that they are seeded as one batch."""
    ref, ox, idx = small
    big = synth.reads_fixed(ref, 3000, 150, False, p_sub=0.01, p_indel=0.001, seed=12)
    tiny = []
    for q in range(60):
        kind = q % 5
        if kind == 0:
            tiny.append((np.zeros(0, np.uint8), np.zeros(0, np.uint32)))
            continue
        m = 1 + q % 3
        lo, hi = (8, 18) if kind == 1 else (19, 300)
        rs = synth.reads_uniform_len(ref, m, lo, hi, seed=2000 + q)
        tiny.append((rs.seq.copy(), rs.lengths.copy()))
    srv = mbw.Server(idx, n_workers=1, max_batch_reads=100_000)
    tb = srv.submit(big.seq, big.lengths)
    ts = [srv.submit(s, l) for s, l in tiny]
    s, p, _ = srv.wait(tb)
    compare_with_oracle(s, p, ox.seed(big.seq, big.offsets))
    shared = 0
    for (seq, lens), t in zip(tiny, ts):
        s, p, info = srv.wait(t)
        offs = np.concatenate([[0], np.cumsum(lens.astype(np.uint64))]).astype(np.uint64)
        if len(lens) == 0:
            assert len(s) == 0 and len(p) == 0
        else:
            compare_with_oracle(s, p, ox.seed(seq, offs))
            if lens.max() < 19:
                assert len(s) == 0
        shared += info["batch_reads"] > len(lens)
    assert shared >= 40
    srv.close()


def _slice(rs, a, b):
    """Reads [a, b) of a ReadSet as (seq, lengths, offsets from 0)."""
    o0, o1 = int(rs.offsets[a]), int(rs.offsets[b])
    return (rs.seq[o0:o1].copy(), rs.lengths[a:b].copy(),
            (rs.offsets[a:b + 1] - rs.offsets[a]).astype(np.uint64))


def _repeat_reference(copies=300, unit=400, div=0.01, seed=41):
    """10 kbp of random sequence, then `copies` copies of one `unit`-base repeat, each with `div`
    substitutions: reads from it have seeds with hundreds of positions."""
    rng = np.random.default_rng(seed)
    u = rng.integers(0, 4, unit).astype(np.uint8)
    parts = [rng.integers(0, 4, 10_000).astype(np.uint8)]
    for _ in range(copies):
        c = u.copy()
        m = rng.random(unit) < div
        c[m] = (c[m] + rng.integers(1, 4, int(m.sum()))) % 4
        parts.append(c.astype(np.uint8))
    return synth.Reference(np.concatenate(parts), np.zeros((0, 2), np.uint64), 0, seed)


def test_serve_split_on_shortfall():
    """A batch that runs short of its worker's arena (far more positions per read than the sizing
    model assumes) is split and its halves run again: two requests that fit alone but not together,
    and a small one queued with them, all equal the oracle's results alone; a request that cannot
    fit even alone fails with MBW_E_CAPACITY while the small request batched with it succeeds."""
    ref = _repeat_reference()
    ox = oracle.OracleIndex(ref.codes, sa_rate=8)
    idx = mbw.Index.build(ref.codes, sa_sample=8, kmer_k=10)
    pool = synth.reads_fixed(ref, 10000, 150, False, p_sub=0.003, p_indel=0.0, seed=42)
    full = ox.seed(pool.seq, pool.offsets)
    per_read = np.bincount(full.read_id, weights=full.npos, minlength=len(pool)).astype(np.int64)
    cum = np.concatenate([[0], np.cumsum(per_read)])
    srv = mbw.Server(idx, n_workers=1, max_batch_reads=4000, max_batch_bases=600_000)
    P = srv.stats()["pos_cap"]
    assert P > 0 and cum[-1] > 3.3 * P, (P, cum[-1])

    def upto(a, target):   # the first b > a with positions of reads [a, b) >= target
        return int(np.searchsorted(cum, cum[a] + target)) + 1

    cuts = [0]
    for _ in range(3):                 # three requests of 0.6 P positions: no two fit together
        cuts.append(upto(cuts[-1], 0.6 * P))
    reqs = [_slice(pool, a, b) for a, b in zip(cuts[:-1], cuts[1:])] + [_slice(pool, cuts[-1], cuts[-1] + 5)]
    a3 = cuts[-1] + 5
    a4 = upto(a3, 1.3 * P)
    assert a4 + 5 <= len(pool)
    big, small = _slice(pool, a3, a4), _slice(pool, a4, a4 + 5)
    # submitted at once to one worker: while the first runs, the others queue and are batched
    ts = [srv.submit(s, l) for s, l, _ in reqs]
    for (s, l, offs), t in zip(reqs, ts):
        seeds, pos, info = srv.wait(t)
        compare_with_oracle(seeds, pos, ox.seed(s, offs))
    st = srv.stats()
    assert st["split_retries"] >= 1 and st["failed_requests"] == 0
    tb, tsm = srv.submit(big[0], big[1]), srv.submit(small[0], small[1])
    with pytest.raises(mbw.MbwError) as e:
        srv.wait(tb)
    assert e.value.code == mbw.MBW_E_CAPACITY
    seeds, pos, info = srv.wait(tsm)
    compare_with_oracle(seeds, pos, ox.seed(small[0], small[2]))
    assert srv.stats()["failed_requests"] == 1
    srv.close()
    idx.free()


def test_serve_admission_by_device_memory(small):
    """A device budget below what one read needs is refused at open (the message names the least
    size); with arenas of that least size, a request within the read and base budget whose
    estimated work space exceeds the arena is refused at submission with MBW_E_CAPACITY, and the
    server goes on serving the requests that fit; the stats report the arenas."""
    import re
    ref, ox, idx = small
    with pytest.raises(mbw.MbwError) as e:
        mbw.Server(idx, n_workers=2, max_batch_reads=20000, max_batch_bases=3_000_000, device_bytes=1 << 20)
    assert e.value.code == mbw.MBW_E_INVAL
    least = int(re.search(r"at least (\d+) bytes", str(e.value)).group(1))
    srv = mbw.Server(idx, n_workers=2, max_batch_reads=20000, max_batch_bases=3_000_000, device_bytes=2 * least)
    st = srv.stats()
    assert st["device_bytes"] >= 2 * st["workspace_bytes"] > 0 and st["pos_cap"] > 0 and st["seeds_cap"] > 0
    over = synth.reads_fixed(ref, 2000, 150, False, seed=81)
    with pytest.raises(mbw.MbwError) as e:
        srv.submit(over.seq, over.lengths)
    assert e.value.code == mbw.MBW_E_CAPACITY and "work space" in str(e.value)
    oks = [synth.reads_fixed(ref, 20, 150, False, seed=82 + q) for q in range(6)]
    ts = [srv.submit(ok.seq, ok.lengths) for ok in oks]
    for ok, t in zip(oks, ts):
        s, p, info = srv.wait(t)
        compare_with_oracle(s, p, ox.seed(ok.seq, ok.offsets))
    assert srv.stats()["failed_requests"] == 0
    srv.close()


def test_serve_by_reference_and_views(small):
    """Requests queued without a host copy and results read in place (no copy) equal the oracle's;
    the views stay valid until release, while later batches run."""
    ref, ox, idx = small
    reqs = _requests(ref, 12, seed=21)
    srv = mbw.Server(idx, n_workers=2, max_batch_reads=5000)
    ts = [srv.submit(r.seq, r.lengths, copy=False) for r in reqs]
    views = [srv.wait(t, copy=False) for t in ts]
    more = [srv.submit(r.seq, r.lengths, copy=False) for r in reqs[:4]]
    for r, t, (s, p, info) in zip(reqs, ts, views):
        compare_with_oracle(s, p, ox.seed(r.seq, r.offsets))
        srv.release(t)
    for r, t in zip(reqs[:4], more):
        s, p, _ = srv.wait(t)
        compare_with_oracle(s, p, ox.seed(r.seq, r.offsets))
    srv.close()
