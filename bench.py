#!/usr/bin/env python3
"""Throughput benchmark of batched (19,1)-SMEM seeding + sampled-SA locate on one MI355X.

Workload (default): a synthetic 3.1 Gbp reference (55% random sequence, 35% interspersed repeat
families of 300 bp / 6 kbp copies at 2-20% divergence, 10% tandem arrays of 171 bp units at 1-3%
divergence), indexed on the GPU (T = R . revcomp(R) . $, n = 6.2 G; 128-byte occurrence lines of
384 rows; SA sampled every 8 rows; 15-mer interval table, the size picked from the text
length), and 10,000,000 read pairs of 150 bp
(20,000,000 reads) at 0.5% substitutions + 0.05% 1-3 bp indels, 5% of pairs drawn from satellite
arrays.  One step = one ``mbw_seed`` call over the whole batch with the reads already resident in
HBM: encode, both SMEM rounds, sort/dedup, locate of every seed with s <= 500.

The JSON line reports reads/s of the default (wave-cooperative) path, the plain one-read-per-thread
kernel on the same index and reads, the roofline of the dominant kernel (the SMEM kernel: 128-byte
index lines it touches, counted by the kernel itself, over its HIP-event time), and the CPU oracle
(paper algorithms, OpenMP) timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "150bp reads seeded/s on 3.1 Gbp ref vs plain GPU kernel; serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
LINE_BYTES = 128


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def strip_comments(src: str) -> str:
    """C/C++ source without its comments and blank lines, trailing spaces removed: the text the
    compiler acts on, so that a change to a comment keeps the hash below."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    lines = (ln.rstrip() for ln in "".join(out).split("\n"))
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash():
    """Key of the committed counter summary: the seeding and index kernels' sources, comments
    excluded."""
    h = hashlib.sha256()
    for f in ("seed.hip", "mbw_internal.h", "index_build.hip"):
        with open(os.path.join(ROOT, "paper_2606_15357_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def profile_entry(kernel: str, isa_sample: int):
    """The committed counter summary's entry for `kernel`, if it was taken on the current kernel
    sources with the same inverse-SA sampling step (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash() or d.get("isa_sample") != isa_sample:
        return None
    return d.get("kernels", {}).get(kernel) or None


def traffic_from_profile(kernel: str, launches_bytes: float, isa_sample: int):
    """HBM bytes per launch of `kernel` from the committed counter summary (see profile_entry)."""
    k = profile_entry(kernel, isa_sample)
    return k.get("hbm_bytes_per_launch") if k else None


def transactions(smem_entry, loc_entry, ms_smem_step: float, ms_loc: float, ceiling_lps: float):
    """L2 hit rates and HBM read-request rates (one request moves a 128-byte line) of the SMEM
    rounds and locate from the committed counter summary, over this run's kernel times, against the
    random-gather probe's rate; None without a matching summary."""
    if not smem_entry or not loc_entry or "l2" not in smem_entry or "l2" not in loc_entry:
        return None
    sreq = sum(smem_entry["l2"]["hbm_read_requests_by_round"])
    lreq = loc_entry["l2"]["hbm_read_requests_per_launch"]
    s_ps, l_ps = sreq / (ms_smem_step * 1e-3), lreq / (ms_loc * 1e-3)
    return dict(smem=dict(l2_hit_rate_by_round=smem_entry["l2"]["hit_rate_by_round"], hbm_read_requests_per_step=sreq,
                          requests_per_s=round(s_ps), frac_of_probe=round(s_ps / ceiling_lps, 3)),
                locate=dict(l2_hit_rate=loc_entry["l2"]["hit_rate"], hbm_read_requests_per_launch=lreq,
                            requests_per_s=round(l_ps), frac_of_probe=round(l_ps / ceiling_lps, 3)),
                source="profiles/traffic.json (rocprofv3 TCC counters of one step); rates over this run's kernel "
                       "times; frac_of_probe against random_line_ceiling.lines_per_s")


def cpu_baseline(workload: str, ref_codes, n_pairs: int, window: int, threads: int):
    """The oracle (Algorithm 3 + LocateSlow + 10-mer shortcut, OpenMP over reads) on a bounded
    sample: an oracle index over the first `window` bases of the same reference and reads from
    that window drawn with the workload's read model."""
    import oracle
    import synth
    sub = synth.Reference(np.ascontiguousarray(ref_codes[:window]), np.zeros((0, 2), np.uint64), 1, 0)
    t0 = time.time()
    ox = oracle.OracleIndex(sub.codes, sa_rate=8)
    t_build = time.time() - t0
    if workload == "lognormal_100mbp":
        rs = synth.reads_lognormal(sub, n_pairs // 10, seed=4003)
    else:
        rs = synth.reads_fixed(sub, n_pairs, 150, True, p_sub=0.005, p_indel=0.0005, seed=4003)
    t0 = time.time()
    res = ox.seed(rs.seq, rs.offsets, min_len=19, max_occ=500, method=1, kmer_k=10, threads=threads)
    dt = time.time() - t0
    one = rs.subset(np.arange(min(len(rs), 20_000)))
    t0 = time.time()
    ox.seed(one.seq, one.offsets, min_len=19, max_occ=500, method=1, kmer_k=10, threads=1)
    dt1 = time.time() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    cpu_baseline.last_result = (res, window)
    return dict(value=len(rs) / dt, unit="reads/s", cores=threads, kind="oracle", cpu_model=model,
                value_1core=round(len(one) / dt1, 1),
                sample=f"{len(rs)} reads ({int(rs.lengths.sum())} bases, workload read model) against an oracle index "
                       f"of the first {window / 1e6:.0f} Mbp of the same 3.1 Gbp reference (index build "
                       f"{t_build:.1f} s excluded); oracle = serial Algorithm 3 + LocateSlow with the 10-mer "
                       f"shortcut per read, OpenMP over reads; {len(res)} seeds, {res.pos.size} positions; "
                       f"{dt:.1f} s wall; value_1core: the first {len(one)} of these reads on one thread, "
                       f"{dt1:.1f} s")


def rescue_leg(mbw, torch, ctx, ref, reads, dseq, dlen, steps: int, warmup: int, cpu: bool, threads: int,
               window: int):
    """Mate-rescue prefilter (Section 2.7, q = 7, pass at max_t M_t >= 10) on the resident index:
    for every read pair of the batch one candidate window where a proper pair puts the mate (from
    the simulated position of the other mate) and one uniformly random decoy window of the same
    length (about 550 bases), all in device memory; candidates/s over `steps` calls.  The CPU
    baseline runs the oracle (M_t by definition, OpenMP over candidates) on a bounded sample of
    the same recipe over the first `window` bases of the reference."""
    import synth
    cands, decoy = synth.rescue_candidates(reads, len(ref), decoys=True, seed=5000)
    dc = torch.from_numpy(cands.view(np.uint8)).to(dseq.device)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        out = ctx.rescue(dseq, dlen, dc, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [ctx.rescue(dseq, dlen, dc, stream=stream) for _ in range(steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = outs[-1]
    hits, _ = out.download()
    pw = reads.lengths[cands["read_id"]].astype(np.float64) - 6
    ww = cands["win_len"].astype(np.float64) - 6
    cells = float(np.sum(np.maximum(pw, 0) * np.maximum(ww, 0)))
    ms_k = sum(o.ms_kernel for o in outs) / len(outs)
    in_bytes = float(reads.lengths[cands["read_id"]].astype(np.float64).sum() + cands["win_len"].astype(np.float64).sum() / 4
                     + 16 * len(cands))
    res = dict(value=round(len(cands) * steps / el, 1), unit="candidates/s", candidates=len(cands),
               ms_per_step=round(el / steps * 1e3, 2), kernel_ms=round(ms_k, 2), q=7, min_hits=10,
               pass_true=round(float(np.mean(hits["max_hits"][decoy == 0] >= 10)), 4),
               pass_decoy=round(float(np.mean(hits["max_hits"][decoy == 1] >= 10)), 4),
               qmer_pairs_per_s=round(cells / (ms_k * 1e-3), 1),
               input_gbs=round(in_bytes / (ms_k * 1e-3) / 1e9, 1))
    del dc
    if cpu:
        import oracle
        sub = synth.Reference(np.ascontiguousarray(ref.codes[:window]), np.zeros((0, 2), np.uint64), 1, 0)
        rs = synth.reads_fixed(sub, 50_000, 150, True, p_sub=0.005, p_indel=0.0005, seed=5001)
        sc, _ = synth.rescue_candidates(rs, window, decoys=True, seed=5002)
        t0 = time.time()
        oracle.rescue(sub.codes, rs.seq, rs.offsets, sc["read_id"], sc["win_beg"], sc["win_len"], q=7,
                      threads=threads)
        dt = time.time() - t0
        res["cpu_baseline"] = dict(value=round(len(sc) / dt, 1), unit="candidates/s", cores=threads, kind="oracle",
                                   sample=f"{len(sc)} candidates (50,000 pairs of the workload's read model, a true-mate "
                                          f"and a decoy window each) over the first {window / 1e6:.0f} Mbp of the "
                                          f"reference; oracle = M_t counted pair by pair, OpenMP over candidates; "
                                          f"{dt:.1f} s wall")
    return res


def chain_leg(torch, ctx, out, n_reads: int, steps: int, stream):
    """Chaining (Section 2.6) of the whole seeding result of a step: anchors of every located seed,
    sorted per read, the chaining recurrence and the extraction of up to 50 chains per read
    (``mbw_chain``); anchors/s over `steps` calls, the chaining kernel's own time beside the call's."""
    ctx.chain(out, n_reads, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [ctx.chain(out, n_reads, stream=stream) for _ in range(steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ch = res[-1]
    return dict(value=round(ch.n_input_anchors * steps / el, 1), unit="anchors/s",
                reads_per_s=round(n_reads * steps / el, 1), ms_per_call=round(el / steps * 1e3, 2),
                kernel_ms=round(sum(r.ms_kernel for r in res) / len(res), 2), anchors=ch.n_input_anchors,
                chains=ch.n_chains, anchors_in_chains=ch.n_anchors, max_read_anchors=ch.max_read_anchors,
                reads_over_lds=ch.reads_over_lds,
                params="max_gap 5000, 50 predecessors, 50 chains per read, min score 19")


def chain_cpu_baseline(res, seg_len: int, sample: str):
    """The chaining oracle (one thread) on the seeds of the CPU-baseline sample."""
    import oracle
    t0 = time.time()
    chains, _ = oracle.chain(res, seg_len=seg_len)
    dt = time.time() - t0
    return dict(value=round(int(res.pos.size) / dt, 1), unit="anchors/s", cores=1, kind="oracle",
                sample=f"the oracle's seeds of the seeding CPU baseline ({sample}); {int(res.pos.size)} anchors, "
                       f"{chains.size} chains, {dt:.1f} s on one thread")


def latency_leg(mbw, torch, ctx, reads, dseq, dlen, sched: dict, stream):
    """Per-call time of small batches (reads already in HBM): persistent grids sized by the work
    (blocks_per_cu = 0) against grids at the occupancy limit (-1)."""
    rows = []
    for n in (1, 100, 1000, 20_000, 100_000, 400_000):
        if n > len(reads):
            break
        nb = int(reads.offsets[n])
        row = dict(reads=n)
        for name, bpc in (("work_sized_ms", 0), ("occupancy_limit_ms", -1)):
            # automatic wave takes: a fixed take tuned on the full batch would leave most waves of a
            # small batch's grid idle
            kw = dict(sched, blocks_per_cu=bpc, wave_chunk=0)
            for _ in range(2):
                ctx.seed(dseq[:nb], dlen[:n], min_seed_len=19, max_occ=500, stream=stream, **kw)
            ts = []
            for _ in range(7):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.seed(dseq[:nb], dlen[:n], min_seed_len=19, max_occ=500, stream=stream, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            row[name] = round(float(np.median(ts)) * 1e3, 3)
        # the same batch through a captured graph planned for it (work-sized grids; the lengths
        # come from the host, which checks them against the plan, the reads from HBM)
        gkw = dict(unique_ext=sched.get("unique_ext", True), blocks_per_cu=0, wave_chunk=0)
        g = ctx.graph(n, max_bases=nb, max_positions=max(64 * n, 16384), min_seed_len=19, max_occ=500, **gkw)
        hl = reads.lengths[:n]
        try:
            for _ in range(2):
                g.seed(dseq[:nb], hl, stream=stream)
            ts = []
            for _ in range(7):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.seed(dseq[:nb], hl, stream=stream)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            row["graph_ms"] = round(float(np.median(ts)) * 1e3, 3)
        except mbw.MbwError as e:            # a batch beyond its plan: no figure
            row["graph_ms"] = None
            log(f"graph leg at {n} reads: {e}")
        g.free()
        rows.append(row)
    return dict(unit="ms per mbw_seed call (graph_ms: per mbw_graph_seed call on a graph planned for the batch), "
                     "reads in HBM, median of 7", batches=rows)


LOADS = (0.25, 0.5, 0.8)
SERVE_WAVE_CHUNK = 256
MEAN_REQ = (20000.0 - 1.0) / np.log(20000.0)   # mean of the log-uniform 1..20,000 request size


def _serve_points(servers: dict, make_request, n_burst: int, seconds: float, loads=LOADS, seed: int = 0):
    """Closed-loop saturation, then open-loop Poisson arrivals at each fraction of it.

    servers maps a stream name to a Server; make_request() returns (name, reads, lengths), views
    into resident read pools (submitted without a host copy; results read in place and released).
    Saturation = reads of a burst of n_burst requests, all submitted at once, over the time from the
    first submission to the last result.  Each load point offers that fraction of the saturation
    rate for `seconds`; latency = submission to host-visible result on the server's clock."""
    import threading

    def drain(k, t):
        srv = servers[k]
        info = srv.wait(t, copy=False)[2]
        srv.release(t)
        return info

    def submit(k, x, y):
        t = servers[k].submit(x, y, copy=False)
        while t is None:                  # queue full: back off
            time.sleep(0.0002)
            t = servers[k].submit(x, y, copy=False)
        return t

    # warm-up: a burst of the same shape, so that every worker's pinned staging and result buffers
    # have grown to full batches before anything is timed
    warm = [make_request() for _ in range(max(8, n_burst // 2))]
    for k, t in [(k, submit(k, x, y)) for k, x, y in warm]:
        drain(k, t)
    burst = [make_request() for _ in range(n_burst)]
    t0 = time.perf_counter()
    ts = [(k, submit(k, x, y)) for k, x, y in burst]
    submit_s = time.perf_counter() - t0
    for k, t in ts:
        drain(k, t)
    sat_s = time.perf_counter() - t0
    sat = sum(len(y) for _, _, y in burst) / sat_s
    mean_req = float(np.mean([len(y) for _, _, y in burst]))
    rng = np.random.default_rng(7000 + seed)
    points = []
    for frac in loads:
        qps = frac * sat / mean_req
        arrivals = np.cumsum(rng.exponential(1.0 / qps, size=int(qps * seconds * 1.3) + 10))
        arrivals = arrivals[arrivals < seconds]
        reqs = [make_request() for _ in range(arrivals.size)]
        tickets, infos = [], []

        def waiter():
            k = 0
            while k < len(reqs):
                if k >= len(tickets):
                    time.sleep(0.0001)
                    continue
                name, t = tickets[k]
                infos.append((name, drain(name, t)))
                k += 1

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        for a, (k, x, y) in zip(arrivals, reqs):
            d = t0 + a - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets.append((k, submit(k, x, y)))
        th.join()
        wall = time.perf_counter() - t0
        lat = np.array([(i["t_done"] - i["t_submit"]) * 1e3 for _, i in infos])
        nr = sum(len(y) for _, _, y in reqs)
        pt = dict(load=frac, qps=round(qps, 1), requests=len(reqs), reads_per_s=round(nr / wall, 1),
                  p50_ms=round(float(np.percentile(lat, 50)), 3), p99_ms=round(float(np.percentile(lat, 99)), 3))
        for name in servers:
            if len(servers) > 1:
                ln = np.array([(i["t_done"] - i["t_submit"]) * 1e3 for k, i in infos if k == name])
                pt[name] = dict(requests=int(ln.size),
                                p50_ms=round(float(np.percentile(ln, 50)), 3) if ln.size else None,
                                p99_ms=round(float(np.percentile(ln, 99)), 3) if ln.size else None)
        bids = {(k, i["batch_id"]): i["batch_reads"] for k, i in infos}
        pt["batches"] = len(bids)
        pt["mean_batch_reads"] = round(float(np.mean(list(bids.values()))), 1) if bids else 0.0
        points.append(pt)
    return dict(saturation_reads_per_s=round(sat, 1), saturation_burst=dict(requests=n_burst, reads=int(sum(
        len(y) for _, _, y in burst)), seconds=round(sat_s, 3), submit_seconds=round(submit_s, 3)), loads=points)


def serve_leg(mbw, idx, reads, seconds: float, sched: dict, workers: int, max_batch: int, n_burst: int,
              bulk_rate: float):
    """The serving stream on the resident index: requests of log-uniform 1..20,000 reads drawn from
    the workload's reads; closed-loop saturation and p50/p99 at 25/50/80% of it for the wave
    kernel, and the closed-loop saturation of the same server running the plain kernel."""
    n = len(reads)
    rng = np.random.default_rng(3000)

    def request():
        m = int(np.exp(rng.uniform(0.0, np.log(20000.0))))
        r0 = int(rng.integers(0, n - m))
        return "plain", reads.seq[int(reads.offsets[r0]):int(reads.offsets[r0 + m])], reads.lengths[r0:r0 + m]

    cfg = dict(n_workers=workers, max_batch_reads=max_batch, max_batch_bases=max_batch * 160)
    # 256-read wave takes: with several batches on the device at once, each batch then keeps to
    # fewer waves (measured: closed-loop saturation 69-71 M reads/s against 60-63 M with automatic
    # takes, p50 at 25% load 12.8-13.3 ms against 12.0-12.5 ms)
    sched = dict(sched, wave_chunk=SERVE_WAVE_CHUNK)
    srv = mbw.Server(idx, **cfg, **sched)
    try:
        st0 = srv.stats()
        res = _serve_points({"plain": srv}, request, n_burst, seconds)
        st = srv.stats()
    finally:
        srv.close()
    res.update(saturation_frac_of_bulk=round(res["saturation_reads_per_s"] / bulk_rate, 3), workers=workers,
               max_batch_reads=max_batch, device_gb=round(st0["device_bytes"] / 1e9, 2),
               split_retries=st["split_retries"], failed_requests=st["failed_requests"],
               request_size="log-uniform 1..20000 reads", arrivals="Poisson at 25/50/80% of the closed-loop saturation",
               handoff="requests queued without a host copy, results read in place from pinned memory")
    sched_plain = dict(sched)
    sched_plain["kernel"] = mbw.KERNEL_PLAIN
    srv = mbw.Server(idx, **cfg, **sched_plain)
    try:
        pres = _serve_points({"plain": srv}, request, n_burst, seconds, loads=())
    finally:
        srv.close()
    res["plain_kernel"] = dict(saturation_reads_per_s=pres["saturation_reads_per_s"],
                               note="the same server and request stream with the plain (one read per lane) kernel")
    return res


def workload_leg(mbw, torch, synth, name: str, args, steps: int = 3):
    """Another workload of the same path, measured in the same way as the headline: its own index
    (100 Mbp mixed genome), reads resident in HBM, autotuned schedule, `steps` timed calls of the
    wave path after one warm-up, and one call of the plain kernel."""
    t0 = time.time()
    wl = synth.WORKLOADS[name]
    ref = synth.workload_reference(name)
    idx = mbw.Index.build(ref.codes, sa_sample=args.sa_sample, kmer_k=args.kmer, isa_sample=args.isa_sample)
    reads = synth.workload_reads(name, ref)
    dev = torch.device("cuda:0")
    dseq = torch.from_numpy(reads.seq).to(dev)
    dlen = torch.from_numpy(reads.lengths.view(np.int32)).to(dev)
    stream = torch.cuda.current_stream()
    ctx = mbw.Context(idx)
    try:
        best = ctx.tune(dseq, dlen, stream=stream)
        best.pop("ms")
        best.pop("cached", None)

        def step(kernel):
            return ctx.seed(dseq, dlen, min_seed_len=19, max_occ=500, kernel=kernel, stream=stream, **best)

        step(mbw.KERNEL_COOP)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        outs = [step(mbw.KERNEL_COOP) for _ in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        o = outs[-1]
        step(mbw.KERNEL_PLAIN)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        po = step(mbw.KERNEL_PLAIN)
        torch.cuda.synchronize()
        pel = time.perf_counter() - t2
        # the same batch through a captured graph planned for it (the tuned schedule where a graph takes
        # it; capacities from this batch's counts with room to spare)
        graph = None
        gkw = {k: v for k, v in best.items() if k in ("unique_ext", "seg_len", "blocks_per_cu", "wave_chunk")}
        g = ctx.graph(len(reads), max_bases=int(reads.lengths.sum()), max_read_len=int(reads.lengths.max()),
                      max_seeds=2 * int(o.n_seeds) + 1024, max_positions=2 * int(o.n_pos) + 1024, min_seed_len=19,
                      max_occ=500, **gkw)
        try:
            hl = reads.lengths
            go = g.seed(dseq, hl, stream=stream)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            for _ in range(steps):
                go = g.seed(dseq, hl, stream=stream)
            torch.cuda.synchronize()
            gel = time.perf_counter() - t3
            graph = dict(value=round(len(reads) * steps / gel, 1), ms_per_step=round(gel / steps * 1e3, 2),
                         same_counts=bool(go.n_seeds == o.n_seeds and go.n_pos == o.n_pos),
                         launches=int(go.n_smem_launches),
                         note="mbw_graph_seed: the whole call replayed from one captured graph (length bins, "
                              "segments), one host wait per call; sorts and scans span the plan's capacities")
        finally:
            g.free()
        res = dict(workload=wl["desc"], reads=len(reads), bases=int(reads.lengths.sum()),
                   value=round(len(reads) * steps / el, 1), unit="reads/s", ms_per_step=round(el / steps * 1e3, 2),
                   graph=graph,
                   plain_kernel=round(len(reads) / pel, 1), same_result=bool(po.n_seeds == o.n_seeds and po.n_pos == o.n_pos),
                   seeds=int(o.n_seeds), positions=int(o.n_pos), schedule=best, kmer_k=idx.info()["kmer_k"],
                   lines_per_read=round(o.lines_smem / len(reads), 1),
                   lane_use=round(o.lane_iters / max(1, 64 * o.wave_iters), 3),
                   note="index lines of a 100 Mbp genome largely fit the 256 MB last-level cache: no HBM roofline",
                   leg_seconds=round(time.time() - t0, 1))
    finally:
        ctx.free()
        idx.free()
    return res


def serve_bs_leg(mbw, synth, ref, pl_idx, args):
    """Serving with a bisulfite index and a plain index of the same 3.1 Gbp reference resident:
    requests of log-uniform 1..20,000 reads; 90% of them directional bisulfite reads (150 bp,
    read-1 form, seeded against the four-copy index with the strand filter and the seed
    refinement), 10% plain reads of 1-5 kbp (against the plain index); closed-loop saturation of
    the mix, then p50/p99 at 25/50/80% of it."""
    t0 = time.time()
    bs_idx = mbw.Index.build(ref.codes, sa_sample=args.sa_sample, kmer_k=args.kmer, bisulfite=True, isa_sample=8)
    t_bs = time.time() - t0
    log(f"bisulfite index built: {t_bs:.1f} s ({bs_idx.info()['bytes_resident'] / 1e9:.1f} GB)")
    bs_pool = synth.reads_bisulfite(ref, 1_000_000, seed=synth.READ_SEED + 4)
    pl_pool = synth.reads_uniform_len(ref, 20_000, 1000, 5000, p_sub=0.001, p_indel=0.0002, seed=synth.READ_SEED + 5)
    rng = np.random.default_rng(3001)

    def request():
        m = int(np.exp(rng.uniform(0.0, np.log(20000.0))))
        bs = rng.random() < 0.9
        pool = bs_pool if bs else pl_pool
        m = min(m, len(pool) - 1)
        r0 = int(rng.integers(0, len(pool) - m))
        return ("bisulfite" if bs else "plain_long", pool.seq[int(pool.offsets[r0]):int(pool.offsets[r0 + m])],
                pool.lengths[r0:r0 + m])

    srv = {}
    try:
        srv["bisulfite"] = mbw.Server(bs_idx, n_workers=args.bs_workers, max_batch_reads=1_000_000,
                                      max_batch_bases=160_000_000, bs_role=1, bs_refine=True,
                                      wave_chunk=SERVE_WAVE_CHUNK)
        srv["plain_long"] = mbw.Server(pl_idx, n_workers=args.bs_plain_workers, max_batch_reads=20_000,
                                       max_batch_bases=100_000_000, wave_chunk=SERVE_WAVE_CHUNK)
        res = _serve_points(srv, request, args.serve_burst, args.serve_seconds, seed=1)
        dev = sum(s.stats()["device_bytes"] for s in srv.values())
    finally:
        for s in srv.values():
            s.close()
        if "res" not in locals():
            bs_idx.free()
    res.update(metric="reads seeded/s served (bisulfite + plain), p50/p99 request latency", unit="reads/s",
               index_gb=dict(bisulfite=round(bs_idx.info()["bytes_resident"] / 1e9, 1),
                             plain=round(pl_idx.info()["bytes_resident"] / 1e9, 1)),
               index_build_s=round(t_bs, 1), device_gb_servers=round(dev / 1e9, 2),
               workers=dict(bisulfite=args.bs_workers, plain_long=args.bs_plain_workers),
               config="3.1 Gbp synthetic reference; bisulfite 4-copy index (n = 12.4 G + 1) and plain index "
                      "resident; 90% directional bisulfite 150 bp requests (strand filter + seed refinement), 10% "
                      "plain 1-5 kbp; log-uniform 1..20000 reads per request; Poisson arrivals at 25/50/80% of "
                      "the closed-loop saturation")
    bs_idx.free()
    return res


def gather_sweep(mbw):
    """Random 128-byte lines per second of the gather probe at 1-8 waves per SIMD and with the full
    grid ("full"): the rate depends on the number of requests in flight."""
    out = {}
    for w in (1, 2, 3, 4, 5, 6, 8, 0):
        lps, _ = mbw.probe_gather(8 << 30, iters=32, waves_per_simd=w)
        out["full" if w == 0 else str(w)] = round(lps)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="human_3gbp",
                    choices=["human_3gbp", "paired_100mbp", "lognormal_100mbp", "serve_bs_3gbp"],
                    help="human_3gbp (the headline), one of the 100 Mbp workloads, or the bisulfite serving workload")
    ap.add_argument("--ref-len", type=int, default=0, help="reference length (0 = the workload's)")
    ap.add_argument("--pairs", type=int, default=0, help="read pairs / reads (0 = the workload's)")
    ap.add_argument("--sa-sample", type=int, default=8)
    ap.add_argument("--kmer", type=int, default=-1, help="k-mer table size (-1 = from the text length)")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of the plain kernel (0 = skip)")
    ap.add_argument("--cpu-pairs", type=int, default=250_000)
    ap.add_argument("--cpu-window", type=int, default=16_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--isa-sample", type=int, default=1,
                    help="inverse-SA sampling step (0 = no unique-match path; 1 keeps every entry: 49.6 GB at 3.1 Gbp, "
                         "2 %% faster seeding than step 4, which needs 12.4 GB)")
    ap.add_argument("--no-unique", action="store_true", help="extend unique matches base by base")
    ap.add_argument("--probe", action="store_true", help="only run the copy and random-gather probes")
    ap.add_argument("--no-tune", action="store_true", help="default schedule instead of the autotuned one")
    ap.add_argument("--sched", default="", help="a fixed schedule as JSON (keyword arguments of Context.seed, e.g. "
                                                "the autotuner's pick of an earlier run) instead of tuning")
    ap.add_argument("--no-rescue", action="store_true", help="skip the mate-rescue prefilter leg")
    ap.add_argument("--no-chain", action="store_true", help="skip the chaining leg")
    ap.add_argument("--no-latency", action="store_true", help="skip the small-batch latency leg")
    ap.add_argument("--serve-workers", type=int, default=4, help="serving leg: worker threads, one stream each")
    ap.add_argument("--bs-workers", type=int, default=2, help="bisulfite serving: workers of the bisulfite server")
    ap.add_argument("--bs-plain-workers", type=int, default=2,
                    help="bisulfite serving: workers of the plain server (2 + 2 saturate at 11.5 M reads/s of the mix, "
                         "3 + 1 at 6.9 M: the 1-5 kbp requests carry most of the bases)")
    ap.add_argument("--serve-max-batch", type=int, default=1_000_000, help="serving leg: reads per batch at most")
    ap.add_argument("--serve-burst", type=int, default=12000,
                    help="requests in the closed-loop saturation burst (about 2,000 reads each)")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="seconds of open-loop arrivals per load point (0 = skip the serving legs)")
    ap.add_argument("--no-serve-bs", action="store_true", help="skip the bisulfite serving leg")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the 100 Mbp workloads (paired reads, lognormal read lengths)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the seeding path is "
              "data-parallel over reads with a replicated index; this benchmark runs on one GPU.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2606_15357_amd as mbw

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.probe:
        ms = mbw.probe_copy(1 << 30)
        lps, gms = mbw.probe_gather(8 << 30, iters=32)
        sweep = gather_sweep(mbw)
        print(json.dumps(dict(copy_bytes=1 << 30, copy_ms=round(ms, 3), copy_gbs=round(2 * (1 << 30) / ms / 1e6, 1),
                              gather_lines_per_s=lps, gather_gbs_128=round(lps * 128 / 1e9, 1), gather_ms=round(gms, 3),
                              gather_by_waves_per_simd=sweep)))
        return
    if args.workload == "serve_bs_3gbp":
        ref = synth.workload_reference("serve_bs_3gbp", args.ref_len or None)
        pl_idx = mbw.Index.build(ref.codes, sa_sample=args.sa_sample, kmer_k=args.kmer, isa_sample=args.isa_sample)
        res = serve_bs_leg(mbw, synth, ref, pl_idx, args)
        sat = res["saturation_reads_per_s"]
        print(json.dumps(dict(res, value=sat, n_gpus=1, higher_is_better=True, data="synthetic", dtype="u64")),
              flush=True)
        return
    gather_by_waves = gather_sweep(mbw)
    gather_lps = max(gather_by_waves.values())
    t0 = time.time()
    wl = synth.WORKLOADS[args.workload]
    args.ref_len = args.ref_len or wl["ref_len"]
    ref = synth.workload_reference(args.workload, args.ref_len)
    log(f"reference {len(ref)} bases generated in {time.time() - t0:.1f} s")
    t0 = time.time()
    idx = mbw.Index.build(ref.codes, sa_sample=args.sa_sample, kmer_k=args.kmer, isa_sample=args.isa_sample)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    info = idx.info()
    index_build = dict(seconds=round(build_s, 2), text_bases_per_s=round(info["n"] / build_s),
                       n=info["n"], resident_gb=round(info["bytes_resident"] / 1e9, 2),
                       includes="upload of the reference codes, suffix sorting, occurrence lines, SA/ISA samples, "
                                "k-mer table; first call in the process")
    log(f"index built on the GPU in {build_s:.1f} s: n={info['n']} lines={info['n_lines']} "
        f"resident={info['bytes_resident'] / 1e9:.2f} GB")
    t0 = time.time()
    reads = synth.workload_reads(args.workload, ref, args.pairs or None)
    n_reads = len(reads)
    log(f"{n_reads} reads generated in {time.time() - t0:.1f} s")
    dseq = torch.from_numpy(reads.seq).to(dev)
    dlen = torch.from_numpy(reads.lengths.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    ctx = mbw.Context(idx)
    stream = torch.cuda.current_stream()
    sched = dict(unique_ext=not args.no_unique)
    if args.sched:
        sched = json.loads(args.sched)
        log(f"fixed schedule: {sched}")
    elif not args.no_tune:
        t0 = time.time()
        m = min(n_reads, 4_000_000)
        best = ctx.tune(dseq[: int(reads.offsets[m])], dlen[:m], stream=stream)
        tune_ms = best.pop("ms")
        best.pop("cached", None)
        if args.no_unique:
            best["unique_ext"] = False
        sched = best
        log(f"autotuned on {m} reads in {time.time() - t0:.1f} s: {sched} ({tune_ms:.1f} ms)")

    def step(kernel):
        return ctx.seed(dseq, dlen, min_seed_len=19, max_occ=500, kernel=kernel, stream=stream, **sched)

    for _ in range(args.warmup):
        out = step(mbw.KERNEL_COOP)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for _ in range(args.steps):
        outs.append(step(mbw.KERNEL_COOP))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = outs[-1]
    value = n_reads * args.steps / elapsed
    ms_smem = sum(o.ms_smem for o in outs) / len(outs)
    ms_loc = sum(o.ms_locate for o in outs) / len(outs)
    launches = out.n_smem_launches
    lines_smem = out.lines_smem
    lines_loc = out.lines_locate
    log(f"wave path: {value / 1e6:.2f} M reads/s, {elapsed / args.steps * 1e3:.1f} ms/step; seeds {out.n_seeds} "
        f"positions {out.n_pos}; smem {ms_smem:.1f} ms ({launches} launches, {lines_smem} lines, "
        f"{out.wave_iters} wave iterations, lane use {out.lane_iters / max(1, 64 * out.wave_iters):.2f}), "
        f"locate {ms_loc:.1f} ms ({lines_loc} lines)")

    chain = None
    if not args.no_chain:
        chain = chain_leg(torch, ctx, out, n_reads, args.steps, stream)
        log(f"chaining: {chain}")

    plain = None
    if args.plain_steps > 0:
        step(mbw.KERNEL_PLAIN)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pouts = [step(mbw.KERNEL_PLAIN) for _ in range(args.plain_steps)]
        torch.cuda.synchronize()
        pel = time.perf_counter() - t0
        po = pouts[-1]
        plain = dict(value=n_reads * args.plain_steps / pel, unit="reads/s",
                     ms_smem=round(po.ms_smem, 2), ms_locate=round(po.ms_locate, 2),
                     same_result=bool(po.n_seeds == out.n_seeds and po.n_pos == out.n_pos))
        log(f"plain kernel: {plain['value'] / 1e6:.2f} M reads/s")

    # roofline of the dominant kernel (SMEM): algorithmic 128-byte lines over its event time
    smem_bytes = lines_smem * LINE_BYTES
    achieved = smem_bytes / (ms_smem * 1e-3) / 1e9
    traffic = traffic_from_profile("smem", smem_bytes / max(launches, 1), args.isa_sample)
    loc_traffic = traffic_from_profile("locate", 0, args.isa_sample)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel="k_smem_wave<staged> (both SMEM rounds)", launches_per_step=launches,
                    avg_launch_ms=round(ms_smem / max(launches, 1), 3),
                    bytes_per_launch=round(smem_bytes / max(launches, 1)),
                    lines_per_read=round(lines_smem / n_reads, 1),
                    locate=dict(line_accesses_per_read=round(lines_loc / n_reads, 1),
                                line_access_gbs=round(lines_loc * LINE_BYTES / (ms_loc * 1e-3) / 1e9, 1),
                                hbm_gbs=round(loc_traffic / (ms_loc * 1e-3) / 1e9, 1) if loc_traffic else None,
                                note="line_access_gbs counts every 128-byte line access of the walks, L2 hits "
                                     "included (neighbouring rows of one seed share lines), so it is not an HBM "
                                     "rate; hbm_gbs is the counter-measured traffic over the kernel time"),
                    whole_path_hbm_gbs=round((traffic * launches + loc_traffic) / (elapsed / args.steps) / 1e9, 1)
                    if traffic and loc_traffic else None,
                    random_line_ceiling=dict(lines_per_s=round(gather_lps), gbs=round(gather_lps * LINE_BYTES / 1e9, 1),
                                             by_waves_per_simd=gather_by_waves,
                                             probe="one lane x 16 B per random 128-B line, 4 dependent chains per lane, "
                                                   "8 GiB buffer; the best of 1-8 waves per SIMD and the full grid"),
                    frac_of_measured_ceiling=round(lines_smem / (ms_smem * 1e-3) / gather_lps, 3),
                    transactions=transactions(profile_entry("smem", args.isa_sample),
                                              profile_entry("locate", args.isa_sample), ms_smem, ms_loc, gather_lps))

    cpu = None
    if not args.no_cpu:
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        threads = max(1, min(threads, int(os.environ.get("OMP_NUM_THREADS", threads))))
        cpu = cpu_baseline(args.workload, ref.codes, args.cpu_pairs, args.cpu_window, threads)
        cpu["value"] = round(cpu["value"], 1)
        log(f"cpu oracle: {cpu['value']:.0f} reads/s on {cpu['cores']} threads")

    if chain is not None and cpu is not None and getattr(cpu_baseline, "last_result", None):
        res_cpu, window = cpu_baseline.last_result
        chain["cpu_baseline"] = chain_cpu_baseline(res_cpu, window, f"{len(res_cpu)} seeds over the first "
                                                                   f"{window / 1e6:.0f} Mbp")
        log(f"chaining cpu oracle: {chain['cpu_baseline']['value']:.0f} anchors/s")

    rescue = None
    if not args.no_rescue and args.workload in ("human_3gbp", "paired_100mbp"):
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        threads = max(1, min(threads, int(os.environ.get("OMP_NUM_THREADS", threads))))
        rescue = rescue_leg(mbw, torch, ctx, ref, reads, dseq, dlen, args.steps, args.warmup, not args.no_cpu, threads,
                            args.cpu_window)
        log(f"rescue prefilter: {rescue}")

    latency = None
    if not args.no_latency:
        latency = latency_leg(mbw, torch, ctx, reads, dseq, dlen, sched, stream)
        log(f"small batches: {latency}")

    others = None
    if not args.no_other_workloads and args.workload == "human_3gbp":
        others = {}
        for name in ("paired_100mbp", "lognormal_100mbp"):
            others[name] = workload_leg(mbw, torch, synth, name, args)
            log(f"{name}: {others[name]}")

    serve = serve_bs = None
    if args.serve_seconds > 0:
        ctx.free()
        serve = serve_leg(mbw, idx, reads, args.serve_seconds, sched, args.serve_workers, args.serve_max_batch,
                          args.serve_burst, value)
        log(f"serving: {serve}")
        if not args.no_serve_bs and args.workload == "human_3gbp":
            serve_bs = serve_bs_leg(mbw, synth, ref, idx, args)
            log(f"bisulfite serving: {serve_bs}")

    line = dict(metric=METRIC, value=round(value, 1), unit="reads/s", n_gpus=1, steps=args.steps,
                warmup=args.warmup, ms_per_step=round(elapsed / args.steps * 1e3, 2), higher_is_better=True,
                scaling="weak", vs_baseline=None, dtype="u64", data="synthetic",
                config=dict(workload=wl["desc"] + f" ({n_reads} reads, {args.ref_len / 1e6:.0f} Mbp); (19,1)-SMEMs + "
                                     f"re-seeding, max_occ 500",
                            min_seed_len=19, max_occ=500, sa_sample=args.sa_sample, kmer_k=info["kmer_k"],
                            isa_sample=args.isa_sample, unique_ext=not args.no_unique,
                            bases_per_line=384, line_bytes=LINE_BYTES, index_gb=round(info["bytes_resident"] / 1e9, 2)),
                schedule=sched, plain_gpu=plain, roofline=roofline, cpu_baseline=cpu, serve=serve, serve_bs=serve_bs,
                batch_latency=latency, other_workloads=others,
                index_build=index_build, rescue=rescue, chain=chain)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
