"""Test helpers: run the GPU library and the oracle on the same seeded inputs and compare."""
from __future__ import annotations

import struct

import numpy as np

import oracle
import paper_2606_15357_amd as mbw

FIELDS = ("read_id", "qbeg", "qend", "k", "kr", "s", "npos")


def gpu_seed(index, reads, **kw):
    ctx = mbw.Context(index)
    out = ctx.seed(reads.seq, reads.lengths, **kw)
    seeds, pos = out.download()
    ctx.free()
    return out, seeds, pos


def gpu_canonical(seeds, pos):
    s, flat = mbw.canonical(seeds, pos)
    return s, flat


def compare_with_oracle(seeds, pos, ref_res, check_flags=True):
    """Bit-exact comparison of a GPU result with an oracle SeedResult (canonical order)."""
    s, flat = gpu_canonical(seeds, pos)
    assert len(s) == len(ref_res), (len(s), len(ref_res))
    for f in FIELDS:
        a = s[f].astype(np.uint64)
        b = getattr(ref_res, f).astype(np.uint64)
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0][:5]
            raise AssertionError(f"field {f} differs at {bad}: gpu {a[bad]} oracle {b[bad]}; "
                                 f"rows {[(int(s['read_id'][i]), int(s['qbeg'][i]), int(s['qend'][i])) for i in bad]}")
    if check_flags:
        assert np.array_equal((s["flags"] & 1).astype(np.uint32), ref_res.flags & 1)
    assert np.array_equal(flat, ref_res.pos), "positions differ"


HEADER = struct.Struct("<QII QQQQQ 5Q iiii 64Q ii QQQ QQQQQQ QQ Q")
MAX_SB = 8


def read_index_file(path):
    """Parse an index file written by mbw_index_save (the documented layout)."""
    with open(path, "rb") as f:
        raw = f.read()
    h = HEADER.unpack_from(raw, 0)
    magic, version, bpl, n, len_r, primary, n_lines, n_ssa = h[:8]
    C5 = list(h[8:13])
    r, K, bis, n_sb = h[13:17]
    sb = np.array(h[17:17 + 8 * MAX_SB], dtype=np.uint64).reshape(MAX_SB, 8)[:n_sb]
    off = HEADER.size
    lines = np.frombuffer(raw, dtype=np.uint64, count=n_lines * 16, offset=off).reshape(n_lines, 16)
    off += n_lines * 128
    ssa = np.frombuffer(raw, dtype=np.uint64, count=n_ssa, offset=off)
    off += n_ssa * 8
    kmer = None
    if K:
        kmer = np.frombuffer(raw, dtype=np.uint64, count=2 * 4 ** K, offset=off).reshape(-1, 2)
        off += 16 * 4 ** K
    isa_sample, sb_shift, n_text, n_isa, n_orig = h[17 + 8 * MAX_SB:22 + 8 * MAX_SB]
    text = np.frombuffer(raw, dtype=np.uint64, count=n_text, offset=off)
    off += 8 * n_text
    isa = np.frombuffer(raw, dtype=np.uint64, count=n_isa, offset=off)
    off += 8 * n_isa
    orig = np.frombuffer(raw, dtype=np.uint64, count=n_orig, offset=off)
    off += 8 * n_orig
    contig_bytes = h[28 + 8 * MAX_SB]
    blob = raw[off:off + contig_bytes]
    contigs, o = [], 8
    for _ in range(struct.unpack_from("<Q", blob, 0)[0]):
        st, ln, nl = struct.unpack_from("<QQI", blob, o)
        contigs.append((blob[o + 20:o + 20 + nl].decode(), st, ln))
        o += 20 + nl
    return dict(n=n, len_r=len_r, primary=primary, n_lines=n_lines, C=C5, r=r, K=K, sb=sb, bis=bis, sb_shift=sb_shift,
                lines=lines, ssa=ssa, kmer=kmer, bpl=bpl, isa_sample=isa_sample, text=text, isa=isa, orig=orig,
                contigs=contigs, size=len(raw), end=off + contig_bytes)


def decode_bwt(idx):
    """BWT codes (0..3, $ row as A) from the occurrence lines: six 64-row blocks per line, each a
    u64 of low code bits followed by a u64 of high code bits."""
    lines = idx["lines"]
    lo = lines[:, 4:16:2]
    hi = lines[:, 5:16:2]
    sh = np.arange(64, dtype=np.uint64)
    syms = ((lo[:, :, None] >> sh) & 1) | (((hi[:, :, None] >> sh) & 1) << 1)
    return syms.reshape(-1)[: idx["n"]].astype(np.uint8)


def unpack_kmer(e):
    w0, w1 = int(e[0]), int(e[1])
    k = w0 & ((1 << 40) - 1)
    kr = (w0 >> 40) | ((w1 & 0xFFFF) << 24)
    s = w1 >> 16
    return k, kr, s


_hip = None


def device_to_host(ptr: int, nbytes: int) -> np.ndarray:
    """Bytes of device memory at ptr (hipMemcpy, device to host)."""
    import ctypes
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    out = np.empty(max(int(nbytes), 1), np.uint8)
    rc = _hip.hipMemcpy(out.ctypes.data, ctypes.c_void_p(int(ptr)), int(nbytes), 2)
    assert rc == 0, f"hipMemcpy returned {rc}"
    return out[:nbytes]


def check_line_table(index, log=print):
    """CPU check of a resident index's occurrence lines and superblock table against their
    definitions, with numpy popcounts of the bit planes (none of the library's rank code):
    rows past n are zero; each sub-checkpoint holds the A, C, G counts of the line's first 64b
    rows; each line header holds the counts from its superblock's first row (zero at every
    2^sb_lines_log2-line boundary); each superblock entry holds the A, C, G, T counts before it and
    their suffix sums; and the totals over all n rows match C ($ counted as A)."""
    info = index.info()
    n, nl, sh, nsb = int(info["n"]), int(info["n_lines"]), int(info["sb_lines_log2"]), int(info["n_superblocks"])
    Cc = [int(x) for x in info["C"]]
    assert nsb == ((nl - 1) >> sh) + 1
    lines_ptr = index.device_arrays()[0]
    sbt = device_to_host(index.superblock_table(), nsb * 64).view(np.uint64).reshape(nsb, 8).astype(np.int64)
    chunk = 1 << min(21, sh)            # chunks never straddle a superblock boundary
    run = np.zeros(3, np.int64)         # A, C, G since the superblock's first row
    total = np.zeros(4, np.int64)       # A, C, G, T before the chunk
    full = np.uint64(0xFFFFFFFFFFFFFFFF)
    for L0 in range(0, nl, chunk):
        m = min(chunk, nl - L0)
        if L0 % (1 << sh) == 0:
            sb = L0 >> sh
            run[:] = 0
            assert np.array_equal(sbt[sb, :4], total), (sb, sbt[sb], total)
            for c in range(4):
                assert sbt[sb, 4 + c] == total[c + 1:].sum(), (sb, c)
        raw = device_to_host(lines_ptr + L0 * 128, m * 128)
        u32 = raw.view(np.uint32).reshape(m, 32)
        u64 = raw.view(np.uint64).reshape(m, 16)
        lo, hi = u64[:, 4::2], u64[:, 5::2]
        first = np.arange(L0, L0 + m, dtype=np.int64)[:, None] * 384 + np.arange(6, dtype=np.int64)[None, :] * 64
        nvalid = np.clip(n - first, 0, 64)
        mask = np.where(nvalid >= 64, full,
                        (np.uint64(1) << np.minimum(nvalid, 63).astype(np.uint64)) - np.uint64(1))
        assert not np.any((lo | hi) & ~mask), "bits set in rows past n"
        cA = np.bitwise_count(~lo & ~hi & mask).astype(np.int64)
        cC = np.bitwise_count(lo & ~hi & mask).astype(np.int64)
        cG = np.bitwise_count(~lo & hi & mask).astype(np.int64)
        cT = np.bitwise_count(lo & hi & mask).astype(np.int64)
        blk = np.stack([cA, cC, cG], axis=2)                    # lines x 6 blocks x 3
        sub_exp = np.cumsum(blk, axis=1)[:, :5, :]
        words = np.concatenate([u32[:, 3:4], u32[:, 4:8]], axis=1).astype(np.int64)
        sub_got = np.stack([(words >> s) & 0x1FF for s in (0, 9, 18)], axis=2)
        if not np.array_equal(sub_got, sub_exp):
            bad = np.argwhere(sub_got != sub_exp)[0]
            raise AssertionError(f"sub-checkpoint differs at line {L0 + bad[0]}, b={bad[1] + 1}")
        per_line = blk.sum(axis=1)
        head_exp = run[None, :] + np.cumsum(per_line, axis=0) - per_line
        head_got = u32[:, 0:3].astype(np.int64)
        if not np.array_equal(head_got, head_exp):
            bad = np.argwhere(head_got != head_exp)[0]
            raise AssertionError(f"line header differs at line {L0 + bad[0]}, symbol {bad[1]}")
        run += per_line.sum(axis=0)
        total += np.array([cA.sum(), cC.sum(), cG.sum(), cT.sum()])
    want = np.array([Cc[2] - Cc[1] + 1, Cc[3] - Cc[2], Cc[4] - Cc[3], n - Cc[4]], np.int64)
    assert np.array_equal(total, want), (total, want)
    log(f"line table checked: {nl} lines, {nsb} superblocks of 2^{sh} lines")
