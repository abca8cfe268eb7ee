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


HEADER = struct.Struct("<QII QQQQQ 5Q iiii 64Q ii QQQ QQQQQQ Q")
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
    return dict(n=n, len_r=len_r, primary=primary, n_lines=n_lines, C=C5, r=r, K=K, sb=sb, bis=bis, sb_shift=sb_shift,
                lines=lines, ssa=ssa, kmer=kmer, bpl=bpl, isa_sample=isa_sample, text=text, isa=isa, orig=orig)


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
