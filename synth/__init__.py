"""Seeded synthetic references and reads (shared input generators).

This package holds none of the seeding method's arithmetic: it draws the inputs that both the
CPU oracle and the GPU library consume.  Recipes follow the workload shapes used throughout the
project (see ``WORKLOADS``): a uniform-random genome with a divergent 2 kbp repeat family for the
small case, and a mixed genome (random sequence, interspersed 300 bp / 6 kbp repeat families at
2-20% divergence, tandem 171 bp satellite arrays at 1-3% divergence) for the 100 Mbp and
3.1 Gbp cases.  Reads carry substitutions and 1-3 bp indels.

Everything is a pure function of (recipe, size, seed); the C kernel (``synth.c``) runs with
OpenMP and its output is independent of the thread count.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libmbwsynth.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``synth.c`` into ``libmbwsynth.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    L = C.CDLL(_LIB)
    u64, u32, i32, dbl, vp = C.c_uint64, C.c_uint32, C.c_int, C.c_double, C.c_void_p
    L.synth_ref_plan.restype = vp
    L.synth_ref_plan.argtypes = [i32, u64, u64]
    L.synth_ref_len.restype = u64
    L.synth_ref_len.argtypes = [vp]
    L.synth_ref_fill.argtypes = [vp, vp]
    L.synth_ref_sats.restype = u64
    L.synth_ref_sats.argtypes = [vp, vp]
    L.synth_ref_free.argtypes = [vp]
    L.synth_reads_fixed.argtypes = [vp, u64, vp, u64, dbl, u64, u32, i32, dbl, dbl, dbl, dbl, u64,
                                     vp, vp, vp, vp]
    L.synth_read_lengths.argtypes = [u64, dbl, dbl, u32, u32, u64, vp]
    L.synth_reads_var.argtypes = [vp, u64, u64, vp, vp, dbl, dbl, u64, vp, vp, vp]
    L.synth_reads_bs.argtypes = [vp, u64, u64, u32, dbl, dbl, dbl, dbl, u64, vp, vp, vp, vp]
    _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------------------------------
# references

REF_SEED = 1000
READ_SEED = 2000


@dataclass
class Reference:
    codes: np.ndarray          # uint8, values 0..3 (A C G T)
    sats: np.ndarray           # uint64 [k, 2] satellite intervals [beg, end)
    recipe: int
    seed: int

    def __len__(self):
        return int(self.codes.size)


def reference(recipe: int, length: int, seed: int) -> Reference:
    """Synthetic reference.  recipe 0: random + 20 copies of a 2 kbp repeat at 5% divergence
    (length = ``length`` + the copies); recipe 1: the mixed genome, exactly ``length`` bases."""
    L = _load()
    h = L.synth_ref_plan(int(recipe), int(length), int(seed))
    try:
        n = int(L.synth_ref_len(h))
        out = np.empty(n, dtype=np.uint8)
        L.synth_ref_fill(h, _ptr(out))
        k = int(L.synth_ref_sats(h, None))
        sats = np.zeros((k, 2), dtype=np.uint64)
        if k:
            L.synth_ref_sats(h, _ptr(sats))
    finally:
        L.synth_ref_free(h)
    return Reference(out, sats, recipe, seed)


def random_reference(length: int, seed: int) -> Reference:
    """Uniform i.i.d. ACGT reference (recipe 0 without repeat copies is not exposed; this draws
    from the same generator with a single random segment)."""
    rng = np.random.default_rng(seed)
    return Reference(rng.integers(0, 4, size=length, dtype=np.uint8), np.zeros((0, 2), np.uint64), -1, seed)


# ------------------------------------------------------------------------------------------
# reads

@dataclass
class ReadSet:
    seq: np.ndarray        # uint8 ASCII, concatenated
    lengths: np.ndarray    # uint32 per read
    offsets: np.ndarray    # uint64, n+1 (CSR)
    tpos: np.ndarray       # uint64 truth start of the source fragment on the reference
    tstrand: np.ndarray    # uint8 truth strand (1 = reverse complement)

    def __len__(self):
        return int(self.lengths.size)

    def read(self, i: int) -> bytes:
        return self.seq[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()

    def subset(self, idx) -> "ReadSet":
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.lengths[idx]
        offs = np.zeros(idx.size + 1, dtype=np.uint64)
        np.cumsum(lens, out=offs[1:])
        seq = np.empty(int(offs[-1]), dtype=np.uint8)
        for j, i in enumerate(idx):
            seq[int(offs[j]):int(offs[j + 1])] = self.seq[int(self.offsets[i]):int(self.offsets[i + 1])]
        return ReadSet(seq, lens.astype(np.uint32), offs, self.tpos[idx], self.tstrand[idx])


def _compact_fixed(buf: np.ndarray, lens: np.ndarray, rlen: int):
    n = lens.size
    offs = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    if np.all(lens == rlen):
        return buf.reshape(-1)[: n * rlen].copy(), offs
    mask = np.arange(rlen, dtype=np.uint32)[None, :] < lens[:, None]
    return buf.reshape(n, rlen)[mask].copy(), offs


def reads_fixed(ref: Reference, n_frag: int, rlen: int = 150, paired: bool = False,
                ins_mean: float = 400.0, ins_sd: float = 50.0, p_sub: float = 0.005,
                p_indel: float = 0.0005, sat_frac: float = 0.0, seed: int = READ_SEED) -> ReadSet:
    """Fixed-length reads from uniform positions on both strands; paired reads give 2*n_frag reads
    (mate = reverse complement of the insert end, insert ~ round(N(ins_mean, ins_sd)))."""
    L = _load()
    nr = n_frag * (2 if paired else 1)
    buf = np.empty(nr * rlen, dtype=np.uint8)
    lens = np.empty(nr, dtype=np.uint32)
    tpos = np.empty(nr, dtype=np.uint64)
    tstr = np.empty(nr, dtype=np.uint8)
    sats = np.ascontiguousarray(ref.sats, dtype=np.uint64)
    L.synth_reads_fixed(_ptr(ref.codes), len(ref), _ptr(sats) if sats.size else None, sats.shape[0],
                        float(sat_frac), int(n_frag), int(rlen), int(paired), float(ins_mean),
                        float(ins_sd), float(p_sub), float(p_indel), int(seed), _ptr(buf), _ptr(lens),
                        _ptr(tpos), _ptr(tstr))
    seq, offs = _compact_fixed(buf, lens, rlen)
    return ReadSet(seq, lens, offs, tpos, tstr)


def reads_lognormal(ref: Reference, n: int, median: float = 300.0, sigma: float = 0.75,
                    lo: int = 100, hi: int = 5000, p_sub: float = 0.001, p_indel: float = 0.0002,
                    seed: int = READ_SEED) -> ReadSet:
    """Single-end reads with lengths exp(N(ln median, sigma^2)) resampled into [lo, hi]."""
    L = _load()
    lens = np.empty(n, dtype=np.uint32)
    L.synth_read_lengths(int(n), float(median), float(sigma), int(lo), int(hi), int(seed), _ptr(lens))
    offs = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    seq = np.empty(int(offs[-1]), dtype=np.uint8)
    tpos = np.empty(n, dtype=np.uint64)
    tstr = np.empty(n, dtype=np.uint8)
    L.synth_reads_var(_ptr(ref.codes), len(ref), int(n), _ptr(lens), _ptr(offs), float(p_sub),
                      float(p_indel), int(seed), _ptr(seq), _ptr(tpos), _ptr(tstr))
    return ReadSet(seq, lens, offs, tpos, tstr)


def reads_uniform_len(ref: Reference, n: int, lo: int, hi: int, p_sub: float = 0.001,
                      p_indel: float = 0.0002, seed: int = READ_SEED) -> ReadSet:
    """Single-end reads with lengths U[lo, hi]."""
    L = _load()
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi + 1, size=n).astype(np.uint32)
    offs = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    seq = np.empty(int(offs[-1]), dtype=np.uint8)
    tpos = np.empty(n, dtype=np.uint64)
    tstr = np.empty(n, dtype=np.uint8)
    L.synth_reads_var(_ptr(ref.codes), len(ref), int(n), _ptr(lens), _ptr(offs), float(p_sub),
                      float(p_indel), int(seed), _ptr(seq), _ptr(tpos), _ptr(tstr))
    return ReadSet(seq, lens, offs, tpos, tstr)


def reads_bisulfite(ref: Reference, n: int, rlen: int = 150, p_cpg: float = 0.20,
                    p_noncpg: float = 0.70, p_sub: float = 0.005, p_indel: float = 0.0005,
                    seed: int = READ_SEED) -> ReadSet:
    """Directional bisulfite reads (read-1 form): OT/OB strand 50/50; on the source strand each C
    becomes T with probability p_cpg in CpG context, p_noncpg elsewhere; then sequencing errors."""
    L = _load()
    buf = np.empty(n * rlen, dtype=np.uint8)
    lens = np.empty(n, dtype=np.uint32)
    tpos = np.empty(n, dtype=np.uint64)
    tstr = np.empty(n, dtype=np.uint8)
    L.synth_reads_bs(_ptr(ref.codes), len(ref), int(n), int(rlen), float(p_cpg), float(p_noncpg),
                     float(p_sub), float(p_indel), int(seed), _ptr(buf), _ptr(lens), _ptr(tpos), _ptr(tstr))
    seq, offs = _compact_fixed(buf, lens, rlen)
    return ReadSet(seq, lens, offs, tpos, tstr)


def concat(a: ReadSet, b: ReadSet) -> ReadSet:
    lens = np.concatenate([a.lengths, b.lengths])
    offs = np.zeros(lens.size + 1, dtype=np.uint64)
    np.cumsum(lens, out=offs[1:])
    return ReadSet(np.concatenate([a.seq, b.seq]), lens, offs, np.concatenate([a.tpos, b.tpos]),
                   np.concatenate([a.tstrand, b.tstrand]))


# ------------------------------------------------------------------------------------------
# the five workloads (reference recipe, size and seed; read model)

RESCUE_CAND_DTYPE = np.dtype([("read_id", "<u4"), ("win_len", "<u4"), ("win_beg", "<u8")])


def rescue_candidates(reads: ReadSet, ref_len: int, decoys: bool = True, seed: int = 0, ins_mean: float = 400.0,
                      ins_sd: float = 50.0, rlen: int = 150):
    """Mate-rescue candidates for a paired read set from ``reads_fixed(..., paired=True)``: for
    every pair, the mate whose text position is known from the simulation (read 1 of a forward
    fragment at ``tpos``, read 2 of a reverse one at ``tpos + 32``) stands for the mapped read,
    and the other mate is looked for in the window where a proper pair puts it: with T = R .
    revcomp(R) and an insert of il bases, a mate of the read at text position p starts at
    2|R| - p - il, so the window is [2|R| - p - ins_mean - 4 ins_sd, + 8 ins_sd + rlen) clipped to
    [0, 2|R|).  With ``decoys`` every true candidate is followed by one for the same read at a
    uniformly random window of the same length.  Returns (candidates, decoy flags)."""
    n_pairs = len(reads) // 2
    two_l = 2 * int(ref_len)
    rev = reads.tstrand[0::2][:n_pairs].astype(np.int64)
    st = reads.tpos[0::2][:n_pairs].astype(np.int64)
    p = np.where(rev == 0, st, st + 32)
    mate = np.where(rev == 0, 2 * np.arange(n_pairs) + 1, 2 * np.arange(n_pairs))
    b = two_l - p - int(round(ins_mean + 4 * ins_sd))
    e = b + int(round(8 * ins_sd)) + int(rlen)
    b = np.clip(b, 0, two_l)
    e = np.clip(e, 0, two_l)
    k = 2 if decoys else 1
    out = np.zeros(n_pairs * k, dtype=RESCUE_CAND_DTYPE)
    flag = np.zeros(n_pairs * k, dtype=np.uint8)
    out["read_id"][0::k] = mate
    out["win_beg"][0::k] = b
    out["win_len"][0::k] = e - b
    if decoys:
        rng = np.random.default_rng(seed)
        wl = e - b
        out["read_id"][1::2] = mate
        out["win_len"][1::2] = wl
        out["win_beg"][1::2] = (rng.random(n_pairs) * (two_l - wl + 1)).astype(np.int64)
        flag[1::2] = 1
    return out, flag


WORKLOADS = {
    "small_1mbp": dict(desc="1 Mbp random + 20x2 kbp repeat @5%; 10,000 x 150 bp single-end, 0.5% sub, "
                            "0.05% indel; min seed 19, max_occ 500", recipe=0, ref_len=1_000_000, seed=0),
    "paired_100mbp": dict(desc="100 Mbp mixed genome; 1,000,000 pairs x 150 bp, insert N(400,50), 0.5% sub, "
                               "0.05% indel", recipe=1, ref_len=100_000_000, seed=1),
    "lognormal_100mbp": dict(desc="100 Mbp mixed genome; 500,000 reads, lognormal length 100-5000 bp "
                                  "(median 300), 0.1% sub, 0.02% indel", recipe=1, ref_len=100_000_000, seed=1,
                             read_seed=2),
    "human_3gbp": dict(desc="3.1 Gbp mixed genome; 10,000,000 pairs x 150 bp at 0.5% error, 5% from "
                            "satellites", recipe=1, ref_len=3_100_000_000, seed=3),
    "serve_bs_3gbp": dict(desc="3.1 Gbp mixed genome, bisulfite 3-base index + plain index; Poisson request "
                               "stream", recipe=1, ref_len=3_100_000_000, seed=3, read_seed=4),
}


def workload_reference(name: str, ref_len: int | None = None) -> Reference:
    w = WORKLOADS[name]
    return reference(w["recipe"], ref_len or w["ref_len"], REF_SEED + w["seed"])


def workload_reads(name: str, ref: Reference, n: int | None = None) -> ReadSet:
    """Reads of workload ``name``; ``n`` overrides the read (or pair) count for bounded samples."""
    w = WORKLOADS[name]
    seed = READ_SEED + w.get("read_seed", w["seed"])
    if name == "small_1mbp":
        return reads_fixed(ref, n or 10_000, 150, False, p_sub=0.005, p_indel=0.0005, seed=seed)
    if name == "paired_100mbp":
        return reads_fixed(ref, n or 1_000_000, 150, True, p_sub=0.005, p_indel=0.0005, seed=seed)
    if name == "lognormal_100mbp":
        return reads_lognormal(ref, n or 500_000, seed=seed)
    if name == "human_3gbp":
        return reads_fixed(ref, n or 10_000_000, 150, True, p_sub=0.005, p_indel=0.0005,
                           sat_frac=0.05, seed=seed)
    raise ValueError("serve_bs_3gbp reads are drawn per request (see reads_bisulfite)")
