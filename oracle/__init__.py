"""ORACLE — test infrastructure only.

A plain CPU statement of the seeding path (see ``oracle.c`` for the paper passages each function
follows).  Only the tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg
may import this package; the product library never does, and the two share no code.

Three oracles:
  * method 0 (O1): full suffix array by sorting; intervals, SMEMs and positions from their
    definitions (Section 2.1).
  * method 1 (O2): FM-index with Algorithm 1, serial Algorithm 3, Algorithm 2 LocateSlow over
    a sampled SA; counts the index lines a given line layout would touch.
  * ``scan_seed`` (O3): no index; one pass over T finds every occurrence of every q-mer of a
    sample of reads, and direct extension gives the SMEM set, s and the exact positions from the
    definitions (Section 2.2).  For references too large to sort on the host; ds-interval bounds
    are not produced (k = k' = 2^64 - 1).

Also: ``bs_refine`` (Section 2.9 seed refinement at read-C-over-reference-T bases),
``rescue`` / ``rescue_diagonals`` (Section 2.7 mate-rescue prefilter, M_t counted pair by pair) and
``chain`` / ``chain_dp`` (Section 2.6: minimap2's chaining recurrence over variable-length seeds,
up to 50 chains per read).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("min_len", C.c_int), ("min_occ", C.c_int), ("max_occ", C.c_int), ("reseed", C.c_int),
                ("reseed_len", C.c_int), ("reseed_occ", C.c_int), ("bs_role", C.c_int),
                ("method", C.c_int), ("kmer_k", C.c_int), ("bases_per_line", C.c_int)]


class _ChainOpts(C.Structure):
    _fields_ = [("max_gap", C.c_int), ("max_pred", C.c_int), ("max_chains", C.c_int), ("min_score", C.c_int)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    L = C.CDLL(_LIB)
    u64, i32, vp, u8 = C.c_uint64, C.c_int, C.c_void_p, C.c_uint8
    L.orc_build.restype = vp
    L.orc_build.argtypes = [vp, u64, i32, i32]
    L.orc_free.argtypes = [vp]
    for f in ("orc_n", "orc_primary"):
        getattr(L, f).restype = u64
        getattr(L, f).argtypes = [vp]
    for f in ("orc_copy_text", "orc_copy_sa", "orc_copy_bwt", "orc_copy_c"):
        getattr(L, f).argtypes = [vp, vp]
    L.orc_interval_ascii.argtypes = [vp, vp, u64, vp]
    L.orc_seed.restype = vp
    L.orc_seed.argtypes = [vp, vp, vp, u64, C.POINTER(_Opts), i32]
    L.orc_result_nseeds.restype = u64
    L.orc_result_nseeds.argtypes = [vp]
    L.orc_result_npos.restype = u64
    L.orc_result_npos.argtypes = [vp]
    L.orc_result_copy.argtypes = [vp] + [vp] * 10
    L.orc_result_lines.argtypes = [vp, vp]
    L.orc_result_free.argtypes = [vp]
    L.orc_backward.argtypes = [vp, vp, u8]
    L.orc_forward.argtypes = [vp, vp, u8]
    L.orc_pi.restype = u64
    L.orc_pi.argtypes = [vp, u8, u64]
    L.orc_locate_slow.restype = u64
    L.orc_locate_slow.argtypes = [vp, u64]
    L.orc_scan_seed.restype = vp
    L.orc_scan_seed.argtypes = [vp, u64, i32, vp, vp, u64, C.POINTER(_Opts), i32]
    L.orc_bs_refine.restype = u64
    L.orc_bs_refine.argtypes = [vp, u64, vp, vp, vp, vp, vp, vp, vp, u64, vp, i32, i32, C.POINTER(vp)]
    L.orc_rescue_diag_ascii.argtypes = [vp, u64, vp, u64, i32, i32, vp]
    L.orc_rescue.restype = i32
    L.orc_rescue.argtypes = [vp, u64, i32, vp, vp, u64, vp, vp, vp, u64, i32, i32, vp, vp, i32]
    L.orc_free_ptr.argtypes = [vp]
    L.orc_chain_dp.argtypes = [vp, vp, vp, vp, u64, i32, i32, vp, vp]
    L.orc_chain.restype = u64
    L.orc_chain.argtypes = [vp, vp, vp, vp, vp, u64, vp, u64, C.POINTER(_ChainOpts)] + [C.POINTER(vp)] * 8 + [vp]
    _lib = L
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


# oracle symbol codes: $ = 0, A..T = 1..4
SYM = {"$": 0, "A": 1, "C": 2, "G": 3, "T": 4}


@dataclass
class SeedResult:
    """Seeds sorted by (read_id, qbeg, qend); positions of seed t are pos[pos_off[t] : pos_off[t] + npos[t]],
    ascending.  flags bit 0: occurrence count above max_occ, so not located."""
    read_id: np.ndarray
    qbeg: np.ndarray
    qend: np.ndarray
    k: np.ndarray
    kr: np.ndarray
    s: np.ndarray
    npos: np.ndarray
    flags: np.ndarray
    pos_off: np.ndarray
    pos: np.ndarray
    lines: dict = field(default_factory=dict)

    def __len__(self):
        return int(self.read_id.size)


class OracleIndex:
    """T = R . revcomp(R) . $ (or the four-copy bisulfite text) with its full SA, BWT and an
    FM-index sampled every ``sa_rate`` rows."""

    def __init__(self, ref_codes: np.ndarray, bisulfite: bool = False, sa_rate: int = 8):
        L = _load()
        self._ref = np.ascontiguousarray(ref_codes, dtype=np.uint8)
        self.len_r = int(self._ref.size)
        self.bisulfite = bool(bisulfite)
        self.sa_rate = int(sa_rate)
        self._h = L.orc_build(_p(self._ref), self.len_r, int(bisulfite), int(sa_rate))
        self.n = int(L.orc_n(self._h))
        self.primary = int(L.orc_primary(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    # raw structures (tests) -------------------------------------------------------------
    def text(self) -> np.ndarray:
        out = np.empty(self.n, np.uint8)
        _lib.orc_copy_text(self._h, _p(out))
        return out

    def sa(self) -> np.ndarray:
        out = np.empty(self.n, np.uint64)
        _lib.orc_copy_sa(self._h, _p(out))
        return out

    def bwt(self) -> np.ndarray:
        out = np.empty(self.n, np.uint8)
        _lib.orc_copy_bwt(self._h, _p(out))
        return out

    def C(self) -> np.ndarray:
        out = np.empty(6, np.uint64)
        _lib.orc_copy_c(self._h, _p(out))
        return out

    def interval(self, pattern: str | bytes):
        """ds-interval (lo(P), lo(revcomp P), occ(P)) of an ASCII pattern, by definition."""
        b = pattern.encode() if isinstance(pattern, str) else bytes(pattern)
        a = np.frombuffer(b, dtype=np.uint8).copy() if b else np.zeros(1, np.uint8)
        out = np.zeros(3, np.uint64)
        _lib.orc_interval_ascii(self._h, _p(a), len(b), _p(out))
        return tuple(int(x) for x in out)

    def backward(self, iv, a: int):
        v = np.array(iv, dtype=np.uint64)
        _lib.orc_backward(self._h, _p(v), int(a))
        return tuple(int(x) for x in v)

    def forward(self, iv, a: int):
        v = np.array(iv, dtype=np.uint64)
        _lib.orc_forward(self._h, _p(v), int(a))
        return tuple(int(x) for x in v)

    def pi(self, a: int, k: int) -> int:
        return int(_lib.orc_pi(self._h, int(a), int(k)))

    def locate_slow(self, k: int) -> int:
        return int(_lib.orc_locate_slow(self._h, int(k)))

    # seeding ------------------------------------------------------------------------------
    def seed(self, seq: np.ndarray, offsets: np.ndarray, min_len: int = 19, min_occ: int = 1,
             max_occ: int = 500, reseed: bool = True, reseed_len: int = 38, reseed_occ: int = 10,
             bs_role: int = 0, method: int = 0, kmer_k: int = 0, bases_per_line: int = 0,
             threads: int = 0) -> SeedResult:
        seq = np.ascontiguousarray(seq, dtype=np.uint8)
        if seq.size == 0:
            seq = np.zeros(1, np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        nr = offsets.size - 1
        o = _Opts(int(min_len), int(min_occ), int(max_occ), int(bool(reseed)), int(reseed_len),
                  int(reseed_occ), int(bs_role), int(method), int(kmer_k), int(bases_per_line))
        h = _lib.orc_seed(self._h, _p(seq), _p(offsets), nr, C.byref(o), int(threads))
        return _result(h)


def _result(h) -> SeedResult:
    try:
        ns = int(_lib.orc_result_nseeds(h))
        np_ = int(_lib.orc_result_npos(h))
        a = dict(read_id=np.empty(ns, np.uint32), qbeg=np.empty(ns, np.uint32), qend=np.empty(ns, np.uint32),
                 k=np.empty(ns, np.uint64), kr=np.empty(ns, np.uint64), s=np.empty(ns, np.uint64),
                 npos=np.empty(ns, np.uint32), flags=np.empty(ns, np.uint32),
                 pos_off=np.empty(ns, np.uint64), pos=np.empty(np_, np.uint64))
        names = ("read_id", "qbeg", "qend", "k", "kr", "s", "npos", "flags", "pos_off", "pos")
        bufs = [a[x] if a[x].size else np.zeros(1, a[x].dtype) for x in names]
        _lib.orc_result_copy(h, *[_p(b) for b in bufs])
        for name, b in zip(names, bufs):
            a[name] = b[: a[name].size]
        ln = np.zeros(5, np.uint64)
        _lib.orc_result_lines(h, _p(ln))
        lines = dict(lines=int(ln[0]), kmer_lookups=int(ln[1]), sa_reads=int(ln[2]), steps=int(ln[3]),
                     lf_steps=int(ln[4]))
    finally:
        _lib.orc_result_free(h)
    return SeedResult(lines=lines, **a)


def scan_seed(ref_codes: np.ndarray, seq: np.ndarray, offsets: np.ndarray, bisulfite: bool = False,
              min_len: int = 19, min_occ: int = 1, max_occ: int = 500, reseed: bool = True,
              reseed_len: int = 38, reseed_occ: int = 10, bs_role: int = 0, threads: int = 0) -> SeedResult:
    """O3: SMEMs of both rounds, s and positions of a (small) read set over T = R . revcomp(R) . $
    (or the bisulfite text) by one scan of T, without an index.  Needs min(l, reseed_len / 2)
    between 1 and 32; k and k' come back as 2^64 - 1."""
    L = _load()
    ref = np.ascontiguousarray(ref_codes, dtype=np.uint8)
    seq = np.ascontiguousarray(seq, dtype=np.uint8)
    if seq.size == 0:
        seq = np.zeros(1, np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    q = min(min_len, reseed_len // 2) if reseed else min_len
    if not 1 <= q <= 32:
        raise ValueError("scan oracle needs a q-mer length between 1 and 32")
    o = _Opts(int(min_len), int(min_occ), int(max_occ), int(bool(reseed)), int(reseed_len), int(reseed_occ),
              int(bs_role), 2, 0, 0)
    h = L.orc_scan_seed(_p(ref), ref.size, int(bool(bisulfite)), _p(seq), _p(offsets), offsets.size - 1,
                        C.byref(o), int(threads))
    if not h:
        raise ValueError("scan oracle rejected its arguments")
    return _result(h)


PIECE_DTYPE = np.dtype([("read_id", "<u4"), ("qbeg", "<u4"), ("qend", "<u4"), ("seed", "<u4"), ("pos", "<u8")])


def bs_refine(ref_codes: np.ndarray, seq: np.ndarray, offsets: np.ndarray, res: SeedResult, role: int,
              min_len: int = 19) -> np.ndarray:
    """Bisulfite seed refinement (Section 2.9) of a bisulfite seeding result: every retained (seed,
    position) pair split at read-C-over-reference-T bases (read 2: G over A) of the original
    sequences, pieces of >= min_len kept.  Returns PIECE_DTYPE records sorted by (read, qbeg,
    qend, pos); ``seed`` is the index of the source seed in ``res``."""
    L = _load()
    ref = np.ascontiguousarray(ref_codes, dtype=np.uint8)
    seq = np.ascontiguousarray(seq, dtype=np.uint8)
    if seq.size == 0:
        seq = np.zeros(1, np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    arrs = [np.ascontiguousarray(a) if a.size else np.zeros(1, a.dtype) for a in
            (res.read_id, res.qbeg, res.qend, res.pos_off, res.npos, res.pos)]
    out = C.c_void_p()
    n = L.orc_bs_refine(_p(ref), ref.size, _p(seq), _p(offsets), *[_p(a) for a in arrs[:5]], len(res), _p(arrs[5]),
                        int(role), int(min_len), C.byref(out))
    pieces = np.zeros(n, dtype=PIECE_DTYPE)
    if n:
        C.memmove(pieces.ctypes.data, out.value, n * PIECE_DTYPE.itemsize)
    L.orc_free_ptr(out)
    return pieces


def seed_reads(index: OracleIndex, reads, **kw) -> SeedResult:
    """Convenience: seed a ``synth.ReadSet``-like object (``seq``, ``offsets``)."""
    return index.seed(reads.seq, reads.offsets, **kw)


def rescue_diagonals(read: bytes | str, window: bytes | str, q: int = 7, role: int = 0) -> np.ndarray:
    """Mate-rescue prefilter (Section 2.7) for one read and one window given as ASCII: the vector
    M_t = #{(i, j): P[i, i+q) = W[j, j+q), j - i = t}, element t + |P| - q, counted from the
    definition.  Empty when |P| < q or |W| < q."""
    L = _load()
    p = np.frombuffer(read.encode() if isinstance(read, str) else bytes(read), dtype=np.uint8).copy()
    w = np.frombuffer(window.encode() if isinstance(window, str) else bytes(window), dtype=np.uint8).copy()
    nd = p.size + w.size - 2 * q + 1 if p.size >= q and w.size >= q else 0
    M = np.zeros(max(nd, 1), dtype=np.uint32)
    pp = p if p.size else np.zeros(1, np.uint8)
    ww = w if w.size else np.zeros(1, np.uint8)
    L.orc_rescue_diag_ascii(_p(pp), p.size, _p(ww), w.size, int(q), int(role), _p(M))
    return M[:nd]


def rescue(ref_codes: np.ndarray, seq: np.ndarray, offsets: np.ndarray, read_id, win_beg, win_len, q: int = 7,
           role: int = 0, bisulfite: bool = False, threads: int = 0):
    """Mate-rescue prefilter (Section 2.7) for candidates (read read_id[c], window
    T[win_beg[c], win_beg[c] + win_len[c]) of the text of ``ref_codes``): returns (max_hits u32,
    best_t i32), best_t the smallest t with M_t = max_hits (0 when that is 0)."""
    L = _load()
    ref = np.ascontiguousarray(ref_codes, dtype=np.uint8)
    seq = np.ascontiguousarray(seq, dtype=np.uint8)
    if seq.size == 0:
        seq = np.zeros(1, np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    rid = np.ascontiguousarray(read_id, dtype=np.uint32)
    beg = np.ascontiguousarray(win_beg, dtype=np.uint64)
    wl = np.ascontiguousarray(win_len, dtype=np.uint32)
    n = rid.size
    mh = np.zeros(max(n, 1), np.uint32)
    bt = np.zeros(max(n, 1), np.int32)
    pad = [a if a.size else np.zeros(1, a.dtype) for a in (rid, beg, wl)]
    rc = L.orc_rescue(_p(ref), ref.size, int(bisulfite), _p(seq), _p(offsets), offsets.size - 1, _p(pad[0]),
                      _p(pad[1]), _p(pad[2]), n, int(q), int(role), _p(mh), _p(bt), int(threads))
    if rc != 0:
        raise ValueError("rescue candidate out of range")
    return mh[:n], bt[:n]


CHAIN_DTYPE = np.dtype([("read_id", "<u4"), ("score", "<i4"), ("n_anchors", "<u4"), ("copy", "<u4"),
                        ("anchor_off", "<u8")])
ANCHOR_DTYPE = np.dtype([("qbeg", "<u4"), ("qend", "<u4"), ("pos", "<u8")])


def chain_dp(x, y, w, g, max_gap: int = 5000, max_pred: int = 50):
    """f and predecessor p (-1: none) of anchors already in chaining order (x, y, w ascending)."""
    L = _load()
    x = np.ascontiguousarray(x, dtype=np.uint64)
    y = np.ascontiguousarray(y, dtype=np.uint32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    g = np.ascontiguousarray(g, dtype=np.uint32)
    n = x.size
    f = np.zeros(max(n, 1), np.int32)
    p = np.zeros(max(n, 1), np.int64)
    pad = [a if a.size else np.zeros(1, a.dtype) for a in (x, y, w, g)]
    L.orc_chain_dp(*[_p(a) for a in pad], n, int(max_gap), int(max_pred), _p(f), _p(p))
    return f[:n], p[:n]


def chain(res: SeedResult, seg_len: int, max_gap: int = 5000, max_pred: int = 50, max_chains: int = 50,
          min_score: int = 19):
    """Chains (Section 2.6) of every read of a seeding result whose seeds are sorted by read:
    (CHAIN_DTYPE records in read and rank order, ANCHOR_DTYPE records of the chains' anchors, each
    chain's anchors ascending).  ``seg_len`` is the length of one copy of the reference in T (|R|)."""
    L = _load()
    arrs = [np.ascontiguousarray(a) if a.size else np.zeros(1, a.dtype) for a in
            (res.read_id, res.qbeg, res.qend, res.pos_off, res.npos)]
    pos = np.ascontiguousarray(res.pos) if res.pos.size else np.zeros(1, np.uint64)
    o = _ChainOpts(int(max_gap), int(max_pred), int(max_chains), int(min_score))
    ptrs = [C.c_void_p() for _ in range(8)]
    na = C.c_uint64()
    nc = L.orc_chain(*[_p(a) for a in arrs], len(res), _p(pos), int(seg_len), C.byref(o), *[C.byref(q) for q in ptrs],
                     C.byref(na))
    na = na.value
    chains = np.zeros(nc, CHAIN_DTYPE)
    anchors = np.zeros(na, ANCHOR_DTYPE)
    def take(q, ctype, n):
        return np.ctypeslib.as_array(C.cast(q, C.POINTER(ctype)), shape=(n,)).copy() if n else None

    if nc:
        for name, q, ct in (("read_id", ptrs[0], C.c_uint32), ("score", ptrs[1], C.c_int32),
                            ("n_anchors", ptrs[2], C.c_uint32), ("copy", ptrs[3], C.c_uint32),
                            ("anchor_off", ptrs[4], C.c_uint64)):
            chains[name] = take(q, ct, nc)
    if na:
        for name, q, ct in (("qbeg", ptrs[5], C.c_uint32), ("qend", ptrs[6], C.c_uint32), ("pos", ptrs[7], C.c_uint64)):
            anchors[name] = take(q, ct, na)
    for q in ptrs:
        L.orc_free_ptr(q)
    return chains, anchors


# ---- reference text from ASCII (Section 2.1: bases other than A, C, G, T become random bases) ----
_SM_GAMMA = 0x9E3779B97F4A7C15
_SM_MASK = (1 << 64) - 1


def splitmix64(seed: int, n: int) -> np.ndarray:
    """The first n outputs of SplitMix64 (Steele, Lea and Flood, 2014) with state `seed`: the state
    advances by the golden-ratio increment 0x9E3779B97F4A7C15, and each output is the state after
    the step through the variant-13 mixer (xor-shift 30, multiply, xor-shift 27, multiply,
    xor-shift 31)."""
    with np.errstate(over="ignore"):
        z = (np.uint64(seed & _SM_MASK) + np.arange(1, n + 1, dtype=np.uint64) * np.uint64(_SM_GAMMA))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def codes_from_ascii(ref: bytes | np.ndarray, rng_seed: int = 0) -> np.ndarray:
    """Reference codes 0..3 from ASCII: A, C, G, T in either case are 0, 1, 2, 3; any other byte at
    position i becomes the low two bits of output i of SplitMix64 seeded with rng_seed (the reading
    S5 of the random replacement)."""
    a = np.frombuffer(bytes(ref), np.uint8) if not isinstance(ref, np.ndarray) else ref.astype(np.uint8)
    table = np.full(256, 255, np.uint8)
    for ch, v in zip(b"ACGT", range(4)):
        table[ch] = v
        table[ch + 32] = v
    codes = table[a]
    amb = np.nonzero(codes == 255)[0]
    if amb.size:
        draws = splitmix64(rng_seed, int(amb.max()) + 1)
        codes[amb] = (draws[amb] & np.uint64(3)).astype(np.uint8)
    return codes
