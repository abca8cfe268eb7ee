"""Python binding of the mbw C-ABI (``include/mbw.h``): argument marshalling only.

Every step of index construction and seeding runs in the HIP library ``libmbw.so`` built for
gfx950; this module only loads it and moves arguments across the boundary.  If the library is
missing it raises instead of computing anything itself.

PyTorch is optional plumbing: reads may be passed as torch CUDA tensors (device pointers are
handed to the library) and ``stream`` may be a ``torch.cuda.Stream``.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
import hashlib
import json
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbw.so")

MBW_OK = 0
MBW_E_INVAL = -1
MBW_E_NOMEM = -2
MBW_E_HIP = -3
MBW_E_IO = -4
MBW_E_FORMAT = -5
MBW_E_CAPACITY = -6
MBW_E_BUSY = -7

KERNEL_COOP = 0
KERNEL_PLAIN = 1
SEED_UNLOCATED = 1
SEED_ROUND2 = 2

# the symbols include/mbw.h declares
EXPORTS = ["mbw_strerror", "mbw_last_error", "mbw_index_build", "mbw_index_save", "mbw_index_load",
           "mbw_index_free", "mbw_index_info", "mbw_index_device_arrays", "mbw_index_superblock_table", "mbw_index_build_fasta", "mbw_index_contigs", "mbw_index_contig", "mbw_ref_to_contig", "mbw_ctx_create", "mbw_ctx_free",
           "mbw_seed", "mbw_result_download", "mbw_pos_to_ref", "mbw_tune",
           "mbw_result_download_pieces", "mbw_serve_open", "mbw_serve_submit", "mbw_serve_submit_nocopy", "mbw_serve_wait", "mbw_serve_release", "mbw_serve_stats",
           "mbw_serve_close", "mbw_rescue_filter", "mbw_rescue_download", "mbw_debug_set_mem_limit", "mbw_chain",
           "mbw_chain_download", "mbw_seed_into", "mbw_seed_static", "mbw_graph_create", "mbw_graph_info",
           "mbw_graph_seed", "mbw_graph_free"]


class MbwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mbw error {code}: {msg}")
        self.code = code


class BuildOpts(C.Structure):
    _fields_ = [("sa_sample", C.c_int), ("kmer_k", C.c_int), ("bisulfite", C.c_int), ("ref_is_codes", C.c_int),
                ("rng_seed", C.c_uint64), ("device", C.c_int), ("isa_sample", C.c_int), ("sb_lines_log2", C.c_int)]


class IndexInfo(C.Structure):
    _fields_ = [("n", C.c_uint64), ("len_r", C.c_uint64), ("primary", C.c_uint64), ("n_lines", C.c_uint64),
                ("bytes_resident", C.c_uint64), ("C", C.c_uint64 * 5), ("bases_per_line", C.c_int),
                ("line_bytes", C.c_int), ("sa_sample", C.c_int), ("kmer_k", C.c_int), ("bisulfite", C.c_int),
                ("device", C.c_int), ("isa_sample", C.c_int), ("sb_lines_log2", C.c_int), ("n_superblocks", C.c_int)]


class GraphPlan(C.Structure):
    _fields_ = [("max_reads", C.c_uint64), ("max_bases", C.c_uint64), ("max_seeds", C.c_uint64),
                ("max_subqueries", C.c_uint64), ("max_positions", C.c_uint64), ("max_read_len", C.c_uint64),
                ("max_pieces", C.c_uint64)]


class SeedOpts(C.Structure):
    _fields_ = [("min_occ", C.c_int), ("reseed", C.c_int), ("reseed_len", C.c_int), ("reseed_occ", C.c_int),
                ("bs_role", C.c_int), ("kernel", C.c_int), ("use_kmer", C.c_int), ("blocks_per_cu", C.c_int),
                ("no_stage", C.c_int), ("unique_ext", C.c_int), ("seg_len", C.c_int), ("bs_refine", C.c_int),
                ("wave_chunk", C.c_int), ("unique_defer", C.c_int)]


class ServeCfg(C.Structure):
    _fields_ = [("n_workers", C.c_int), ("max_batch_reads", C.c_uint64), ("max_batch_bases", C.c_uint64),
                ("max_queued_bases", C.c_uint64), ("min_seed_len", C.c_int), ("max_occ", C.c_int),
                ("opts", SeedOpts), ("device", C.c_int), ("device_bytes", C.c_uint64)]


class ServeResult(C.Structure):
    _fields_ = [("n_seeds", C.c_uint64), ("n_pos", C.c_uint64), ("seeds", C.c_void_p), ("pos", C.c_void_p),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("batch_id", C.c_uint64), ("batch_reads", C.c_uint64), ("n_pieces", C.c_uint64),
                ("pieces", C.c_void_p), ("attempts", C.c_uint32), ("reserved", C.c_uint32)]


class ServeStats(C.Structure):
    _fields_ = [("batches", C.c_uint64), ("batch_reads", C.c_uint64), ("queued", C.c_uint64),
                ("split_retries", C.c_uint64), ("failed_requests", C.c_uint64), ("device_bytes", C.c_uint64),
                ("workspace_bytes", C.c_uint64), ("seeds_cap", C.c_uint64), ("pos_cap", C.c_uint64),
                ("pieces_cap", C.c_uint64)]


class RescueOpts(C.Structure):
    _fields_ = [("q", C.c_int), ("min_hits", C.c_int), ("bs_role", C.c_int)]


class RescueResult(C.Structure):
    _fields_ = [("n_cands", C.c_uint64), ("n_pass", C.c_uint64), ("hits", C.c_void_p), ("pass_", C.c_void_p),
                ("ms_kernel", C.c_float), ("ms_total", C.c_float)]


class SeedBuffers(C.Structure):
    _fields_ = [("workspace", C.c_void_p), ("workspace_bytes", C.c_uint64), ("seeds", C.c_void_p),
                ("seeds_cap", C.c_uint64), ("pos", C.c_void_p), ("pos_cap", C.c_uint64), ("pieces", C.c_void_p),
                ("pieces_cap", C.c_uint64), ("workspace_needed", C.c_uint64), ("seeds_needed", C.c_uint64),
                ("pos_needed", C.c_uint64), ("pieces_needed", C.c_uint64)]


class ChainOpts(C.Structure):
    _fields_ = [("max_gap", C.c_int), ("max_pred", C.c_int), ("max_chains", C.c_int), ("min_score", C.c_int)]


class ChainResult(C.Structure):
    _fields_ = [("n_chains", C.c_uint64), ("n_anchors", C.c_uint64), ("n_input_anchors", C.c_uint64),
                ("chains", C.c_void_p), ("anchors", C.c_void_p), ("ms_kernel", C.c_float), ("ms_total", C.c_float),
                ("max_read_anchors", C.c_uint64), ("reads_over_lds", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [("n_seeds", C.c_uint64), ("n_pos", C.c_uint64), ("seeds", C.c_void_p), ("pos", C.c_void_p),
                ("lines_smem", C.c_uint64), ("lines_locate", C.c_uint64), ("steps", C.c_uint64),
                ("lf_steps", C.c_uint64), ("ms_smem", C.c_float), ("ms_locate", C.c_float), ("ms_total", C.c_float),
                ("n_smem_launches", C.c_int), ("wave_iters", C.c_uint64), ("lane_iters", C.c_uint64),
                ("max_chain", C.c_uint64), ("n_pieces", C.c_uint64), ("pieces", C.c_void_p)]


SEED_DTYPE = np.dtype([("read_id", "<u4"), ("qbeg", "<u4"), ("qend", "<u4"), ("flags", "<u4"), ("k", "<u8"),
                       ("kr", "<u8"), ("s", "<u8"), ("pos_off", "<u8"), ("npos", "<u4"), ("reserved", "<u4")])
assert SEED_DTYPE.itemsize == 56
PIECE_DTYPE = np.dtype([("read_id", "<u4"), ("qbeg", "<u4"), ("qend", "<u4"), ("seed", "<u4"), ("pos", "<u8")])
RESCUE_CAND_DTYPE = np.dtype([("read_id", "<u4"), ("win_len", "<u4"), ("win_beg", "<u8")])
RESCUE_HIT_DTYPE = np.dtype([("max_hits", "<u4"), ("best_t", "<i4")])
CHAIN_DTYPE = np.dtype([("read_id", "<u4"), ("n_anchors", "<u4"), ("score", "<i4"), ("copy", "<u4"),
                        ("anchor_off", "<u8")])
ANCHOR_DTYPE = np.dtype([("qbeg", "<u4"), ("qend", "<u4"), ("pos", "<u8")])

_lib = None


def load_library():
    """Load libmbw.so; raises if it has not been built (no fallback of any kind)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_15357_amd.build` "
                          "(or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, u64, i32 = C.c_void_p, C.c_uint64, C.c_int
    L.mbw_strerror.restype = C.c_char_p
    L.mbw_strerror.argtypes = [i32]
    L.mbw_last_error.restype = C.c_char_p
    L.mbw_last_error.argtypes = []
    L.mbw_index_build.argtypes = [vp, u64, C.POINTER(BuildOpts), C.POINTER(vp)]
    L.mbw_index_save.argtypes = [vp, C.c_char_p]
    L.mbw_index_load.argtypes = [C.c_char_p, i32, C.POINTER(vp)]
    L.mbw_index_free.argtypes = [vp]
    L.mbw_index_free.restype = None
    L.mbw_index_info.argtypes = [vp, C.POINTER(IndexInfo)]
    L.mbw_index_device_arrays.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
    L.mbw_index_superblock_table.argtypes = [vp, C.POINTER(vp)]
    L.mbw_index_build_fasta.argtypes = [C.c_char_p, C.POINTER(BuildOpts), C.POINTER(vp)]
    L.mbw_index_contigs.argtypes = [vp, C.POINTER(C.c_uint64)]
    L.mbw_index_contig.argtypes = [vp, u64, C.POINTER(C.c_char_p), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    L.mbw_ref_to_contig.argtypes = [vp, u64, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    L.mbw_ctx_create.argtypes = [vp, C.POINTER(vp)]
    L.mbw_ctx_free.argtypes = [vp]
    L.mbw_ctx_free.restype = None
    L.mbw_seed.argtypes = [vp, vp, vp, u64, i32, i32, C.POINTER(SeedOpts), vp, C.POINTER(Result)]
    L.mbw_seed_into.argtypes = [vp, vp, vp, u64, i32, i32, C.POINTER(SeedOpts), vp, C.POINTER(SeedBuffers),
                                C.POINTER(Result)]
    L.mbw_seed_static.argtypes = L.mbw_seed_into.argtypes
    L.mbw_result_download.argtypes = [vp, C.POINTER(Result), vp, vp]
    L.mbw_result_download_pieces.argtypes = [vp, C.POINTER(Result), vp]
    L.mbw_pos_to_ref.argtypes = [vp, u64, C.c_uint32, C.POINTER(C.c_int), C.POINTER(C.c_uint64)]
    L.mbw_tune.argtypes = [vp, vp, vp, u64, i32, i32, C.POINTER(SeedOpts), vp, C.POINTER(SeedOpts), C.POINTER(C.c_float)]
    L.mbw_serve_open.argtypes = [vp, C.POINTER(ServeCfg), C.POINTER(vp)]
    L.mbw_serve_submit.argtypes = [vp, vp, vp, u64, C.POINTER(C.c_uint64)]
    L.mbw_serve_submit_nocopy.argtypes = [vp, vp, vp, u64, C.POINTER(C.c_uint64)]
    L.mbw_serve_wait.argtypes = [vp, u64, i32, C.POINTER(ServeResult)]
    L.mbw_serve_release.argtypes = [vp, u64]
    L.mbw_serve_stats.argtypes = [vp, C.POINTER(ServeStats)]
    L.mbw_serve_close.argtypes = [vp]
    L.mbw_serve_close.restype = None
    L.mbw_rescue_filter.argtypes = [vp, vp, vp, u64, vp, u64, C.POINTER(RescueOpts), vp, C.POINTER(RescueResult)]
    L.mbw_rescue_download.argtypes = [vp, C.POINTER(RescueResult), vp, vp]
    L.mbw_debug_set_mem_limit.argtypes = [u64]
    L.mbw_chain.argtypes = [vp, C.POINTER(Result), u64, C.POINTER(ChainOpts), vp, C.POINTER(ChainResult)]
    L.mbw_chain_download.argtypes = [vp, C.POINTER(ChainResult), vp, vp]
    L.mbw_graph_create.argtypes = [vp, C.POINTER(GraphPlan), i32, i32, C.POINTER(SeedOpts), C.POINTER(vp)]
    L.mbw_graph_info.argtypes = [vp, C.POINTER(GraphPlan)]
    L.mbw_graph_seed.argtypes = [vp, vp, vp, u64, vp, C.POINTER(Result)]
    L.mbw_graph_free.argtypes = [vp]
    L.mbw_graph_free.restype = None
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


_lib_id = None


def _library_id() -> str:
    """Hash of the built library file (tuner cache entries of another build do not apply)."""
    global _lib_id
    if _lib_id is None:
        h = hashlib.sha1()
        with open(LIB_PATH, "rb") as fh:
            for chunk in iter(lambda: fh.read(1 << 20), b""):
                h.update(chunk)
        _lib_id = h.hexdigest()[:16]
    return _lib_id


def _read_json(path: str) -> dict:
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _check(rc):
    if rc != MBW_OK:
        msg = _lib.mbw_last_error().decode(errors="replace")
        raise MbwError(rc, msg or _lib.mbw_strerror(rc).decode())


def _ptr(x):
    """Address of a numpy array, torch tensor or raw int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    raise TypeError(type(x))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Index:
    """A resident FM-index (``mbw_index``)."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle) if isinstance(handle, int) else handle
        self._lib = load_library()

    @classmethod
    def build(cls, ref, sa_sample: int = 8, kmer_k: int = 10, bisulfite: bool = False, device: int = 0,
              rng_seed: int = 0, isa_sample: int = 4, sb_lines_log2: int = 0):
        """``ref``: numpy uint8 codes 0..3 or ASCII bytes / str.  ``isa_sample`` > 0 also keeps the
        packed text and inverse-SA samples for direct extension of unique matches.
        ``sb_lines_log2``: occurrence lines per superblock as a power of two (0 = 2^23)."""
        L = load_library()
        if isinstance(ref, str):
            ref = ref.encode()
        if isinstance(ref, (bytes, bytearray)):
            arr = np.frombuffer(bytes(ref), dtype=np.uint8)
            codes = 0
        else:
            arr = np.ascontiguousarray(ref, dtype=np.uint8)
            codes = 1
        o = BuildOpts(int(sa_sample), int(kmer_k), int(bool(bisulfite)), codes, int(rng_seed), int(device),
                      int(isa_sample), int(sb_lines_log2))
        h = C.c_void_p()
        _check(L.mbw_index_build(arr.ctypes.data if arr.size else None, arr.size, C.byref(o), C.byref(h)))
        return cls(h)

    @classmethod
    def build_fasta(cls, path: str, sa_sample: int = 8, kmer_k: int = 10, bisulfite: bool = False, device: int = 0,
                    rng_seed: int = 0, isa_sample: int = 4, sb_lines_log2: int = 0):
        """Build from a FASTA file (records back to back; see ``contigs``)."""
        L = load_library()
        o = BuildOpts(int(sa_sample), int(kmer_k), int(bool(bisulfite)), 0, int(rng_seed), int(device),
                      int(isa_sample), int(sb_lines_log2))
        h = C.c_void_p()
        _check(L.mbw_index_build_fasta(path.encode(), C.byref(o), C.byref(h)))
        return cls(h)

    def contigs(self):
        """[(name, start, length)] of the reference's records, start and length in R."""
        n = C.c_uint64()
        _check(self._lib.mbw_index_contigs(self._h, C.byref(n)))
        out = []
        for i in range(n.value):
            nm, st, ln = C.c_char_p(), C.c_uint64(), C.c_uint64()
            _check(self._lib.mbw_index_contig(self._h, i, C.byref(nm), C.byref(st), C.byref(ln)))
            out.append((nm.value.decode(errors="replace"), st.value, ln.value))
        return out

    def ref_to_contig(self, ref_pos: int):
        """(record index, offset in it) of a position of R."""
        c, o = C.c_uint64(), C.c_uint64()
        _check(self._lib.mbw_ref_to_contig(self._h, int(ref_pos), C.byref(c), C.byref(o)))
        return c.value, o.value

    @classmethod
    def load(cls, path: str, device: int = 0):
        L = load_library()
        h = C.c_void_p()
        _check(L.mbw_index_load(path.encode(), int(device), C.byref(h)))
        return cls(h)

    def save(self, path: str):
        _check(self._lib.mbw_index_save(self._h, path.encode()))

    def info(self) -> dict:
        i = IndexInfo()
        _check(self._lib.mbw_index_info(self._h, C.byref(i)))
        d = {f: getattr(i, f) for f, _ in IndexInfo._fields_}
        d["C"] = list(i.C)
        return d

    def device_arrays(self):
        a, b, c = C.c_void_p(), C.c_void_p(), C.c_void_p()
        _check(self._lib.mbw_index_device_arrays(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def superblock_table(self):
        """Device pointer to the superblock table (n_superblocks x 8 u64)."""
        a = C.c_void_p()
        _check(self._lib.mbw_index_superblock_table(self._h, C.byref(a)))
        return a.value

    def pos_to_ref(self, pos: int, length: int):
        s, p = C.c_int(), C.c_uint64()
        _check(self._lib.mbw_pos_to_ref(self._h, int(pos), int(length), C.byref(s), C.byref(p)))
        return s.value, p.value

    def free(self):
        if self._h:
            self._lib.mbw_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


@dataclass
class SeedOutput:
    n_seeds: int
    n_pos: int
    seeds_ptr: int
    pos_ptr: int
    lines_smem: int
    lines_locate: int
    steps: int
    lf_steps: int
    ms_smem: float
    ms_locate: float
    ms_total: float
    n_smem_launches: int
    wave_iters: int
    lane_iters: int
    max_chain: int
    _res: Result
    _ctx: "Context"

    def download_pieces(self):
        """Refined bisulfite pieces (PIECE_DTYPE) on the host (``bs_refine=True``)."""
        n = int(self._res.n_pieces)
        out = np.zeros(n, dtype=PIECE_DTYPE)
        _check(self._ctx._lib.mbw_result_download_pieces(self._ctx._h, C.byref(self._res), out.ctypes.data if n else None))
        return out

    def download(self):
        """(seeds structured array, positions uint64 array) on the host."""
        seeds = np.zeros(self.n_seeds, dtype=SEED_DTYPE)
        pos = np.zeros(self.n_pos, dtype=np.uint64)
        _check(self._ctx._lib.mbw_result_download(self._ctx._h, C.byref(self._res),
                                                  seeds.ctypes.data if self.n_seeds else None,
                                                  pos.ctypes.data if self.n_pos else None))
        return seeds, pos


@dataclass
class ChainOutput:
    n_chains: int
    n_anchors: int
    n_input_anchors: int
    ms_kernel: float
    ms_total: float
    max_read_anchors: int
    reads_over_lds: int
    _res: ChainResult
    _ctx: "Context"

    def download(self):
        """(chains as CHAIN_DTYPE records by read and rank, their anchors as ANCHOR_DTYPE) on the host."""
        chains = np.zeros(self.n_chains, dtype=CHAIN_DTYPE)
        anchors = np.zeros(self.n_anchors, dtype=ANCHOR_DTYPE)
        _check(self._ctx._lib.mbw_chain_download(self._ctx._h, C.byref(self._res),
                                                 chains.ctypes.data if self.n_chains else None,
                                                 anchors.ctypes.data if self.n_anchors else None))
        return chains, anchors


@dataclass
class RescueOutput:
    n_cands: int
    n_pass: int
    hits_ptr: int
    pass_ptr: int
    ms_kernel: float
    ms_total: float
    _res: RescueResult
    _ctx: "Context"

    def download(self):
        """(hits as RESCUE_HIT_DTYPE records, passing candidate indices as uint32) on the host."""
        hits = np.zeros(self.n_cands, dtype=RESCUE_HIT_DTYPE)
        passed = np.zeros(self.n_pass, dtype=np.uint32)
        _check(self._ctx._lib.mbw_rescue_download(self._ctx._h, C.byref(self._res),
                                                  hits.ctypes.data if self.n_cands else None,
                                                  passed.ctypes.data if self.n_pass else None))
        return hits, passed


class Graph:
    """A captured seeding graph (``mbw_graph_*``) of a context; results point into its buffers until
    its next call."""

    def __init__(self, ctx, h):
        self._ctx = ctx
        self._lib = ctx._lib
        self._h = h

    def plan(self) -> dict:
        p = GraphPlan()
        _check(self._lib.mbw_graph_info(self._h, C.byref(p)))
        return {f: int(getattr(p, f)) for f, _ in GraphPlan._fields_}

    def seed(self, reads, lengths, stream=None) -> "SeedOutput":
        if not self._h:
            raise MbwError(MBW_E_INVAL, "graph already freed")
        n = int(lengths.numel() if hasattr(lengths, "numel") else len(lengths))
        if isinstance(lengths, np.ndarray):
            lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
        if isinstance(reads, np.ndarray):
            reads = np.ascontiguousarray(reads, dtype=np.uint8)
        res = Result()
        _check(self._lib.mbw_graph_seed(self._h, _ptr(reads) if n else None, _ptr(lengths) if n else None, n,
                                        _stream_handle(stream), C.byref(res)))
        return SeedOutput(res.n_seeds, res.n_pos, res.seeds or 0, res.pos or 0, res.lines_smem, res.lines_locate,
                          res.steps, res.lf_steps, res.ms_smem, res.ms_locate, res.ms_total, res.n_smem_launches,
                          res.wave_iters, res.lane_iters, res.max_chain, res, self._ctx)

    def free(self):
        if self._h:
            self._lib.mbw_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Context:
    """Work space for a stream of ``mbw_seed`` / ``mbw_rescue_filter`` calls against one index."""

    def __init__(self, index: Index):
        self._lib = load_library()
        self.index = index
        h = C.c_void_p()
        _check(self._lib.mbw_ctx_create(index._h, C.byref(h)))
        self._h = h
        self._graphs = weakref.WeakSet()   # graphs of this context: freed before it

    def seed(self, reads, lengths, min_seed_len: int = 19, max_occ: int = 500, min_occ: int = 1,
             reseed: bool = True, reseed_len: int = 38, reseed_occ: int = 10, bs_role: int = 0,
             kernel: int = KERNEL_COOP, use_kmer: bool = True, blocks_per_cu: int = 0, stage: bool = True,
             unique_ext: bool = True, seg_len: int = 0, bs_refine: bool = False, wave_chunk: int = 0,
             unique_defer: int = 0, stream=None) -> SeedOutput:
        """``reads``: concatenated ASCII (numpy uint8 on the host or a torch uint8 CUDA tensor);
        ``lengths``: uint32 per read (numpy or torch)."""
        n = int(lengths.numel() if hasattr(lengths, "numel") else len(lengths))
        if isinstance(lengths, np.ndarray):
            lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
        if isinstance(reads, np.ndarray):
            reads = np.ascontiguousarray(reads, dtype=np.uint8)
        o = SeedOpts(int(min_occ), int(bool(reseed)), int(reseed_len), int(reseed_occ), int(bs_role), int(kernel),
                     int(bool(use_kmer)), int(blocks_per_cu), int(not stage), int(bool(unique_ext)), int(seg_len),
                     int(bool(bs_refine)), int(wave_chunk), int(unique_defer))
        res = Result()
        rp = _ptr(reads) if n else None
        lp = _ptr(lengths) if n else None
        _check(self._lib.mbw_seed(self._h, rp, lp, n, int(min_seed_len), int(max_occ), C.byref(o),
                                  _stream_handle(stream), C.byref(res)))
        return SeedOutput(res.n_seeds, res.n_pos, res.seeds or 0, res.pos or 0, res.lines_smem, res.lines_locate,
                          res.steps, res.lf_steps, res.ms_smem, res.ms_locate, res.ms_total, res.n_smem_launches,
                          res.wave_iters, res.lane_iters, res.max_chain, res, self)

    def seed_into(self, reads, lengths, workspace, seeds, pos, pieces=None, min_seed_len: int = 19, max_occ: int = 500,
                  stream=None, entry: str = "mbw_seed_into", **kw):
        """``mbw_seed_into``: the same result as :meth:`seed` in caller-owned device buffers (torch
        uint8 tensors, or (pointer, bytes) pairs): ``workspace`` for every temporary, ``seeds``
        (56-byte records), ``pos`` (uint64), ``pieces`` (24-byte records, bisulfite refinement).
        Returns (SeedOutput, SeedBuffers with the ``*_needed`` sizes); an MbwError with code
        MBW_E_CAPACITY carries the buffers as ``.buffers``."""
        def span(x, item):
            if x is None:
                return None, 0
            if isinstance(x, tuple):
                return x[0], x[1] // item
            return x.data_ptr(), x.numel() * x.element_size() // item
        n = int(lengths.numel() if hasattr(lengths, "numel") else len(lengths))
        if isinstance(lengths, np.ndarray):
            lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
        if isinstance(reads, np.ndarray):
            reads = np.ascontiguousarray(reads, dtype=np.uint8)
        o = self._opts(kw)
        wp, wb = span(workspace, 1)
        sp, sc = span(seeds, SEED_DTYPE.itemsize)
        pp, pc = span(pos, 8)
        qp, qc = span(pieces, PIECE_DTYPE.itemsize)
        b = SeedBuffers(wp, wb, sp, sc, pp, pc, qp, qc, 0, 0, 0, 0)
        res = Result()
        rc = getattr(self._lib, entry)(self._h, _ptr(reads) if n else None, _ptr(lengths) if n else None, n,
                                       int(min_seed_len), int(max_occ), C.byref(o), _stream_handle(stream), C.byref(b),
                                       C.byref(res))
        if rc != MBW_OK:
            err = MbwError(rc, self._lib.mbw_last_error().decode(errors="replace"))
            err.buffers = b
            raise err
        return (SeedOutput(res.n_seeds, res.n_pos, res.seeds or 0, res.pos or 0, res.lines_smem, res.lines_locate,
                           res.steps, res.lf_steps, res.ms_smem, res.ms_locate, res.ms_total, res.n_smem_launches,
                           res.wave_iters, res.lane_iters, res.max_chain, res, self), b)

    def seed_static(self, reads, lengths, seeds, pos, pieces=None, min_seed_len: int = 19, max_occ: int = 500,
                    stream=None, **kw):
        """``mbw_seed_static``: :meth:`seed_into` on the library's static device work space (no
        allocation); ``reads`` and ``lengths`` must be device tensors."""
        return self.seed_into(reads, lengths, None, seeds, pos, pieces, min_seed_len=min_seed_len, max_occ=max_occ,
                              stream=stream, entry="mbw_seed_static", **kw)

    @staticmethod
    def _opts(kw):
        return SeedOpts(int(kw.get("min_occ", 1)), int(bool(kw.get("reseed", True))), int(kw.get("reseed_len", 38)),
                        int(kw.get("reseed_occ", 10)), int(kw.get("bs_role", 0)), int(kw.get("kernel", KERNEL_COOP)),
                        int(bool(kw.get("use_kmer", True))), int(kw.get("blocks_per_cu", 0)),
                        int(not kw.get("stage", True)), int(bool(kw.get("unique_ext", True))), int(kw.get("seg_len", 0)),
                        int(bool(kw.get("bs_refine", False))), int(kw.get("wave_chunk", 0)),
                        int(kw.get("unique_defer", 0)))

    def rescue(self, reads, lengths, cands, q: int = 7, min_hits: int = 10, bs_role: int = 0,
               stream=None) -> RescueOutput:
        """Mate-rescue prefilter (``mbw_rescue_filter``).  ``cands``: RESCUE_CAND_DTYPE records on
        the host, or a torch uint8/int64 CUDA tensor holding them (16 bytes each)."""
        n = int(lengths.numel() if hasattr(lengths, "numel") else len(lengths))
        if isinstance(lengths, np.ndarray):
            lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
        if isinstance(reads, np.ndarray):
            reads = np.ascontiguousarray(reads, dtype=np.uint8)
        if isinstance(cands, np.ndarray):
            cands = np.ascontiguousarray(cands)
            if cands.dtype != RESCUE_CAND_DTYPE:
                raise TypeError("candidates must be RESCUE_CAND_DTYPE records")
            nc = cands.size
        else:
            nc = cands.numel() * cands.element_size() // RESCUE_CAND_DTYPE.itemsize
        o = RescueOpts(int(q), int(min_hits), int(bs_role))
        res = RescueResult()
        _check(self._lib.mbw_rescue_filter(self._h, _ptr(reads) if n else None, _ptr(lengths) if n else None, n,
                                           _ptr(cands) if nc else None, nc, C.byref(o), _stream_handle(stream),
                                           C.byref(res)))
        return RescueOutput(res.n_cands, res.n_pass, res.hits or 0, res.pass_ or 0, res.ms_kernel, res.ms_total,
                            res, self)

    def chain(self, seeds: SeedOutput, n_reads: int, max_gap: int = 5000, max_pred: int = 50, max_chains: int = 50,
              min_score: int = 19, stream=None) -> ChainOutput:
        """Chains of the located seeds of a seeding result of this context (``mbw_chain``)."""
        o = ChainOpts(int(max_gap), int(max_pred), int(max_chains), int(min_score))
        res = ChainResult()
        _check(self._lib.mbw_chain(self._h, C.byref(seeds._res), int(n_reads), C.byref(o), _stream_handle(stream),
                                   C.byref(res)))
        return ChainOutput(res.n_chains, res.n_anchors, res.n_input_anchors, res.ms_kernel, res.ms_total,
                           res.max_read_anchors, res.reads_over_lds, res, self)

    def graph(self, max_reads: int, max_bases: int = 0, max_seeds: int = 0, max_subqueries: int = 0,
              max_positions: int = 0, max_read_len: int = 0, max_pieces: int = 0, min_seed_len: int = 19,
              max_occ: int = 500, **kw) -> "Graph":
        """``mbw_graph_create``: the seeding path captured once as a HIP graph for batches of at most
        ``max_reads`` reads of at most ``max_read_len`` bases (0: 160; options as for :meth:`seed`)."""
        plan = GraphPlan(int(max_reads), int(max_bases), int(max_seeds), int(max_subqueries), int(max_positions),
                         int(max_read_len), int(max_pieces))
        h = C.c_void_p()
        _check(self._lib.mbw_graph_create(self._h, C.byref(plan), int(min_seed_len), int(max_occ),
                                          C.byref(self._opts(kw)), C.byref(h)))
        g = Graph(self, h)
        self._graphs.add(g)
        return g

    def tune(self, reads, lengths, min_seed_len: int = 19, max_occ: int = 500, stream=None, cache=None,
             **base) -> dict:
        """Time candidate schedules on this batch (``mbw_tune``); returns the fastest as keyword
        arguments for :meth:`seed` plus ``ms`` (its device time).  With ``cache`` (a JSON file
        path) the pick is stored under a key made of the library build, the index parameters, the
        seeding parameters and a coarse profile of the batch's read lengths (log2 buckets of the
        median and the longest read); a later call with the same key returns the stored pick
        without timing anything (``cached`` is then True)."""
        n = int(lengths.numel() if hasattr(lengths, "numel") else len(lengths))
        key = None
        if cache:
            key = self._tune_key(lengths, min_seed_len, max_occ, base)
            stored = _read_json(cache)
            if key in stored:
                return dict(stored[key], cached=True)
        b = SeedOpts(int(base.get("min_occ", 1)), int(bool(base.get("reseed", True))), int(base.get("reseed_len", 38)),
                     int(base.get("reseed_occ", 10)), int(base.get("bs_role", 0)), KERNEL_COOP,
                     int(bool(base.get("use_kmer", True))), 0, 0, 1, 0, 0)
        best = SeedOpts()
        ms = C.c_float()
        _check(self._lib.mbw_tune(self._h, _ptr(reads) if n else None, _ptr(lengths) if n else None, n,
                                  int(min_seed_len), int(max_occ), C.byref(b), _stream_handle(stream), C.byref(best),
                                  C.byref(ms)))
        res = dict(stage=not best.no_stage, seg_len=best.seg_len, blocks_per_cu=best.blocks_per_cu,
                   unique_ext=bool(best.unique_ext), wave_chunk=best.wave_chunk, ms=ms.value)
        if cache:
            stored = _read_json(cache)
            stored[key] = res
            tmp = f"{cache}.tmp{os.getpid()}"
            with open(tmp, "w") as fh:
                json.dump(stored, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(res, cached=False)

    def _tune_key(self, lengths, min_seed_len, max_occ, base) -> str:
        if hasattr(lengths, "cpu"):
            lengths = lengths.cpu().numpy()
        lens = np.asarray(lengths).astype(np.int64)
        med = int(np.median(lens)) if lens.size else 0
        mx = int(lens.max()) if lens.size else 0
        info = self.index.info()
        parts = [_library_id(), f"n={info['n']}", f"r={info['sa_sample']}", f"K={info['kmer_k']}",
                 f"ri={info['isa_sample']}", f"bs={info['bisulfite']}", f"l={min_seed_len}", f"max_occ={max_occ}",
                 "opts=" + ",".join(f"{k}={base[k]}" for k in sorted(base)),
                 f"median_log2={med.bit_length()}", f"max_log2={mx.bit_length()}"]
        return "|".join(parts)

    def free(self):
        if self._h:
            for g in list(self._graphs):   # a graph is freed before its context
                g.free()
            self._lib.mbw_ctx_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def set_mem_limit(nbytes: int) -> None:
    """Debug: cap the device work space of every context (0 = no cap); for allocation-failure
    tests."""
    _check(load_library().mbw_debug_set_mem_limit(int(nbytes)))


_probe = None


def _probe_library():
    """The measurement helper library (libmbw_probe.so, built beside libmbw.so)."""
    global _probe
    if _probe is None:
        path = os.path.join(HERE, "libmbw_probe.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_2606_15357_amd.build`")
        P = C.CDLL(path)
        P.mbwprobe_copy.argtypes = [C.c_int, C.c_uint64, C.POINTER(C.c_float)]
        P.mbwprobe_gather.argtypes = [C.c_int, C.c_uint64, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_float)]
        P.mbwprobe_last_error.restype = C.c_char_p
        _probe = P
    return _probe


def _probe_check(rc):
    if rc != 0:
        raise MbwError(rc, _probe_library().mbwprobe_last_error().decode(errors="replace"))


def probe_copy(nbytes: int = 1 << 30, device: int = 0) -> float:
    """Kernel time (ms) of one streaming copy of `nbytes` bytes (profiler counter calibration)."""
    ms = C.c_float()
    _probe_check(_probe_library().mbwprobe_copy(int(device), int(nbytes), C.byref(ms)))
    return ms.value


def probe_gather(nbytes: int = 16 << 30, iters: int = 64, waves_per_simd: int = 0, device: int = 0):
    """Random 128-byte lines served per second over a power-of-two buffer of at most `nbytes` (one
    lane per line, four dependent chains per lane); `waves_per_simd` 1..8 launches that many blocks
    of 256 threads per CU (0: 8,192 blocks), with the same number of fetches in every setting."""
    lps, ms = C.c_double(), C.c_float()
    _probe_check(_probe_library().mbwprobe_gather(int(device), int(nbytes), int(iters), int(waves_per_simd),
                                                  C.byref(lps), C.byref(ms)))
    return lps.value, ms.value


def canonical(seeds: np.ndarray, pos: np.ndarray):
    """Seeds in (read_id, qbeg, qend) order with each seed's positions sorted ascending, as flat
    arrays: (records without pos_off, concatenated positions)."""
    order = np.lexsort((seeds["qend"], seeds["qbeg"], seeds["read_id"]))
    s = seeds[order]
    chunks = [np.sort(pos[int(o):int(o) + int(c)]) for o, c in zip(s["pos_off"], s["npos"])]
    flat = np.concatenate(chunks) if chunks else np.zeros(0, np.uint64)
    return s, flat


def _view(ptr, n: int, dtype: np.dtype) -> np.ndarray:
    """A numpy array over n records at host address ptr (no copy)."""
    if not n or not ptr:
        return np.zeros(0, dtype=dtype)
    return np.frombuffer((C.c_char * (int(n) * dtype.itemsize)).from_address(ptr), dtype=dtype)


_live_servers = weakref.WeakSet()


@atexit.register
def _close_servers():
    """Servers still open when the interpreter exits are closed first (their workers finish the
    queued requests), so that no worker thread is left running while the process tears down."""
    for srv in list(_live_servers):
        try:
            srv.close()
        except Exception:
            pass


class Server:
    """Request loop over a resident index (``mbw_serve_*``): submit reads, wait for each
    request's seeds and positions; batches of several requests overlap on the device.  Each worker
    holds a fixed device arena (``device_bytes`` for all of them together; 0 = sized for a full
    batch); requests that can never fit one are refused with MBW_E_CAPACITY."""

    def __init__(self, index: Index, n_workers: int = 2, max_batch_reads: int = 1 << 18,
                 max_batch_bases: int = 1 << 26, max_queued_bases: int = 1 << 32, min_seed_len: int = 19,
                 max_occ: int = 500, device_bytes: int = 0, **opts):
        self._lib = load_library()
        self.index = index
        o = SeedOpts(int(opts.get("min_occ", 1)), int(bool(opts.get("reseed", True))), int(opts.get("reseed_len", 38)),
                     int(opts.get("reseed_occ", 10)), int(opts.get("bs_role", 0)), int(opts.get("kernel", KERNEL_COOP)),
                     int(bool(opts.get("use_kmer", True))), int(opts.get("blocks_per_cu", 0)),
                     int(not opts.get("stage", True)), int(bool(opts.get("unique_ext", True))), int(opts.get("seg_len", 0)),
                     int(bool(opts.get("bs_refine", False))), int(opts.get("wave_chunk", 0)),
                     int(opts.get("unique_defer", 0)))
        cfg = ServeCfg(int(n_workers), int(max_batch_reads), int(max_batch_bases), int(max_queued_bases),
                       int(min_seed_len), int(max_occ), o, int(index.info()["device"]), int(device_bytes))
        self._held = {}   # ticket -> arrays of a request submitted without a copy
        h = C.c_void_p()
        _check(self._lib.mbw_serve_open(index._h, C.byref(cfg), C.byref(h)))
        self._h = h
        _live_servers.add(self)

    def submit(self, reads: np.ndarray, lengths: np.ndarray, copy: bool = True):
        """Queue a request; returns its ticket, or None when the queue is full (MBW_E_BUSY).
        copy=False queues the arrays themselves (no host copy): they are kept referenced here and
        must not be modified until the request is waited for."""
        reads = np.ascontiguousarray(reads, dtype=np.uint8)
        lengths = np.ascontiguousarray(lengths, dtype=np.uint32)
        t = C.c_uint64()
        fn = self._lib.mbw_serve_submit if copy else self._lib.mbw_serve_submit_nocopy
        rc = fn(self._h, reads.ctypes.data if reads.size else None, lengths.ctypes.data if lengths.size else None,
                lengths.size, C.byref(t))
        if rc == MBW_E_BUSY:
            return None
        _check(rc)
        if not copy:
            self._held[t.value] = (reads, lengths)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1, release: bool = True, copy: bool = True):
        """(seeds, positions, info) of a request, or None if not finished within timeout_ms; info has
        the timing, the batch, the device batches tried and, for a bisulfite server with bs_refine,
        the refined pieces (PIECE_DTYPE, read_id and seed counted within the request).
        copy=False returns arrays over the server's pinned result buffer without copying; they stay
        valid until ``release(ticket)``, which the caller then must call (release is ignored)."""
        r = ServeResult()
        rc = self._lib.mbw_serve_wait(self._h, int(ticket), int(timeout_ms), C.byref(r))
        if rc == MBW_E_BUSY:
            return None
        self._held.pop(int(ticket), None)
        if rc != MBW_OK:
            err = MbwError(rc, self._lib.mbw_last_error().decode(errors="replace"))
            err.attempts = r.attempts
            if release:   # the request failed: free it and report
                self._lib.mbw_serve_release(self._h, int(ticket))
            raise err
        if copy:
            seeds = np.zeros(r.n_seeds, dtype=SEED_DTYPE)
            pos = np.zeros(r.n_pos, dtype=np.uint64)
            if r.n_seeds:
                C.memmove(seeds.ctypes.data, r.seeds, r.n_seeds * SEED_DTYPE.itemsize)
            if r.n_pos:
                C.memmove(pos.ctypes.data, r.pos, r.n_pos * 8)
            pieces = np.zeros(r.n_pieces, dtype=PIECE_DTYPE)
            if r.n_pieces:
                C.memmove(pieces.ctypes.data, r.pieces, r.n_pieces * PIECE_DTYPE.itemsize)
        else:
            seeds = _view(r.seeds, r.n_seeds, SEED_DTYPE)
            pos = _view(r.pos, r.n_pos, np.dtype(np.uint64))
            pieces = _view(r.pieces, r.n_pieces, PIECE_DTYPE)
        info = dict(t_submit=r.t_submit, t_start=r.t_start, t_done=r.t_done, batch_id=r.batch_id,
                    batch_reads=r.batch_reads, attempts=r.attempts, pieces=pieces)
        if release and copy:
            _check(self._lib.mbw_serve_release(self._h, int(ticket)))
        return seeds, pos, info

    def release(self, ticket: int):
        """Free a finished request (after wait(copy=False): its arrays become invalid)."""
        _check(self._lib.mbw_serve_release(self._h, int(ticket)))

    def stats(self):
        st = ServeStats()
        _check(self._lib.mbw_serve_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServeStats._fields_}

    def close(self):
        if self._h:
            self._lib.mbw_serve_close(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
