"""The C-ABI library loads and exports every entry point include/mbw.h declares (CPU only;
no compute call is made except the ones that fail before touching a GPU)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mbw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mbw_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("mbw_index_build", "mbw_index_load", "mbw_seed", "mbw_index_free", "mbw_ctx_create"):
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2606_15357_amd as mbw
    L = mbw.load_library()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(mbw.EXPORTS) == declared_functions()


def test_strerror_and_bad_file(tmp_path):
    import paper_2606_15357_amd as mbw
    L = mbw.load_library()
    assert L.mbw_strerror(mbw.MBW_E_FORMAT) == b"bad index file format"
    p = tmp_path / "bad.mbw"
    p.write_bytes(b"not an index" * 20)
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.load(str(p))
    assert e.value.code == mbw.MBW_E_FORMAT
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.load(str(tmp_path / "missing.mbw"))
    assert e.value.code == mbw.MBW_E_IO


def test_invalid_build_options():
    import paper_2606_15357_amd as mbw
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.build(np.zeros(10, np.uint8), sa_sample=0)
    assert e.value.code == mbw.MBW_E_INVAL
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.build(np.zeros(10, np.uint8), kmer_k=16)
    assert e.value.code == mbw.MBW_E_INVAL
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.build(np.zeros(10, np.uint8), kmer_k=-2)
    assert e.value.code == mbw.MBW_E_INVAL


def _header(n=1001, r=8, **over):
    """An index file header (the documented layout, version 7) with consistent fields and a valid
    header checksum, for a plain index of n rows without k-mer table, text or inverse-SA samples;
    `over` replaces named fields (the checksum is computed afterwards)."""
    from mbw_helpers import HEADER
    f = dict(n=n, len_r=(n - 1) // 2, primary=0, n_lines=n // 384 + 1, n_ssa=(n + r - 1) // r,
             C=[0, 1, 1 + (n - 1) // 4, 1 + (n - 1) // 2, 1 + 3 * (n - 1) // 4], r=r, bis=0, sb_shift=23,
             contig_bytes=32)
    f.update(over)
    n_sb = f.get("n_sb", ((f["n_lines"] - 1) >> f["sb_shift"]) + 1)
    fields = ([0x3158444E4957424D, 7, 384, f["n"], f["len_r"], f["primary"], f["n_lines"], f["n_ssa"], *f["C"],
               f["r"], 0, f["bis"], n_sb] + [0] * 64 + [0, f["sb_shift"], 0, 0, 0] + [0] * 6 +
              [f["contig_bytes"], 0] + [0])
    raw = bytearray(HEADER.pack(*fields))
    h = 1469598103934665603
    for b in raw[:-8]:
        h = ((h ^ b) * 1099511628211) & (2 ** 64 - 1)
    raw[-8:] = h.to_bytes(8, "little")
    return bytes(raw), f["n_lines"] * 128 + f["n_ssa"] * 8 + f["contig_bytes"]


@pytest.mark.parametrize("delta", [-8, 8])
def test_load_refuses_a_file_of_the_wrong_size(tmp_path, delta):
    """The file size is checked against the header before any device memory is allocated."""
    import paper_2606_15357_amd as mbw
    hd, payload = _header()
    p = tmp_path / "sized.mbw"
    p.write_bytes(hd + b"\0" * (payload + delta))
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.load(str(p))
    assert e.value.code == mbw.MBW_E_FORMAT
    assert ("truncated" if delta < 0 else "differs") in str(e.value)
    bad = bytearray(hd)
    bad[8] ^= 1                                        # version field: header checksum fails
    p.write_bytes(bytes(bad) + b"\0" * payload)
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.load(str(p))
    assert e.value.code == mbw.MBW_E_FORMAT and "header" in str(e.value)


@pytest.mark.parametrize("over", [
    dict(sb_shift=0), dict(sb_shift=24), dict(sb_shift=1, n=2 ** 13 + 1, len_r=2 ** 12, n_lines=22, n_ssa=1025),
    dict(n_sb=9), dict(primary=1001), dict(C=[0, 1, 500, 400, 900]), dict(C=[0, 0, 250, 500, 750]),
    dict(C=[0, 1, 250, 500, 1002]), dict(n=2 ** 39 + 1, len_r=2 ** 38, n_lines=(2 ** 39 + 1) // 384 + 1,
                                           n_ssa=2 ** 36 + 1, sb_shift=23), dict(len_r=7), dict(bis=2),
    dict(contig_bytes=0), dict(contig_bytes=28)])
def test_load_refuses_header_fields_beyond_the_builder_limits(tmp_path, over):
    """A header whose checksum is right but whose fields break the builder's limits (more than 8
    superblocks, which the kernels' LDS table cannot hold; a superblock shift outside 1..23; n at or
    above 2^39; primary >= n; C decreasing, without its single $ row or above n; n not 2|R|+1; a
    record table size that cannot hold one record or is not whole words) is refused before any
    device allocation, whatever follows it in the file."""
    import paper_2606_15357_amd as mbw
    hd, payload = _header(**over)
    p = tmp_path / "crafted.mbw"
    p.write_bytes(hd + b"\0" * min(payload, 1 << 20))
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.load(str(p))
    assert e.value.code == mbw.MBW_E_FORMAT and "header" in str(e.value)


def test_consistent_crafted_header_passes_the_field_checks(tmp_path):
    """The crafted header of the tests above is itself acceptable: with the wrong payload size the
    load gets past the field checks and fails on the size."""
    import paper_2606_15357_amd as mbw
    hd, payload = _header()
    p = tmp_path / "ok.mbw"
    p.write_bytes(hd + b"\0" * (payload + 8))
    with pytest.raises(mbw.MbwError) as e:
        mbw.Index.load(str(p))
    assert "differs" in str(e.value)
