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


def _header(n=1000, r=8):
    """An index file header (the documented layout) with consistent fields and a valid header
    checksum, for an index of n rows without k-mer table, text or inverse-SA samples."""
    from mbw_helpers import HEADER
    n_lines = n // 384 + 1
    fields = [0x3158444E4957424D, 5, 384, n, (n - 1) // 2, 0, n_lines, (n + r - 1) // r, 0, 0, 0, 0, 0,
              r, 0, 0, ((n_lines - 1) >> 23) + 1] + [0] * 64 + [0, 0, 0, 0, 0] + [0] * 6 + [0]
    raw = bytearray(HEADER.pack(*fields))
    h = 1469598103934665603
    for b in raw[:-8]:
        h = ((h ^ b) * 1099511628211) & (2 ** 64 - 1)
    raw[-8:] = h.to_bytes(8, "little")
    return bytes(raw), n_lines * 128 + ((n + r - 1) // r) * 8


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
