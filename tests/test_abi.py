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
