"""The C-ABI library and the oracle build here (no GPU) and libhgv.so exports every
function include/hgv.h declares; the Python binding binds the same names.  No compute
call is made."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hgv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    names = re.findall(r"\b(hgv_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hgv_create", "hgv_zhegvx", "hgv_zhegvx_batched", "hgv_zpotrf", "hgv_zhegst",
                     "hgv_zhe2hb", "hgv_zhb2st", "hgv_dstedc", "hgv_zunmtr_q2", "hgv_zunmtr_q1",
                     "hgv_ztrsm_lh", "hgv_zhegvx_backward"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1207_1773_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_1207_1773_amd import build
        build.build()
    lib = ctypes.CDLL(LIB_PATH)
    missing = [nm for nm in declared_functions() if not hasattr(lib, nm)]
    assert not missing, missing


def test_binding_covers_the_header():
    import paper_1207_1773_amd as h
    names = declared_functions()
    assert sorted(h.EXPORTS) == names
    for nm in names:
        assert callable(getattr(h, nm)), nm


def test_status_strings_without_gpu():
    import paper_1207_1773_amd as h
    lib = h.load()
    lib.hgv_status_string.restype = ctypes.c_char_p
    for st in range(0, 8):
        assert isinstance(lib.hgv_status_string(st), bytes)


def test_oracle_builds():
    import oracle
    oracle.build()
    assert oracle._load() is not None
