"""The C-ABI library loads and exports every symbol include/hgp.h declares
(no GPU needed: nothing here launches work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hgp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hgp_[a-z_]+)\s*\(", txt)) - {"hgp_alloc_fn", "hgp_free_fn"})


def test_header_declares_entry_points():
    names = _declared()
    for n in ["hgp_create", "hgp_load_csr", "hgp_set_limits", "hgp_coarsen", "hgp_refine", "hgp_evaluate",
              "hgp_get_partition", "hgp_get_phi", "hgp_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2605_20497_amd import LIB_PATH, EXPORTED
    if not os.path.exists(LIB_PATH):
        pytest.fail("libhgp.so is not built: run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    for n in _declared():
        assert hasattr(L, n), n
    assert sorted(EXPORTED) == _declared()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2605_20497_amd as P
    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        P.lib()
