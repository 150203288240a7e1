"""The C-ABI library loads and exports every function include/ovsign.h declares
(no compute calls: runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_names():
    hdr = open(os.path.join(ROOT, "include", "ovsign.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(ovs_[a-z_0-9]+)\s*\(", hdr)))


def test_header_declares_entry_points():
    names = header_names()
    for required in ("ovs_lattice_create", "ovs_set_links", "ovs_set_params", "ovs_apply",
                     "ovs_deflation_set", "ovs_sign_apply"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_0810_4228_amd as ovs
    lib = ovs.load()
    missing = [n for n in header_names() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(ovs.EXPORTED) == set(header_names())


def test_status_strings():
    import paper_0810_4228_amd as ovs
    assert ovs.status_string(0) == "ok"
    assert "invalid" in ovs.status_string(-1)


def test_binding_has_no_fallback(monkeypatch, tmp_path):
    import paper_0810_4228_amd as ovs
    monkeypatch.setattr(ovs, "_lib", None)
    monkeypatch.setattr(ovs, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        ovs.load()
