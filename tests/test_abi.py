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


def test_small_eig_host():
    """The library's host eigensolver (Rayleigh-Ritz step) against numpy (no GPU)."""
    import numpy as np

    import paper_0810_4228_amd as ovs
    rng = np.random.default_rng(3)
    for n in (1, 2, 9, 48):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        lam, V = ovs.small_eig(A)
        assert np.abs(A @ V - V * lam).max() <= 1e-12 * np.abs(A).max()
        assert np.allclose(np.linalg.norm(V, axis=0), 1.0)
        assert np.abs(np.sort_complex(lam) - np.sort_complex(np.linalg.eigvals(A))).max() < 1e-11
    # defective-ish upper triangular with clustered diagonal
    T = np.triu(rng.standard_normal((20, 20)), 1) + np.diag(np.repeat([0.5, -0.5], 10) + 1e-3 * np.arange(20))
    lam, V = ovs.small_eig(T.astype(complex))
    assert np.abs(np.sort(lam.real) - np.sort(np.diag(T))).max() < 1e-9


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with status 2 and a
    message saying so, before touching a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
