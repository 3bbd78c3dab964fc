"""CPU checks of the C ABI library: it loads, and exports every entry point
that include/lst.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lst.h")


def declared_entry_points():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lst_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for n in ("lst_create", "lst_load_geometry", "lst_load_model", "lst_build_objects",
              "lst_build_objects_batched", "lst_score", "lst_workspace_size", "lst_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2403_13166_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for n in declared_entry_points():
        assert hasattr(lib, n), n
    assert sorted(binding.EXPORTED) == declared_entry_points()
    # status strings need no device
    L = binding.lib()
    assert binding.lst_status_string(binding.LST_E_CAPACITY) == "capacity exceeded"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2403_13166_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError):
        binding.lib()


def test_runtime_requires_a_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2403_13166_amd.runtime import Builder
    with pytest.raises(RuntimeError):
        Builder(b"", b"", 0)


def test_product_code_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2403_13166_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", txt, re.M), f
                assert "lst_oracle" not in txt, f
