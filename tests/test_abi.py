"""The C-ABI library loads and exports every symbol include/dcs.h declares
(CPU only: no compute call is made without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dcs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dcs_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    import paper_1610_05141_amd as m
    assert sorted(m.EXPORTED_SYMBOLS) == _declared()


def test_library_exports_every_declared_symbol():
    import paper_1610_05141_amd as m
    assert os.path.exists(m.LIB_PATH), "libdcs.so not built"
    L = ctypes.CDLL(m.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_status_strings_and_host_only_entry_points():
    import paper_1610_05141_amd as m
    L = m.lib()
    for code in range(7):
        assert L.dcs_status_string(code)
    # Host-side computations that need no device.
    assert m.bernoulli_capacity_hint(0.01, 1 << 36) > int(0.01 * (1 << 36))
    assert m.bernoulli_capacity_hint(1.0, 100) == 100


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1610_05141_amd as m
    monkeypatch.setattr(m, "_lib", None)
    monkeypatch.setattr(m, "LIB_PATH", str(tmp_path / "nope.so"))
    try:
        m.lib()
    except FileNotFoundError:
        pass
    else:
        raise AssertionError("expected FileNotFoundError")
