"""CPU checks of the C-ABI: the library loads and exports every entry point
that include/fg.h declares (no compute call: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fg.h")).read()
    return sorted(set(re.findall(r"^(?:fg_status|const char \*)\s*(fg_\w+)\s*\(", src, re.M)))


def test_header_declares_boundary():
    names = declared_symbols()
    for required in ("fg_assemble", "fg_pcg_solve", "fg_cohesive_update", "fg_flow_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2410_17133_amd import fg
    path = fg.LIB_PATH
    if not os.path.exists(path):
        pytest.skip("libfg.so not built")
    L = ctypes.CDLL(path)
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing
    assert set(declared_symbols()) <= set(fg.SYMBOLS)


def test_binding_rejects_missing_library(tmp_path, monkeypatch):
    from paper_2410_17133_amd import fg
    monkeypatch.setattr(fg, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(fg, "_lib", None)
    with pytest.raises(fg.FgError):
        fg.lib()
